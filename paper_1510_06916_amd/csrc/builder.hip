// DSSS construction on the GPU (Sec. III-A "Sharding"): every edge is placed in
// its sub-shard, sub-shards are destination-sorted (ties by source), shards are
// stored contiguously, and the offset tables are derived. The sort is a
// hand-written LSD radix sort over 64-bit keys whose bit fields are, from the
// top: destination tile, source interval, then destination within the tile and
// source within the interval (source first for the source-major ablation
// order). The edge word is the key's low L + t bits.
#include <algorithm>
#include <cstring>

#include "nxg_internal.h"

namespace nxg {
namespace {

constexpr int kRsBlock = 256;  // threads of the radix-sort kernels (4 wavefronts)
constexpr int kRsItems = 8;    // keys per thread per step
constexpr uint32_t kPad = 0xFFFFFFFFu;
constexpr uint32_t kMarker = 0x80000000u;
constexpr uint32_t kHeader = 0x40000000u;  // pair layout: names the run's source
constexpr uint32_t kPairW = 0x20000000u;   // pair layout: two destinations of that source

__device__ inline int lane_id() { return threadIdx.x & 63; }
__device__ inline uint64_t lanemask_lt() { return (1ull << lane_id()) - 1ull; }

// deg[id] += 1 for every valid lane of the wave, with one atomic per run of
// equal ids in consecutive lanes (sorted inputs put a vertex's edges side by
// side, so a hub's count no longer takes one contended atomic per edge). All
// 64 lanes must call it.
__device__ inline void add_degree_runs(int32_t* deg, uint32_t id, bool valid) {
    const int lane = lane_id();
    const uint32_t prev = (uint32_t)__shfl_up((int)id, 1);
    const bool prev_valid = __shfl_up((int)valid, 1) != 0;
    const bool head = valid && (lane == 0 || !prev_valid || prev != id);
    const uint64_t bound = __ballot(head) | __ballot(!valid);
    if (head) {
        const uint64_t after = lane == 63 ? 0ull : bound >> (lane + 1);
        const int len = after ? __builtin_ctzll(after) + 1 : 64 - lane;
        atomicAdd(&deg[id], len);
    }
}

// Lanes of the wavefront holding the same 8-bit digit as this lane.
__device__ inline uint64_t match_digit(uint32_t digit, uint64_t valid) {
    uint64_t peers = valid;
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        uint32_t bit = (digit >> b) & 1u;
        uint64_t bal = __ballot(bit);
        peers &= bit ? bal : ~bal;
    }
    return peers;
}

struct KeyGeom {
    int32_t n, I, T, P, L, t, order;
};

// Validates ids and forms keys; payload = input edge index. With sym != 0 the
// input is E followed by reverse(E) (2m keys). rev != 0 swaps src and dst.
__global__ void k_make_keys(const int32_t* __restrict__ src, const int32_t* __restrict__ dst,
                            int64_t m, int sym, int rev, KeyGeom g, uint64_t* __restrict__ keys,
                            uint32_t* __restrict__ vals, int32_t* __restrict__ err) {
    const int64_t total = sym ? 2 * m : m;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        int64_t k = e < m ? e : e - m;
        int32_t s = src[k], d = dst[k];
        if ((e >= m) != (rev != 0)) {
            int32_t x = s;
            s = d;
            d = x;
        }
        if (s < 0 || s >= g.n || d < 0 || d >= g.n) {
            atomicOr(err, 1);
            s = 0;
            d = 0;
        }
        uint32_t tau = (uint32_t)d >> g.t;
        uint32_t dt = (uint32_t)d & ((1u << g.t) - 1u);
        uint32_t i = (uint32_t)s / (uint32_t)g.I;
        uint32_t sl = (uint32_t)s - i * (uint32_t)g.I;
        uint64_t grp = (uint64_t)tau * (uint64_t)g.P + i;
        uint64_t low = g.order == NXG_ORDER_SRC ? (((uint64_t)sl << g.t) | dt)
                                                : (((uint64_t)dt << g.L) | sl);
        keys[e] = (grp << (g.t + g.L)) | low;
        if (vals) vals[e] = (uint32_t)k;
    }
}

// ---- LSD radix sort, 8-bit digits ---------------------------------------

__global__ __launch_bounds__(kRsBlock) void k_rs_count(const uint64_t* __restrict__ keys,
                                                        int64_t m, int64_t per_block, int shift,
                                                        uint32_t* __restrict__ hist, int nb) {
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t b0 = (int64_t)blockIdx.x * per_block;
    const int64_t b1 = min(m, b0 + per_block);
    for (int64_t e0 = b0; e0 < b1; e0 += kRsBlock) {
        int64_t e = e0 + threadIdx.x;
        bool valid = e < b1;
        uint32_t dig = valid ? (uint32_t)(keys[e] >> shift) & 255u : 0u;
        uint64_t peers = match_digit(dig, __ballot(valid));
        if (valid && (peers & lanemask_lt()) == 0) atomicAdd(&h[dig], (uint32_t)__popcll(peers));
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * nb + blockIdx.x] = h[threadIdx.x];
}

// Exclusive scan of N uint32 counts into int64 offsets, one block of 1024.
// Exclusive prefix sums of N uint32 counts into int64 offsets, in three
// launches: each block scans its segment of kScanSeg counts (read and written
// through LDS, so global accesses are coalesced) and stores the segment's
// total; one block scans the totals; every element then adds its segment's
// offset.
constexpr int kScanSeg = 4096;  // counts per block: 1024 threads x 4

__global__ __launch_bounds__(1024) void k_scan_seg(const uint32_t* __restrict__ in, int64_t* __restrict__ out,
                                                   int64_t N, int64_t* __restrict__ seg_total) {
    __shared__ uint32_t v[kScanSeg];
    __shared__ int64_t part[1024];
    const int64_t s0 = (int64_t)blockIdx.x * kScanSeg;
    for (int i = threadIdx.x; i < kScanSeg; i += 1024) v[i] = s0 + i < N ? in[s0 + i] : 0u;
    __syncthreads();
    const int a = threadIdx.x * 4;
    int64_t sum = (int64_t)v[a] + v[a + 1] + v[a + 2] + v[a + 3];
    part[threadIdx.x] = sum;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const int64_t x = threadIdx.x >= off ? part[threadIdx.x - off] : 0;
        __syncthreads();
        part[threadIdx.x] += x;
        __syncthreads();
    }
    int64_t run = threadIdx.x ? part[threadIdx.x - 1] : 0;
    int64_t ex[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        ex[k] = run;
        run += v[a + k];
    }
    __syncthreads();
    __shared__ int64_t res[kScanSeg / 2];
    // write the 4096 results in two halves through LDS, coalesced
    for (int h = 0; h < 2; ++h) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int i = a + k - h * (kScanSeg / 2);
            if (i >= 0 && i < kScanSeg / 2) res[i] = ex[k];
        }
        __syncthreads();
        for (int i = threadIdx.x; i < kScanSeg / 2; i += 1024) {
            const int64_t gi = s0 + h * (kScanSeg / 2) + i;
            if (gi < N) out[gi] = res[i];
        }
        __syncthreads();
    }
    if (threadIdx.x == 1023) seg_total[blockIdx.x] = part[1023];
}

// Exclusive scan of the segment totals in place (one block); the grand total
// to *total when given.
__global__ __launch_bounds__(1024) void k_scan_totals(int64_t* __restrict__ seg, int nseg,
                                                      int64_t* __restrict__ total) {
    __shared__ int64_t part[1024];
    const int per = (nseg + 1023) / 1024;
    const int a = threadIdx.x * per, b = min(nseg, a + per);
    int64_t sum = 0;
    for (int i = a; i < b; ++i) sum += seg[i];
    part[threadIdx.x] = sum;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const int64_t x = threadIdx.x >= off ? part[threadIdx.x - off] : 0;
        __syncthreads();
        part[threadIdx.x] += x;
        __syncthreads();
    }
    int64_t run = threadIdx.x ? part[threadIdx.x - 1] : 0;
    for (int i = a; i < b; ++i) {
        const int64_t x = seg[i];
        seg[i] = run;
        run += x;
    }
    if (total && threadIdx.x == 1023) *total = part[1023];
}

__global__ void k_scan_add(int64_t* __restrict__ out, int64_t N, const int64_t* __restrict__ seg) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x)
        out[i] += seg[i / kScanSeg];
}

// out[i] = sum of in[0, i) for i < N; *total (device, nullable) = sum of all.
void scan_u32(const uint32_t* in, int64_t* out, int64_t N, int64_t* total, hipStream_t s) {
    const int nseg = (int)std::max<int64_t>(1, (N + kScanSeg - 1) / kScanSeg);
    DevBuf seg;
    seg.alloc(sizeof(int64_t) * nseg, s);
    hipLaunchKernelGGL(k_scan_seg, dim3(nseg), dim3(1024), 0, s, in, out, N, seg.as<int64_t>());
    NXG_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_scan_totals, dim3(1), dim3(1024), 0, s, seg.as<int64_t>(), nseg, total);
    NXG_CHECK_LAUNCH();
    if (nseg > 1) {
        hipLaunchKernelGGL(k_scan_add, dim3((unsigned)std::min<int64_t>((N + 255) / 256, 8192)), dim3(256), 0, s, out, N, seg.as<int64_t>());
        NXG_CHECK_LAUNCH();
    }
}

// Stable scatter: inside a block keys are ranked in input order (step, thread).
template <bool kVal>
__global__ __launch_bounds__(kRsBlock) void k_rs_scatter(
    const uint64_t* __restrict__ kin, const uint32_t* __restrict__ vin,
    uint64_t* __restrict__ kout, uint32_t* __restrict__ vout, int64_t m, int64_t per_block,
    int shift, const int64_t* __restrict__ offs, int nb) {
    __shared__ int64_t run[256];
    __shared__ uint32_t wc[4][256];
    __shared__ int64_t wo[4][256];
    const int tid = threadIdx.x, wave = tid >> 6;
    run[tid] = offs[(int64_t)tid * nb + blockIdx.x];
#pragma unroll
    for (int w = 0; w < 4; ++w) wc[w][tid] = 0;
    __syncthreads();
    const int64_t b0 = (int64_t)blockIdx.x * per_block;
    const int64_t b1 = min(m, b0 + per_block);
    for (int64_t s0 = b0; s0 < b1; s0 += (int64_t)kRsBlock * kRsItems) {
        uint64_t key[kRsItems];
        uint32_t val[kRsItems];
#pragma unroll
        for (int k = 0; k < kRsItems; ++k) {
            int64_t e = s0 + (int64_t)k * kRsBlock + tid;
            key[k] = e < b1 ? kin[e] : 0ull;
            val[k] = (kVal && e < b1) ? vin[e] : 0u;
        }
#pragma unroll
        for (int k = 0; k < kRsItems; ++k) {
            int64_t e = s0 + (int64_t)k * kRsBlock + tid;
            bool valid = e < b1;
            uint32_t dig = (uint32_t)(key[k] >> shift) & 255u;
            uint64_t peers = match_digit(dig, __ballot(valid));
            uint64_t lower = peers & lanemask_lt();
            if (valid && lower == 0) wc[wave][dig] = (uint32_t)__popcll(peers);
            __syncthreads();
            {
                int64_t r = run[tid];
#pragma unroll
                for (int w = 0; w < 4; ++w) {
                    wo[w][tid] = r;
                    r += wc[w][tid];
                    wc[w][tid] = 0;
                }
                run[tid] = r;
            }
            __syncthreads();
            if (valid) {
                int64_t pos = wo[wave][dig] + __popcll(lower);
                kout[pos] = key[k];
                if (kVal) vout[pos] = val[k];
            }
        }
    }
}

// ---- de-duplication of a sorted key array (stable compaction) -----------

__global__ __launch_bounds__(kRsBlock) void k_uniq_count(const uint64_t* __restrict__ keys,
                                                          int64_t m, int64_t per_block,
                                                          uint32_t* __restrict__ cnt) {
    __shared__ uint32_t c;
    if (threadIdx.x == 0) c = 0;
    __syncthreads();
    const int64_t b0 = (int64_t)blockIdx.x * per_block;
    const int64_t b1 = min(m, b0 + per_block);
    uint32_t mine = 0;
    for (int64_t e = b0 + threadIdx.x; e < b1; e += kRsBlock)
        mine += (e == 0 || keys[e] != keys[e - 1]) ? 1u : 0u;
    atomicAdd(&c, mine);
    __syncthreads();
    if (threadIdx.x == 0) cnt[blockIdx.x] = c;
}

template <bool kVal>
__global__ __launch_bounds__(kRsBlock) void k_uniq_scatter(
    const uint64_t* __restrict__ kin, const uint32_t* __restrict__ vin,
    uint64_t* __restrict__ kout, uint32_t* __restrict__ vout, int64_t m, int64_t per_block,
    const int64_t* __restrict__ boff) {
    __shared__ uint32_t wsum[4];
    __shared__ int64_t run;
    const int tid = threadIdx.x, wave = tid >> 6;
    if (tid == 0) run = boff[blockIdx.x];
    __syncthreads();
    const int64_t b0 = (int64_t)blockIdx.x * per_block;
    const int64_t b1 = min(m, b0 + per_block);
    for (int64_t e0 = b0; e0 < b1; e0 += kRsBlock) {
        int64_t e = e0 + tid;
        bool keep = e < b1 && (e == 0 || kin[e] != kin[e - 1]);
        uint64_t bal = __ballot(keep);
        if (lane_id() == 0) wsum[wave] = (uint32_t)__popcll(bal);
        __syncthreads();
        int64_t before = run;
        for (int w = 0; w < wave; ++w) before += wsum[w];
        if (keep) {
            int64_t pos = before + __popcll(bal & lanemask_lt());
            kout[pos] = kin[e];
            if (kVal) vout[pos] = vin[e];
        }
        __syncthreads();
        if (tid == 0) run += wsum[0] + wsum[1] + wsum[2] + wsum[3];
        __syncthreads();
    }
}

// ---- layout ---------------------------------------------------------------

__global__ void k_outdeg(const uint64_t* __restrict__ keys, int64_t m, KeyGeom g,
                         int32_t* __restrict__ deg) {
    // wave-uniform loop: every lane reaches the wave operations of add_degree_runs
    for (int64_t e0 = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63); e0 < m;
         e0 += (int64_t)gridDim.x * blockDim.x) {
        const int64_t e = e0 + lane_id();
        const bool valid = e < m;
        uint32_t id = 0;
        if (valid) {
            uint64_t k = keys[e];
            uint32_t i = (uint32_t)((k >> (g.t + g.L)) % (uint64_t)g.P);
            uint32_t sl = g.order == NXG_ORDER_SRC ? (uint32_t)(k >> g.t) & ((1u << g.L) - 1u)
                                                   : (uint32_t)k & ((1u << g.L) - 1u);
            id = i * (uint32_t)g.I + sl;
        }
        add_degree_runs(deg, id, valid);
    }
}

// group_edge[g] = first sorted index whose group is >= g, for g in [0, G].
__global__ void k_group_bounds(const uint64_t* __restrict__ keys, int64_t m, int64_t G, int sh,
                               int64_t* __restrict__ gbeg) {
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g <= G;
         g += (int64_t)gridDim.x * blockDim.x) {
        int64_t lo = 0, hi = m;
        while (lo < hi) {
            int64_t mid = (lo + hi) >> 1;
            if ((int64_t)(keys[mid] >> sh) < g)
                lo = mid + 1;
            else
                hi = mid;
        }
        gbeg[g] = lo;
    }
}

// One block per tile: word offsets of the tile's groups (relative to the
// tile), the tile's word count and its edge count.
// With pw (pair layout) a group's words are the marker plus what its edges
// emit, pw[end] - pw[begin]; otherwise one word per edge plus the marker.
__device__ inline int64_t group_words(const int64_t* __restrict__ gbeg,
                                      const int64_t* __restrict__ pw, int64_t g) {
    const int64_t c = gbeg[g + 1] - gbeg[g];
    if (!c) return 0;
    return 1 + (pw ? pw[gbeg[g + 1]] - pw[gbeg[g]] : c);
}

__global__ __launch_bounds__(1024) void k_tile_words(const int64_t* __restrict__ gbeg, int P,
                                                     const int64_t* __restrict__ pw,
                                                     int64_t* __restrict__ gword,
                                                     int64_t* __restrict__ tile_words,
                                                     int64_t* __restrict__ tile_edges) {
    __shared__ int64_t part[1024];
    const int64_t tau = blockIdx.x;
    const int64_t g0 = tau * P;
    const int per = (P + 1023) / 1024;
    const int a = threadIdx.x * per, b = min(P, a + per);
    int64_t s = 0;
    for (int i = a; i < b; ++i) s += group_words(gbeg, pw, g0 + i);
    part[threadIdx.x] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        int64_t v = threadIdx.x >= off ? part[threadIdx.x - off] : 0;
        __syncthreads();
        part[threadIdx.x] += v;
        __syncthreads();
    }
    int64_t run = threadIdx.x ? part[threadIdx.x - 1] : 0;
    for (int i = a; i < b; ++i) {
        gword[g0 + i] = run;
        run += group_words(gbeg, pw, g0 + i);
    }
    if (threadIdx.x == 1023) {
        tile_words[tau] = part[1023];
        tile_edges[tau] = gbeg[g0 + P] - gbeg[g0];
    }
}

__global__ void k_group_word_abs(int64_t* __restrict__ gword, const int64_t* __restrict__ tchunk,
                                 int64_t G, int P, int C, int64_t total_words) {
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g <= G;
         g += (int64_t)gridDim.x * blockDim.x) {
        if (g == G)
            gword[g] = total_words;
        else
            gword[g] += tchunk[g / P] * (int64_t)C;
    }
}

template <class T>
__global__ void k_fill(T* __restrict__ p, int64_t n, T v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_scatter_words(const uint64_t* __restrict__ keys,
                                const uint32_t* __restrict__ vals, int64_t m, int sh, int P,
                                const int64_t* __restrict__ gbeg,
                                const int64_t* __restrict__ gword, uint32_t* __restrict__ words,
                                int32_t* __restrict__ perm, const float* __restrict__ win,
                                float* __restrict__ wout) {
    const uint64_t low = (1ull << sh) - 1ull;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m;
         e += (int64_t)gridDim.x * blockDim.x) {
        uint64_t k = keys[e];
        int64_t g = (int64_t)(k >> sh);
        int64_t pos = gword[g] + 1 + (e - gbeg[g]);
        words[pos] = (uint32_t)(k & low);
        if (perm) perm[pos] = (int32_t)vals[e];
        if (wout) wout[pos] = win[vals[e]];
    }
}

__global__ void k_markers(const int64_t* __restrict__ gbeg, const int64_t* __restrict__ gword,
                          int64_t G, int P, uint32_t* __restrict__ words) {
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < G;
         g += (int64_t)gridDim.x * blockDim.x) {
        if (gbeg[g + 1] > gbeg[g]) words[gword[g]] = kMarker | (uint32_t)(g % P);
    }
}

// ---- pair layout (NXG_BUILD_PAIRS, source order) ---------------------------
// A run is the edges of one source into one tile: equal key >> t, consecutive
// in the sorted keys. An edge at an even index pairs with the next edge when
// that one is of the same run (one word: kPairW | dst | dst' << 14), and the
// run's first pair is preceded by a header word (kHeader | source field). An
// edge neither pairing nor paired keeps its plain word. Every flag is decided
// from the edge's neighbours, so the words of an edge are known locally.
struct PairFlags {
    bool hdr, pair, plain;
};
__device__ inline PairFlags pair_flags(const uint64_t* __restrict__ keys, int64_t m, int t, int64_t e) {
    const uint64_t r = keys[e] >> t;
    const bool sn = e + 1 < m && (keys[e + 1] >> t) == r;
    const bool sp = e > 0 && (keys[e - 1] >> t) == r;
    const bool sp2 = e > 1 && (keys[e - 2] >> t) == r;
    const bool even = (e & 1) == 0;
    PairFlags f;
    f.pair = even && sn;
    f.plain = even ? !sn : !sp;
    f.hdr = f.pair && (!sp || !sp2);
    return f;
}
constexpr int kPB = 4096;  // sorted edges per block of the word-count scan

// Words emitted by each block of kPB sorted edges.
__global__ __launch_bounds__(256) void k_pair_count(const uint64_t* __restrict__ keys, int64_t m, int t,
                                                    int64_t* __restrict__ bsum) {
    __shared__ int64_t red[4];
    int64_t s = 0;
    for (int i = threadIdx.x; i < kPB; i += 256) {
        const int64_t e = (int64_t)blockIdx.x * kPB + i;
        if (e < m) {
            const PairFlags f = pair_flags(keys, m, t, e);
            s += (int)f.hdr + (int)f.pair + (int)f.plain;
        }
    }
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if (lane_id() == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) bsum[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// pw[e] = words emitted by sorted edges [0, e), for e in [0, m]; boff holds the
// blocks' exclusive offsets (boff[nblocks] = total). Thread j of a block takes
// 16 consecutive edges.
__global__ __launch_bounds__(256) void k_pair_prefix(const uint64_t* __restrict__ keys, int64_t m, int t,
                                                     const int64_t* __restrict__ boff,
                                                     int64_t nblocks, int64_t* __restrict__ pw) {
    __shared__ int64_t wsum[4];
    const int64_t e0 = (int64_t)blockIdx.x * kPB + threadIdx.x * 16;
    int c[16];
    int64_t s = 0;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        const int64_t e = e0 + k;
        c[k] = 0;
        if (e < m) {
            const PairFlags f = pair_flags(keys, m, t, e);
            c[k] = (int)f.hdr + (int)f.pair + (int)f.plain;
        }
        s += c[k];
    }
    const int lane = lane_id(), wave = threadIdx.x >> 6;
    int64_t v = s;  // inclusive scan over the wave
    for (int o = 1; o < 64; o <<= 1) {
        const int64_t a = __shfl_up(v, o);
        if (lane >= o) v += a;
    }
    if (lane == 63) wsum[wave] = v;
    __syncthreads();
    int64_t run = boff[blockIdx.x] + v - s;
    for (int w = 0; w < wave; ++w) run += wsum[w];
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        const int64_t e = e0 + k;
        if (e < m) pw[e] = run;
        run += c[k];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) pw[m] = boff[nblocks];
}

// Writes the words of the pair layout (markers and padding come separately).
__global__ void k_pair_words(const uint64_t* __restrict__ keys, int64_t m, int sh, int t,
                             const int64_t* __restrict__ gbeg, const int64_t* __restrict__ gword,
                             const int64_t* __restrict__ pw, uint32_t* __restrict__ words) {
    const uint64_t low_mask = (1ull << sh) - 1ull;
    const uint32_t tmask = (1u << t) - 1u;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m;
         e += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t k = keys[e];
        const int64_t g = (int64_t)(k >> sh);
        int64_t pos = gword[g] + 1 + (pw[e] - pw[gbeg[g]]);
        const uint32_t low = (uint32_t)(k & low_mask);
        const PairFlags f = pair_flags(keys, m, t, e);
        if (f.hdr) words[pos++] = kHeader | (low >> t);
        if (f.pair)
            words[pos] = kPairW | (low & tmask) | (((uint32_t)keys[e + 1] & tmask) << 14);
        else if (f.plain)
            words[pos] = low;
    }
}

// Pair layout: the source field named by the header in effect at each chunk's
// first word, when that word is a pair (its run's header lies before the
// chunk); 0 otherwise. The walk back only crosses pairs of the same run.
__global__ void k_chunk_src(const uint32_t* __restrict__ words, int64_t n_chunks, int C,
                            int32_t* __restrict__ csrc) {
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n_chunks;
         c += (int64_t)gridDim.x * blockDim.x) {
        int64_t q = c * (int64_t)C;
        int32_t v = 0;
        if ((words[q] >> 29) == 1u) {
            while (q > 0 && (words[q] >> 29) == 1u) --q;
            if ((words[q] >> 30) == 1u) v = (int32_t)(words[q] & ~kHeader);
        }
        csrc[c] = v;
    }
}

// Largest group g in [g0, g0 + P) with gword[g] <= pos (gword is monotone).
__device__ inline int64_t last_group_at(const int64_t* gword, int64_t g0, int P, int64_t pos) {
    int64_t lo = g0, hi = g0 + P;  // answer in [g0, g0+P)
    while (hi - lo > 1) {
        int64_t mid = (lo + hi) >> 1;
        if (gword[mid] <= pos)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

// Per chunk: the source interval in effect at its first word, and its tile.
__global__ void k_chunk_rows(const int64_t* __restrict__ tchunk, int n_tiles,
                             const int64_t* __restrict__ gword, int P, int C,
                             int64_t n_chunks, int32_t* __restrict__ crow,
                             int32_t* __restrict__ ctile) {
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n_chunks;
         c += (int64_t)gridDim.x * blockDim.x) {
        // tile owning chunk c: last tau with tchunk[tau] <= c
        int lo = 0, hi = n_tiles;
        while (hi - lo > 1) {
            int mid = (lo + hi) >> 1;
            if (tchunk[mid] <= c)
                lo = mid;
            else
                hi = mid;
        }
        const int64_t g0 = (int64_t)lo * P;
        const int64_t first = c * (int64_t)C;
        // a chunk's first word precedes the tile's padding, where trailing empty
        // groups sit, so the search lands on the non-empty group in effect
        crow[c] = (int32_t)(last_group_at(gword, g0, P, first) - g0);
        ctile[c] = lo;
    }
}

// Decodes the stream back to edges (one thread per chunk), for export, and
// counts the edges of every logical sub-shard SS_{i.j} (index j*P + i).
__global__ void k_decode(const uint32_t* __restrict__ words, const int64_t* __restrict__ tchunk,
                         int n_tiles, const int32_t* __restrict__ crow,
                         const int64_t* __restrict__ gbeg, const int64_t* __restrict__ gword,
                         KeyGeom g, int C, int64_t n_chunks, const int32_t* __restrict__ perm_in,
                         int32_t* __restrict__ osrc, int32_t* __restrict__ odst,
                         int32_t* __restrict__ operm, unsigned long long* __restrict__ lcount) {
    const uint32_t lmask = (1u << g.L) - 1u, tmask = (1u << g.t) - 1u;
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n_chunks;
         c += (int64_t)gridDim.x * blockDim.x) {
        int lo = 0, hi = n_tiles;
        while (hi - lo > 1) {
            int mid = (lo + hi) >> 1;
            if (tchunk[mid] <= c)
                lo = mid;
            else
                hi = mid;
        }
        const int64_t tau = lo;
        const int64_t g0 = tau * g.P;
        const int64_t tbase = tau << g.t;
        int64_t row = crow[c];
        for (int64_t pos = c * (int64_t)C; pos < (c + 1) * (int64_t)C; ++pos) {
            uint32_t w = words[pos];
            if (w & kMarker) {
                row = w & ~kMarker;
                continue;
            }
            int64_t grp = g0 + row;
            int64_t e = gbeg[grp] + (pos - gword[grp] - 1);
            uint32_t sl = g.order == NXG_ORDER_SRC ? (w >> g.t) & lmask : w & lmask;
            uint32_t dt = g.order == NXG_ORDER_SRC ? w & tmask : (w >> g.L) & tmask;
            int64_t sv = row * g.I + sl, dv = tbase + dt;
            if (osrc) osrc[e] = (int32_t)sv;
            if (odst) odst[e] = (int32_t)dv;
            if (operm) operm[e] = perm_in[pos];
            if (lcount) atomicAdd(&lcount[(dv / g.I) * g.P + row], 1ull);
        }
    }
}

__global__ __launch_bounds__(1024) void k_scan_i64_inplace_excl(int64_t* __restrict__ a,
                                                                int64_t N) {
    // a[0..N) counts -> a[0..N] exclusive offsets (a[N] = total); one block.
    __shared__ int64_t part[1024];
    const int64_t per = (N + 1023) / 1024;
    const int64_t lo = threadIdx.x * per, hi = min(N, lo + per);
    int64_t s = 0;
    for (int64_t i = lo; i < hi; ++i) s += a[i];
    part[threadIdx.x] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        int64_t v = threadIdx.x >= off ? part[threadIdx.x - off] : 0;
        __syncthreads();
        part[threadIdx.x] += v;
        __syncthreads();
    }
    int64_t run = threadIdx.x ? part[threadIdx.x - 1] : 0;
    for (int64_t i = lo; i < hi; ++i) {
        int64_t v = a[i];
        a[i] = run;
        run += v;
    }
    __syncthreads();
    if (threadIdx.x == 0) a[N] = part[1023];
}

inline int grid_for(int64_t work, int threads = 256) {
    int64_t b = (work + threads - 1) / threads;
    if (b < 1) b = 1;
    if (b > 16384) b = 16384;
    return (int)b;
}

int ceil_log2(int64_t x) {
    int b = 0;
    while ((int64_t(1) << b) < x) ++b;
    return b;
}

// Sorts keys (and optional payload) in place; returns which buffer holds the result.
int radix_sort(DevBuf* kb, DevBuf* vb, int64_t m, int bits, hipStream_t s) {
    if (m <= 1 || bits <= 0) return 0;
    const int64_t tile = (int64_t)kRsBlock * kRsItems;
    int64_t nb64 = std::min<int64_t>(2048, (m + tile - 1) / tile);
    const int nb = (int)std::max<int64_t>(1, nb64);
    int64_t per_block = (m + nb - 1) / nb;
    per_block = (per_block + tile - 1) / tile * tile;
    DevBuf hist, offs;
    hist.alloc(sizeof(uint32_t) * 256 * nb, s);
    offs.alloc(sizeof(int64_t) * 256 * nb, s);
    int cur = 0;
    const bool hv = vb[0].p != nullptr;
    for (int shift = 0; shift < bits; shift += 8) {
        hipLaunchKernelGGL(k_rs_count, dim3(nb), dim3(kRsBlock), 0, s, kb[cur].as<uint64_t>(), m,
                           per_block, shift, hist.as<uint32_t>(), nb);
        NXG_CHECK_LAUNCH();
        scan_u32(hist.as<uint32_t>(), offs.as<int64_t>(), (int64_t)256 * nb, nullptr, s);
        if (hv)
            hipLaunchKernelGGL(k_rs_scatter<true>, dim3(nb), dim3(kRsBlock), 0, s,
                               kb[cur].as<uint64_t>(), vb[cur].as<uint32_t>(),
                               kb[cur ^ 1].as<uint64_t>(), vb[cur ^ 1].as<uint32_t>(), m,
                               per_block, shift, offs.as<int64_t>(), nb);
        else
            hipLaunchKernelGGL(k_rs_scatter<false>, dim3(nb), dim3(kRsBlock), 0, s,
                               kb[cur].as<uint64_t>(), (const uint32_t*)nullptr,
                               kb[cur ^ 1].as<uint64_t>(), (uint32_t*)nullptr, m, per_block,
                               shift, offs.as<int64_t>(), nb);
        NXG_CHECK_LAUNCH();
        cur ^= 1;
    }
    return cur;
}

// Stable de-duplication of sorted keys from buffer `cur` into `cur ^ 1`.
int64_t dedup(DevBuf* kb, DevBuf* vb, int cur, int64_t m, hipStream_t s) {
    if (m == 0) return 0;
    const int64_t tile = kRsBlock * 16;
    const int nb = (int)std::max<int64_t>(1, std::min<int64_t>(2048, (m + tile - 1) / tile));
    int64_t per_block = (m + nb - 1) / nb;
    DevBuf cnt, off;
    cnt.alloc(sizeof(uint32_t) * nb, s);
    off.alloc(sizeof(int64_t) * (nb + 1), s);
    hipLaunchKernelGGL(k_uniq_count, dim3(nb), dim3(kRsBlock), 0, s, kb[cur].as<uint64_t>(), m,
                       per_block, cnt.as<uint32_t>());
    NXG_CHECK_LAUNCH();
    scan_u32(cnt.as<uint32_t>(), off.as<int64_t>(), (int64_t)nb, off.as<int64_t>() + nb, s);
    if (vb[0].p)
        hipLaunchKernelGGL(k_uniq_scatter<true>, dim3(nb), dim3(kRsBlock), 0, s,
                           kb[cur].as<uint64_t>(), vb[cur].as<uint32_t>(),
                           kb[cur ^ 1].as<uint64_t>(), vb[cur ^ 1].as<uint32_t>(), m, per_block,
                           off.as<int64_t>());
    else
        hipLaunchKernelGGL(k_uniq_scatter<false>, dim3(nb), dim3(kRsBlock), 0, s,
                           kb[cur].as<uint64_t>(), (const uint32_t*)nullptr,
                           kb[cur ^ 1].as<uint64_t>(), (uint32_t*)nullptr, m, per_block,
                           off.as<int64_t>());
    NXG_CHECK_LAUNCH();
    int64_t mu = 0;
    NXG_HIP(hipMemcpyAsync(&mu, off.as<int64_t>() + nb, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    NXG_HIP(hipStreamSynchronize(s));
    return mu;
}

// ---- vertex renumbering (NXG_BUILD_RELABEL) --------------------------------

// Degree of every input id (out-degree; plus in-degree when both != 0). The
// ids index the array, so they are validated here.
__global__ void k_input_degree(const int32_t* __restrict__ src, const int32_t* __restrict__ dst,
                               int64_t m, int32_t n, int both, uint32_t* __restrict__ deg,
                               int32_t* __restrict__ err) {
    // wave-uniform loop: every lane reaches the wave operations of add_degree_runs
    for (int64_t e0 = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63); e0 < m;
         e0 += (int64_t)gridDim.x * blockDim.x) {
        const int64_t e = e0 + lane_id();
        bool valid = e < m;
        int32_t sv = 0, dv = 0;
        if (valid) {
            sv = src[e];
            dv = dst[e];
            if (sv < 0 || sv >= n || dv < 0 || dv >= n) {
                atomicOr(err, 1);
                valid = false;
            }
        }
        add_degree_runs(reinterpret_cast<int32_t*>(deg), (uint32_t)sv, valid);
        if (both) add_degree_runs(reinterpret_cast<int32_t*>(deg), (uint32_t)dv, valid);
    }
}

// Sort keys of the new order: dropped ids last (bit 63), then degree descending
// (when deg is given), then id ascending (bits 0..30).
__global__ void k_vertex_keys(const uint32_t* __restrict__ deg, const uint32_t* __restrict__ any,
                              int32_t n, uint64_t* __restrict__ keys) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t dropped = (any && any[v] == 0) ? 1ull : 0ull;
        const uint64_t high = deg ? (uint64_t)(0xFFFFFFFFu - deg[v]) : 0ull;
        keys[v] = (dropped << 63) | (high << 31) | (uint64_t)v;
    }
}

// Vertices with at least one edge (block partial counts).
__global__ __launch_bounds__(256) void k_count_kept(const uint32_t* __restrict__ any, int32_t n,
                                                    unsigned long long* __restrict__ count) {
    int c = 0;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x)
        c += any[v] != 0;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off);
    if (lane_id() == 0 && c) atomicAdd(count, (unsigned long long)c);
}

// new2old[k] = id at sorted position k (k < kept); old2new[id] = its position,
// or -1 for the ids sorted past the kept ones.
__global__ void k_vertex_maps(const uint64_t* __restrict__ sorted, int32_t n, int32_t kept,
                              int32_t* __restrict__ new2old, int32_t* __restrict__ old2new) {
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n;
         k += (int64_t)gridDim.x * blockDim.x) {
        const int32_t v = (int32_t)(sorted[k] & 0x7FFFFFFFu);
        if (k < kept) new2old[k] = v;
        old2new[v] = k < kept ? (int32_t)k : -1;
    }
}

__global__ void k_relabel_edges(const int32_t* __restrict__ src, const int32_t* __restrict__ dst,
                                int64_t m, const int32_t* __restrict__ old2new,
                                int32_t* __restrict__ src2, int32_t* __restrict__ dst2) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m;
         e += (int64_t)gridDim.x * blockDim.x) {
        src2[e] = old2new[src[e]];
        dst2[e] = old2new[dst[e]];
    }
}

}  // namespace

void plan_geometry(const nxg_build_desc& d, int device, bool spread, Layout& L) {
    const int64_t n = d.n;
    // default: 8-byte accumulators, enough for every program (PageRank sums in
    // FP64; BFS/WCC need only 4)
    int vb = d.value_bytes ? d.value_bytes : 8;
    if (vb < 1 || vb > 65536) fail(NXG_EINVAL, "value_bytes out of range");
    const int budget = lds_budget_bytes(device);
    int64_t tmax = 1;
    while (tmax * 2 * vb <= budget && tmax * 2 <= (1 << 20)) tmax *= 2;
    if (tmax * vb > budget) fail(NXG_EINVAL, "value_bytes too large for the LDS of one workgroup");
    int64_t I = d.interval;
    if (I < 0) fail(NXG_EINVAL, "interval must be >= 0");
    if (d.flags & NXG_BUILD_SCATTER) {
        // one tile over all vertices, source order; the interval shrinks until
        // the source and destination fields fit one word
        const int t = ceil_log2(n);
        if (t > 30) fail(NXG_EINVAL, "n too large for a SCATTER layout");
        const int64_t imax = std::min<int64_t>(n, (int64_t)1 << (31 - t));
        if (I == 0 || I > imax) I = imax;
        L.n = (int32_t)n;
        L.I = (int32_t)I;
        L.P = (int32_t)((n + I - 1) / I);
        L.L = ceil_log2(I);
        L.T = (int32_t)1 << t;
        L.t = t;
        L.n_tiles = 1;
        if (L.P > (1 << 27)) fail(NXG_EINVAL, "too many source intervals");
        L.order = NXG_ORDER_SRC;
        int64_t C = d.chunk ? d.chunk : 2048;
        if (C < 256 || C > 65536 || (C & (C - 1))) fail(NXG_EINVAL, "chunk must be a power of two in [256, 65536]");
        L.C = (int32_t)C;
        return;
    }
    if (I == 0) {
        // square DSSS with the interval equal to the largest tile that fits in LDS,
        // but never fewer than ~sqrt(n) vertices per interval (keeps P <= I)
        I = tmax;
        while (I * I < n) I *= 2;
        if (I > n) I = n;
    }
    if (I > n) I = n;
    L.n = (int32_t)n;
    L.I = (int32_t)I;
    L.P = (int32_t)((n + I - 1) / I);
    L.L = ceil_log2(I);
    if (L.L > 30) fail(NXG_EINVAL, "interval too large");
    int64_t T = d.tile;
    if (T < 0 || (T & (T - 1))) fail(NXG_EINVAL, "tile must be 0 or a power of two");
    if (T == 0) {
        T = tmax;
        // the planner's tile: the largest that fits, halved (down to 256) until
        // there are at least as many tiles as compute units, so a graph of a few
        // million vertices still occupies the whole chip (not for graphs that
        // share launches: those fill the chip together)
        int cus = 0;
        if (spread && hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess)
            while (T > 256 && (n + T - 1) / T < cus) T >>= 1;
    }
    if (T * vb > budget) fail(NXG_EINVAL, "tile * value_bytes exceeds the LDS of one workgroup");
    // destination tiles are global ranges [tau*T, (tau+1)*T); a tile may hold
    // several intervals (T > I) or part of one (T < I)
    while (T > 1 && (T >> 1) >= n) T >>= 1;
    while (L.L + ceil_log2(T) > 31) T >>= 1;
    if (T < 1) T = 1;
    L.T = (int32_t)T;
    L.t = ceil_log2(T);
    int64_t nt = (n + T - 1) / T;
    if (nt > (int64_t)1 << 24) fail(NXG_EINVAL, "too many destination tiles");
    int64_t G = nt * L.P;
    if (G > (int64_t)1 << 27) fail(NXG_EINVAL, "too many (tile, source interval) groups (P too large)");
    if (ceil_log2(G) + L.t + L.L > 64) fail(NXG_EINVAL, "key does not fit in 64 bits");
    L.n_tiles = (int32_t)nt;
    if (d.order != NXG_ORDER_DST && d.order != NXG_ORDER_SRC) fail(NXG_EINVAL, "unknown order");
    L.order = d.order;
    int64_t C = d.chunk;
    if (C == 0) {
        int64_t per_tile = (d.m + nt - 1) / std::max<int64_t>(nt, 1);
        C = per_tile >= 65536 ? 2048 : (per_tile >= 8192 ? 1024 : 256);
    }
    if (C < 256 || C > 65536 || (C & (C - 1))) fail(NXG_EINVAL, "chunk must be a power of two in [256, 65536]");
    L.C = (int32_t)C;
    if (d.flags & NXG_BUILD_PAIRS) {
        // two destination fields in a word under three flag bits, and plain
        // words clear of the flag bits
        if (L.order != NXG_ORDER_SRC) fail(NXG_EINVAL, "NXG_BUILD_PAIRS needs NXG_ORDER_SRC");
        if (L.t > 14) fail(NXG_EINVAL, "NXG_BUILD_PAIRS needs a tile of at most 16384 vertices");
        if (L.L + L.t > 29) fail(NXG_EINVAL, "NXG_BUILD_PAIRS needs L + t <= 29 (smaller interval)");
        L.pairs = true;
    }
}

void build_layout(const nxg_build_desc& d, bool reversed, hipStream_t s, Layout& L, bool spread) {
    int device = 0;
    NXG_HIP(hipGetDevice(&device));
    plan_geometry(d, device, spread, L);
    const bool sym = (d.flags & NXG_BUILD_SYMMETRIZE) != 0;
    const bool dedup_req = sym || (d.flags & NXG_BUILD_DEDUP);
    const bool want_perm = (d.flags & NXG_BUILD_KEEP_PERM) != 0;
    const bool want_w = d.d_weight != nullptr;
    const bool payload = want_perm || want_w;
    const int64_t mt = sym ? 2 * d.m : d.m;

    KeyGeom g{L.n, L.I, L.T, L.P, L.L, L.t, L.order};
    const int64_t G = (int64_t)L.n_tiles * L.P;
    const int sh = L.t + L.L;
    const int bits = ceil_log2(std::max<int64_t>(G, 2)) + sh;

    DevBuf kb[2], vb[2], err;
    kb[0].alloc(sizeof(uint64_t) * std::max<int64_t>(mt, 1), s);
    kb[1].alloc(sizeof(uint64_t) * std::max<int64_t>(mt, 1), s);
    if (payload) {
        vb[0].alloc(sizeof(uint32_t) * std::max<int64_t>(mt, 1), s);
        vb[1].alloc(sizeof(uint32_t) * std::max<int64_t>(mt, 1), s);
    }
    err.alloc(sizeof(int32_t), s);
    NXG_HIP(hipMemsetAsync(err.p, 0, sizeof(int32_t), s));
    if (mt > 0) {
        hipLaunchKernelGGL(k_make_keys, dim3(grid_for(mt)), dim3(256), 0, s, d.d_src, d.d_dst,
                           d.m, sym ? 1 : 0, reversed ? 1 : 0, g, kb[0].as<uint64_t>(),
                           payload ? vb[0].as<uint32_t>() : nullptr, err.as<int32_t>());
        NXG_CHECK_LAUNCH();
    }
    int32_t herr = 0;
    NXG_HIP(hipMemcpyAsync(&herr, err.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    NXG_HIP(hipStreamSynchronize(s));
    if (herr) fail(NXG_EINVAL, "edge id outside [0, n)");

    int cur = radix_sort(kb, vb, mt, bits, s);
    int64_t m = mt;
    if (dedup_req && mt > 0) {
        m = dedup(kb, vb, cur, mt, s);
        cur ^= 1;
    }
    L.m = m;
    const uint64_t* keys = kb[cur].as<uint64_t>();
    const uint32_t* vals = payload ? vb[cur].as<uint32_t>() : nullptr;

    // out-degree of the stored graph
    L.outdeg.alloc(sizeof(int32_t) * L.n, s);
    NXG_HIP(hipMemsetAsync(L.outdeg.p, 0, sizeof(int32_t) * L.n, s));
    if (m > 0) {
        hipLaunchKernelGGL(k_outdeg, dim3(grid_for(m)), dim3(256), 0, s, keys, m, g,
                           L.outdeg.as<int32_t>());
        NXG_CHECK_LAUNCH();
    }
    // groups
    L.group_edge.alloc(sizeof(int64_t) * (G + 1), s);
    L.group_word.alloc(sizeof(int64_t) * (G + 1), s);
    hipLaunchKernelGGL(k_group_bounds, dim3(grid_for(G + 1)), dim3(256), 0, s, keys, m, G, sh,
                       L.group_edge.as<int64_t>());
    NXG_CHECK_LAUNCH();
    // pair layout: words emitted before each sorted edge
    DevBuf pw;
    if (L.pairs) {
        const int64_t nbk = std::max<int64_t>(1, (m + kPB - 1) / kPB);
        DevBuf boff;
        boff.alloc(sizeof(int64_t) * (nbk + 1), s);
        pw.alloc(sizeof(int64_t) * (m + 1), s);
        if (m > 0) {
            hipLaunchKernelGGL(k_pair_count, dim3((unsigned)nbk), dim3(256), 0, s, keys, m, L.t,
                               boff.as<int64_t>());
            NXG_CHECK_LAUNCH();
        } else {
            NXG_HIP(hipMemsetAsync(boff.p, 0, sizeof(int64_t) * (nbk + 1), s));
        }
        hipLaunchKernelGGL(k_scan_i64_inplace_excl, dim3(1), dim3(1024), 0, s, boff.as<int64_t>(), nbk);
        NXG_CHECK_LAUNCH();
        hipLaunchKernelGGL(k_pair_prefix, dim3((unsigned)nbk), dim3(256), 0, s, keys, m, L.t,
                           boff.as<int64_t>(), nbk, pw.as<int64_t>());
        NXG_CHECK_LAUNCH();
    }
    DevBuf twords, tedges;
    twords.alloc(sizeof(int64_t) * L.n_tiles, s);
    tedges.alloc(sizeof(int64_t) * L.n_tiles, s);
    hipLaunchKernelGGL(k_tile_words, dim3(L.n_tiles), dim3(1024), 0, s,
                       L.group_edge.as<int64_t>(), L.P, L.pairs ? pw.as<int64_t>() : nullptr,
                       L.group_word.as<int64_t>(), twords.as<int64_t>(), tedges.as<int64_t>());
    NXG_CHECK_LAUNCH();
    std::vector<int64_t> hw(L.n_tiles), he(L.n_tiles);
    NXG_HIP(hipMemcpyAsync(hw.data(), twords.p, sizeof(int64_t) * L.n_tiles, hipMemcpyDeviceToHost, s));
    NXG_HIP(hipMemcpyAsync(he.data(), tedges.p, sizeof(int64_t) * L.n_tiles, hipMemcpyDeviceToHost, s));
    NXG_HIP(hipStreamSynchronize(s));
    L.h_tile_chunk.assign(L.n_tiles + 1, 0);
    L.h_tile_edges = he;
    L.max_tile_edges = 0;
    for (int tau = 0; tau < L.n_tiles; ++tau) {
        L.h_tile_chunk[tau + 1] = L.h_tile_chunk[tau] + (hw[tau] + L.C - 1) / L.C;
        L.max_tile_edges = std::max(L.max_tile_edges, he[tau]);
    }
    L.n_chunks = L.h_tile_chunk[L.n_tiles];
    L.n_words = L.n_chunks * L.C;
    L.tile_chunk.alloc(sizeof(int64_t) * (L.n_tiles + 1), s);
    NXG_HIP(hipMemcpyAsync(L.tile_chunk.p, L.h_tile_chunk.data(), sizeof(int64_t) * (L.n_tiles + 1),
                           hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_group_word_abs, dim3(grid_for(G + 1)), dim3(256), 0, s,
                       L.group_word.as<int64_t>(), L.tile_chunk.as<int64_t>(), G, L.P, L.C,
                       L.n_words);
    NXG_CHECK_LAUNCH();
    // words
    L.words.alloc(sizeof(uint32_t) * std::max<int64_t>(L.n_words, 1), s);
    if (L.n_words > 0) {
        hipLaunchKernelGGL(k_fill<uint32_t>, dim3(grid_for(L.n_words)), dim3(256), 0, s,
                           L.words.as<uint32_t>(), L.n_words, kPad);
        NXG_CHECK_LAUNCH();
    }
    if (want_perm) {
        L.perm.alloc(sizeof(int32_t) * std::max<int64_t>(L.n_words, 1), s);
        hipLaunchKernelGGL(k_fill<int32_t>, dim3(grid_for(L.n_words)), dim3(256), 0, s,
                           L.perm.as<int32_t>(), L.n_words, (int32_t)-1);
        NXG_CHECK_LAUNCH();
        L.has_perm = true;
    }
    if (want_w) {
        L.weight.alloc(sizeof(float) * std::max<int64_t>(L.n_words, 1), s);
        hipLaunchKernelGGL(k_fill<float>, dim3(grid_for(L.n_words)), dim3(256), 0, s,
                           L.weight.as<float>(), L.n_words, 0.0f);
        NXG_CHECK_LAUNCH();
        L.has_weight = true;
    }
    if (m > 0) {
        if (L.pairs)
            hipLaunchKernelGGL(k_pair_words, dim3(grid_for(m)), dim3(256), 0, s, keys, m, sh, L.t,
                               L.group_edge.as<int64_t>(), L.group_word.as<int64_t>(), pw.as<int64_t>(),
                               L.words.as<uint32_t>());
        else
            hipLaunchKernelGGL(k_scatter_words, dim3(grid_for(m)), dim3(256), 0, s, keys, vals, m, sh,
                               L.P, L.group_edge.as<int64_t>(), L.group_word.as<int64_t>(),
                               L.words.as<uint32_t>(), want_perm ? L.perm.as<int32_t>() : nullptr,
                               d.d_weight, want_w ? L.weight.as<float>() : nullptr);
        NXG_CHECK_LAUNCH();
        hipLaunchKernelGGL(k_markers, dim3(grid_for(G)), dim3(256), 0, s,
                           L.group_edge.as<int64_t>(), L.group_word.as<int64_t>(), G, L.P,
                           L.words.as<uint32_t>());
        NXG_CHECK_LAUNCH();
    }
    L.chunk_row.alloc(sizeof(int32_t) * std::max<int64_t>(L.n_chunks, 1), s);
    L.chunk_tile.alloc(sizeof(int32_t) * std::max<int64_t>(L.n_chunks, 1), s);
    if (L.n_chunks > 0) {
        hipLaunchKernelGGL(k_chunk_rows, dim3(grid_for(L.n_chunks)), dim3(256), 0, s,
                           L.tile_chunk.as<int64_t>(), L.n_tiles,
                           L.group_word.as<int64_t>(), L.P,
                           L.C, L.n_chunks, L.chunk_row.as<int32_t>(),
                           L.chunk_tile.as<int32_t>());
        NXG_CHECK_LAUNCH();
    }
    if (L.pairs) {
        L.chunk_src.alloc(sizeof(int32_t) * std::max<int64_t>(L.n_chunks, 1), s);
        if (L.n_chunks > 0) {
            hipLaunchKernelGGL(k_chunk_src, dim3(grid_for(L.n_chunks)), dim3(256), 0, s,
                               L.words.as<uint32_t>(), L.n_chunks, L.C, L.chunk_src.as<int32_t>());
            NXG_CHECK_LAUNCH();
        }
    }
    NXG_HIP(hipStreamSynchronize(s));
}

int32_t relabel_input(const nxg_build_desc& d, hipStream_t s, bool by_degree, bool drop,
                      DevBuf& new2old, DevBuf& old2new, DevBuf& src2, DevBuf& dst2) {
    const int32_t n = d.n;
    const int64_t m = d.m;
    DevBuf deg, any, err, cnt, kb[2], vb[2];
    deg.alloc(sizeof(uint32_t) * n, s);
    err.alloc(sizeof(int32_t), s);
    NXG_HIP(hipMemsetAsync(deg.p, 0, sizeof(uint32_t) * n, s));
    NXG_HIP(hipMemsetAsync(err.p, 0, sizeof(int32_t), s));
    // ordering degree: out-degree (plus in-degree for a symmetrised build)
    if (m > 0) {
        hipLaunchKernelGGL(k_input_degree, dim3(grid_for(m)), dim3(256), 0, s, d.d_src, d.d_dst, m,
                           n, (d.flags & NXG_BUILD_SYMMETRIZE) ? 1 : 0, deg.as<uint32_t>(),
                           err.as<int32_t>());
        NXG_CHECK_LAUNCH();
    }
    // with drop: any edge at all, in or out
    const uint32_t* anyp = nullptr;
    if (drop) {
        if (d.flags & NXG_BUILD_SYMMETRIZE) {
            anyp = deg.as<uint32_t>();
        } else {
            any.alloc(sizeof(uint32_t) * n, s);
            NXG_HIP(hipMemsetAsync(any.p, 0, sizeof(uint32_t) * n, s));
            if (m > 0) {
                hipLaunchKernelGGL(k_input_degree, dim3(grid_for(m)), dim3(256), 0, s, d.d_src, d.d_dst,
                                   m, n, 1, any.as<uint32_t>(), err.as<int32_t>());
                NXG_CHECK_LAUNCH();
            }
            anyp = any.as<uint32_t>();
        }
    }
    int32_t herr = 0;
    NXG_HIP(hipMemcpyAsync(&herr, err.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    NXG_HIP(hipStreamSynchronize(s));
    if (herr) fail(NXG_EINVAL, "edge id outside [0, n)");
    int32_t kept = n;
    if (drop) {
        cnt.alloc(sizeof(unsigned long long), s);
        NXG_HIP(hipMemsetAsync(cnt.p, 0, sizeof(unsigned long long), s));
        hipLaunchKernelGGL(k_count_kept, dim3(grid_for(n)), dim3(256), 0, s, anyp, n,
                           cnt.as<unsigned long long>());
        NXG_CHECK_LAUNCH();
        unsigned long long hk = 0;
        NXG_HIP(hipMemcpyAsync(&hk, cnt.p, sizeof(hk), hipMemcpyDeviceToHost, s));
        NXG_HIP(hipStreamSynchronize(s));
        kept = (int32_t)hk;
        if (kept < 1) fail(NXG_EINVAL, "NXG_BUILD_DEGREE needs at least one edge");
    }
    kb[0].alloc(sizeof(uint64_t) * n, s);
    kb[1].alloc(sizeof(uint64_t) * n, s);
    hipLaunchKernelGGL(k_vertex_keys, dim3(grid_for(n)), dim3(256), 0, s,
                       by_degree ? deg.as<uint32_t>() : (const uint32_t*)nullptr, anyp, n,
                       kb[0].as<uint64_t>());
    NXG_CHECK_LAUNCH();
    const int cur = radix_sort(kb, vb, n, 64, s);
    new2old.alloc(sizeof(int32_t) * kept, s);
    old2new.alloc(sizeof(int32_t) * n, s);
    hipLaunchKernelGGL(k_vertex_maps, dim3(grid_for(n)), dim3(256), 0, s, kb[cur].as<uint64_t>(), n, kept,
                       new2old.as<int32_t>(), old2new.as<int32_t>());
    NXG_CHECK_LAUNCH();
    src2.alloc(sizeof(int32_t) * std::max<int64_t>(m, 1), s);
    dst2.alloc(sizeof(int32_t) * std::max<int64_t>(m, 1), s);
    if (m > 0) {
        hipLaunchKernelGGL(k_relabel_edges, dim3(grid_for(m)), dim3(256), 0, s, d.d_src, d.d_dst, m,
                           old2new.as<int32_t>(), src2.as<int32_t>(), dst2.as<int32_t>());
        NXG_CHECK_LAUNCH();
    }
    NXG_HIP(hipStreamSynchronize(s));
    return kept;
}

void export_layout(const Layout& L, int64_t* d_offsets, int32_t* d_src, int32_t* d_dst,
                   int32_t* d_perm, hipStream_t s) {
    KeyGeom g{L.n, L.I, L.T, L.P, L.L, L.t, L.order};
    if (d_perm && !L.has_perm) fail(NXG_EINVAL, "export of perm needs NXG_BUILD_KEEP_PERM");
    const int64_t PP = (int64_t)L.P * L.P;
    if (d_offsets) NXG_HIP(hipMemsetAsync(d_offsets, 0, sizeof(int64_t) * (PP + 1), s));
    if ((d_offsets || d_src || d_dst || d_perm) && L.n_chunks > 0) {
        hipLaunchKernelGGL(k_decode, dim3(grid_for(L.n_chunks, 64)), dim3(64), 0, s,
                           L.words.as<uint32_t>(), L.tile_chunk.as<int64_t>(), L.n_tiles,
                           L.chunk_row.as<int32_t>(), L.group_edge.as<int64_t>(),
                           L.group_word.as<int64_t>(), g, L.C, L.n_chunks,
                           L.has_perm ? L.perm.as<int32_t>() : nullptr, d_src, d_dst, d_perm,
                           (unsigned long long*)d_offsets);
        NXG_CHECK_LAUNCH();
    }
    if (d_offsets) {
        hipLaunchKernelGGL(k_scan_i64_inplace_excl, dim3(1), dim3(1024), 0, s, d_offsets, PP);
        NXG_CHECK_LAUNCH();
    }
    NXG_HIP(hipStreamSynchronize(s));
}

}  // namespace nxg
