// One DSSS iteration on the GPU (Alg. 1 with the single-phase update of Alg. 5
// and, for destination tiles split over several workgroups, the two-phase
// update of Alg. 6).
//
// A workgroup owns one piece of one destination tile: its accumulators live in
// LDS, and its wavefronts stream the tile's edge words chunk by chunk. They
// follow the source-interval markers, gather the source values and add
// (PageRank) or min-reduce (BFS, WCC) into LDS -- the write-conflict-free
// destination ownership of Sec. III-D. The 64 lanes of a load take 64
// consecutive edges: in destination order runs of equal destination are summed
// across the wave before they reach LDS; in source order the lanes of a gather
// read adjacent sources. A tile handled by one
// workgroup applies the vertex update straight from LDS (single phase). A tile
// split into k pieces writes k partial arrays (the hub of Sec. III-B2), which a
// second launch sums in piece order and applies (two phase); a third launch
// reduces the per-iteration scalars (dangling mass, residual, activity) in a
// fixed order, so they are independent of scheduling.
#include <algorithm>
#include <memory>
#include <type_traits>
#include <cmath>
#include <cstring>

#include "nxg_internal.h"

namespace nxg {
// Chunks per work item when the caller does not choose: about one item per
// CU's share of the stream, but never so few that a piece's partial sums
// (slot_bytes, written and read back once) exceed an eighth of the stream
// bytes it covers.
int default_piece(int64_t chunks, int C, size_t slot_bytes, int cus) {
    const int64_t share = chunks / std::max(1, cus);
    const int64_t floor_ = (int64_t)(8 * slot_bytes / (4 * (size_t)C)) + 1;
    return (int)std::max<int64_t>(16, std::max(share, floor_));
}

namespace {

constexpr uint32_t kMarker = 0x80000000u;
constexpr uint32_t kNoDst = 0xFFFFFFFFu;  // decoded destination of a marker or padding word
constexpr int32_t kInf = INT32_MAX;
constexpr int kSpill = 64;  // LDS accumulators past the tile: lane l's discard slot T + l
// A split tile is finished in segments of kFinSeg vertices, one workgroup of
// kFinWG threads (one vertex per thread) each, so a heavy tile's FromHub is
// spread over many CUs and needs only kFinSeg accumulators of LDS.
constexpr int kFinSeg = 256, kFinWG = 256;
// workgroups of the two-step BFS output reduction
constexpr int kFinalBlocks = 256;

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ inline int lane_id() { return threadIdx.x & 63; }

// Third word of a raw buffer resource on gfx9-class GPUs (no format, no swizzle).
constexpr int kBufWord3 = 0x00020000;

// One sub-block of padding words (and of zero weights), read by loads that fall
// outside the edge stream so that no load needs a branch or a select. Never
// written; not const, so that they sit in global memory like the stream and a
// choice between the two stays a global load (a generic one would make the
// compiler wait for every load in flight before the next LDS operation).
__device__ __align__(16) uint32_t kPadWords[256] = {
#define NXG_PAD8 0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu
#define NXG_PAD64 NXG_PAD8, NXG_PAD8, NXG_PAD8, NXG_PAD8, NXG_PAD8, NXG_PAD8, NXG_PAD8, NXG_PAD8
    NXG_PAD64, NXG_PAD64, NXG_PAD64, NXG_PAD64
#undef NXG_PAD64
#undef NXG_PAD8
};
__device__ __align__(16) float kPadZeros[256] = {};

// A gathered value by byte offset from a buffer resource; offsets past the
// buffer's size read 0.
template <typename T>
__device__ inline T load_val(__amdgpu_buffer_rsrc_t r, uint32_t off);
template <>
__device__ inline float load_val<float>(__amdgpu_buffer_rsrc_t r, uint32_t off) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}
template <>
__device__ inline int32_t load_val<int32_t>(__amdgpu_buffer_rsrc_t r, uint32_t off) {
    return (int32_t)__builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0);
}
template <>
__device__ inline double load_val<double>(__amdgpu_buffer_rsrc_t r, uint32_t off) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
template <>
__device__ inline uint64_t load_val<uint64_t>(__amdgpu_buffer_rsrc_t r, uint32_t off) {
    return (uint64_t)__builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0);
}

struct Geo {
    const uint32_t* words;
    const int32_t* chunk_row;
    const int32_t* chunk_src;  // pair layout: header source at each chunk's first word
    const Item* items;
    const int32_t* deg;
    int32_t n, I, P, L, T, t, n_tiles, C;
    int32_t sshift, dshift;  // bit offsets of the source and destination fields
    int32_t order;           // NXG_ORDER_* of the stream
    // two-phase partials
    void* partial;
    double* tile_s;      // [n_sslots * 3]: per tile, then per finishing segment
    int32_t n_sslots;
    int32_t* tile_flag;  // [n_tiles]
    // compacted active chunk lists (BFS/WCC), nullable
    const int64_t* clist;
    const int32_t* ccount;
    // with lists: a split tile listing at most this many chunks is done whole
    // by its piece 0 in that round (no hub partials, no finishing segment work)
    int64_t split_min;
};

// Per-iteration control block in device memory.
struct Ctl {
    double* stats;        // [4 * (max_iters + 1)]: [k*4+0] scalar entering iteration k,
                          // [k*4+1] residual of iteration k, [k*4+2] norm, [k*4+3] changed
    int32_t* done;        // set once the tolerance is met (PageRank) / nothing changed
    int32_t k;            // iteration index
    double tol;
};

// ---------------------------------------------------------------------------
// Programs
// ---------------------------------------------------------------------------

// PageRank with W = 1/outdeg. The gathered array holds x_u / outdeg_u (x_u for
// dangling u, which is never gathered), so no separate x vector is kept.
// Destination sums accumulate in FP64 in LDS whatever the value type: on gfx950
// the LDS FP64 atomic add sustains several times the throughput of the FP32
// one, and the sums of high in-degree vertices keep FP64 accuracy.
template <typename V>
struct ProgPR {
    using acc_t = double;
    using val_t = V;
    static constexpr bool kSum = true, kWeights = false, kActivity = false;
    const V* cur;
    V* nxt;
    const V* tele;   // nullable: uniform
    V* xout;         // nullable: write x on this iteration
    double d;
    __device__ acc_t identity() const { return (acc_t)0; }
    __device__ acc_t from_val(V v, float) const { return (acc_t)v; }
    __device__ acc_t gather(uint32_t src, float w) const { return from_val(cur[src], w); }
    __device__ bool row_active(uint32_t) const { return true; }
    static __device__ bool converged(double resid, double, double tol) { return resid <= tol; }
    // the apply's loads, issued for several vertices before any is used
    struct Ld {
        V c, t;
    };
    __device__ Ld load(int64_t v) const { return Ld{cur[v], tele ? tele[v] : (V)0}; }
    // sv[0]: dangling mass of x^{k+1}; sv[1]: |x^{k+1} - x^k|_1; sv[2]: sum of x^{k+1}
    __device__ void apply(int64_t v, const Ld& l, acc_t acc, int32_t dg, double scal, int32_t n,
                          double* sv, int&) const {
        double xo = dg ? (double)l.c * dg : (double)l.c;
        double tv = tele ? (double)l.t : 1.0 / n;
        double xn = d * ((double)acc + scal / n) + (1.0 - d) * tv;
        V xr = (V)xn;
        sv[1] += fabs((double)xr - xo);
        sv[2] += (double)xr;
        if (dg == 0) sv[0] += (double)xr;
        nxt[v] = dg ? (V)((double)xr / dg) : xr;
        if (xout) xout[v] = xr;
    }
    __device__ void pass(int64_t v, int32_t dg) const {
        nxt[v] = cur[v];
        if (xout) xout[v] = dg ? (V)((double)cur[v] * dg) : cur[v];
    }
};

// Plain PageRank over the pair layout (NXG_BUILD_PAIRS): the same program; the
// iteration decodes header and pair words as well.
template <typename V>
struct ProgPRP : ProgPR<V> {
    static constexpr bool kPairs = true;
};

// Whether a program's stream is the pair layout.
template <class P, class = void>
struct pairs_of : std::false_type {};
template <class P>
struct pairs_of<P, std::void_t<decltype(P::kPairs)>> : std::bool_constant<P::kPairs> {};

// Mixed-phase update (Alg. 7, Sec. III-B3) with host memory as the slower
// tier: a PageRank program (plain or weighted) whose launch covers only the
// source intervals [r_lo, r_hi) of each tile, and whose items do one of three
// things with their sums: store them in a slot of g.partial (a shard hub in
// host memory, or a resident tile's device accumulators), add them into such a
// slot, or apply the update after adding hub slots [slot, slot + npieces).
// When a store or add item is one of npieces > 1 pieces of a heavy tile, the
// pieces add with device-scope atomics (a stored slot is cleared first).
// The apply reads the old value from `own` (the values of the tile's vertices,
// wherever they live), so a tile whose values are in host memory can gather
// resident sources.
constexpr int kMpuApply = 0, kMpuStore = 1, kMpuAdd = 2;
template <class Base>
struct ProgMPU : Base {
    static constexpr bool kRowRange = true;
    using V = typename Base::val_t;
    uint32_t r_lo, r_hi;
    int32_t mode;
    const V* own;  // the apply's old gathered values, by vertex id
    __device__ bool row_in(uint32_t r) const { return r - r_lo < r_hi - r_lo; }
    __device__ typename Base::Ld load(int64_t v) const {
        return typename Base::Ld{own[v], this->tele ? this->tele[v] : (V)0};
    }
};

// Whether a program restricts its launch to a range of source intervals.
template <class P, class = void>
struct row_range_of : std::false_type {};
template <class P>
struct row_range_of<P, std::void_t<decltype(P::kRowRange)>> : std::bool_constant<P::kRowRange> {};

// Whether a program's accumulators start from the current values and an edge
// into a destination that already holds a value is skipped (no gather).
template <class P, class = void>
struct early_exit_of : std::false_type {};
template <class P>
struct early_exit_of<P, std::void_t<decltype(P::kEarlyExit)>> : std::bool_constant<P::kEarlyExit> {};

// PageRank with the stored edge weights: gathers x_u and multiplies by w_e
// (FP64 accumulation as above).
template <typename V>
struct ProgPRW {
    using acc_t = double;
    using val_t = V;
    static constexpr bool kSum = true, kWeights = true, kActivity = false;
    const V* cur;
    V* nxt;
    const V* tele;
    V* xout;
    const float* w;  // [n_words] weights in stream order
    double d;
    __device__ acc_t identity() const { return (acc_t)0; }
    __device__ acc_t from_val(V v, float we) const { return (acc_t)we * (acc_t)v; }
    __device__ acc_t gather(uint32_t src, float we) const { return from_val(cur[src], we); }
    __device__ bool row_active(uint32_t) const { return true; }
    static __device__ bool converged(double resid, double, double tol) { return resid <= tol; }
    struct Ld {
        V c, t;
    };
    __device__ Ld load(int64_t v) const { return Ld{cur[v], tele ? tele[v] : (V)0}; }
    __device__ void apply(int64_t v, const Ld& l, acc_t acc, int32_t dg, double scal, int32_t n,
                          double* sv, int&) const {
        double xo = (double)l.c;
        double tv = tele ? (double)l.t : 1.0 / n;
        double xn = d * ((double)acc + scal / n) + (1.0 - d) * tv;
        V xr = (V)xn;
        sv[1] += fabs((double)xr - xo);
        sv[2] += (double)xr;
        if (dg == 0) sv[0] += (double)xr;
        nxt[v] = xr;
        if (xout) xout[v] = xr;
    }
    __device__ void pass(int64_t v, int32_t) const {
        nxt[v] = cur[v];
        if (xout) xout[v] = cur[v];
    }
};

// BFS (Alg. 3): a reached source offers level + 1; min-reduce.
struct ProgBFS {
    using acc_t = int32_t;
    using val_t = int32_t;
    static constexpr bool kSum = false, kWeights = false, kActivity = true;
    // Bottom-up early exit: rounds are level-synchronous, so an unreached
    // destination can only be offered level r + 1 in round r + 1 (a source with
    // a smaller level would have reached it in an earlier round). The first
    // offer it takes is therefore final, and so is the level of a vertex reached
    // before; the tile's accumulators start from the current levels and the
    // remaining edges into a destination that holds a level read nothing.
    static constexpr bool kEarlyExit = true;
    const int32_t* cur;
    int32_t* nxt;
    uint8_t* chg;  // [n >> bs] block flags: a vertex of the block changed in this round
    uint8_t* opn;  // [n >> bs] block flags: a vertex of the block is still unreached
    int32_t bs;    // log2 of the vertices per activity block
    __device__ acc_t identity() const { return kInf; }
    __device__ acc_t from_val(int32_t l, float) const { return l == kInf ? kInf : l + 1; }
    __device__ acc_t gather(uint32_t src, float w) const { return from_val(cur[src], w); }
    // Chunks none of whose sources changed in the previous round, or none of
    // whose destinations is still unreached, are left out of the compacted
    // chunk list; the edges of a kept chunk are all processed (an unchanged
    // source offers what it offered before, which cannot lower a destination).
    __device__ bool row_active(uint32_t) const { return true; }
    static __device__ bool converged(double, double, double) { return false; }
    struct Ld {
        int32_t c;
    };
    __device__ Ld load(int64_t v) const { return Ld{cur[v]}; }
    // flag bit 0: the level changed; bit 1: the vertex is still unreached
    __device__ void apply(int64_t v, const Ld& l, acc_t acc, int32_t, double, int32_t, double*,
                          int& flag) const {
        int32_t o = l.c;
        int32_t nv = acc < o ? acc : o;
        nxt[v] = nv;
        flag = (nv != o ? 1 : 0) | (nv == kInf ? 2 : 0);
    }
    __device__ void pass(int64_t v, int32_t) const { nxt[v] = cur[v]; }
};

// WCC by min-label propagation on the symmetrised graph.
struct ProgWCC {
    using acc_t = int32_t;
    using val_t = int32_t;
    static constexpr bool kSum = false, kWeights = false, kActivity = true;
    const int32_t* cur;
    int32_t* nxt;
    uint8_t* chg;  // [n >> bs] block flags: a vertex of the block changed in this round
    uint8_t* opn;  // unused (a label may fall in any round)
    int32_t bs;
    __device__ acc_t identity() const { return kInf; }
    __device__ acc_t from_val(int32_t l, float) const { return l; }
    __device__ acc_t gather(uint32_t src, float w) const { return from_val(cur[src], w); }
    // Chunks none of whose sources changed in the previous round are left out
    // of the compacted chunk list (see ProgBFS).
    __device__ bool row_active(uint32_t) const { return true; }
    static __device__ bool converged(double, double, double) { return false; }
    struct Ld {
        int32_t c;
    };
    __device__ Ld load(int64_t v) const { return Ld{cur[v]}; }
    // flag bit 0: the label changed
    __device__ void apply(int64_t v, const Ld& l, acc_t acc, int32_t, double, int32_t, double*,
                          int& flag) const {
        int32_t o = l.c;
        int32_t nv = acc < o ? acc : o;
        nxt[v] = nv;
        flag = nv != o ? 1 : 0;
    }
    __device__ void pass(int64_t v, int32_t) const { nxt[v] = cur[v]; }
};

// Up to 64 BFS at once, one per root: a vertex's state is the set of roots
// that have reached it (bit b: root b), gathered as a 64-bit mask and combined
// by OR. Rounds are level-synchronous: in round r a vertex gains exactly the
// roots at distance r (a root that reached an in-neighbour before round r - 1
// would have reached the vertex before round r), so its new bits take level r.
// Levels go to lev[v * B + b]; the mask is the monotone state of the ping-pong.
struct ProgMSBFS {
    using acc_t = uint64_t;
    using val_t = uint64_t;
    static constexpr bool kSum = false, kWeights = false, kActivity = true;
    const uint64_t* cur;
    uint64_t* nxt;
    uint8_t* chg;
    uint8_t* opn;  // unused
    int32_t bs;
    int32_t* lev;
    int32_t B;
    int32_t round;
    uint64_t full;  // the mask of all B roots
    __device__ acc_t identity() const { return 0ull; }
    __device__ acc_t from_val(uint64_t m, float) const { return m; }
    __device__ acc_t gather(uint32_t src, float w) const { return from_val(cur[src], w); }
    __device__ bool row_active(uint32_t) const { return true; }
    static __device__ bool converged(double, double, double) { return false; }
    struct Ld {
        uint64_t c;
    };
    __device__ Ld load(int64_t v) const { return Ld{cur[v]}; }
    __device__ void apply(int64_t v, const Ld& l, acc_t acc, int32_t, double, int32_t, double*,
                          int& flag) const {
        const uint64_t o = l.c;
        uint64_t nw = acc & ~o & full;
        nxt[v] = o | nw;
        flag = nw ? 1 : 0;
        while (nw) {
            lev[v * B + __builtin_ctzll(nw)] = round;
            nw &= nw - 1;
        }
    }
    __device__ void pass(int64_t v, int32_t) const { nxt[v] = cur[v]; }
};

// Strongly connected components (named among the targeted queries of
// Sec. IV-D, with no algorithm given) by colouring, in rounds over the
// vertices not yet assigned to a component:
//   forward  col[v] starts at v's caller id and takes the minimum over the
//            edges u -> v between unassigned vertices: at the fixed point it is
//            the smallest caller id among the unassigned vertices reaching v;
//   backward the vertex whose caller id is its colour (the colour's root)
//            joins; over the reversed layout v joins when an out-neighbour w
//            that joined has col[w] == col[v]. The joined vertices of colour c
//            are those of colour c that reach c: c's component, whose smallest
//            caller id is c (every member has the same ancestors);
//   assign   joined vertices take label col[v] and leave.
// An assigned vertex holds colour kInf, which offers nothing and never changes.
struct ProgSCCF {
    using acc_t = int32_t;
    using val_t = int32_t;
    static constexpr bool kSum = false, kWeights = false, kActivity = true;
    const int32_t* cur;
    int32_t* nxt;
    uint8_t* chg;
    uint8_t* opn;  // unused
    int32_t bs;
    __device__ acc_t identity() const { return kInf; }
    __device__ acc_t from_val(int32_t c, float) const { return c; }
    __device__ acc_t gather(uint32_t src, float w) const { return from_val(cur[src], w); }
    __device__ bool row_active(uint32_t) const { return true; }
    static __device__ bool converged(double, double, double) { return false; }
    struct Ld {
        int32_t c;
    };
    __device__ Ld load(int64_t v) const { return Ld{cur[v]}; }
    __device__ void apply(int64_t v, const Ld& l, acc_t acc, int32_t, double, int32_t, double*,
                          int& flag) const {
        const int32_t o = l.c;
        const int32_t nv = o == kInf ? kInf : (acc < o ? acc : o);
        nxt[v] = nv;
        flag = nv != o ? 1 : 0;
    }
    __device__ void pass(int64_t v, int32_t) const { nxt[v] = cur[v]; }
};

// The backward step on the reversed layout. A joined vertex holds
// kInf - 1 - col[v], any other kInf (colours are in [0, n), so the two never
// meet), and the minimum offered to v is kInf - 1 minus the largest colour
// among its joined out-neighbours. Along a forward edge v -> w between
// unassigned vertices col[w] <= col[v] (w has every ancestor of v), so v joins
// exactly when that minimum is kInf - 1 - col[v].
struct ProgSCCB {
    using acc_t = int32_t;
    using val_t = int32_t;
    static constexpr bool kSum = false, kWeights = false, kActivity = true;
    const int32_t* cur;
    int32_t* nxt;
    uint8_t* chg;
    uint8_t* opn;  // unused
    int32_t bs;
    const int32_t* col;
    __device__ acc_t identity() const { return kInf; }
    __device__ acc_t from_val(int32_t q, float) const { return q; }
    __device__ acc_t gather(uint32_t src, float w) const { return from_val(cur[src], w); }
    __device__ bool row_active(uint32_t) const { return true; }
    static __device__ bool converged(double, double, double) { return false; }
    struct Ld {
        int32_t q, c;
    };
    __device__ Ld load(int64_t v) const { return Ld{cur[v], col[v]}; }
    __device__ void apply(int64_t v, const Ld& l, acc_t acc, int32_t, double, int32_t, double*,
                          int& flag) const {
        const int32_t o = l.q;
        const int32_t nv = o != kInf ? o : ((l.c != kInf && acc == kInf - 1 - l.c) ? acc : kInf);
        nxt[v] = nv;
        flag = nv != o ? 1 : 0;
    }
    __device__ void pass(int64_t v, int32_t) const { nxt[v] = cur[v]; }
};

// Adjoint of weighted PageRank, iterated on the reversed graph: the gathered
// array is lambda (indexed by the forward destination), the edge carries the
// forward weight, and the tile owns forward sources u:
//   lambda'_u = g_u + d * sum_{e: u->v} w_e lambda_v + d * [outdeg_u = 0] * S / n,
// S = sum_v lambda_v of the previous iterate. sv[0] = sum of lambda' (next S),
// sv[1] = |lambda' - lambda|_1, sv[2] = |lambda'|_1 (relative stopping test).
struct ProgADJ {
    using acc_t = double;
    using val_t = double;
    static constexpr bool kSum = true, kWeights = true, kActivity = false;
    const double* cur;
    double* nxt;
    const double* gvec;
    double* xout;
    const float* w;
    double d;
    __device__ acc_t identity() const { return 0.0; }
    __device__ acc_t from_val(double v, float we) const { return (double)we * v; }
    __device__ acc_t gather(uint32_t src, float we) const { return from_val(cur[src], we); }
    __device__ bool row_active(uint32_t) const { return true; }
    static __device__ bool converged(double resid, double norm, double tol) {
        return resid <= tol * norm;
    }
    struct Ld {
        double c, g;
    };
    __device__ Ld load(int64_t v) const { return Ld{cur[v], gvec[v]}; }
    __device__ void apply(int64_t v, const Ld& l, acc_t acc, int32_t dg, double scal, int32_t n,
                          double* sv, int&) const {
        double lo = l.c;
        double ln = l.g + d * acc + (dg == 0 ? d * scal / n : 0.0);
        sv[0] += ln;
        sv[1] += fabs(ln - lo);
        sv[2] += fabs(ln);
        nxt[v] = ln;
        if (xout) xout[v] = ln;
    }
    __device__ void pass(int64_t v, int32_t) const {
        nxt[v] = cur[v];
        if (xout) xout[v] = cur[v];
    }
};

__device__ inline void lds_combine(float* p, float v, bool) { atomicAdd(p, v); }
__device__ inline void lds_combine(double* p, double v, bool) { atomicAdd(p, v); }
__device__ inline void lds_combine(int32_t* p, int32_t v, bool sum) {
    if (sum)
        atomicAdd(p, v);
    else
        atomicMin(p, v);
}
// 64-bit accumulators are bit sets (one bit per BFS root), combined by OR.
__device__ inline void lds_combine(uint64_t* p, uint64_t v, bool) {
    if (v) atomicOr((unsigned long long*)p, (unsigned long long)v);
}

// Device-scope atomics on the hub of a split tile (native FP64 add, int min).
__device__ inline void global_combine(double* p, double v, bool) { unsafeAtomicAdd(p, v); }
__device__ inline void global_combine(int32_t* p, int32_t v, bool sum) {
    if (sum)
        atomicAdd(p, v);
    else
        atomicMin(p, v);
}

template <bool kSum, typename A>
__device__ inline A combine(A a, A b) {
    if constexpr (std::is_same<A, uint64_t>::value)
        return a | b;  // bit sets
    else if constexpr (kSum)
        return a + b;
    else
        return b < a ? b : a;
}

// DPP controls of gfx9: row_shr:n (0x110 + n) shifts inside rows of 16 lanes,
// row_bcast:15 / row_bcast:31 pass lane 15 of each row (lane 31) to the rows
// after it, wave_shr:1 shifts the whole wave by one lane. A lane with no source
// keeps `old`.
constexpr int kDppRowShr = 0x110, kDppRowBcast15 = 0x142, kDppRowBcast31 = 0x143, kDppWaveShr1 = 0x138;

template <int kCtl, int kRowMask>
__device__ inline uint32_t dpp_u32(uint32_t old, uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp((int)old, (int)v, kCtl, kRowMask, 0xF, false);
}
template <int kCtl, int kRowMask>
__device__ inline int32_t dpp_val(int32_t old, int32_t v) {
    return __builtin_amdgcn_update_dpp(old, v, kCtl, kRowMask, 0xF, false);
}
template <int kCtl, int kRowMask>
__device__ inline uint64_t dpp_val(uint64_t o, uint64_t x) {
    const uint32_t lo = dpp_u32<kCtl, kRowMask>((uint32_t)o, (uint32_t)x);
    const uint32_t hi = dpp_u32<kCtl, kRowMask>((uint32_t)(o >> 32), (uint32_t)(x >> 32));
    return ((uint64_t)hi << 32) | lo;
}
template <int kCtl, int kRowMask>
__device__ inline double dpp_val(double old, double v) {
    return __builtin_bit_cast(double, dpp_val<kCtl, kRowMask>(__builtin_bit_cast(uint64_t, old),
                                                              __builtin_bit_cast(uint64_t, v)));
}

// Segmented reduction across a wave: the lanes of every run (consecutive lanes
// start..lane, `start` being the run's first lane) are combined so that each
// lane ends with the combination of its run up to itself -- the run's last lane
// holds the run's total. Steps of 1, 2, 4 and 8 lanes inside rows of 16, then
// the last lane of each row passed on to the rows after it.
template <bool kSum, typename A>
__device__ inline A run_reduce(A v, int start, int lane, A ident) {
    A s;
    s = dpp_val<kDppRowShr + 1, 0xF>(ident, v);
    if (lane - 1 >= start) v = combine<kSum>(v, s);
    s = dpp_val<kDppRowShr + 2, 0xF>(ident, v);
    if (lane - 2 >= start) v = combine<kSum>(v, s);
    s = dpp_val<kDppRowShr + 4, 0xF>(ident, v);
    if (lane - 4 >= start) v = combine<kSum>(v, s);
    s = dpp_val<kDppRowShr + 8, 0xF>(ident, v);
    if (lane - 8 >= start) v = combine<kSum>(v, s);
    // rows 1 and 3 take lane 15 / 47, when their run began in the row before
    s = dpp_val<kDppRowBcast15, 0xA>(ident, v);
    if (start < (lane & ~15)) v = combine<kSum>(v, s);
    // rows 2 and 3 take lane 31, when their run began in row 0 or 1
    s = dpp_val<kDppRowBcast31, 0xC>(ident, v);
    if (lane >= 32 && start < 32) v = combine<kSum>(v, s);
    return v;
}

__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// ---------------------------------------------------------------------------
// The edge kernel
// ---------------------------------------------------------------------------
// One iteration is three launches, ordered by the stream, so no workgroup
// ever waits for another and no workgroup needs a device-scope fence (on
// gfx950 each one writes back the XCD's L2):
//   k_iterate  one workgroup per work item (a tile, or a piece of a heavy
//              tile): streams the item's chunks into LDS accumulators; a whole
//              tile applies the update at once, a piece stores its partial in
//              its slot of the tile's hub (Alg. 6 ToHub);
//   k_finish   one workgroup per split tile: sums the hub slots in piece order
//              (FromHub) and applies the update;
//   k_reduce   one workgroup: sums the per-tile scalars in tile order into the
//              next iteration's dangling mass, the residual and the stop flag.

// Applies the update to vertices [base, base + len) from the accumulators
// acc[0, len) in LDS and stores their scalars (dangling mass, residual, norm,
// changed flag) in scalar slot `slot`.
template <class Prog, int WG>
__device__ void apply_range(const Geo& g, const Ctl& ctl, const Prog& prog, int64_t base, int64_t len,
                            int slot, typename Prog::acc_t* acc) {
    __shared__ double red[3][WG / 64];
    __shared__ int sflag;
    const int lane = lane_id(), wave = threadIdx.x >> 6;
    if (threadIdx.x == 0) sflag = 0;
    __syncthreads();
    const double scal = ctl.stats[ctl.k * 4 + 0];
    double sv[3] = {0.0, 0.0, 0.0};
    int flag = 0;
    // kAR vertices per thread at a time: all their loads are issued (vertices
    // past the tile reload the first one) before the first update is computed
    constexpr int kAR = 4;
    if constexpr (Prog::kActivity) {
        // Block activity (Sec. II-B at a finer grain): the first lane of each
        // block of 2^bs vertices stores the block's flags (changed; unreached).
        // base is a multiple of the block size and a wave's lanes hold
        // consecutive vertices, so a block lies inside one wave. A block not
        // flagged as changed holds the same values in both buffers; if nothing
        // reaches it in this round either it is skipped (no loads, no stores,
        // flags unchanged). acc == NULL: nothing reaches the range at all.
        // The range's flags from the previous round are first copied to LDS
        // (at most kMaxBlk blocks: the range is at most a tile).
        const int bl = 1 << prog.bs;  // <= 64
        const int first = lane & ~(bl - 1);
        const uint64_t bm = (bl == 64 ? ~0ull : (1ull << bl) - 1ull) << first;
        constexpr int kMaxBlk = 1024;
        __shared__ uint8_t was_s[kMaxBlk];
        const int64_t b0 = base >> prog.bs;
        const int nblk = (int)min((int64_t)kMaxBlk, (len + bl - 1) >> prog.bs);
        for (int i = threadIdx.x; i < nblk; i += WG) was_s[i] = prog.chg[b0 + i];
        __syncthreads();
        for (int64_t x0 = threadIdx.x; x0 < len; x0 += kAR * WG) {
            typename Prog::Ld ld[kAR];
            bool need[kAR];
#pragma unroll
            for (int r = 0; r < kAR; ++r) {
                const int64_t x = x0 + r * WG;
                const bool in = x < len;
                const int64_t xs = in ? x : x0;
                const bool arrived = in && acc && acc[xs] != prog.identity();
                const uint64_t am = __ballot(arrived);
                const bool was = was_s[xs >> prog.bs] != 0;
                need[r] = in && (was || (am & bm) != 0);
                if (need[r]) ld[r] = prog.load(base + x);
            }
#pragma unroll
            for (int r = 0; r < kAR; ++r) {
                const int64_t x = x0 + r * WG;
                if (x >= len) break;
                if (!need[r]) continue;  // uniform over the block
                int ch = 0;
                prog.apply(base + x, ld[r], acc ? acc[x] : prog.identity(), 0, scal, g.n, sv, ch);
                const uint64_t cm = __ballot(ch & 1), om = __ballot(ch & 2);
                if (lane == first) {
                    const int64_t b = (base + x) >> prog.bs;
                    prog.chg[b] = (cm & bm) != 0;
                    if (prog.opn) prog.opn[b] = (om & bm) != 0;
                }
                if (ch & 1) flag = 1;
            }
        }
    } else {
    for (int64_t x0 = threadIdx.x; x0 < len; x0 += kAR * WG) {
        typename Prog::Ld ld[kAR];
        int32_t dgv[kAR];
#pragma unroll
        for (int r = 0; r < kAR; ++r) {
            const int64_t x = x0 + r * WG < len ? x0 + r * WG : x0;
            ld[r] = prog.load(base + x);
            dgv[r] = g.deg[base + x];
        }
#pragma unroll
        for (int r = 0; r < kAR; ++r) {
            const int64_t x = x0 + r * WG;
            if (x >= len) break;
            prog.apply(base + x, ld[r], acc[x], dgv[r], scal, g.n, sv, flag);
        }
    }
    }
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        sv[q] = wave_sum(sv[q]);
        if (lane == 0) red[q][wave] = sv[q];
    }
    if (flag) sflag = 1;
    __syncthreads();
    if (threadIdx.x == 0) {
        if constexpr (Prog::kActivity) {
            // no scalars; the round's changed flag (cleared before the round) is
            // raised directly, so no reduction launch follows
            if (sflag) ctl.stats[ctl.k * 4 + 3] = 1.0;
        } else {
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                double a = 0.0;
                for (int w = 0; w < WG / 64; ++w) a += red[q][w];
                g.tile_s[3 * slot + q] = a;
            }
            g.tile_flag[slot] = sflag;
        }
    }
}

// Sums the scalar slots of one iteration in slot order (k_reduce's body).
template <class Prog, int WG>
__device__ void reduce_tiles(const Geo& g, const Ctl& ctl) {
    __shared__ double red[3][WG / 64];
    __shared__ int sflag;
    const int lane = lane_id(), wave = threadIdx.x >> 6;
    if (threadIdx.x == 0) sflag = 0;
    __syncthreads();
    double tv[3] = {0.0, 0.0, 0.0};
    int f = 0;
    for (int x = threadIdx.x; x < g.n_sslots; x += WG) {
#pragma unroll
        for (int q = 0; q < 3; ++q) tv[q] += g.tile_s[3 * x + q];
        f |= g.tile_flag[x];
    }
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        tv[q] = wave_sum(tv[q]);
        if (lane == 0) red[q][wave] = tv[q];
    }
    if (f) sflag = 1;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t3[3];
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            t3[q] = 0.0;
            for (int w = 0; w < WG / 64; ++w) t3[q] += red[q][w];
        }
        ctl.stats[(ctl.k + 1) * 4 + 0] = t3[0];
        ctl.stats[ctl.k * 4 + 1] = t3[1];
        ctl.stats[ctl.k * 4 + 2] = t3[2];
        ctl.stats[ctl.k * 4 + 3] = sflag ? 1.0 : 0.0;
        if (ctl.tol > 0.0 && Prog::converged(t3[1], t3[2], ctl.tol)) *ctl.done = 1;
    }
}

// Sums the hub slots of a split tile in piece order into LDS (FromHub), over
// the segment's vertices.
template <class Prog, int WG>
__device__ void gather_hub(const Geo& g, const Prog& prog, const FinSeg& it, typename Prog::acc_t* acc) {
    using acc_t = typename Prog::acc_t;
    const int64_t len = it.vlen;
    // sixteen slots per pass so the loads of a thread are independent
    const acc_t* p0 = reinterpret_cast<const acc_t*>(g.partial) + (int64_t)it.slot * g.T + it.v0;
    for (int64_t x = threadIdx.x; x < len; x += WG) {
        acc_t sum = prog.identity();
        int p = 0;
        for (; p + 16 <= it.npieces; p += 16) {
            acc_t v[16];
#pragma unroll
            for (int q = 0; q < 16; ++q) v[q] = __builtin_nontemporal_load(p0 + (int64_t)(p + q) * g.T + x);
#pragma unroll
            for (int q = 0; q < 16; ++q) sum = combine<Prog::kSum>(sum, v[q]);
        }
        for (; p < it.npieces; ++p)
            sum = combine<Prog::kSum>(sum, __builtin_nontemporal_load(p0 + (int64_t)p * g.T + x));
        acc[x] = sum;
    }
    __syncthreads();
}

// Processes one work item (a tile, or a piece of a heavy tile) of one iteration.
template <class Prog, int WG, bool kDstOrder>
__device__ void iterate_item(const Geo& g, const Ctl& ctl, const Prog& prog, const Item& it,
                             unsigned char* smem) {
    using acc_t = typename Prog::acc_t;
    acc_t* acc = reinterpret_cast<acc_t*>(smem);

    const int tile = it.tile;
    const int64_t base = (int64_t)tile << g.t;
    int64_t len = min((int64_t)g.T, (int64_t)g.n - base);
    if (len < 0) len = 0;

    // Once converged (tolerance met) the remaining iterations only carry the
    // vector over so the final buffer is the one the caller expects.
    if (*ctl.done) {
        if (it.piece == 0)
            for (int64_t x = threadIdx.x; x < len; x += WG) prog.pass(base + x, g.deg[base + x]);
        return;
    }

    // chunk source: explicit range, or this piece's share of the tile's compacted list
    int64_t c_lo = it.c0, c_hi = it.c1;
    const int64_t* list = nullptr;
    int npieces = it.npieces;
    if (g.clist) {
        const int64_t cnt = g.ccount[tile];
        if (npieces > 1 && cnt <= g.split_min) {
            if (it.piece > 0) return;  // piece 0 takes the whole (short) list
            npieces = 1;
        }
        list = g.clist + it.c0;  // tile's first chunk = list origin
        c_lo = cnt * it.piece / npieces;
        c_hi = cnt * (it.piece + 1) / npieces;
        if constexpr (Prog::kActivity) {
            if (cnt == 0) {  // nothing reaches the tile: no accumulators to clear
                apply_range<Prog, WG>(g, ctl, prog, base, len, tile, nullptr);
                return;
            }
        }
    }

    if constexpr (early_exit_of<Prog>::value) {
        for (int64_t x = threadIdx.x; x < len; x += WG) acc[x] = prog.cur[base + x];
    } else {
        for (int64_t x = threadIdx.x; x < len; x += WG) acc[x] = prog.identity();
    }
    __syncthreads();

    // the wave index is uniform: chunk indices and interval rows then live in
    // scalar registers and their loads go through the scalar cache
    const int lane = lane_id(), wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint64_t lt = (1ull << lane) - 1ull;
    const uint32_t lmask = (1u << g.L) - 1u;
    const uint32_t tmask = (1u << g.t) - 1u;
    const int steps = g.C >> 8;

    // Both edge orders share one loop. Load k of a lane reads word 64k + lane of
    // a 256-word sub-block, so the 64 lanes of a load, a gather and an LDS
    // reduction hold 64 consecutive edges: in source order their sources are
    // adjacent (a gather touches few cache lines); in destination order runs of
    // equal destination lie in consecutive lanes and are summed across the wave
    // before they reach LDS. The wave walks its units (kU sub-blocks of one
    // chunk) through two word buffers, and gathers run one unit ahead of the
    // reductions: a unit's gathers are issued before the previous unit's LDS
    // reductions, so each lane keeps two units of gathers and two units of word
    // loads in flight (the 6-bit load counter holds exactly that many).
    //
    // Per word the decode keeps two 32-bit numbers: the byte offset of the
    // gathered value from the value array's base, and the LDS slot it adds
    // into. Gathers are buffer loads with 32-bit offsets; a marker or padding
    // word asks for an offset past the array and reads 0 (the hardware's range
    // check), so a summing program needs no select for non-edges, and such
    // words add into the lane's own discard slot past the tile.
    auto stream = [&](auto dst_tag) {
        constexpr bool kDst = decltype(dst_tag)::value;
        using val_t = typename Prog::val_t;
        // 16 edges per lane and unit in source order; 8 when weights, 8-byte values
        // or the cross-lane run sums of the destination order need the registers
        constexpr int kU = (Prog::kWeights || sizeof(val_t) > 4 || kDst) ? 2 : 4, kQ = 4 * kU;
        // pair layout (source order only): header words set the source of the
        // pair words after them (carried across lanes and units like the
        // interval markers), and a pair word adds its one gathered value to two
        // destinations
        constexpr bool kPairs = pairs_of<Prog>::value && !kDst;
        constexpr bool kRows = row_range_of<Prog>::value;
        constexpr uint32_t kVs = sizeof(val_t) == 8 ? 3u : 2u;  // log2 of the value bytes
        constexpr uint32_t kOOB = 0xFFFFFFF0u;                 // past any value array
        // destination order: a slice whose 64 edges form at most this many runs
        // of equal destination is summed across the wave first
        constexpr int kRunSlice = 16;
        const uint32_t* const wordsp = g.words;
        const int64_t Cw = g.C;
        const int32_t* const rowp = g.chunk_row;
        const float* wtsp = nullptr;
        if constexpr (Prog::kWeights) wtsp = prog.w;
        const __amdgpu_buffer_rsrc_t vrs = __builtin_amdgcn_make_buffer_rsrc(
            (void*)prog.cur, (short)0, (int)((uint32_t)g.n << kVs), kBufWord3);
        const uint32_t ival = (uint32_t)g.I;  // interval size (any size, not only powers of two)
        const uint32_t disc = (uint32_t)g.T + lane;   // this lane's discard slot
        // loader cursor: chunk (index into the item's range or list) and sub-block
        int64_t lci = c_lo + wave;
        int ls = 0;
        int64_t lprev = lci;  // chunk of the last unit loaded (a valid address)
        uint32_t wA[kQ], wB[kQ];
        float fA[kQ], fB[kQ];
        bool vA = false, vB = false, nA = false, nB = false;  // valid, starts a chunk
        uint32_t rA = 0, rB = 0;                              // chunk's first interval
        uint32_t sA = 0, sB = 0;  // pair layout: header source at the chunk's first word
        // Issues the loads of the next unit. Every load is unconditional, so the
        // code has no branch around memory operations and the compiler keeps
        // exact counts of the loads in flight: a sub-block outside the stream
        // (past the wave's range, or past the chunk's end) is read from a
        // constant block of padding words (weights: zeros) instead.
        auto next = [&](uint32_t* wo, float* fo, bool& valid, bool& starts, uint32_t& r0, uint32_t& s0) {
            valid = lci < c_hi;
            const int64_t cl = valid ? lci : lprev;
            const int sl = valid ? ls : 0;
            starts = sl == 0;
            int64_t c_ = cl;
            if constexpr (Prog::kActivity) c_ = list ? list[cl] : cl;
            r0 = (uint32_t)rowp[c_];
            if constexpr (kPairs) s0 = (uint32_t)g.chunk_src[c_];
            const int64_t base = c_ * Cw + (int64_t)sl * 256;
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                const bool in = valid && sl + u < steps;
                const uint32_t* wb = in ? wordsp + base + u * 256 : kPadWords;
                const float* fb = nullptr;
                if constexpr (Prog::kWeights) fb = in ? wtsp + base + u * 256 : kPadZeros;
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    wo[4 * u + k] = __builtin_nontemporal_load(wb + k * 64 + lane);
                    if constexpr (Prog::kWeights)
                        fo[4 * u + k] = __builtin_nontemporal_load(fb + k * 64 + lane);
                    else
                        fo[4 * u + k] = 0.f;
                }
            }
            if (valid) {
                lprev = lci;
                ls += kU;
                if (ls >= steps) {
                    ls = 0;
                    lci += WG / 64;
                }
            }
        };
        if (lci >= c_hi) return;
        next(wA, fA, vA, nA, rA, sA);
        next(wB, fB, vB, nB, rB, sB);
        uint32_t row = 0, hsrc = 0;
        // decode: offsets of the gathers and LDS slots of one unit's words
        auto decode = [&](const uint32_t* w_, bool starts, uint32_t r0, uint32_t s0, uint32_t* off,
                          uint32_t* li, uint32_t* li2) {
            if (starts) {
                row = r0;
                if constexpr (kPairs) hsrc = s0;
            }
#pragma unroll
            for (int q = 0; q < kQ; ++q) {
                const uint32_t w = w_[q];
                // markers and padding have bit 31 set; the lane's interval is the
                // last marker at or before it in the slice, else the carried one
                const uint64_t mm = __ballot((int32_t)w < 0);
                // byte offset of the interval's first value: a scalar unless the
                // slice holds a marker
                uint32_t rb = (uint32_t)__builtin_amdgcn_readfirstlane((int)((row * ival) << kVs));
                uint32_t rl = row;  // the lane's source interval
                if (mm) {
                    const uint64_t upto = mm & (lt | (1ull << lane));
                    const uint32_t got = __shfl(w & ~kMarker, upto ? 63 - __clzll(upto) : lane);
                    rl = upto ? got : row;
                    rb = (rl * ival) << kVs;
                    row = (uint32_t)__builtin_amdgcn_readlane((int)(w & ~kMarker), 63 - __clzll(mm));
                }
                // a launch over a range of source intervals treats the words of
                // other intervals as padding
                bool in_rows = true;
                if constexpr (kRows) in_rows = prog.row_in(rl);
                if constexpr (kPairs) {
                    // word kinds by the top three bits: 1xx marker or padding,
                    // 01x header, 001 pair, 000 plain edge
                    const uint32_t kind = w >> 29;
                    const uint64_t hm = __ballot(kind == 2u || kind == 3u);
                    uint32_t sv = hsrc;
                    if (hm) {
                        const uint64_t upto = hm & (lt | (1ull << lane));
                        const uint32_t got = __shfl(w & 0x3FFFFFFFu, upto ? 63 - __clzll(upto) : lane);
                        sv = upto ? got : hsrc;
                        hsrc = (uint32_t)__builtin_amdgcn_readlane((int)(w & 0x3FFFFFFFu), 63 - __clzll(hm));
                    }
                    const bool pr = kind == 1u, pl = kind == 0u;
                    const uint32_t loc = pr ? sv : __builtin_amdgcn_ubfe(w, (uint32_t)g.sshift, (uint32_t)g.L);
                    off[q] = (pr || pl) ? (loc << kVs) + rb : kOOB;
                    li[q] = (pr || pl) ? (w & tmask) : disc;
                    li2[q] = pr ? ((w >> 14) & tmask) : disc;
                } else {
                    bool e = (int32_t)w >= 0 && in_rows;
                    const uint32_t dl = __builtin_amdgcn_ubfe(w, (uint32_t)g.dshift, (uint32_t)g.t);
                    // (dl < T for any word, so the read stays in the array; a
                    // value written by another wave after it is only a missed skip)
                    if constexpr (early_exit_of<Prog>::value) e = e && acc[dl] == prog.identity();
                    off[q] = e ? (__builtin_amdgcn_ubfe(w, (uint32_t)g.sshift, (uint32_t)g.L) << kVs) + rb : kOOB;
                    li[q] = e ? dl : disc;
                }
            }
        };
        auto gather = [&](const uint32_t* off, const float* f_, val_t* raw, float* wq) {
#pragma unroll
            for (int q = 0; q < kQ; ++q) {
                wq[q] = f_[q];
                raw[q] = load_val<val_t>(vrs, off[q]);  // non-edges read 0
            }
        };
        // branch-free reductions: a summing program adds the gathered 0 of a
        // non-edge to the lane's discard slot; a minimum program offers its
        // identity there (a conditional block around the gathered value would let
        // the compiler sink a gather into it and wait on every load in flight)
        auto reduce = [&](const val_t* raw, const float* wq, const uint32_t* li, const uint32_t* li2) {
#pragma unroll
            for (int q = 0; q < kQ; ++q) {
                acc_t v = prog.from_val(raw[q], wq[q]);
                if constexpr (!Prog::kSum) v = li[q] != disc ? v : prog.identity();
                uint32_t slot = li[q];
                if constexpr (kDst) {
                    // Runs of equal destination (the slice's keys; a marker or
                    // padding lane has its own slot, so it ends any run) are summed
                    // across the wave into their last lane, which alone adds to
                    // LDS, when the slice has few enough runs for that to pay
                    const uint32_t kp = dpp_u32<kDppWaveShr1, 0xF>(~slot, slot);
                    const uint64_t heads = __ballot(kp != slot);
                    if (__popcll(heads) <= kRunSlice) {
                        const int start = 63 - (int)__clzll(heads & ((2ull << lane) - 1ull));
                        v = run_reduce<Prog::kSum>(v, start, lane, prog.identity());
                        const bool tail = lane == 63 || (((heads >> lane) >> 1) & 1ull);
                        slot = tail ? slot : disc;
                        v = tail ? v : prog.identity();
                    }
                }
                lds_combine(&acc[slot], v, Prog::kSum);
                if constexpr (kPairs) {
                    if (__ballot(li2[q] != disc)) lds_combine(&acc[li2[q]], v, Prog::kSum);
                }
            }
        };
        uint32_t off[kQ], lA[kQ], lB[kQ], l2A[kPairs ? kQ : 1], l2B[kPairs ? kQ : 1];
        val_t gA[kQ], gB[kQ];
        float qA[kQ], qB[kQ];
        // unit 0 decoded and its gathers issued; its buffer takes unit 2
        decode(wA, nA, rA, sA, off, lA, l2A);
        gather(off, fA, gA, qA);
        bool okA = vA, okB = false;  // the unit held in gA / gB is part of the stream
        next(wA, fA, vA, nA, rA, sA);
        while (okA) {
            decode(wB, nB, rB, sB, off, lB, l2B);
            gather(off, fB, gB, qB);
            okB = vB;
            next(wB, fB, vB, nB, rB, sB);
            reduce(gA, qA, lA, l2A);
            if (!okB) break;
            decode(wA, nA, rA, sA, off, lA, l2A);
            gather(off, fA, gA, qA);
            okA = vA;
            next(wA, fA, vA, nA, rA, sA);
            reduce(gB, qB, lB, l2B);
        }
    };
    stream(std::integral_constant<bool, kDstOrder>{});
    __syncthreads();

    if constexpr (row_range_of<Prog>::value) {
        // mixed-phase update: the tile's sums go to its slot (store or add), or
        // the hub slots after it are added and the update applied
        acc_t* hub = reinterpret_cast<acc_t*>(g.partial) + (int64_t)it.slot * g.T;
        if (prog.mode != kMpuApply && it.npieces > 1) {
            for (int64_t x = threadIdx.x; x < len; x += WG)
                if (acc[x] != (acc_t)0) unsafeAtomicAdd(&hub[x], acc[x]);
            return;
        }
        if (prog.mode == kMpuStore) {
            for (int64_t x = threadIdx.x; x < len; x += WG) hub[x] = acc[x];
            return;
        }
        if (prog.mode == kMpuAdd) {
            for (int64_t x = threadIdx.x; x < len; x += WG) hub[x] += acc[x];
            return;
        }
        for (int64_t x = threadIdx.x; x < len; x += WG) {
            acc_t sum = acc[x];
            for (int p = 0; p < it.npieces; ++p) sum += hub[(int64_t)p * g.T + x];
            acc[x] = sum;
        }
        __syncthreads();
        apply_range<Prog, WG>(g, ctl, prog, base, len, tile, acc);
        return;
    }

    // a piece stores its partial in its hub slot; k_finish combines them (its
    // segments carry the tile's scalars, the tile's own slot holds zeros)
    if (npieces > 1) {
        acc_t* part = reinterpret_cast<acc_t*>(g.partial) + (int64_t)(it.slot + it.piece) * g.T;
        for (int64_t x = threadIdx.x; x < len; x += WG) part[x] = acc[x];
        if (it.piece == 0 && threadIdx.x == 0) {
            for (int q = 0; q < 3; ++q) g.tile_s[3 * tile + q] = 0.0;
            g.tile_flag[tile] = 0;
        }
        return;
    }
    apply_range<Prog, WG>(g, ctl, prog, base, len, tile, acc);
}

// kDstOrder: the stream's sub-shards are in destination order (runs of equal
// destination summed across the wave); a kernel of its own per order, so each
// loop gets its own register allocation.
template <class Prog, int WG, bool kDstOrder>
__global__ __launch_bounds__(WG) void k_iterate(Geo g, Ctl ctl, Prog prog) {
    extern __shared__ __align__(16) unsigned char smem[];
    iterate_item<Prog, WG, kDstOrder>(g, ctl, prog, g.items[blockIdx.x], smem);
}

// One workgroup per vertex segment of a split tile.
template <class Prog, int WG>
__global__ __launch_bounds__(WG) void k_finish(Geo g, Ctl ctl, Prog prog, const FinSeg* __restrict__ fin) {
    extern __shared__ __align__(16) unsigned char smem[];
    if (*ctl.done) return;  // converged: the pieces have carried the vectors over
    const FinSeg f = fin[blockIdx.x];
    if (g.clist && g.ccount[f.tile] <= g.split_min) {
        // the tile was done whole this round: the segment's scalar slot is empty
        if (threadIdx.x == 0) {
            for (int q = 0; q < 3; ++q) g.tile_s[3 * f.sslot + q] = 0.0;
            g.tile_flag[f.sslot] = 0;
        }
        return;
    }
    typename Prog::acc_t* acc = reinterpret_cast<typename Prog::acc_t*>(smem);
    gather_hub<Prog, WG>(g, prog, f, acc);
    apply_range<Prog, WG>(g, ctl, prog, ((int64_t)f.tile << g.t) + f.v0, f.vlen, f.sslot, acc);
}

template <class Prog, int WG>
__global__ __launch_bounds__(WG) void k_reduce(Geo g, Ctl ctl) {
    if (*ctl.done) return;
    reduce_tiles<Prog, WG>(g, ctl);
}

// ---------------------------------------------------------------------------
// Many graphs per launch: one launch per iteration covers the work items (tile
// pieces) of every graph, heaviest first across all graphs; workgroup w reads
// its item and the item's graph. As for one graph, the split tiles of all graphs are
// finished by a second launch and each graph's scalars are reduced by a third
// (one workgroup per graph), so no workgroup ever waits for another.
// ---------------------------------------------------------------------------
struct MultiGraph {
    Geo geo;
    double* stats;     // [4 * (iters + 2)]
    float* buf0;
    float* buf1;
    float* xout;       // [n] result (in internal ids for a relabeled graph)
    int32_t* done0;    // a zero word (no tolerance stop in this mode)
    int32_t n_items;   // work items of this graph
    const int32_t* o2n;  // relabeled graph: caller id -> internal id, else NULL
    float* user;         // the caller's result buffer (written from xout when o2n is set)
};

template <int WG, bool kDstOrder>
__global__ __launch_bounds__(WG) void k_multi_iter(const MultiGraph* __restrict__ graphs,
                                                   const int32_t* __restrict__ item_graph,
                                                   const Item* __restrict__ items, int k, int iters,
                                                   double damping) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int r = blockIdx.x;
    const MultiGraph& mg = graphs[item_graph[r]];
    Ctl ctl{mg.stats, mg.done0, k, 0.0};
    ProgPR<float> prog{(k & 1) ? mg.buf1 : mg.buf0, (k & 1) ? mg.buf0 : mg.buf1, nullptr,
                       k == iters - 1 ? mg.xout : nullptr, damping};
    iterate_item<ProgPR<float>, WG, kDstOrder>(mg.geo, ctl, prog, items[r], smem);
}

// A finishing segment of graph `graph`.
struct MultiFin {
    int32_t graph;
    FinSeg f;
};

template <int WG>
__global__ __launch_bounds__(WG) void k_multi_finish(const MultiGraph* __restrict__ graphs,
                                                     const MultiFin* __restrict__ fin, int k, int iters,
                                                     double damping) {
    extern __shared__ __align__(16) unsigned char smem[];
    const MultiFin f = fin[blockIdx.x];
    const MultiGraph& mg = graphs[f.graph];
    Ctl ctl{mg.stats, mg.done0, k, 0.0};
    ProgPR<float> prog{(k & 1) ? mg.buf1 : mg.buf0, (k & 1) ? mg.buf0 : mg.buf1, nullptr,
                       k == iters - 1 ? mg.xout : nullptr, damping};
    double* acc = reinterpret_cast<double*>(smem);
    gather_hub<ProgPR<float>, WG>(mg.geo, prog, f.f, acc);
    apply_range<ProgPR<float>, WG>(mg.geo, ctl, prog, ((int64_t)f.f.tile << mg.geo.t) + f.f.v0, f.f.vlen,
                                   f.f.sslot, acc);
}

// kMultiBlocks workgroups per graph for the start and the final mapping.
constexpr int kMultiBlocks = 16;

// x^0 = 1/n (gathered array x^0 / outdeg) and per-block dangling partial sums;
// block b works on graph b / kMultiBlocks.
__global__ __launch_bounds__(256) void k_multi_init(const MultiGraph* __restrict__ graphs,
                                                    double* __restrict__ part) {
    __shared__ double red[4];
    const MultiGraph& mg = graphs[blockIdx.x / kMultiBlocks];
    const int j = blockIdx.x % kMultiBlocks;
    const int32_t n = mg.geo.n;
    const float x = (float)(1.0 / n);
    double sdang = 0.0;
    for (int64_t v = (int64_t)j * 256 + threadIdx.x; v < n; v += kMultiBlocks * 256) {
        const int32_t dg = mg.geo.deg[v];
        if (dg == 0) sdang += (double)x;
        mg.buf0[v] = dg ? (float)((double)x / dg) : x;
    }
    sdang = wave_sum(sdang);
    if (lane_id() == 0) red[threadIdx.x >> 6] = sdang;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// The dangling mass entering iteration 0 of every graph: its blocks' partial
// sums in block order (one thread per graph).
__global__ void k_multi_init_sum(const MultiGraph* __restrict__ graphs, int G, const double* __restrict__ part) {
    for (int gi = blockIdx.x * blockDim.x + threadIdx.x; gi < G; gi += gridDim.x * blockDim.x) {
        double sum = 0.0;
        for (int j = 0; j < kMultiBlocks; ++j) sum += part[gi * kMultiBlocks + j];
        graphs[gi].stats[0] = sum;
    }
}

// The result of every relabeled graph into the caller's ids (kMultiBlocks
// workgroups per graph).
__global__ __launch_bounds__(256) void k_multi_emit(const MultiGraph* __restrict__ graphs) {
    const MultiGraph& mg = graphs[blockIdx.x / kMultiBlocks];
    if (!mg.o2n) return;
    const int j = blockIdx.x % kMultiBlocks;
    for (int64_t v = (int64_t)j * 256 + threadIdx.x; v < mg.geo.n; v += kMultiBlocks * 256)
        mg.user[v] = mg.xout[mg.o2n[v]];
}

// The last iteration's residual of every graph, gathered for one copy to the host.
__global__ void k_multi_residuals(const MultiGraph* __restrict__ graphs, int G, int k, double* __restrict__ out) {
    for (int i = threadIdx.x; i < G; i += blockDim.x) out[i] = graphs[i].stats[4 * k + 1];
}

// One workgroup per graph: that graph's scalars in tile order.
__global__ __launch_bounds__(1024) void k_multi_reduce(const MultiGraph* __restrict__ graphs, int k) {
    const MultiGraph& mg = graphs[blockIdx.x];
    Ctl ctl{mg.stats, mg.done0, k, 0.0};
    reduce_tiles<ProgPR<float>, 1024>(mg.geo, ctl);
}

// ---------------------------------------------------------------------------
// Initialisation, activity and end-of-run kernels
// ---------------------------------------------------------------------------

// x^0 = t (or the caller's x^0), gathered array = x^0 / outdeg; per-block
// partial dangling mass.
template <typename V>
__global__ __launch_bounds__(256) void k_init_pr(int32_t n, const int32_t* __restrict__ deg,
                                                 const V* __restrict__ tele,
                                                 const V* __restrict__ x0, int divide,
                                                 V* __restrict__ cur, double* __restrict__ part) {
    __shared__ double red[4];
    double s = 0.0;
    for (int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x; v < n; v += (int64_t)gridDim.x * 256) {
        V x = x0 ? x0[v] : (tele ? tele[v] : (V)(1.0 / n));
        int32_t dg = deg[v];
        if (dg == 0) s += (double)x;
        cur[v] = (divide && dg) ? (V)((double)x / dg) : x;
    }
    s = wave_sum(s);
    if (lane_id() == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// *out = the sum of part[0, nb), by one wave (64 threads): lane l sums
// part[l], part[l + 64], ... in order, then the lanes are combined by a fixed
// butterfly, so the result does not depend on scheduling.
__global__ void k_sum_parts(const double* __restrict__ part, int nb, double* __restrict__ out) {
    double s = 0.0;
    for (int b = threadIdx.x; b < nb; b += 64) s += part[b];
    s = wave_sum(s);
    if (threadIdx.x == 0) *out = s;
}

// ---------------------------------------------------------------------------
// Coarse-grained, source-sorted comparison (NXG_RUN_SCATTER): the stream is the
// whole edge list in (source, destination) order, one wave per chunk, and every
// edge adds its source's share to its destination with a device-scope FP64
// atomic in global memory (the paper's lock-based scheme of Sec. IV-B1).
// ---------------------------------------------------------------------------
template <typename V, bool kW>
__global__ __launch_bounds__(256) void k_scatter(const uint32_t* __restrict__ words,
                                                 const int32_t* __restrict__ chunk_row, int64_t n_chunks,
                                                 int C, int I, int Lb, int t, const V* __restrict__ cur,
                                                 const float* __restrict__ wts, double* __restrict__ y) {
    const int lane = lane_id();
    const uint64_t lt = (1ull << lane) - 1ull;
    const uint32_t lmask = (1u << Lb) - 1u, tmask = (1u << t) - 1u;
    const int64_t nwaves = ((int64_t)gridDim.x * 256) >> 6;
    for (int64_t c = __builtin_amdgcn_readfirstlane((int)(((int64_t)blockIdx.x * 256 + threadIdx.x) >> 6));
         c < n_chunks; c += nwaves) {
        uint32_t row = (uint32_t)chunk_row[c];
        const int64_t base = c * (int64_t)C;
        for (int s0 = 0; s0 < C; s0 += 64) {
            const uint32_t w = __builtin_nontemporal_load(words + base + s0 + lane);
            const uint64_t mm = __ballot((w >> 31) != 0);
            uint32_t r = row;
            if (mm) {
                const uint64_t upto = mm & (lt | (1ull << lane));
                const uint32_t got = __shfl(w & ~kMarker, upto ? 63 - __clzll(upto) : lane);
                r = upto ? got : row;
                row = (uint32_t)__builtin_amdgcn_readlane((int)(w & ~kMarker), 63 - __clzll(mm));
            }
            if ((w >> 31) == 0) {
                const uint32_t src = r * (uint32_t)I + ((w >> t) & lmask);
                double v = (double)cur[src];
                if constexpr (kW) v *= (double)wts[base + s0 + lane];
                unsafeAtomicAdd(&y[w & tmask], v);
            }
        }
    }
}

// The update of every vertex from the global sums y (which it clears for the
// next iteration), with per-block partial scalars [3] (dangling mass, residual,
// sum) as in the tiled apply. divide: the gathered array is x / outdeg.
template <typename V>
__global__ __launch_bounds__(256) void k_scatter_apply(int32_t n, double* __restrict__ y,
                                                       const int32_t* __restrict__ deg,
                                                       const V* __restrict__ cur, V* __restrict__ nxt,
                                                       const V* __restrict__ tele, V* __restrict__ xout,
                                                       double d, int divide, const double* __restrict__ scal,
                                                       double* __restrict__ part) {
    __shared__ double red[3][4];
    double sv[3] = {0.0, 0.0, 0.0};
    const double delta = *scal;
    for (int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x; v < n; v += (int64_t)gridDim.x * 256) {
        const double acc = y[v];
        y[v] = 0.0;
        const int32_t dg = deg[v];
        const double c = (double)cur[v];
        const double xo = (divide && dg) ? c * dg : c;
        const double tv = tele ? (double)tele[v] : 1.0 / n;
        const V xr = (V)(d * (acc + delta / n) + (1.0 - d) * tv);
        sv[1] += fabs((double)xr - xo);
        sv[2] += (double)xr;
        if (dg == 0) sv[0] += (double)xr;
        nxt[v] = (divide && dg) ? (V)((double)xr / dg) : xr;
        if (xout) xout[v] = xr;
    }
    const int lane = lane_id(), wave = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        sv[q] = wave_sum(sv[q]);
        if (lane == 0) red[q][wave] = sv[q];
    }
    __syncthreads();
    if (threadIdx.x < 3) part[blockIdx.x * 3 + threadIdx.x] = red[threadIdx.x][0] + red[threadIdx.x][1] +
                                                              red[threadIdx.x][2] + red[threadIdx.x][3];
}

// Block partials in block order: delta entering k + 1, residual and sum of k.
__global__ void k_scatter_reduce(const double* __restrict__ part, int nb, double* __restrict__ stats, int k,
                                 double tol, int32_t* __restrict__ done) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double t3[3] = {0.0, 0.0, 0.0};
    for (int b = 0; b < nb; ++b)
        for (int q = 0; q < 3; ++q) t3[q] += part[b * 3 + q];
    stats[(k + 1) * 4 + 0] = t3[0];
    stats[k * 4 + 1] = t3[1];
    stats[k * 4 + 2] = t3[2];
    if (tol > 0.0 && t3[1] <= tol) *done = 1;
}

// x from the gathered array (x / outdeg where divide is set).
template <typename V>
__global__ void k_unscale(int32_t n, const int32_t* __restrict__ deg, const V* __restrict__ cur, int divide,
                          V* __restrict__ out) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
        out[v] = (divide && deg[v]) ? (V)((double)cur[v] * deg[v]) : cur[v];
}

// Levels into both buffers (a block not flagged as changed must agree in the
// two). Block flags before the first round: only the root's block has
// changed, and every block may hold an unreached vertex. The root comes in the
// caller's ids (o2n maps it; -1: an id without edges, which reaches nothing).
// Zeroes the streamed-chunk count.
__global__ void k_init_bfs(int32_t n, int32_t root_caller, const int32_t* __restrict__ o2n,
                           int32_t* __restrict__ lev, int32_t* __restrict__ lev1,
                           uint8_t* __restrict__ chg, uint8_t* __restrict__ opn, int bs,
                           unsigned long long* __restrict__ streamed) {
    const int32_t root = o2n ? o2n[root_caller] : root_caller;
    const int64_t nb = ((int64_t)n + (1 << bs) - 1) >> bs;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x) {
        lev[v] = lev1[v] = v == root ? 0 : kInf;
        if (v < nb) {
            chg[v] = (root >= 0 && v == (root >> bs)) ? 1 : 0;
            opn[v] = 1;
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) *streamed = 0;
}

// Labels start as the vertex's caller id (its own id, or new2old[v] in a
// relabeled build), so the fixed point is the minimum caller id of the component.
// Every block counts as changed before the first round (labels go into both
// buffers, as for BFS).
__global__ void k_init_wcc(int32_t n, int32_t* __restrict__ lab, int32_t* __restrict__ lab1,
                           uint8_t* __restrict__ chg, int bs, const int32_t* __restrict__ ids,
                           unsigned long long* __restrict__ streamed) {
    const int64_t nb = ((int64_t)n + (1 << bs) - 1) >> bs;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x) {
        lab[v] = lab1[v] = ids ? ids[v] : (int32_t)v;
        if (v < nb) chg[v] = 1;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) *streamed = 0;
}

__global__ void k_set_root(int32_t* __restrict__ lev, int32_t root) {
    if (threadIdx.x == 0) lev[root] = 0;
}

// Per chunk, the smallest and largest source and destination (global ids) of
// its edges, {slo, shi, dlo, dhi} (a chunk without edges gets
// {INT32_MAX, -1, INT32_MAX, -1}). One wave per chunk: lane l reads words
// l, l + 64, ... and follows the interval markers as the iteration does.
__global__ __launch_bounds__(256) void k_chunk_ranges(const uint32_t* __restrict__ words,
                                                      const int32_t* __restrict__ crow,
                                                      const int32_t* __restrict__ ctile,
                                                      int64_t n_chunks, int C, int I, int L, int t,
                                                      int sshift, int dshift, int4* __restrict__ out) {
    const int lane = lane_id();
    const uint64_t lt = (1ull << lane) - 1ull;
    const int64_t c = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (c >= n_chunks) return;  // uniform over the wave
    const int64_t tb = (int64_t)ctile[c] << t;
    const uint32_t lmask = (1u << L) - 1u, tmask = (1u << t) - 1u;
    uint32_t row = (uint32_t)crow[c];
    int32_t slo = INT32_MAX, shi = -1, dlo = INT32_MAX, dhi = -1;
    for (int j = 0; j < C / 64; ++j) {
        const uint32_t w = words[c * (int64_t)C + j * 64 + lane];
        const bool mk = (w >> 31) != 0 && w != 0xFFFFFFFFu;  // a marker (not padding)
        const uint64_t mm = __ballot(mk);
        uint32_t r = row;
        if (mm) {
            const uint64_t upto = mm & (lt | (1ull << lane));
            const uint32_t got = __shfl(w & ~kMarker, upto ? 63 - __clzll(upto) : lane);
            r = upto ? got : row;
            row = (uint32_t)__builtin_amdgcn_readlane((int)(w & ~kMarker), 63 - __clzll(mm));
        }
        if ((w >> 31) == 0) {
            const int32_t sv = (int32_t)((int64_t)r * I + ((w >> sshift) & lmask));
            const int32_t dv = (int32_t)(tb + ((w >> dshift) & tmask));
            slo = min(slo, sv);
            shi = max(shi, sv);
            dlo = min(dlo, dv);
            dhi = max(dhi, dv);
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
        slo = min(slo, __shfl_xor(slo, o));
        shi = max(shi, __shfl_xor(shi, o));
        dlo = min(dlo, __shfl_xor(dlo, o));
        dhi = max(dhi, __shfl_xor(dhi, o));
    }
    if (lane == 0) out[c] = make_int4(slo, shi, dlo, dhi);
}

// Block activity prefix counts, per segment of `seg` blocks (seg a multiple
// of 1024; one workgroup per segment): for x in [0, nb], pre[x] = number of
// flagged blocks in [x - x % seg, x), and tot[x / seg] = the segment's count
// (a flag past nb reads as 0). Done for the changed flags (f0) and, when f1 is
// not NULL, for the unreached flags. Workgroup 0 adds the previous round's
// per-tile list lengths to *streamed (when not NULL), clears them for the
// compaction to append to, and clears the round's changed flag.
__device__ void count_and_clear(int32_t* __restrict__ ccount, int n_tiles,
                                unsigned long long* __restrict__ streamed) {
    __shared__ unsigned long long red[16];
    unsigned long long sum = 0;
    for (int x = threadIdx.x; x < n_tiles; x += blockDim.x) {
        sum += (unsigned long long)ccount[x];
        ccount[x] = 0;
    }
    for (int o = 32; o > 0; o >>= 1) sum += __shfl_xor(sum, o);
    if (lane_id() == 0) red[threadIdx.x >> 6] = sum;
    __syncthreads();
    if (threadIdx.x == 0 && streamed) {
        unsigned long long a = 0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) a += red[w];
        *streamed += a;
    }
}

__global__ __launch_bounds__(1024) void k_blkscan(const uint8_t* __restrict__ f0,
                                                  const uint8_t* __restrict__ f1, int64_t nb, int seg,
                                                  int32_t* __restrict__ pre0, int32_t* __restrict__ pre1,
                                                  int32_t* __restrict__ tot0, int32_t* __restrict__ tot1,
                                                  int32_t* __restrict__ ccount, int n_tiles,
                                                  unsigned long long* __restrict__ streamed,
                                                  double* __restrict__ changed) {
    __shared__ int32_t part[2][16];
    if (blockIdx.x == 0) {
        count_and_clear(ccount, n_tiles, streamed);
        if (threadIdx.x == 0) *changed = 0.0;
    }
    const int per = seg / 1024;
    const int64_t a = (int64_t)blockIdx.x * seg + (int64_t)threadIdx.x * per;
    int32_t s0 = 0, s1 = 0;
    for (int k = 0; k < per; ++k) {
        const int64_t x = a + k;
        if (x < nb) {
            s0 += f0[x] != 0;
            if (f1) s1 += f1[x] != 0;
        }
    }
    // workgroup exclusive scan: inside each wave by shuffles, then over the
    // 16 wave totals
    const int lane = lane_id(), wave = threadIdx.x >> 6;
    int32_t v0 = s0, v1 = s1;
    for (int o = 1; o < 64; o <<= 1) {
        const int32_t a0 = __shfl_up(v0, o), a1 = __shfl_up(v1, o);
        if (lane >= o) {
            v0 += a0;
            v1 += a1;
        }
    }
    if (lane == 63) {
        part[0][wave] = v0;
        part[1][wave] = v1;
    }
    __syncthreads();
    int32_t r0 = v0 - s0, r1 = v1 - s1, all0 = 0, all1 = 0;
    for (int w = 0; w < 16; ++w) {
        if (w < wave) {
            r0 += part[0][w];
            r1 += part[1][w];
        }
        all0 += part[0][w];
        all1 += part[1][w];
    }
    for (int k = 0; k < per; ++k) {
        const int64_t x = a + k;
        if (x > nb) break;
        pre0[x] = r0;
        if (f1) pre1[x] = r1;
        if (x < nb) {
            r0 += f0[x] != 0;
            if (f1) r1 += f1[x] != 0;
        }
    }
    if (threadIdx.x == 0) {
        tot0[blockIdx.x] = all0;
        if (f1) tot1[blockIdx.x] = all1;
    }
}

// Frontier compaction: per tile, the chunks that hold a source changed in the
// previous round and (BFS, pre1 not NULL) a destination still unreached,
// stored from the tile's first chunk on. A chunk's source and destination
// ranges are tested against the block prefix counts (k_blkscan), so a kept
// chunk may still hold only unchanged sources or reached destinations between
// its extremes: a superset of the chunks that can lower a value. One thread
// per chunk; the lanes of a wave that belong to one tile take their places
// with a single atomic on the tile's count, so the order inside a tile's list
// varies from run to run. BFS and WCC take integer minima, so their results
// do not depend on it.
__global__ __launch_bounds__(256) void k_compact(const int64_t* __restrict__ tchunk,
                                                 const int32_t* __restrict__ ctile,
                                                 int64_t n_chunks, const int4* __restrict__ crng, int bs,
                                                 int seg, int nseg, const int32_t* __restrict__ pre0,
                                                 const int32_t* __restrict__ tot0,
                                                 const int32_t* __restrict__ pre1,
                                                 const int32_t* __restrict__ tot1,
                                                 int64_t* __restrict__ clist,
                                                 int32_t* __restrict__ ccount) {
    // exclusive prefix of the segment counts (nseg <= 256)
    __shared__ int32_t off[2][257];
    {
        const int x = threadIdx.x;
        off[0][x + 1] = x < nseg ? tot0[x] : 0;
        off[1][x + 1] = (pre1 && x < nseg) ? tot1[x] : 0;
        if (x == 0) off[0][0] = off[1][0] = 0;
        __syncthreads();
        for (int o = 1; o < 256; o <<= 1) {
            const int32_t v0 = x >= o ? off[0][x + 1 - o] : 0;
            const int32_t v1 = x >= o ? off[1][x + 1 - o] : 0;
            __syncthreads();
            off[0][x + 1] += v0;
            off[1][x + 1] += v1;
            __syncthreads();
        }
    }
    // flagged blocks before block x (x in [0, nb]; seg is a power of two)
    const int lseg = 31 - __clz(seg);
    auto before = [&](int q, int64_t x) -> int32_t {
        return off[q][x >> lseg] + (q ? pre1[x] : pre0[x]);
    };
    const int lane = lane_id();
    for (int64_t c0 = (int64_t)blockIdx.x * 256; c0 < n_chunks; c0 += (int64_t)gridDim.x * 256) {
        const int64_t c = c0 + threadIdx.x;
        bool keep = false;
        int tile = 0;
        int64_t origin = 0;
        if (c < n_chunks) {
            // the loads of the two tests are independent (issued together), as
            // is the list origin's
            tile = ctile[c];
            const int4 r = crng[c];
            origin = tchunk[tile];
            const int64_t s0 = (int64_t)r.x >> bs, s1 = ((int64_t)r.y >> bs) + 1;
            const int64_t d0 = (int64_t)r.z >> bs, d1 = ((int64_t)r.w >> bs) + 1;
            const bool any = r.y >= r.x;
            const int64_t e0 = any ? s0 : 0, e1 = any ? s1 : 0;
            const int64_t f0 = any ? d0 : 0, f1 = any ? d1 : 0;
            keep = any && before(0, e1) - before(0, e0) > 0;
            if (pre1) keep = keep && before(1, f1) - before(1, f0) > 0;
        }
        uint64_t pending = __ballot(keep);
        while (pending) {  // one round per distinct tile among the kept lanes
            const int leader = __builtin_ctzll(pending);
            const int t = __shfl(tile, leader);
            const uint64_t mine = __ballot(keep && tile == t);
            int32_t base = 0;
            if (lane == leader) base = atomicAdd(&ccount[t], __popcll(mine));
            base = __shfl(base, leader);
            if (keep && tile == t) clist[origin + base + __popcll(mine & ((1ull << lane) - 1ull))] = c;
            pending &= ~mine;
        }
    }
}

// Adds the last round's per-tile list lengths to *streamed (when not NULL).
__global__ __launch_bounds__(1024) void k_count_streamed(int32_t* __restrict__ ccount, int n_tiles,
                                                         unsigned long long* __restrict__ streamed) {
    count_and_clear(ccount, n_tiles, streamed);
}

// BFS output (Alg. 4) plus the reached-edge count used for TEPS: per-block
// partials (part[b] reached edges, part[kFinalBlocks + b] largest level) ...
__global__ __launch_bounds__(256) void k_bfs_final(int32_t n, const int32_t* __restrict__ lev,
                                                   const int32_t* __restrict__ deg,
                                                   unsigned long long* __restrict__ part) {
    __shared__ unsigned long long red[2][4];
    int32_t mx = 0;
    unsigned long long r = 0;
    for (int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x; v < n; v += (int64_t)gridDim.x * 256) {
        int32_t l = lev[v];
        if (l != kInf) {
            mx = l > mx ? l : mx;
            r += (unsigned long long)deg[v];
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
        mx = max(mx, __shfl_xor(mx, o));
        r += __shfl_xor(r, o);
    }
    if (lane_id() == 0) {
        red[0][threadIdx.x >> 6] = r;
        red[1][threadIdx.x >> 6] = (unsigned long long)mx;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long a = 0, b = 0;
        for (int w = 0; w < 4; ++w) {
            a += red[0][w];
            b = red[1][w] > b ? red[1][w] : b;
        }
        part[blockIdx.x] = a;
        part[kFinalBlocks + blockIdx.x] = b;
    }
}

// ... combined by one workgroup of kFinalBlocks threads into part[-2] (reached
// edges) and part[-1] (largest level).
__global__ __launch_bounds__(kFinalBlocks) void k_bfs_final_sum(unsigned long long* __restrict__ part) {
    __shared__ unsigned long long red[2][kFinalBlocks / 64];
    unsigned long long a = part[threadIdx.x], b = part[kFinalBlocks + threadIdx.x];
    for (int o = 32; o > 0; o >>= 1) {
        a += __shfl_xor(a, o);
        const unsigned long long y = __shfl_xor(b, o);
        b = y > b ? y : b;
    }
    if (lane_id() == 0) {
        red[0][threadIdx.x >> 6] = a;
        red[1][threadIdx.x >> 6] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long s = 0, m = 0;
        for (int w = 0; w < kFinalBlocks / 64; ++w) {
            s += red[0][w];
            m = red[1][w] > m ? red[1][w] : m;
        }
        part[-2] = s;
        part[-1] = m;
    }
}

// lambda^0 = g, and per-block partial sums of g (S^0).
__global__ __launch_bounds__(256) void k_init_adj(int32_t n, const double* __restrict__ gx,
                                                  double* __restrict__ cur,
                                                  double* __restrict__ part) {
    __shared__ double red[4];
    double s = 0.0;
    for (int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x; v < n; v += (int64_t)gridDim.x * 256) {
        cur[v] = gx[v];
        s += gx[v];
    }
    s = wave_sum(s);
    if (lane_id() == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// Extrapolation of a geometrically converging iterate along its last step:
// cur <- cur + c * (cur - prev), plus per-block partial sums of the result.
__global__ __launch_bounds__(256) void k_extrapolate(int32_t n, double* __restrict__ cur,
                                                     const double* __restrict__ prev, double c,
                                                     double* __restrict__ part) {
    __shared__ double red[4];
    double s = 0.0;
    for (int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x; v < n; v += (int64_t)gridDim.x * 256) {
        const double x = cur[v];
        const double y = x + c * (x - prev[v]);
        cur[v] = y;
        s += y;
    }
    s = wave_sum(s);
    if (lane_id() == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// dL/dw_e = d * x*[src_e] * lambda[dst_e], written at the input position of
// edge e (through the kept permutation). One wavefront per chunk; the source
// interval of every word is recovered from the markers as in k_iterate.
__global__ __launch_bounds__(256) void k_edge_grad(
    const uint32_t* __restrict__ words, const int32_t* __restrict__ crow,
    const int64_t* __restrict__ tchunk, int n_tiles, int64_t n_chunks, int C, int I, int L, int t,
    int sshift, int dshift, const int32_t* __restrict__ perm, const double* __restrict__ xs,
    const double* __restrict__ lam, double d, float* __restrict__ gw) {
    const int lane = lane_id();
    const uint64_t lt = (1ull << lane) - 1ull;
    const uint32_t lmask = (1u << L) - 1u, tmask = (1u << t) - 1u;
    const int64_t nw = (int64_t)gridDim.x * (blockDim.x >> 6);
    for (int64_t c = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); c < n_chunks; c += nw) {
        int lo = 0, hi = n_tiles;
        while (hi - lo > 1) {
            int mid = (lo + hi) >> 1;
            if (tchunk[mid] <= c)
                lo = mid;
            else
                hi = mid;
        }
        const int64_t tbase = (int64_t)lo << t;
        uint32_t row = (uint32_t)crow[c];
        const u32x4* wp = reinterpret_cast<const u32x4*>(words + c * (int64_t)C);
        for (int s = 0; s < (C >> 8); ++s) {
            const u32x4 w4 = wp[s * 64 + lane];
            const uint32_t w[4] = {w4.x, w4.y, w4.z, w4.w};
            const uint64_t mm = __ballot(((w[0] | w[1] | w[2] | w[3]) >> 31) != 0);
            uint32_t r = row;
            if (mm) {
                uint32_t last = 0;
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    if (w[k] & kMarker) last = w[k] & ~kMarker;
                const uint64_t prev = mm & lt;
                const uint32_t got = __shfl(last, prev ? 63 - __clzll(prev) : lane);
                r = prev ? got : row;
                row = (uint32_t)__builtin_amdgcn_readlane((int)(last), 63 - __clzll(mm));
            }
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                if (w[k] & kMarker) {
                    r = w[k] & ~kMarker;
                    continue;
                }
                const int64_t pos = c * (int64_t)C + (int64_t)s * 256 + lane * 4 + k;
                const int64_t src = (int64_t)r * I + ((w[k] >> sshift) & lmask);
                const int64_t dst = tbase + ((w[k] >> dshift) & tmask);
                gw[perm[pos]] = (float)(d * xs[src] * lam[dst]);
            }
        }
    }
}

// Vertex data between caller ids and the internal ids of a relabeled build:
// out[k*w + c] = f * in[idx[k]*w + c]. idx = new2old brings caller data in,
// idx = old2new hands results back; an id dropped by degreeing (idx[k] < 0)
// gets `fill`, or its own id k when own_id is set.
template <typename T>
__global__ __launch_bounds__(256) void k_permute_rows(const T* __restrict__ in,
                                                      const int32_t* __restrict__ idx, int64_t n,
                                                      int w, T f, T fill, int own_id,
                                                      T* __restrict__ out) {
    for (int64_t x = (int64_t)blockIdx.x * 256 + threadIdx.x; x < n * w;
         x += (int64_t)gridDim.x * 256) {
        const int64_t k = x / w;
        const int64_t c = x - k * w;
        const int32_t j = idx[k];
        out[x] = j >= 0 ? f * in[(int64_t)j * w + c] : (own_id ? (T)k : fill);
    }
}

__global__ void k_scale_copy(const double* __restrict__ a, double f, double* __restrict__ b, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        b[i] = f * a[i];
}


// ---------------------------------------------------------------------------
// Batched personalised PageRank: B value columns per vertex, stored [n, B]
// row-major. A wavefront processes one edge per step with lane b handling
// column b, so the source row is one coalesced load; sums along a run of equal
// destination stay in registers and reach the LDS accumulators [T, B] (FP64)
// once per run. Column b teleports to seeds[b] (one-hot), or uniformly when no
// seeds are given; the dangling mass and the residual are kept per column.
// ---------------------------------------------------------------------------
struct BCtl {
    double* stats;   // [(max_iters + 2) * 3 * B]: per iteration, per column: delta, resid, sum
    int32_t* done;
    int32_t k;
    double tol;
};

// The update of one tile from its accumulators acc[T][B] (lane = column), and
// the tile's per-column scalars (dangling mass, residual, sum) in tile_sb.
template <int WG>
__device__ void apply_batched(const Geo& g, const BCtl& ctl, const float* __restrict__ cur,
                              float* __restrict__ nxt, float* __restrict__ xout,
                              const int32_t* __restrict__ seeds, int B, double d,
                              double* __restrict__ tile_sb, int tile, double* acc) {
    const int lane = lane_id(), wave = threadIdx.x >> 6;
    const bool col = lane < B;
    const int cl = col ? lane : B - 1;
    const int64_t base = (int64_t)tile << g.t;
    int64_t len = min((int64_t)g.T, (int64_t)g.n - base);
    if (len < 0) len = 0;
    const double* sc = ctl.stats + (int64_t)ctl.k * 3 * B;
    const double delta = col ? sc[lane] : 0.0;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    const int32_t seed = (col && seeds) ? seeds[lane] : -1;
    // kR rows per wave at a time, their loads issued before the first update
    // (rows past the tile reload the wave's first row)
    constexpr int kR = 8;
    for (int64_t v0 = wave; v0 < len; v0 += kR * (WG / 64)) {
        float cv[kR];
        int32_t dgv[kR];
#pragma unroll
        for (int r = 0; r < kR; ++r) {
            const int64_t v = v0 + r * (WG / 64) < len ? v0 + r * (WG / 64) : v0;
            cv[r] = cur[(base + v) * B + cl];
            dgv[r] = g.deg[base + v];
        }
#pragma unroll
        for (int r = 0; r < kR; ++r) {
            const int64_t v = v0 + r * (WG / 64);
            if (v >= len || !col) continue;
            const int64_t gv = base + v;
            const int64_t o = gv * B + lane;
            const int32_t dg = dgv[r];
            const double xo = dg ? (double)cv[r] * dg : (double)cv[r];
            const double tv = seeds ? (gv == seed ? 1.0 : 0.0) : 1.0 / g.n;
            const double xn = d * (acc[v * B + lane] + delta / g.n) + (1.0 - d) * tv;
            const float xr = (float)xn;
            s1 += fabs((double)xr - xo);
            s2 += (double)xr;
            if (dg == 0) s0 += (double)xr;
            nxt[o] = dg ? (float)((double)xr / dg) : xr;
            if (xout) xout[o] = xr;
        }
    }
    __syncthreads();  // acc is reused as the reduction buffer
    double* red = acc;
    red[(0 * (WG / 64) + wave) * 64 + lane] = s0;
    red[(1 * (WG / 64) + wave) * 64 + lane] = s1;
    red[(2 * (WG / 64) + wave) * 64 + lane] = s2;
    __syncthreads();
    if (threadIdx.x < 3 * 64) {
        const int q = threadIdx.x >> 6, b = threadIdx.x & 63;
        double a = 0.0;
        for (int w = 0; w < WG / 64; ++w) a += red[(q * (WG / 64) + w) * 64 + b];
        if (b < B) tile_sb[((int64_t)tile * 3 + q) * B + b] = a;
    }
}

template <int WG>
__global__ __launch_bounds__(WG) void k_iterate_batched(Geo g, BCtl ctl, const float* __restrict__ cur,
                                                        float* __restrict__ nxt, float* __restrict__ xout,
                                                        const int32_t* __restrict__ seeds, int B,
                                                        double d, double* __restrict__ tile_sb) {
    extern __shared__ __align__(16) unsigned char smem[];
    double* acc = reinterpret_cast<double*>(smem);  // [T][B]
    const Item it = g.items[blockIdx.x];
    const int tile = it.tile;
    const int64_t base = (int64_t)tile << g.t;
    int64_t len = min((int64_t)g.T, (int64_t)g.n - base);
    if (len < 0) len = 0;
    // the wave index is uniform: chunk indices and interval rows then live in
    // scalar registers and their loads go through the scalar cache
    const int lane = lane_id(), wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint64_t lt = (1ull << lane) - 1ull;
    const bool col = lane < B;
    if (*ctl.done) {  // converged earlier: carry the vectors over
        if (it.piece == 0)
            for (int64_t v = wave; v < len; v += WG / 64)
                if (col) {
                    const int64_t o = (base + v) * B + lane;
                    nxt[o] = cur[o];
                    if (xout) {
                        const int32_t dg = g.deg[base + v];
                        xout[o] = dg ? (float)((double)cur[o] * dg) : cur[o];
                    }
                }
        return;
    }
    for (int64_t x = threadIdx.x; x < len * B; x += WG) acc[x] = 0.0;
    __syncthreads();
    const uint32_t lmask = (1u << g.L) - 1u, tmask = (1u << g.t) - 1u;
    // The wave walks the 64-word slices of its chunks (all in this item's tile).
    // A slice is decoded lane-parallel (one word per lane); its 64 edges are then
    // taken in two halves of 32, with the edge fields read out as wave-uniform
    // scalars, so a gather is one coalesced row load (lane = column) from a scalar
    // base. Gathers are unconditional (non-edges read row 0), and the next half's
    // 32 are issued before the current half's are used, so up to 64 rows per
    // wave are in flight; words are loaded two slices ahead. A run of equal
    // destinations is summed in registers and reaches the LDS accumulator once.
    constexpr int kH = 32;
    const int cl = col ? lane : B - 1;  // lanes past B read a valid column and discard it
    const int spc = g.C >> 6;           // slices per chunk
    const int64_t nch = it.c1 - it.c0 > wave ? (it.c1 - it.c0 - wave + WG / 64 - 1) / (WG / 64) : 0;
    const int64_t K = nch * spc;        // slices of this wave
    if (K > 0) {
        const uint32_t* const wbase = g.words;
        // word address of this wave's slice k (k clamped to the last one)
        auto slice_ptr = [&](int64_t k) -> const uint32_t* {
            const int64_t kc = k < K ? k : K - 1;
            const int64_t c = it.c0 + wave + (kc / spc) * (WG / 64);
            return wbase + c * (int64_t)g.C + (kc % spc) * 64;
        };
        uint32_t row = 0;
        // decodes slice k's words into per-lane source index and tile-local destination
        auto decode = [&](int64_t k, uint32_t wl, uint32_t& src_l, uint32_t& dst_l) {
            if (k % spc == 0) row = (uint32_t)g.chunk_row[it.c0 + wave + (k / spc) * (WG / 64)];
            const uint64_t mm = __ballot((wl >> 31) != 0);
            uint32_t r = row;
            if (mm) {
                const uint64_t upto = mm & (lt | (1ull << lane));
                const uint32_t got = __shfl(wl & ~kMarker, upto ? 63 - __clzll(upto) : lane);
                r = upto ? got : row;
                row = (uint32_t)__builtin_amdgcn_readlane((int)(wl & ~kMarker), 63 - __clzll(mm));
            }
            const bool edge = (wl >> 31) == 0;
            src_l = edge ? r * (uint32_t)g.I + ((wl >> g.sshift) & lmask) : 0u;
            dst_l = edge ? ((wl >> g.dshift) & tmask) : kNoDst;
        };
        auto issue = [&](float* v, uint32_t src_l, int j0) {
#pragma unroll
            for (int q = 0; q < kH; ++q) {
                const uint32_t sj = (uint32_t)__builtin_amdgcn_readlane((int)src_l, j0 + q);
                v[q] = cur[(int64_t)sj * B + cl];
            }
        };
        uint32_t pd = kNoDst;
        double pv = 0.0;
        auto consume = [&](const float* v, uint32_t dst_l, int j0) {
#pragma unroll
            for (int q = 0; q < kH; ++q) {
                const uint32_t dj = (uint32_t)__builtin_amdgcn_readlane((int)dst_l, j0 + q);
                if (dj == kNoDst) continue;
                if (dj != pd) {
                    if (pd != kNoDst && col) atomicAdd(&acc[(int64_t)pd * B + lane], pv);
                    pd = dj;
                    pv = 0.0;
                }
                pv += (double)v[q];
            }
        };
        float vA[kH], vB[kH];
        uint32_t sc, dc;
        uint32_t w0 = __builtin_nontemporal_load(slice_ptr(0) + lane);
        uint32_t wn = __builtin_nontemporal_load(slice_ptr(1) + lane);
        decode(0, w0, sc, dc);
        issue(vA, sc, 0);
        for (int64_t k = 0; k < K; ++k) {
            issue(vB, sc, kH);  // second half of slice k
            consume(vA, dc, 0);
            // first half of slice k + 1; after the last slice the (discarded)
            // gathers all read row 0, with no branch around them
            const bool more = k + 1 < K;
            uint32_t sn, dn;
            decode(more ? k + 1 : k, wn, sn, dn);
            sn = more ? sn : 0u;
            wn = __builtin_nontemporal_load(slice_ptr(k + 2) + lane);
            issue(vA, sn, 0);
            consume(vB, dc, kH);
            sc = sn;
            dc = dn;
        }
        if (pd != kNoDst && col) atomicAdd(&acc[(int64_t)pd * B + lane], pv);
    }
    __syncthreads();
    if (it.npieces > 1) {  // partial to the hub slot; k_finish_batched combines them
        double* part = reinterpret_cast<double*>(g.partial) + (int64_t)(it.slot + it.piece) * g.T * B;
        for (int64_t x = threadIdx.x; x < len * B; x += WG) part[x] = acc[x];
        return;
    }
    apply_batched<WG>(g, ctl, cur, nxt, xout, seeds, B, d, tile_sb, tile, acc);
}

// One workgroup per split tile: hub slots summed in piece order, then the update.
template <int WG>
__global__ __launch_bounds__(WG) void k_finish_batched(Geo g, BCtl ctl, const float* __restrict__ cur,
                                                       float* __restrict__ nxt, float* __restrict__ xout,
                                                       const int32_t* __restrict__ seeds, int B,
                                                       double d, double* __restrict__ tile_sb,
                                                       const Item* __restrict__ fin) {
    extern __shared__ __align__(16) unsigned char smem[];
    double* acc = reinterpret_cast<double*>(smem);  // [T][B]
    if (*ctl.done) return;
    const Item it = fin[blockIdx.x];
    const int64_t base = (int64_t)it.tile << g.t;
    int64_t len = min((int64_t)g.T, (int64_t)g.n - base);
    if (len < 0) len = 0;
    const double* p0 = reinterpret_cast<const double*>(g.partial) + (int64_t)it.slot * g.T * B;
    for (int64_t x = threadIdx.x; x < len * B; x += WG) {
        double sum = 0.0;
        for (int p = 0; p < it.npieces; ++p) sum += __builtin_nontemporal_load(p0 + (int64_t)p * g.T * B + x);
        acc[x] = sum;
    }
    __syncthreads();
    apply_batched<WG>(g, ctl, cur, nxt, xout, seeds, B, d, tile_sb, it.tile, acc);
}

// Per-column scalars of one iteration, in two deterministic passes: block r sums
// tiles [r*per, (r+1)*per) in tile order (thread = (scalar, column)); then one
// block sums the block partials in order and sets the stop flag.
__global__ __launch_bounds__(256) void k_reduce_batched1(const double* __restrict__ tile_sb, int n_tiles,
                                                         int B, int per, const int32_t* __restrict__ done,
                                                         double* __restrict__ part) {
    if (*done) return;
    const int j = threadIdx.x;  // (q, b) = (j / B, j % B)
    if (j >= 3 * B) return;
    const int t0 = blockIdx.x * per, t1 = min(n_tiles, t0 + per);
    double a = 0.0;
    for (int x = t0; x < t1; ++x) a += tile_sb[(int64_t)x * 3 * B + j];
    part[(int64_t)blockIdx.x * 3 * B + j] = a;
}

__global__ __launch_bounds__(256) void k_reduce_batched2(const double* __restrict__ part, int nblocks, int B,
                                                         BCtl ctl) {
    __shared__ double res[64];
    if (*ctl.done) return;
    const int j = threadIdx.x;
    if (j < 3 * B) {
        double a = 0.0;
        for (int r = 0; r < nblocks; ++r) a += part[(int64_t)r * 3 * B + j];
        const int q = j / B, b = j % B;
        double* so = ctl.stats + (int64_t)(q == 0 ? ctl.k + 1 : ctl.k) * 3 * B;
        so[q * B + b] = a;  // q=0: delta entering k+1 at [k+1][0][b]; q=1,2: [k][q][b]
        if (q == 1) res[b] = a;
    }
    __syncthreads();
    if (threadIdx.x == 0 && ctl.tol > 0.0) {
        double mx = 0.0;
        for (int b = 0; b < B; ++b) mx = fmax(mx, res[b]);
        if (mx <= ctl.tol) *ctl.done = 1;
    }
}

// x^0 = t per column (one-hot at seeds[b], or uniform); per-block per-column
// dangling partial sums.
__global__ __launch_bounds__(256) void k_init_batched(int32_t n, int B, const int32_t* __restrict__ deg,
                                                      const int32_t* __restrict__ seeds,
                                                      float* __restrict__ cur,
                                                      double* __restrict__ part) {
    // cur[v*B + b]
    const int64_t total = (int64_t)n * B;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < total; i += (int64_t)gridDim.x * 256) {
        const int64_t v = i / B;
        const int b = (int)(i - v * B);
        const double x = seeds ? (v == seeds[b] ? 1.0 : 0.0) : 1.0 / n;
        const int32_t dg = deg[v];
        cur[i] = dg ? (float)(x / dg) : (float)x;
    }
    (void)part;
}

// delta^0[b] = sum over dangling v of x^0[v][b]. One-hot columns read their
// seed's degree; uniform columns all get (dangling vertices) / n, counted by
// k_count_dangling's fixed grid (per-workgroup counts, integers, so exact in any
// order) and summed here in workgroup order.
constexpr int kDangBlocks = 256;

__global__ __launch_bounds__(256) void k_count_dangling(int32_t n, const int32_t* __restrict__ deg,
                                                        unsigned long long* __restrict__ part) {
    __shared__ unsigned long long red[4];
    unsigned long long c = 0;
    for (int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x; v < n; v += (int64_t)kDangBlocks * 256)
        c += deg[v] == 0 ? 1ull : 0ull;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off);
    if (lane_id() == 0) red[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

__global__ __launch_bounds__(64) void k_init_batched_delta(int32_t n, int B, const int32_t* __restrict__ deg,
                                                           const int32_t* __restrict__ seeds,
                                                           const unsigned long long* __restrict__ part,
                                                           double* __restrict__ stats) {
    if (threadIdx.x >= B) return;
    if (seeds) {
        stats[threadIdx.x] = deg[seeds[threadIdx.x]] == 0 ? 1.0 : 0.0;
        return;
    }
    unsigned long long tot = 0;
    for (int w = 0; w < kDangBlocks; ++w) tot += part[w];
    stats[threadIdx.x] = (double)tot / n;
}

// Weights in stream order from weights in input order (words that hold an edge).
__global__ void k_set_weights(const int32_t* __restrict__ perm, int64_t n_words,
                              const float* __restrict__ win, float* __restrict__ wout) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_words;
         i += (int64_t)gridDim.x * blockDim.x) {
        int32_t e = perm[i];
        wout[i] = e >= 0 ? win[e] : 0.0f;
    }
}

template <typename V>
__global__ void k_fill_val(V* __restrict__ p, int64_t n, V v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

template <typename V>
__global__ void k_copy(const V* __restrict__ a, V* __restrict__ b, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        b[i] = a[i];
}

inline int grid_for(int64_t work, int threads = 256, int cap = 8192) {
    int64_t b = (work + threads - 1) / threads;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return (int)b;
}

// Sets n elements to v with a kernel (no memset node, so it can be captured).
template <typename V>
void fill(V* p, int64_t n, V v, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_fill_val<V>, dim3(grid_for(n)), dim3(256), 0, s, p, n, v);
    NXG_CHECK_LAUNCH();
}

// Where a run's workspace comes from: the allocator (no arena), or a device
// region the caller owns, carved into 256-byte aligned pieces. A measuring
// arena touches nothing and only counts the bytes the run would take.
struct Arena {
    unsigned char* base = nullptr;
    size_t cap = 0, used = 0;
    bool measure = false;
    hipEvent_t e0 = nullptr, e1 = nullptr;  // timing events the region's owner keeps
    void take(DevBuf& b, size_t bytes) {
        bytes = bytes ? bytes : 16;
        const size_t off = (used + 255) & ~(size_t)255;
        used = off + bytes;
        if (measure) return;
        if (used > cap) fail(NXG_EINVAL, "run workspace exceeds the scratch region");
        b.borrow(base + off, bytes);
    }
};

inline void take(DevBuf& b, size_t bytes, hipStream_t s, Arena* a) {
    if (a)
        a->take(b, bytes);
    else
        b.alloc(bytes, s);
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------

int env_int(const char* name, int dflt) {
    const char* v = getenv(name);
    return v && *v ? atoi(v) : dflt;
}

int num_cus(int device) {
    int cu = 0;
    if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || cu < 1)
        cu = 256;
    return cu;
}

// Splits every tile into pieces of at most piece_chunks chunks; heavy tiles
// first. With whole_tiles every piece carries the tile's full chunk range (the
// pieces then split the tile's compacted active list at run time).
// Fisher-Yates shuffle driven by splitmix64 (a fixed, seeded order).
template <class T>
void shuffle_items(std::vector<T>& v, uint64_t seed) {
    uint64_t x = seed;
    for (size_t i = v.size(); i > 1; --i) {
        x += 0x9E3779B97F4A7C15ull;
        uint64_t z = x;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        z ^= z >> 31;
        std::swap(v[i - 1], v[(size_t)(z % i)]);
    }
}

// A cache entry added to a handle before it is complete: if an error is thrown
// while it is being set up, it is taken out again, so no later run finds it
// half made.
struct PendingEntry {
    nxg_dsss* g;
    Cached* c;
    PendingEntry(nxg_dsss* g_, Cached* c_) : g(g_), c(c_) {}
    PendingEntry(const PendingEntry&) = delete;
    PendingEntry& operator=(const PendingEntry&) = delete;
    ~PendingEntry() {
        if (!c) return;
        auto it = std::find(g->cached.begin(), g->cached.end(), c);
        if (it != g->cached.end()) g->cached.erase(it);
        delete c;
    }
    void commit() { c = nullptr; }
};

// Captured runs kept per handle and kind; a new capture beyond this releases
// the least recently used one of its kind.
constexpr int kMaxCaptures = 8;

// Moves cached entry e to the back of the handle's list (most recently used).
void touch_cached(nxg_dsss* g, Cached* e) {
    auto it = std::find(g->cached.begin(), g->cached.end(), e);
    if (it != g->cached.end()) {
        g->cached.erase(it);
        g->cached.push_back(e);
    }
}

// Before a new capture of kind C: if the handle already keeps kMaxCaptures of
// them, releases the least recently used (after the device has drained, since
// its graph may still be running on some stream).
template <class C>
void evict_captures(nxg_dsss* g) {
    int cnt = 0;
    for (Cached* c : g->cached)
        if (dynamic_cast<C*>(c)) ++cnt;
    if (cnt < kMaxCaptures) return;
    NXG_HIP(hipDeviceSynchronize());
    for (auto it = g->cached.begin(); it != g->cached.end(); ++it)
        if (dynamic_cast<C*>(*it)) {
            delete *it;
            g->cached.erase(it);
            return;
        }
}

Plan* find_plan(nxg_dsss* g, const Layout& L, int piece_chunks, bool whole_tiles, bool tile_order) {
    for (Plan* p : g->plans)
        if (p->layout == &L && p->piece_chunks == piece_chunks && p->whole_tiles == whole_tiles &&
            p->tile_order == tile_order)
            return p;
    return nullptr;
}

Plan* get_plan(nxg_dsss* g, const Layout& L, int piece_chunks, bool whole_tiles, hipStream_t s,
               bool tile_order = false) {
    if (Plan* q = find_plan(g, L, piece_chunks, whole_tiles, tile_order)) return q;
    std::unique_ptr<Plan> owner(new Plan());  // released to the handle once complete
    Plan* p = owner.get();
    p->layout = &L;
    p->tile_order = tile_order;
    p->piece_chunks = piece_chunks;
    p->whole_tiles = whole_tiles;
    std::vector<Item> items;
    int slots = 0;
    for (int tau = 0; tau < L.n_tiles; ++tau) {
        int64_t c0 = L.h_tile_chunk[tau], c1 = L.h_tile_chunk[tau + 1];
        int64_t nc = c1 - c0;
        int np = 1;
        // (a negative piece_chunks only keys the whole-tile plans apart)
        const int64_t pcs = piece_chunks < 0 ? -(int64_t)piece_chunks : piece_chunks;
        if (pcs > 0 && nc > pcs) np = (int)((nc + pcs - 1) / pcs);
        int slot = np > 1 ? slots : -1;
        if (np > 1) slots += np;
        for (int pc = 0; pc < np; ++pc) {
            Item it;
            it.tile = tau;
            it.piece = pc;
            it.npieces = np;
            it.slot = slot;
            if (whole_tiles) {
                it.c0 = c0;
                it.c1 = c1;
            } else {
                it.c0 = c0 + nc * pc / np;
                it.c1 = c0 + nc * (pc + 1) / np;
            }
            items.push_back(it);
        }
    }
    if (!tile_order) {
        std::stable_sort(items.begin(), items.end(), [np_whole = whole_tiles](const Item& a, const Item& b) {
            int64_t wa = np_whole ? (a.c1 - a.c0) / a.npieces : a.c1 - a.c0;
            int64_t wb = np_whole ? (b.c1 - b.c0) / b.npieces : b.c1 - b.c0;
            return wa > wb;
        });
        // debug schedule: the work items (and below the finishing segments) in a
        // seeded random order instead, to show the results do not depend on it
        if (g->flags & NXG_BUILD_SHUFFLE_SCHEDULE) shuffle_items(items, 0x9E3779B97F4A7C15ull ^ items.size());
    }
    p->h_items = items;
    p->n_slots = slots;
    p->items.alloc(sizeof(Item) * std::max<size_t>(items.size(), 1), s);
    NXG_HIP(hipMemcpyAsync(p->items.p, items.data(), sizeof(Item) * items.size(),
                           hipMemcpyHostToDevice, s));
    for (const Item& it : items)
        if (it.npieces > 1 && it.piece == 0) p->h_fin.push_back(it);
    p->fin.alloc(sizeof(Item) * std::max<size_t>(p->h_fin.size(), 1), s);
    if (!p->h_fin.empty())
        NXG_HIP(hipMemcpyAsync(p->fin.p, p->h_fin.data(), sizeof(Item) * p->h_fin.size(),
                               hipMemcpyHostToDevice, s));
    // segments of kFinSeg vertices; scalar slots n_tiles, n_tiles + 1, ... in list order
    for (const Item& it : p->h_fin) {
        const int64_t base = (int64_t)it.tile * L.T;
        const int64_t len = std::max<int64_t>(0, std::min<int64_t>(L.T, (int64_t)L.n - base));
        for (int64_t v0 = 0; v0 < len; v0 += kFinSeg) {
            FinSeg f;
            f.tile = it.tile;
            f.npieces = it.npieces;
            f.slot = it.slot;
            f.v0 = (int32_t)v0;
            f.vlen = (int32_t)std::min<int64_t>(kFinSeg, len - v0);
            f.sslot = L.n_tiles + (int32_t)p->h_fseg.size();
            p->h_fseg.push_back(f);
        }
    }
    if (g->flags & NXG_BUILD_SHUFFLE_SCHEDULE) {
        // segments in a random order; their scalar slots keep the segment order,
        // so a segment's slot moves with it
        shuffle_items(p->h_fseg, 0xD1B54A32D192ED03ull ^ p->h_fseg.size());
        for (size_t i = 0; i < p->h_fseg.size(); ++i) p->h_fseg[i].sslot = L.n_tiles + (int32_t)i;
    }
    p->fseg.alloc(sizeof(FinSeg) * std::max<size_t>(p->h_fseg.size(), 1), s);
    if (!p->h_fseg.empty())
        NXG_HIP(hipMemcpyAsync(p->fseg.p, p->h_fseg.data(), sizeof(FinSeg) * p->h_fseg.size(),
                               hipMemcpyHostToDevice, s));
    NXG_HIP(hipStreamSynchronize(s));
    g->plans.push_back(owner.release());
    return p;
}

struct Workspace {
    DevBuf buf[2], partial, tile_s, tile_flag, stats, done, blk, bpre, btot, clist,
        ccount, part, bfsout;
    DevBuf mtele, mvals, mseeds, mgx, mxs;  // caller data in internal ids (relabeled builds)
};

// Two timing events, released on every exit path (an error throws).
struct Events {
    hipEvent_t a = nullptr, b = nullptr;
    Events() {
        NXG_HIP(hipEventCreate(&a));
        if (hipEventCreate(&b) != hipSuccess) {
            (void)hipEventDestroy(a);
            a = nullptr;
            fail(NXG_EDEVICE, "hipEventCreate failed");
        }
    }
    Events(const Events&) = delete;
    Events& operator=(const Events&) = delete;
    ~Events() {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
};

// What a multi-graph handle keeps between runs: per-graph workspaces, the
// descriptor and item arrays (device and host).
struct MultiCache : Cached {
    int iters = 0, piece = 0, per_iter = 0, n_fin = 0;
    size_t lds = 0;
    std::vector<Workspace> ws;
    std::vector<MultiGraph> hdesc;
    DevBuf ditems, dgraph, ddesc, dfin, dres, dpart;
    // NXG_RUN_CAPTURE: the run's launches recorded once (they read the graph
    // descriptors, so each run's output buffers reach them through ddesc)
    double cap_damping = 0.0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    void drop_graph() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        exec = nullptr;
        graph = nullptr;
    }
    ~MultiCache() override { drop_graph(); }
};

// Index arrays of a relabeled or degreed build (both NULL otherwise); n is the
// caller's id range (results are handed back over all of it).
struct VMap {
    const int32_t* n2o = nullptr;
    const int32_t* o2n = nullptr;
    int64_t n = 0;
    explicit operator bool() const { return n2o != nullptr; }
};

VMap vmap_of(const nxg_dsss* g) {
    VMap m;
    if (g->relabeled) {
        m.n2o = g->new2old.as<int32_t>();
        m.o2n = g->old2new.as<int32_t>();
        m.n = g->n_caller;
    }
    return m;
}

template <typename T>
void permute_rows(const T* in, const int32_t* idx, int64_t n, int w, T* out, hipStream_t s,
                  T f = (T)1, T fill = (T)0, int own_id = 0) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_permute_rows<T>, dim3(grid_for(n * w, 256, 8192)), dim3(256), 0, s, in, idx,
                       n, w, f, fill, own_id, out);
    NXG_CHECK_LAUNCH();
}

template <class Prog, int WG>
void prepare_iter(size_t lds) {
    static size_t attr_lds = 0;
    if (lds > attr_lds) {
        NXG_HIP(hipFuncSetAttribute((const void*)k_iterate<Prog, WG, false>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        NXG_HIP(hipFuncSetAttribute((const void*)k_iterate<Prog, WG, true>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        attr_lds = lds;
    }
}

// The edge kernel of one iteration for the stream's edge order.
template <class Prog, int WG>
void launch_items(int n_items, size_t lds, hipStream_t s, const Geo& geo, const Ctl& ctl, const Prog& prog) {
    if (geo.order == NXG_ORDER_DST)
        hipLaunchKernelGGL((k_iterate<Prog, WG, true>), dim3(n_items), dim3(WG), lds, s, geo, ctl, prog);
    else
        hipLaunchKernelGGL((k_iterate<Prog, WG, false>), dim3(n_items), dim3(WG), lds, s, geo, ctl, prog);
    NXG_CHECK_LAUNCH();
}

// A host-resident edge stream (NXG_BUILD_HOST_STREAM) is fed to the edge
// kernel through two device staging buffers: the items run in stream order, in
// batches of whole items whose chunks fit one buffer, and the copy of batch j+1
// (on a copy stream) overlaps the edge work of batch j. The batch counter runs
// on across iterations, so the copy of the next iteration's first batch also
// overlaps this iteration's finishing launches.
struct Streamer {
    struct Batch {
        int i0, i1;      // items [i0, i1)
        int64_t c0, c1;  // their chunks [c0, c1)
    };
    const Layout* L = nullptr;
    const Plan* p = nullptr;
    std::vector<Batch> batches;
    DevBuf wst[2], fst[2];
    hipStream_t cs = nullptr;
    hipEvent_t copied[2] = {nullptr, nullptr}, used[2] = {nullptr, nullptr};
    int64_t issued = 0, launched = 0;
    ~Streamer() {
        for (int b = 0; b < 2; ++b) {
            if (copied[b]) (void)hipEventDestroy(copied[b]);
            if (used[b]) (void)hipEventDestroy(used[b]);
        }
        if (cs) (void)hipStreamDestroy(cs);
    }
    void init(const Layout& lay, const Plan& plan, int64_t cap_chunks, hipStream_t s) {
        L = &lay;
        p = &plan;
        const std::vector<Item>& it = plan.h_items;
        for (int i = 0; i < (int)it.size(); ++i) {
            if (it[i].c1 == it[i].c0) {  // an empty tile rides with its neighbours
                if (batches.empty()) batches.push_back(Batch{i, i + 1, it[i].c0, it[i].c1});
                else batches.back().i1 = i + 1;
                continue;
            }
            if (batches.empty() || it[i].c1 - batches.back().c0 > cap_chunks)
                batches.push_back(Batch{i, i + 1, it[i].c0, it[i].c1});
            else {
                batches.back().i1 = i + 1;
                batches.back().c1 = it[i].c1;
            }
        }
        int64_t most = 1;
        for (const Batch& b : batches) most = std::max<int64_t>(most, b.c1 - b.c0);
        for (int b = 0; b < 2; ++b) {
            wst[b].alloc(sizeof(uint32_t) * (size_t)most * lay.C, s);
            if (lay.has_weight) fst[b].alloc(sizeof(float) * (size_t)most * lay.C, s);
            NXG_HIP(hipEventCreateWithFlags(&copied[b], hipEventDisableTiming));
            NXG_HIP(hipEventCreateWithFlags(&used[b], hipEventDisableTiming));
        }
        NXG_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
        NXG_HIP(hipStreamSynchronize(s));  // the staging buffers exist before cs uses them
    }
    // copy of global batch j into buffer j & 1, once the edge work of j - 2 is done
    void issue(int64_t j) {
        const int buf = (int)(j & 1);
        const Batch& b = batches[j % (int64_t)batches.size()];
        if (j >= 2) NXG_HIP(hipStreamWaitEvent(cs, used[buf], 0));
        const size_t off = (size_t)b.c0 * L->C, cnt = (size_t)(b.c1 - b.c0) * L->C;
        if (cnt) {
            NXG_HIP(hipMemcpyAsync(wst[buf].p, L->h_words.as<uint32_t>() + off, sizeof(uint32_t) * cnt,
                                   hipMemcpyHostToDevice, cs));
            if (L->has_weight)
                NXG_HIP(hipMemcpyAsync(fst[buf].p, L->h_weight.as<float>() + off, sizeof(float) * cnt,
                                       hipMemcpyHostToDevice, cs));
        }
        NXG_HIP(hipEventRecord(copied[buf], cs));
    }
    // the edge kernel over every batch of one iteration
    template <class Prog, int WG>
    void launch(const Geo& geo, const Ctl& ctl, const Prog& prog, size_t lds, hipStream_t s) {
        for (size_t bi = 0; bi < batches.size(); ++bi) {
            const int64_t j = launched;
            while (issued <= j) issue(issued++);
            const int buf = (int)(j & 1);
            const Batch& b = batches[bi];
            NXG_HIP(hipStreamWaitEvent(s, copied[buf], 0));
            // the kernel indexes words by global chunk: the buffer holds chunks
            // [c0, c1), so its base is shifted back by c0 chunks (only
            // [c0, c1) is ever read through it)
            Geo gb = geo;
            gb.items = p->items.as<Item>() + b.i0;
            gb.words = reinterpret_cast<const uint32_t*>(reinterpret_cast<uintptr_t>(wst[buf].p) -
                                                         (uintptr_t)b.c0 * L->C * sizeof(uint32_t));
            Prog pb = prog;
            if constexpr (Prog::kWeights)
                pb.w = reinterpret_cast<const float*>(reinterpret_cast<uintptr_t>(fst[buf].p) -
                                                      (uintptr_t)b.c0 * L->C * sizeof(float));
            if (b.i1 > b.i0) launch_items<Prog, WG>(b.i1 - b.i0, lds, s, gb, ctl, pb);
            NXG_HIP(hipEventRecord(used[buf], s));
            ++launched;
            if (issued == launched) issue(issued++);  // the next batch into the other buffer
        }
    }
};

// One iteration: the items, the split tiles, the scalar reduction (no memsets,
// so it can be recorded into a hipGraph).
template <class Prog, int WG>
void launch_iter(const Geo& geo, const Ctl& ctl, const Prog& prog, const Plan& p, size_t lds,
                 hipStream_t s, Streamer* str = nullptr) {
    prepare_iter<Prog, WG>(lds);
    const int n_items = (int)p.h_items.size();
    if (str) {
        str->launch<Prog, WG>(geo, ctl, prog, lds, s);
    } else if (n_items > 0) {
        launch_items<Prog, WG>(n_items, lds, s, geo, ctl, prog);
    }
    if (!p.h_fseg.empty()) {
        hipLaunchKernelGGL((k_finish<Prog, kFinWG>), dim3((int)p.h_fseg.size()), dim3(kFinWG),
                           kFinSeg * sizeof(typename Prog::acc_t), s, geo, ctl, prog, p.fseg.as<FinSeg>());
        NXG_CHECK_LAUNCH();
    }
    if constexpr (!Prog::kActivity) {
        hipLaunchKernelGGL((k_reduce<Prog, 1024>), dim3(1), dim3(1024), 0, s, geo, ctl);
        NXG_CHECK_LAUNCH();
    }
}

// Plain PageRank on either stream layout (the pair layout decodes more word kinds).
template <typename V>
void launch_plain_pr(const Layout& L, const Geo& geo, const Ctl& ctl, const ProgPR<V>& pr, const Plan& p,
                     size_t lds, hipStream_t s, Streamer* str = nullptr) {
    if (L.pairs)
        launch_iter<ProgPRP<V>, 1024>(geo, ctl, ProgPRP<V>{pr}, p, lds, s, str);
    else
        launch_iter<ProgPR<V>, 1024>(geo, ctl, pr, p, lds, s, str);
}

// ab = bytes of one LDS accumulator of the program.
Geo make_geo(const Layout& L, const Plan& p, Workspace& w, size_t ab) {
    Geo g;
    g.words = L.words.as<uint32_t>();
    g.chunk_row = L.chunk_row.as<int32_t>();
    g.chunk_src = L.pairs ? L.chunk_src.as<int32_t>() : nullptr;
    g.items = p.items.as<Item>();
    g.deg = L.outdeg.as<int32_t>();
    g.n = L.n;
    g.I = L.I;
    g.P = L.P;
    g.L = L.L;
    g.T = L.T;
    g.t = L.t;
    g.sshift = L.order == NXG_ORDER_SRC ? L.t : 0;
    g.dshift = L.order == NXG_ORDER_SRC ? 0 : L.L;
    g.order = L.order;
    g.n_tiles = L.n_tiles;
    g.C = L.C;
    g.partial = w.partial.p;
    g.tile_s = w.tile_s.as<double>();
    g.tile_flag = w.tile_flag.as<int32_t>();
    g.n_sslots = L.n_tiles + (int32_t)p.h_fseg.size();
    g.clist = nullptr;
    g.ccount = nullptr;
    g.split_min = 0;
    return g;
}

// Dynamic LDS of one iteration launch: the tile's accumulators plus one
// discard slot per lane.
size_t iter_lds(const Geo&, const Layout& L, size_t ab) { return ((size_t)L.T + kSpill) * ab; }

void alloc_common(Workspace& w, const Layout& L, const Plan& p, size_t vb, int max_iters,
                  hipStream_t s, bool min_identity, Arena* a = nullptr) {
    // one tile-sized partial per piece of a split tile (written before read)
    (void)min_identity;
    const int64_t hub_elems = (int64_t)std::max(p.n_slots, 1) * L.T;
    take(w.partial, (size_t)hub_elems * vb, s, a);
    const size_t slots = (size_t)L.n_tiles + p.h_fseg.size();
    take(w.tile_s, sizeof(double) * 3 * slots, s, a);
    take(w.tile_flag, sizeof(int32_t) * slots, s, a);
    take(w.stats, sizeof(double) * 4 * (size_t)(max_iters + 2), s, a);
    take(w.done, sizeof(int32_t), s, a);
    if (a && a->measure) return;
    // stats and the stop flag start at zero (scratch memory keeps the last run's)
    fill<double>(w.stats.as<double>(), 4 * (int64_t)(max_iters + 2), 0.0, s);
    fill<int32_t>(w.done.as<int32_t>(), 1, 0, s);
}

// A PageRank run recorded into a hipGraph (NXG_RUN_CAPTURE) with the
// workspace it uses; replayed when a later run asks for the same thing.
struct CapturedPR : Cached {
    int program = 0, dtype = 0, iters = 0, piece = 0;
    uint32_t flags = 0;
    double damping = 0.0;
    const void* values = nullptr;
    const void* tele = nullptr;
    const void* stats_out = nullptr;
    Workspace w;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    ~CapturedPR() override {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
    }
};

// A batched personalised PageRank run recorded into a hipGraph (NXG_RUN_CAPTURE)
// with its workspace; replayed when a later run has the same width, iteration
// count, piece size, damping, seed and output buffers. Each call still checks
// the seeds (and maps them to internal ids) before the replay.
struct CapturedBatched : Cached {
    int B = 0, iters = 0, piece = 0;
    double damping = 0.0;
    const void* values = nullptr;
    const void* seeds = nullptr;
    Workspace w;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    ~CapturedBatched() override {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
    }
};

// The run's per-iteration statistics into the caller's device buffer (if any).
void copy_stats_out(const Workspace& w, const nxg_run_desc& d, hipStream_t s) {
    if (!d.d_stats || d.max_iters < 1) return;
    const int64_t cnt = 4 * (int64_t)d.max_iters;
    hipLaunchKernelGGL(k_copy<double>, dim3(grid_for(cnt)), dim3(256), 0, s, w.stats.as<double>(),
                       d.d_stats, cnt);
    NXG_CHECK_LAUNCH();
}

// Enqueues x^0 and max_iters iterations of (weighted) PageRank; no syncs.
template <typename V>
void enqueue_pagerank(const Layout& L, const Plan& p, Workspace& w, const nxg_run_desc& d,
                      bool weighted, const VMap& vm, hipStream_t s) {
    const int nb = grid_for(L.n, 256, 1024);
    const V* tele = (const V*)d.d_teleport;
    V* vals = (V*)d.d_values;
    if (vm) {
        if (tele) {
            permute_rows<V>(tele, vm.n2o, L.n, 1, w.mtele.as<V>(), s);
            tele = w.mtele.as<V>();
        }
        if (d.flags & NXG_RUN_WARM_START) permute_rows<V>(vals, vm.n2o, L.n, 1, w.mvals.as<V>(), s);
        vals = w.mvals.as<V>();
    }
    const V* x0 = (d.flags & NXG_RUN_WARM_START) ? vals : nullptr;
    hipLaunchKernelGGL(k_init_pr<V>, dim3(nb), dim3(256), 0, s, L.n, L.outdeg.as<int32_t>(),
                       tele, x0, weighted ? 0 : 1, w.buf[0].as<V>(), w.part.as<double>());
    NXG_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(64), 0, s, w.part.as<double>(), nb,
                       w.stats.as<double>());
    NXG_CHECK_LAUNCH();
    Geo geo = make_geo(L, p, w, sizeof(double));
    const size_t lds = iter_lds(geo, L, sizeof(double));
    for (int k = 0; k < d.max_iters; ++k) {
        Ctl ctl{w.stats.as<double>(), w.done.as<int32_t>(), k, 0.0};
        const V* cur = w.buf[k & 1].as<V>();
        V* nxt = w.buf[(k + 1) & 1].as<V>();
        V* xout = (k == d.max_iters - 1) ? vals : nullptr;
        if (weighted) {
            ProgPRW<V> pr{cur, nxt, tele, xout, L.weight.as<float>(), d.damping};
            launch_iter<ProgPRW<V>, 1024>(geo, ctl, pr, p, lds, s);
        } else {
            ProgPR<V> pr{cur, nxt, tele, xout, d.damping};
            launch_plain_pr<V>(L, geo, ctl, pr, p, lds, s);
        }
    }
    if (vm) permute_rows<V>(vals, vm.o2n, vm.n, 1, (V*)d.d_values, s);
    copy_stats_out(w, d, s);
}

template <typename V>
nxg_status run_pagerank_captured(nxg_dsss* g, const nxg_run_desc& d, hipStream_t s,
                                 nxg_run_stats* st, int piece) {
    const Layout& L = g->fwd;
    const bool weighted = d.program == NXG_PAGERANK_WEIGHTED;
    if (d.tol > 0) fail(NXG_EINVAL, "NXG_RUN_CAPTURE needs a fixed iteration count (tol <= 0)");
    if (d.max_iters < 1) fail(NXG_EINVAL, "NXG_RUN_CAPTURE needs max_iters >= 1");
    CapturedPR* e = nullptr;
    for (Cached* c : g->cached) {
        CapturedPR* r = dynamic_cast<CapturedPR*>(c);
        if (r && r->program == d.program && r->dtype == d.dtype && r->iters == d.max_iters &&
            r->piece == piece && r->flags == d.flags && r->damping == d.damping &&
            r->values == d.d_values && r->tele == d.d_teleport && r->stats_out == d.d_stats) {
            e = r;
            break;
        }
    }
    if (e) touch_cached(g, e);
    if (!e) {
        evict_captures<CapturedPR>(g);
        Plan* p = get_plan(g, L, piece, false, s);
        std::unique_ptr<CapturedPR> n(new CapturedPR());
        n->program = d.program;
        n->dtype = d.dtype;
        n->iters = d.max_iters;
        n->piece = piece;
        n->flags = d.flags;
        n->damping = d.damping;
        n->values = d.d_values;
        n->tele = d.d_teleport;
        n->stats_out = d.d_stats;
        Workspace& w = n->w;
        alloc_common(w, L, *p, sizeof(double), d.max_iters, s, false);
        w.buf[0].alloc(sizeof(V) * (L.n), s);
        w.buf[1].alloc(sizeof(V) * (L.n), s);
        w.part.alloc(sizeof(double) * grid_for(L.n, 256, 1024), s);
        const VMap vm = vmap_of(g);
        if (vm) {
            w.mvals.alloc(sizeof(V) * L.n, s);
            if (d.d_teleport) w.mtele.alloc(sizeof(V) * L.n, s);
        }
        const size_t lds = iter_lds(make_geo(L, *p, w, sizeof(double)), L, sizeof(double));
        if (weighted)
            prepare_iter<ProgPRW<V>, 1024>(lds);
        else if (L.pairs)
            prepare_iter<ProgPRP<V>, 1024>(lds);
        else
            prepare_iter<ProgPR<V>, 1024>(lds);
        NXG_HIP(hipStreamSynchronize(s));
        if (!g->capture_stream)
            NXG_HIP(hipStreamCreateWithFlags(&g->capture_stream, hipStreamNonBlocking));
        hipStream_t cs = g->capture_stream;
        NXG_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
        try {
            enqueue_pagerank<V>(L, *p, w, d, weighted, vm, cs);
        } catch (...) {
            hipGraph_t dead = nullptr;
            (void)hipStreamEndCapture(cs, &dead);
            if (dead) (void)hipGraphDestroy(dead);
            throw;
        }
        NXG_HIP(hipStreamEndCapture(cs, &n->graph));
        NXG_HIP(hipGraphInstantiate(&n->exec, n->graph, nullptr, nullptr, 0));
        e = n.release();
        g->cached.push_back(e);
    }
    std::unique_ptr<Events> ev;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (st) {
        ev.reset(new Events());
        e0 = ev->a;
        e1 = ev->b;
        NXG_HIP(hipEventRecord(e0, s));
    }
    NXG_HIP(hipGraphLaunch(e->exec, s));
    if (st) {
        NXG_HIP(hipEventRecord(e1, s));
        std::vector<double> hs(4 * (size_t)(d.max_iters + 2));
        NXG_HIP(hipMemcpyAsync(hs.data(), e->w.stats.p, sizeof(double) * hs.size(),
                               hipMemcpyDeviceToHost, s));
        NXG_HIP(hipStreamSynchronize(s));
        float ms = 0.f;
        NXG_HIP(hipEventSynchronize(e1));
        NXG_HIP(hipEventElapsedTime(&ms, e0, e1));
        memset(st, 0, sizeof(*st));
        st->iterations = d.max_iters;
        st->residual = hs[4 * (d.max_iters - 1) + 1];
        st->device_ms = ms;
    }
    return NXG_OK;
}

// PageRank by coarse-grained push over the source-sorted stream (NXG_RUN_SCATTER).
template <typename V>
nxg_status run_scatter(nxg_dsss* g, const nxg_run_desc& d, hipStream_t s, nxg_run_stats* st) {
    const Layout& L = g->fwd;
    const bool weighted = d.program == NXG_PAGERANK_WEIGHTED;
    if (!(g->flags & NXG_BUILD_SCATTER)) fail(NXG_EINVAL, "NXG_RUN_SCATTER needs a NXG_BUILD_SCATTER layout");
    if (d.flags & NXG_RUN_CAPTURE) fail(NXG_EINVAL, "NXG_RUN_SCATTER runs cannot be captured");
    if (weighted && !L.has_weight) fail(NXG_EINVAL, "weighted PageRank needs a build with weights");
    const int max_iters = d.max_iters;
    Workspace w;
    w.buf[0].alloc(sizeof(V) * L.n, s);
    w.buf[1].alloc(sizeof(V) * L.n, s);
    w.partial.alloc(sizeof(double) * L.n, s);  // the global sums y
    NXG_HIP(hipMemsetAsync(w.partial.p, 0, sizeof(double) * L.n, s));
    const int nb = grid_for(L.n, 256, 1024);
    w.part.alloc(sizeof(double) * 3 * nb, s);
    const size_t nstat = 4 * (size_t)(max_iters + 2);
    w.stats.alloc(sizeof(double) * nstat, s);
    NXG_HIP(hipMemsetAsync(w.stats.p, 0, sizeof(double) * nstat, s));
    w.done.alloc(sizeof(int32_t), s);
    NXG_HIP(hipMemsetAsync(w.done.p, 0, sizeof(int32_t), s));
    const V* tele = (const V*)d.d_teleport;
    V* vals = (V*)d.d_values;
    const V* x0 = (d.flags & NXG_RUN_WARM_START) ? vals : nullptr;
    const int divide = weighted ? 0 : 1;
    hipLaunchKernelGGL(k_init_pr<V>, dim3(nb), dim3(256), 0, s, L.n, L.outdeg.as<int32_t>(), tele, x0, divide,
                       w.buf[0].as<V>(), w.part.as<double>());
    NXG_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(64), 0, s, w.part.as<double>(), nb, w.stats.as<double>());
    NXG_CHECK_LAUNCH();
    const int sgrid = grid_for(L.n_chunks * 64, 256, 16384);
    Events ev;
    hipEvent_t e0 = ev.a, e1 = ev.b;
    NXG_HIP(hipEventRecord(e0, s));
    int k = 0, done_h = 0;
    for (; k < max_iters; ++k) {
        const V* cur = w.buf[k & 1].as<V>();
        V* nxt = w.buf[(k + 1) & 1].as<V>();
        if (L.n_chunks > 0) {
            if (weighted)
                hipLaunchKernelGGL((k_scatter<V, true>), dim3(sgrid), dim3(256), 0, s, L.words.as<uint32_t>(),
                                   L.chunk_row.as<int32_t>(), L.n_chunks, L.C, L.I, L.L, L.t, cur,
                                   L.weight.as<float>(), w.partial.as<double>());
            else
                hipLaunchKernelGGL((k_scatter<V, false>), dim3(sgrid), dim3(256), 0, s, L.words.as<uint32_t>(),
                                   L.chunk_row.as<int32_t>(), L.n_chunks, L.C, L.I, L.L, L.t, cur,
                                   (const float*)nullptr, w.partial.as<double>());
            NXG_CHECK_LAUNCH();
        }
        // with a tolerance every iteration writes x, so the last one run is the result
        V* xout = (d.tol > 0 || k == max_iters - 1) ? vals : nullptr;
        hipLaunchKernelGGL(k_scatter_apply<V>, dim3(nb), dim3(256), 0, s, L.n, w.partial.as<double>(),
                           L.outdeg.as<int32_t>(), cur, nxt, tele, xout, d.damping, divide,
                           w.stats.as<double>() + 4 * k, w.part.as<double>());
        NXG_CHECK_LAUNCH();
        hipLaunchKernelGGL(k_scatter_reduce, dim3(1), dim3(64), 0, s, w.part.as<double>(), nb,
                           w.stats.as<double>(), k, d.tol, w.done.as<int32_t>());
        NXG_CHECK_LAUNCH();
        if (d.tol > 0) {
            NXG_HIP(hipMemcpyAsync(&done_h, w.done.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
            NXG_HIP(hipStreamSynchronize(s));
            if (done_h) {
                ++k;
                break;
            }
        }
    }
    if (max_iters == 0) {
        hipLaunchKernelGGL(k_unscale<V>, dim3(grid_for(L.n)), dim3(256), 0, s, L.n, L.outdeg.as<int32_t>(),
                           w.buf[0].as<V>(), divide, vals);
        NXG_CHECK_LAUNCH();
    }
    NXG_HIP(hipEventRecord(e1, s));
    std::vector<double> hs(nstat);
    NXG_HIP(hipMemcpyAsync(hs.data(), w.stats.p, sizeof(double) * nstat, hipMemcpyDeviceToHost, s));
    NXG_HIP(hipStreamSynchronize(s));
    float ms = 0.f;
    NXG_HIP(hipEventSynchronize(e1));
    NXG_HIP(hipEventElapsedTime(&ms, e0, e1));
    const bool conv = d.tol > 0 && done_h;
    if (st) {
        memset(st, 0, sizeof(*st));
        st->iterations = k;
        st->converged = conv ? 1 : 0;
        st->residual = k > 0 ? hs[4 * (k - 1) + 1] : 0.0;
        st->device_ms = ms;
    }
    return (d.tol > 0 && !conv) ? NXG_ENOTCONV : NXG_OK;
}

// The workspace of one PageRank run (allocated, carved out of an arena, or
// only measured by a measuring arena).
template <typename V>
void pr_workspace(Workspace& w, const Layout& L, const Plan& p, int max_iters, bool relabeled,
                  bool tele, hipStream_t s, Arena* a) {
    alloc_common(w, L, p, sizeof(double), max_iters, s, false, a);
    take(w.buf[0], sizeof(V) * (size_t)L.n, s, a);
    take(w.buf[1], sizeof(V) * (size_t)L.n, s, a);
    take(w.part, sizeof(double) * grid_for(L.n, 256, 1024), s, a);
    if (relabeled) {
        take(w.mvals, sizeof(V) * (size_t)L.n, s, a);
        if (tele) take(w.mtele, sizeof(V) * (size_t)L.n, s, a);
    }
}

// First iteration (of iters) whose residual met tol, or -1; *resid receives the
// residual of the last iteration counted. Reads the device stats in blocks into
// a fixed host array.
int first_converged(const double* d_stats, int iters, double tol, hipStream_t s, double* resid) {
    constexpr int kBlk = 64;
    double h[4 * kBlk];
    int conv = -1;
    *resid = 0.0;
    if (iters <= 0) return conv;
    if (tol <= 0) {  // no stop test: only the last residual
        NXG_HIP(hipMemcpyAsync(h, d_stats + 4 * (size_t)(iters - 1) + 1, sizeof(double),
                               hipMemcpyDeviceToHost, s));
        NXG_HIP(hipStreamSynchronize(s));
        *resid = h[0];
        return conv;
    }
    for (int i0 = 0; i0 < iters; i0 += kBlk) {
        const int cnt = std::min(kBlk, iters - i0);
        NXG_HIP(hipMemcpyAsync(h, d_stats + 4 * (size_t)i0, sizeof(double) * 4 * cnt,
                               hipMemcpyDeviceToHost, s));
        NXG_HIP(hipStreamSynchronize(s));
        for (int j = 0; j < cnt; ++j) {
            *resid = h[4 * j + 1];
            if (h[4 * j + 1] <= tol) return i0 + j;
        }
    }
    return conv;
}

// PageRank (plain or weighted) run. With an arena the workspace is carved out of
// the arena's region and the run allocates nothing: the plan must already exist
// and the arena supplies the timing events.
template <typename V>
nxg_status run_pagerank(nxg_dsss* g, const nxg_run_desc& d, hipStream_t s, nxg_run_stats* st,
                        Arena* arena = nullptr) {
    const Layout& L = g->fwd;
    const bool weighted = d.program == NXG_PAGERANK_WEIGHTED;
    if (weighted && !L.has_weight) fail(NXG_EINVAL, "weighted PageRank needs a build with weights");
    const size_t vb = sizeof(V);
    const size_t ab = sizeof(double);  // LDS accumulator bytes per destination
    if (((size_t)L.T + kSpill) * ab > (size_t)lds_budget_bytes(g->device))
        fail(NXG_EINVAL, "destination tile does not fit in LDS (PageRank accumulates 8 bytes per "
                         "vertex); rebuild with value_bytes = 8");
    const int cus = num_cus(g->device);
    int piece = d.piece_chunks > 0 ? d.piece_chunks : env_int("NXG_PIECE_CHUNKS", 0);
    if (piece <= 0) piece = default_piece(L.n_chunks, L.C, (size_t)L.T * ab, cus);
    std::unique_ptr<Streamer> str;
    if (L.host_stream) {
        if (arena) fail(NXG_EINVAL, "a HOST_STREAM handle cannot run without allocating");
        if (d.flags & NXG_RUN_CAPTURE) fail(NXG_EINVAL, "HOST_STREAM runs cannot be captured");
        // staging buffer size; pieces never exceed one buffer
        const int64_t mb = std::max(1, env_int("NXG_STREAM_MB", 256));
        const int64_t cap = std::max<int64_t>(1, mb * (1 << 20) / ((int64_t)L.C * 4));
        piece = (int)std::min<int64_t>(piece, cap);
        str.reset(new Streamer());
        Plan* sp = get_plan(g, L, piece, false, s, true);
        str->init(L, *sp, cap, s);
    } else if (d.flags & NXG_RUN_CAPTURE) {
        if (arena) fail(NXG_EINVAL, "NXG_RUN_CAPTURE is not available without allocating");
        return run_pagerank_captured<V>(g, d, s, st, piece);
    }
    Plan* p = nullptr;
    if (arena) {
        p = find_plan(g, L, piece, false, false);
        if (!p)
            fail(NXG_EINVAL, "no iteration plan for " + std::to_string(piece) +
                                 " chunks per piece on this handle (the build prepares the "
                                 "planner's; run nxg_run once with this piece size first)");
    } else {
        p = get_plan(g, L, piece, false, s, L.host_stream);
    }
    const int max_iters = d.max_iters;
    // a relabeled build works on copies in internal ids
    const VMap vm = vmap_of(g);
    Workspace w;
    if (arena) {
        Arena probe;
        probe.measure = true;
        pr_workspace<V>(w, L, *p, max_iters, (bool)vm, d.d_teleport != nullptr, s, &probe);
        if (probe.used > arena->cap)
            fail(NXG_EINVAL, "the run needs " + std::to_string(probe.used) +
                                 " bytes of workspace; the scratch region holds " +
                                 std::to_string(arena->cap));
    }
    pr_workspace<V>(w, L, *p, max_iters, (bool)vm, d.d_teleport != nullptr, s, arena);
    const int nb = grid_for(L.n, 256, 1024);
    const V* tele = (const V*)d.d_teleport;
    V* vals = (V*)d.d_values;
    if (vm) {
        if (tele) {
            permute_rows<V>(tele, vm.n2o, L.n, 1, w.mtele.as<V>(), s);
            tele = w.mtele.as<V>();
        }
        if (d.flags & NXG_RUN_WARM_START) permute_rows<V>(vals, vm.n2o, L.n, 1, w.mvals.as<V>(), s);
        vals = w.mvals.as<V>();
    }
    const V* x0 = (d.flags & NXG_RUN_WARM_START) ? vals : nullptr;
    hipLaunchKernelGGL(k_init_pr<V>, dim3(nb), dim3(256), 0, s, L.n, L.outdeg.as<int32_t>(), tele,
                       x0, weighted ? 0 : 1, w.buf[0].as<V>(), w.part.as<double>());
    NXG_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(64), 0, s, w.part.as<double>(), nb,
                       w.stats.as<double>());
    NXG_CHECK_LAUNCH();
    Geo geo = make_geo(L, *p, w, ab);
    const size_t lds = iter_lds(geo, L, ab);
    std::unique_ptr<Events> ev;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (arena) {
        e0 = arena->e0;
        e1 = arena->e1;
    } else {
        ev.reset(new Events());
        e0 = ev->a;
        e1 = ev->b;
    }
    NXG_HIP(hipEventRecord(e0, s));
    int k = 0;
    int done_h = 0;
    const int block = d.tol > 0 ? std::max(1, env_int("NXG_SYNC_BLOCK", 8)) : max_iters;
    while (k < max_iters) {
        int kend = std::min(max_iters, k + block);
        for (; k < kend; ++k) {
            Ctl ctl{w.stats.as<double>(), w.done.as<int32_t>(), k, d.tol};
            const V* cur = w.buf[k & 1].as<V>();
            V* nxt = w.buf[(k + 1) & 1].as<V>();
            V* xout = (k == max_iters - 1) ? vals : nullptr;
            if (weighted) {
                ProgPRW<V> pr{cur, nxt, tele, xout, L.weight.as<float>(), d.damping};
                launch_iter<ProgPRW<V>, 1024>(geo, ctl, pr, *p, lds, s, str.get());
            } else {
                ProgPR<V> pr{cur, nxt, tele, xout, d.damping};
                launch_plain_pr<V>(L, geo, ctl, pr, *p, lds, s, str.get());
            }
        }
        if (d.tol > 0 && k < max_iters) {
            NXG_HIP(hipMemcpyAsync(&done_h, w.done.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
            NXG_HIP(hipStreamSynchronize(s));
            if (done_h) break;
        }
    }
    if (k < max_iters || max_iters == 0) {
        // converged early (or no iteration asked): the newest vector is buf[k & 1]
        const V* cur = w.buf[k & 1].as<V>();
        if (weighted) {
            hipLaunchKernelGGL(k_copy<V>, dim3(grid_for(L.n)), dim3(256), 0, s, cur, vals,
                               (int64_t)L.n);
        } else {
            // x = gathered value * outdeg; reuse the carry-over path of the kernel
            Ctl ctl{w.stats.as<double>(), w.done.as<int32_t>(), k, d.tol};
            ProgPR<V> pr{cur, w.buf[(k + 1) & 1].as<V>(), nullptr, vals, d.damping};
            fill<int32_t>(w.done.as<int32_t>(), 1, -1, s);
            launch_plain_pr<V>(L, geo, ctl, pr, *p, lds, s);
        }
        NXG_CHECK_LAUNCH();
    }
    if (vm) permute_rows<V>(vals, vm.o2n, vm.n, 1, (V*)d.d_values, s);
    copy_stats_out(w, d, s);
    NXG_HIP(hipEventRecord(e1, s));
    nxg_status rc = NXG_OK;
    if (st || d.tol > 0) {
        double resid = 0.0;
        // with early exit the kernels after convergence only carried data over
        const int conv_at = first_converged(w.stats.as<double>(), k, d.tol, s, &resid);
        const int iters = conv_at >= 0 ? conv_at + 1 : k;
        float ms = 0.f;
        NXG_HIP(hipEventSynchronize(e1));
        NXG_HIP(hipEventElapsedTime(&ms, e0, e1));
        if (st) {
            memset(st, 0, sizeof(*st));
            st->iterations = iters;
            st->converged = conv_at >= 0 ? 1 : 0;
            st->residual = iters > 0 ? resid : 0.0;
            st->device_ms = ms;
        }
        if (d.tol > 0 && conv_at < 0) rc = NXG_ENOTCONV;
    }
    // the buffers are released through the allocator on the same stream (so
    // stream-ordered allocators see the frees after the kernels); a carved
    // workspace is not released at all
    NXG_HIP(hipStreamSynchronize(s));
    return rc;
}

// ---------------------------------------------------------------------------
// Mixed-phase update with host memory as the slower tier (NXG_RUN_MPU)
// ---------------------------------------------------------------------------
// The first Q source intervals (vertices [0, R), R = Q * I, a whole number of
// tiles) keep their ping-pong values in device memory; the others keep them in
// pinned host memory and are staged into a one-interval device buffer when
// their row of sub-shards is processed. Sub-shards whose source and
// destination are both outside the resident range go through shard hubs in
// host memory (Alg. 6's ToHub / FromHub); all others update in place. One
// iteration follows Alg. 7:
//   P1  resident tiles, resident source rows: sums stored in the tiles' device
//       accumulators;
//   P2  for each non-resident row i (its values staged): resident tiles add
//       into their accumulators, non-resident tiles store hub slot (tile, i);
//   P3  non-resident tiles: resident source rows, plus their hub slots in row
//       order, then the update, written to host memory;
//   P4  resident tiles: the update from their accumulators.
// The scalar reduction then works as in every other run.

// x^0 (or the caller's x^0) as gathered values, split at vertex R between the
// device array and the host array (indexed from R); per-block dangling mass.
template <typename V>
__global__ __launch_bounds__(256) void k_init_mpu(int32_t n, int64_t R, const int32_t* __restrict__ deg,
                                                  const V* __restrict__ tele, const V* __restrict__ x0,
                                                  int divide, V* __restrict__ cur_d, V* __restrict__ cur_h,
                                                  double* __restrict__ part) {
    __shared__ double red[4];
    double s = 0.0;
    for (int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x; v < n; v += (int64_t)gridDim.x * 256) {
        const V x = x0 ? x0[v] : (tele ? tele[v] : (V)(1.0 / n));
        const int32_t dg = deg[v];
        if (dg == 0) s += (double)x;
        const V c = (divide && dg) ? (V)((double)x / dg) : x;
        if (v < R)
            cur_d[v] = c;
        else
            cur_h[v - R] = c;
    }
    s = wave_sum(s);
    if (lane_id() == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// x^0 into the caller's output (a run of zero iterations).
template <typename V>
__global__ void k_x0_out(int32_t n, const V* __restrict__ tele, V* __restrict__ x) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
        x[v] = tele ? tele[v] : (V)(1.0 / n);
}

// Device address of pinned host memory.
void* host_dev_ptr(const HostBuf& h) {
    void* dp = nullptr;
    NXG_HIP(hipHostGetDevicePointer(&dp, h.p, 0));
    return dp;
}

// Clears the FP64 slots [list[b] * T, list[b] * T + T) of `acc`, one workgroup each.
__global__ __launch_bounds__(256) void k_zero_slots(const int32_t* __restrict__ list, double* __restrict__ acc,
                                                    int64_t T) {
    double* p = acc + (int64_t)list[blockIdx.x] * T;
    for (int64_t x = threadIdx.x; x < T; x += 256) p[x] = 0.0;
}

template <typename V>
nxg_status run_pagerank_mpu(nxg_dsss* g, const nxg_run_desc& d, hipStream_t s, nxg_run_stats* st) {
    const Layout& L = g->fwd;
    const bool weighted = d.program == NXG_PAGERANK_WEIGHTED;
    if (weighted && !L.has_weight) fail(NXG_EINVAL, "weighted PageRank needs a build with weights");
    if (g->relabeled) fail(NXG_EUNSUPPORTED, "NXG_RUN_MPU needs natural vertex ids (no RELABEL or DEGREE build)");
    if (L.host_stream || L.pairs || (g->flags & NXG_BUILD_SCATTER))
        fail(NXG_EUNSUPPORTED, "NXG_RUN_MPU runs on plain device-resident layouts");
    if (d.flags & (NXG_RUN_CAPTURE | NXG_RUN_SCATTER | NXG_RUN_PERSISTENT))
        fail(NXG_EINVAL, "NXG_RUN_MPU cannot be combined with CAPTURE, SCATTER or PERSISTENT");
    if (L.I & (L.I - 1)) fail(NXG_EUNSUPPORTED, "NXG_RUN_MPU needs an interval size that is a power of two");
    if (((size_t)L.T + kSpill) * sizeof(double) > (size_t)lds_budget_bytes(g->device))
        fail(NXG_EINVAL, "destination tile does not fit in LDS; rebuild with value_bytes = 8");
    if ((int64_t)L.n_tiles * L.P > ((int64_t)1 << 24))
        fail(NXG_EUNSUPPORTED, "too many sub-shards for the mixed-phase schedule; use larger intervals or tiles");
    int64_t budget = d.vertex_budget;
    if (budget <= 0) budget = (int64_t)env_int("NXG_VERTEX_BUDGET_MB", 0) << 20;
    if (budget <= 0)
        fail(NXG_EINVAL, "NXG_RUN_MPU needs a device memory budget (vertex_budget, or NXG_VERTEX_BUDGET_MB)");
    const int64_t n = L.n, I = L.I, T = L.T, P = L.P, vb = sizeof(V);
    // Planner (Sec. III-B3: Q <= B_M / (2 n B_a / P)): each resident vertex costs
    // its two values and an FP64 accumulator, plus one staged interval; the
    // resident range moves in whole intervals and whole tiles
    const int64_t unit = std::max(I, T);
    int64_t R = (budget - I * vb) / (2 * vb + 8);
    R = std::max<int64_t>(0, R / unit * unit);
    const int64_t n_up = (n + unit - 1) / unit * unit;
    if (R >= n_up) R = n_up;
    const int64_t Q = std::min<int64_t>(P, R / I);
    const int64_t Rv = std::min<int64_t>(R, n);                 // resident vertices
    const int64_t Qt = std::min<int64_t>(L.n_tiles, R / T);     // resident tiles
    const int64_t Nt = L.n_tiles - Qt, Nr = P - Q;              // non-resident tiles and rows
    // group word positions (host) -> chunk ranges of (tile, source rows [a, b))
    std::vector<int64_t> gw((size_t)L.n_tiles * P + 1);
    NXG_HIP(hipMemcpyAsync(gw.data(), L.group_word.p, sizeof(int64_t) * gw.size(), hipMemcpyDeviceToHost, s));
    NXG_HIP(hipStreamSynchronize(s));
    auto range = [&](int64_t tau, int64_t a, int64_t b, Item& it) {
        const int64_t w0 = gw[tau * P + a], w1 = gw[tau * P + b];
        it.c0 = w0 / L.C;
        it.c1 = w1 > w0 ? (w1 + L.C - 1) / L.C : it.c0;
    };
    auto item = [](int64_t tau, int64_t slot, int np) {
        Item it;
        it.tile = (int32_t)tau;
        it.piece = 0;
        it.npieces = np;
        it.slot = (int32_t)slot;
        it.c0 = it.c1 = 0;
        return it;
    };
    // Pieces: an item longer than pc chunks is cut into pieces of about pc
    // chunks, so a heavy tile (natural ids of a skewed graph put a twentieth of
    // the edges in the first tile) does not hold a launch for one workgroup.
    // Pieces of a resident tile add into its accumulators atomically (npieces
    // marks them; P1's are cleared first); pieces of a (non-resident tile, row)
    // each store into a hub slot of their own.
    const int cus = num_cus(g->device);
    const int64_t pc_env = env_int("NXG_PIECE_CHUNKS", 0);
    auto piece_len = [&](int64_t list_chunks) {
        if (pc_env > 0) return pc_env;
        return std::max<int64_t>(8, (list_chunks + 2 * cus - 1) / (2 * cus));
    };
    auto chunks_of = [&](int64_t tau, int64_t a, int64_t b) {
        Item it;
        range(tau, a, b, it);
        return it.c1 - it.c0;
    };
    auto cut = [](const Item& it, int64_t pc, std::vector<Item>& out, bool own_slots) {
        const int64_t nc = it.c1 - it.c0;
        const int64_t k = nc > pc ? (nc + pc - 1) / pc : 1;
        for (int64_t p = 0; p < k; ++p) {
            Item q = it;
            q.c0 = it.c0 + nc * p / k;
            q.c1 = it.c0 + nc * (p + 1) / k;
            if (own_slots)
                q.slot = it.slot + (int32_t)p;
            else
                q.npieces = (int32_t)k;
            out.push_back(q);
        }
        return k;
    };
    std::vector<int32_t> zero_tiles;  // resident tiles whose P1 pieces add atomically
    // item lists: P1, P2a(i), P2b(i) for each non-resident row, P3, P4
    std::vector<Item> items;
    std::vector<int64_t> off;  // first item of each list
    off.push_back((int64_t)items.size());
    {
        int64_t lc = 0;
        for (int64_t tau = 0; tau < Qt; ++tau) lc += chunks_of(tau, 0, Q);
        const int64_t pc = piece_len(lc);
        for (int64_t tau = 0; tau < Qt; ++tau) {  // P1: every resident tile's slot is written
            Item it = item(tau, tau, 1);
            range(tau, 0, Q, it);
            if (cut(it, pc, items, false) > 1) zero_tiles.push_back((int32_t)tau);
        }
    }
    // hub slots of the non-resident tiles, tile-major: for tile tau the pieces
    // of rows Q .. P-1 in order (at least one per row, empty ones store zeros)
    std::vector<int64_t> tslot((size_t)Nt + 1, 0), row_slots((size_t)Nr, 0), row_pc((size_t)Nr, 1);
    for (int64_t i = Q; i < P; ++i) {
        int64_t lc = 0;
        for (int64_t tau = Qt; tau < L.n_tiles; ++tau) lc += chunks_of(tau, i, i + 1);
        row_pc[i - Q] = piece_len(lc);
    }
    for (int64_t tau = Qt; tau < L.n_tiles; ++tau) {
        int64_t k = 0;
        for (int64_t i = Q; i < P; ++i) {
            const int64_t nc = chunks_of(tau, i, i + 1), pc = row_pc[i - Q];
            const int64_t kk = nc > pc ? (nc + pc - 1) / pc : 1;
            k += kk;
            row_slots[i - Q] += kk;
        }
        tslot[tau - Qt + 1] = tslot[tau - Qt] + k;
    }
    const int64_t hub_slots = tslot[Nt];
    if (hub_slots * T * 8 > ((int64_t)16 << 30))
        fail(NXG_EUNSUPPORTED, "shard hubs would exceed 16 GiB of host memory; raise the budget");
    if (hub_slots > INT32_MAX) fail(NXG_EUNSUPPORTED, "too many shard hub slots");
    std::vector<int64_t> next_slot(tslot.begin(), tslot.end() - 1);
    for (int64_t i = Q; i < P; ++i) {
        off.push_back((int64_t)items.size());
        {
            int64_t lc = 0;
            for (int64_t tau = 0; tau < Qt; ++tau) lc += chunks_of(tau, i, i + 1);
            const int64_t pc = piece_len(lc);
            for (int64_t tau = 0; tau < Qt; ++tau) {  // P2a: only tiles the row reaches
                Item it = item(tau, tau, 1);
                range(tau, i, i + 1, it);
                if (it.c1 > it.c0) cut(it, pc, items, false);
            }
        }
        off.push_back((int64_t)items.size());
        for (int64_t tau = Qt; tau < L.n_tiles; ++tau) {  // P2b: every hub slot is written
            Item it = item(tau, next_slot[tau - Qt], 1);
            range(tau, i, i + 1, it);
            next_slot[tau - Qt] += cut(it, row_pc[i - Q], items, true);
        }
    }
    off.push_back((int64_t)items.size());
    for (int64_t tau = Qt; tau < L.n_tiles; ++tau) {  // P3
        Item it = item(tau, tslot[tau - Qt], (int)(tslot[tau - Qt + 1] - tslot[tau - Qt]));
        range(tau, 0, Q, it);
        items.push_back(it);
    }
    off.push_back((int64_t)items.size());
    for (int64_t tau = 0; tau < Qt; ++tau) items.push_back(item(tau, tau, 1));  // P4
    off.push_back((int64_t)items.size());
    // each launch takes its items heaviest first (every item names its own slot)
    for (size_t l = 0; l + 1 < off.size(); ++l)
        std::stable_sort(items.begin() + off[l], items.begin() + off[l + 1],
                         [](const Item& a, const Item& b) { return a.c1 - a.c0 > b.c1 - b.c0; });
    // device and host memory of the run
    DevBuf ditems, cur_d, nxt_d, acc_d, stage, tile_s, tile_flag, stats, done, zero, part, zslots;
    ditems.alloc(sizeof(Item) * std::max<size_t>(items.size(), 1), s);
    zslots.alloc(sizeof(int32_t) * std::max<size_t>(zero_tiles.size(), 1), s);
    if (!zero_tiles.empty())
        NXG_HIP(hipMemcpyAsync(zslots.p, zero_tiles.data(), sizeof(int32_t) * zero_tiles.size(),
                               hipMemcpyHostToDevice, s));
    NXG_HIP(hipMemcpyAsync(ditems.p, items.data(), sizeof(Item) * items.size(), hipMemcpyHostToDevice, s));
    cur_d.alloc(vb * std::max<int64_t>(Rv, 1), s);
    nxt_d.alloc(vb * std::max<int64_t>(Rv, 1), s);
    acc_d.alloc(sizeof(double) * std::max<int64_t>(Qt * T, 1), s);
    stage.alloc(vb * I, s);
    tile_s.alloc(sizeof(double) * 3 * L.n_tiles, s);
    tile_flag.alloc(sizeof(int32_t) * L.n_tiles, s);
    const int max_iters = d.max_iters;
    stats.alloc(sizeof(double) * 4 * (size_t)(max_iters + 2), s);
    fill<double>(stats.as<double>(), 4 * (int64_t)(max_iters + 2), 0.0, s);
    done.alloc(sizeof(int32_t), s);
    fill<int32_t>(done.as<int32_t>(), 1, 0, s);
    zero.alloc(sizeof(int32_t), s);  // the edge kernels' stop flag, never set
    fill<int32_t>(zero.as<int32_t>(), 1, 0, s);
    const int nb = grid_for(n, 256, 1024);
    part.alloc(sizeof(double) * nb, s);
    HostBuf cur_h, nxt_h, hub_h;
    cur_h.alloc(vb * std::max<int64_t>(n - Rv, 1));
    nxt_h.alloc(vb * std::max<int64_t>(n - Rv, 1));
    hub_h.alloc(sizeof(double) * std::max<int64_t>(hub_slots * T, 1));
    V* curh = static_cast<V*>(host_dev_ptr(cur_h));
    V* nxth = static_cast<V*>(host_dev_ptr(nxt_h));
    double* hubd = static_cast<double*>(host_dev_ptr(hub_h));
    const V* tele = (const V*)d.d_teleport;
    V* vals = (V*)d.d_values;
    const V* x0 = (d.flags & NXG_RUN_WARM_START) ? vals : nullptr;
    hipLaunchKernelGGL(k_init_mpu<V>, dim3(nb), dim3(256), 0, s, (int32_t)n, Rv, L.outdeg.as<int32_t>(), tele,
                       x0, weighted ? 0 : 1, cur_d.as<V>(), curh, part.as<double>());
    NXG_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(64), 0, s, part.as<double>(), nb, stats.as<double>());
    NXG_CHECK_LAUNCH();
    if (max_iters == 0 && !x0) {
        hipLaunchKernelGGL(k_x0_out<V>, dim3(grid_for(n)), dim3(256), 0, s, (int32_t)n, tele, vals);
        NXG_CHECK_LAUNCH();
    }
    Geo geo;
    memset(&geo, 0, sizeof(geo));
    geo.words = L.words.as<uint32_t>();
    geo.chunk_row = L.chunk_row.as<int32_t>();
    geo.deg = L.outdeg.as<int32_t>();
    geo.n = L.n;
    geo.I = L.I;
    geo.P = L.P;
    geo.L = L.L;
    geo.T = L.T;
    geo.t = L.t;
    geo.sshift = L.order == NXG_ORDER_SRC ? L.t : 0;
    geo.dshift = L.order == NXG_ORDER_SRC ? 0 : L.L;
    geo.order = L.order;
    geo.n_tiles = L.n_tiles;
    geo.C = L.C;
    geo.tile_s = tile_s.as<double>();
    geo.n_sslots = L.n_tiles;
    geo.tile_flag = tile_flag.as<int32_t>();
    const size_t lds = ((size_t)L.T + kSpill) * sizeof(double);
    using Base = std::conditional_t<std::is_same<V, float>::value, ProgPR<float>, ProgPR<double>>;
    using BaseW = std::conditional_t<std::is_same<V, float>::value, ProgPRW<float>, ProgPRW<double>>;
    int64_t host_rd = 0, host_wr = 0;
    auto launch = [&](int list, const V* cur, const V* own, V* nxt, V* xout, uint32_t r_lo, uint32_t r_hi,
                      int mode, void* slots, const Ctl& ctl) {
        const int64_t a = off[list], b = off[list + 1];
        if (b <= a) return;
        Geo gl = geo;
        gl.items = ditems.as<Item>() + a;
        gl.partial = slots;
        if (weighted) {
            ProgMPU<BaseW> pr;
            static_cast<BaseW&>(pr) = BaseW{cur, nxt, tele, xout, L.weight.as<float>(), d.damping};
            pr.r_lo = r_lo;
            pr.r_hi = r_hi;
            pr.mode = mode;
            pr.own = own;
            prepare_iter<ProgMPU<BaseW>, 1024>(lds);
            launch_items<ProgMPU<BaseW>, 1024>((int)(b - a), lds, s, gl, ctl, pr);
        } else {
            ProgMPU<Base> pr;
            static_cast<Base&>(pr) = Base{cur, nxt, tele, xout, d.damping};
            pr.r_lo = r_lo;
            pr.r_hi = r_hi;
            pr.mode = mode;
            pr.own = own;
            prepare_iter<ProgMPU<Base>, 1024>(lds);
            launch_items<ProgMPU<Base>, 1024>((int)(b - a), lds, s, gl, ctl, pr);
        }
    };
    Events ev;
    NXG_HIP(hipEventRecord(ev.a, s));
    V* cd = cur_d.as<V>();
    V* nd = nxt_d.as<V>();
    V* ch = curh;  // device addresses of the host arrays (kernels)
    V* nh = nxth;
    const V* chost = cur_h.as<V>();  // their host addresses (copies)
    const V* nhost = nxt_h.as<V>();
    int k = 0, done_h = 0;
    const int list_p3 = 1 + 2 * (int)Nr, list_p4 = list_p3 + 1;
    for (; k < max_iters; ++k) {
        Ctl ctl{stats.as<double>(), zero.as<int32_t>(), k, d.tol};     // edge kernels: never stop
        Ctl rctl{stats.as<double>(), done.as<int32_t>(), k, d.tol};    // the scalar reduction
        V* xout = (d.tol > 0 || k == max_iters - 1) ? vals : nullptr;
        // P1: resident tiles, resident rows, sums stored in their accumulators
        if (!zero_tiles.empty()) {
            hipLaunchKernelGGL(k_zero_slots, dim3((unsigned)zero_tiles.size()), dim3(256), 0, s,
                               zslots.as<int32_t>(), acc_d.as<double>(), T);
            NXG_CHECK_LAUNCH();
        }
        launch(0, cd, nullptr, nullptr, nullptr, 0u, (uint32_t)Q, kMpuStore, acc_d.p, ctl);
        // P2: the non-resident rows, one staged interval at a time
        for (int64_t i = Q; i < P; ++i) {
            const int64_t cnt = std::min<int64_t>(I, n - i * I);
            NXG_HIP(hipMemcpyAsync(stage.p, chost + (i * I - Rv), vb * cnt, hipMemcpyHostToDevice, s));
            host_rd += vb * cnt;
            const V* sb = stage.as<V>() - i * I;  // indexed by global vertex id
            const int l = 1 + 2 * (int)(i - Q);
            launch(l, sb, nullptr, nullptr, nullptr, (uint32_t)i, (uint32_t)(i + 1), kMpuAdd, acc_d.p, ctl);
            launch(l + 1, sb, nullptr, nullptr, nullptr, (uint32_t)i, (uint32_t)(i + 1), kMpuStore, hubd, ctl);
            host_wr += row_slots[i - Q] * T * 8;
        }
        // P3: non-resident tiles: resident rows, hub slots, update into host memory
        launch(list_p3, cd, ch - Rv, nh - Rv, xout, 0u, (uint32_t)Q, kMpuApply, hubd, ctl);
        host_rd += hub_slots * T * 8 + (n - Rv) * vb;
        host_wr += (n - Rv) * vb;
        // P4: resident tiles from their accumulators
        launch(list_p4, cd, cd, nd, xout, 0u, 0u, kMpuApply, acc_d.p, ctl);
        hipLaunchKernelGGL((k_reduce<ProgPR<V>, 1024>), dim3(1), dim3(1024), 0, s, geo, rctl);
        NXG_CHECK_LAUNCH();
        std::swap(cd, nd);
        std::swap(ch, nh);
        std::swap(chost, nhost);
        if (d.tol > 0) {
            NXG_HIP(hipMemcpyAsync(&done_h, done.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
            NXG_HIP(hipStreamSynchronize(s));
            if (done_h) {
                ++k;
                break;
            }
        }
    }
    NXG_HIP(hipEventRecord(ev.b, s));
    nxg_status rc = NXG_OK;
    double resid = 0.0;
    const int conv_at = first_converged(stats.as<double>(), k, d.tol, s, &resid);
    const int iters = conv_at >= 0 ? conv_at + 1 : k;
    float ms = 0.f;
    NXG_HIP(hipEventSynchronize(ev.b));
    NXG_HIP(hipEventElapsedTime(&ms, ev.a, ev.b));
    if (st) {
        memset(st, 0, sizeof(*st));
        st->iterations = iters;
        st->converged = conv_at >= 0 ? 1 : 0;
        st->residual = iters > 0 ? resid : 0.0;
        st->device_ms = ms;
        st->resident_intervals = (int32_t)Q;
        st->host_read_bytes = host_rd;
        st->host_write_bytes = host_wr;
    }
    if (d.tol > 0 && conv_at < 0) rc = NXG_ENOTCONV;
    NXG_HIP(hipStreamSynchronize(s));
    return rc;
}

// The chunk ranges the compaction tests, made once per layout.
void ensure_chunk_ranges(Layout& L, hipStream_t s) {
    if (L.chunk_rng.p || L.n_chunks == 0) return;
    DevBuf r;
    r.alloc(sizeof(int4) * (size_t)L.n_chunks, s);
    const int sshift = L.order == NXG_ORDER_SRC ? L.t : 0;
    const int dshift = L.order == NXG_ORDER_SRC ? 0 : L.L;
    hipLaunchKernelGGL(k_chunk_ranges, dim3((unsigned)((L.n_chunks + 3) / 4)), dim3(256), 0, s,
                       L.words.as<uint32_t>(), L.chunk_row.as<int32_t>(), L.chunk_tile.as<int32_t>(),
                       L.n_chunks, L.C, L.I, L.L, L.t, sshift, dshift, r.as<int4>());
    NXG_CHECK_LAUNCH();
    L.chunk_rng = std::move(r);
}

// What a handle keeps between BFS (or WCC) runs: the workspace, sized for the
// layout, so a run allocates nothing.
struct MinprogCache : Cached {
    bool bfs = false;
    int piece = 0, block = 0, bs = 0, seg = 0, nseg = 0;
    int64_t nb = 0;
    Workspace w;
};

nxg_status run_minprog(nxg_dsss* g, const nxg_run_desc& d, hipStream_t s, nxg_run_stats* st) {
    const bool bfs = d.program == NXG_BFS;
    if (!bfs && !(g->flags & NXG_BUILD_SYMMETRIZE))
        fail(NXG_EINVAL, "WCC needs a build with NXG_BUILD_SYMMETRIZE");
    const VMap vm = vmap_of(g);
    const int64_t n_out = vm ? vm.n : g->fwd.n;
    if (bfs) {
        if (!d.roots) fail(NXG_EINVAL, "BFS needs roots");
        if (d.batch != 1) fail(NXG_EUNSUPPORTED, "BFS runs one root per call");
        if (d.roots[0] < 0 || d.roots[0] >= n_out) fail(NXG_EINVAL, "BFS root outside [0, n)");
    }
    if (((size_t)g->fwd.T + kSpill) * 4 > (size_t)lds_budget_bytes(g->device) || g->fwd.T > 65536)
        fail(NXG_EINVAL, "tile does not fit in LDS");
    ensure_chunk_ranges(g->fwd, s);
    const Layout& L = g->fwd;
    const int cus = num_cus(g->device);
    int piece = env_int("NXG_PIECE_CHUNKS", 0);
    if (piece <= 0) piece = default_piece(L.n_chunks, L.C, (size_t)L.T * 4, cus);
    Plan* p = get_plan(g, L, -piece, true, s);  // whole-tile ranges; pieces split the active list
    // the host reads the per-round stats a block of rounds at a time, so the
    // device keeps one block of them (max_iters may be as large as n + 1); the
    // first block is longer (a power-law graph settles in about that many rounds)
    const int block = std::max(1, env_int("NXG_SYNC_BLOCK", 4));
    const int first_block = std::max(block, env_int("NXG_SYNC_FIRST", 8));
    MinprogCache* c = nullptr;
    for (Cached* x : g->cached) {
        MinprogCache* m = dynamic_cast<MinprogCache*>(x);
        if (m && m->bfs == bfs && m->piece == piece && m->block == first_block) c = m;
    }
    if (!c) {
        c = new MinprogCache();
        g->cached.push_back(c);
        PendingEntry pend(g, c);
        c->bfs = bfs;
        c->piece = piece;
        c->block = first_block;
        Workspace& w = c->w;
        alloc_common(w, L, *p, 4, first_block, s, true);
        w.buf[0].alloc(sizeof(int32_t) * (L.n), s);
        w.buf[1].alloc(sizeof(int32_t) * (L.n), s);
        // activity blocks of 2^bs vertices (at most a wave of the apply), their
        // flags (changed, then unreached) and prefix counts per segment of `seg`
        // blocks (at most 256 segments)
        c->bs = std::min(6, L.t);
        c->nb = ((int64_t)L.n + (1 << c->bs) - 1) >> c->bs;
        c->seg = 4096;
        while ((c->nb + c->seg) / c->seg > 256) c->seg *= 2;
        c->nseg = (int)((c->nb + c->seg) / c->seg);  // segments over [0, nb]
        w.blk.alloc(2 * (size_t)c->nb, s);
        w.bpre.alloc(sizeof(int32_t) * 2 * (size_t)(c->nb + 1), s);
        w.btot.alloc(sizeof(int32_t) * 2 * (size_t)c->nseg, s);
        w.clist.alloc(sizeof(int64_t) * std::max<int64_t>(L.n_chunks, 1), s);
        w.ccount.alloc(sizeof(int32_t) * L.n_tiles, s);
        // streamed-chunk count, reached edges, maximum level, then the BFS
        // outputs' per-block partials
        w.bfsout.alloc(sizeof(unsigned long long) * (3 + 2 * kFinalBlocks), s);
        pend.commit();
    }
    Workspace& w = c->w;
    const int bs = c->bs, seg = c->seg, nseg = c->nseg;
    const int64_t nb = c->nb;
    uint8_t* chg = w.blk.as<uint8_t>();
    uint8_t* opn = bfs ? chg + nb : nullptr;
    int32_t* pre0 = w.bpre.as<int32_t>();
    int32_t* pre1 = bfs ? pre0 + nb + 1 : nullptr;
    int32_t* tot0 = w.btot.as<int32_t>();
    int32_t* tot1 = bfs ? tot0 + nseg : nullptr;
    unsigned long long* streamed = w.bfsout.as<unsigned long long>();
    const int max_iters = d.max_iters;
    Events ev;
    hipEvent_t e0 = ev.a, e1 = ev.b;
    NXG_HIP(hipEventRecord(e0, s));
    // the root is mapped to its internal id on the device; a root dropped by
    // degreeing (no edges) maps to -1 and reaches nothing but itself
    if (bfs)
        hipLaunchKernelGGL(k_init_bfs, dim3(grid_for(L.n)), dim3(256), 0, s, L.n, d.roots[0], vm.o2n,
                           w.buf[0].as<int32_t>(), w.buf[1].as<int32_t>(), chg, opn, bs, streamed);
    else
        hipLaunchKernelGGL(k_init_wcc, dim3(grid_for(L.n)), dim3(256), 0, s, L.n,
                           w.buf[0].as<int32_t>(), w.buf[1].as<int32_t>(), chg, bs, vm.n2o, streamed);
    NXG_CHECK_LAUNCH();
    Geo geo = make_geo(L, *p, w, 4);
    geo.clist = w.clist.as<int64_t>();
    geo.ccount = w.ccount.as<int32_t>();
    geo.split_min = piece;
    const size_t lds = iter_lds(geo, L, 4);
    int k = 0;
    std::vector<double> hs(4 * (size_t)(first_block + 2));
    bool fixed = false;
    int last_changed = 0;
    // the values after round kk live in buf[kk & 1] (rounds past the fixed point
    // copy): map them out, add the last round's listed chunks to the count, and
    // form the BFS outputs (maximum level, reached edges) in two steps without
    // atomics; the counts come back with the next synchronisation
    unsigned long long out3[3] = {0, 0, 0};  // streamed, reached, max level
    auto finish_work = [&](int kk) {
        NXG_HIP(hipEventRecord(e1, s));
        const int32_t* fin = w.buf[kk & 1].as<int32_t>();
        if (vm) {
            permute_rows<int32_t>(fin, vm.o2n, vm.n, 1, (int32_t*)d.d_values, s, 1, bfs ? kInf : 0,
                                  bfs ? 0 : 1);
            if (bfs)  // a dropped root keeps level 0
                hipLaunchKernelGGL(k_set_root, dim3(1), dim3(64), 0, s, (int32_t*)d.d_values, d.roots[0]);
        } else {
            hipLaunchKernelGGL(k_copy<int32_t>, dim3(grid_for(L.n)), dim3(256), 0, s, fin,
                               (int32_t*)d.d_values, (int64_t)L.n);
        }
        NXG_CHECK_LAUNCH();
        hipLaunchKernelGGL(k_count_streamed, dim3(1), dim3(1024), 0, s, w.ccount.as<int32_t>(), L.n_tiles,
                           kk > 0 ? streamed : nullptr);
        NXG_CHECK_LAUNCH();
        if (bfs) {
            unsigned long long* part = streamed + 3;
            hipLaunchKernelGGL(k_bfs_final, dim3(kFinalBlocks), dim3(256), 0, s, L.n, fin,
                               L.outdeg.as<int32_t>(), part);
            NXG_CHECK_LAUNCH();
            hipLaunchKernelGGL(k_bfs_final_sum, dim3(1), dim3(kFinalBlocks), 0, s, part);
            NXG_CHECK_LAUNCH();
            NXG_HIP(hipMemcpyAsync(out3, streamed, sizeof(out3), hipMemcpyDeviceToHost, s));
        } else {
            NXG_HIP(hipMemcpyAsync(out3, streamed, sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
        }
    };
    bool finished = false;
    while (k < max_iters && !fixed) {
        int kend = std::min(max_iters, k + (k == 0 ? first_block : block));
        int kb = k;
        for (; k < kend; ++k) {
            hipLaunchKernelGGL(k_blkscan, dim3(nseg), dim3(1024), 0, s, chg, opn, nb, seg, pre0, pre1,
                               tot0, tot1, w.ccount.as<int32_t>(), L.n_tiles, k > 0 ? streamed : nullptr,
                               w.stats.as<double>() + 4 * (k - kb) + 3);
            NXG_CHECK_LAUNCH();
            if (L.n_chunks > 0) {
                hipLaunchKernelGGL(k_compact, dim3(grid_for(L.n_chunks, 256, 4096)), dim3(256), 0, s,
                                   L.tile_chunk.as<int64_t>(), L.chunk_tile.as<int32_t>(), L.n_chunks,
                                   L.chunk_rng.as<int4>(), bs, seg, nseg, pre0, tot0, pre1, tot1,
                                   w.clist.as<int64_t>(), w.ccount.as<int32_t>());
            }
            NXG_CHECK_LAUNCH();
            Ctl ctl{w.stats.as<double>(), w.done.as<int32_t>(), k - kb, 0.0};
            const int32_t* cur = w.buf[k & 1].as<int32_t>();
            int32_t* nxt = w.buf[(k + 1) & 1].as<int32_t>();
            if (bfs) {
                ProgBFS pr{cur, nxt, chg, opn, bs};
                launch_iter<ProgBFS, 1024>(geo, ctl, pr, *p, lds, s);
            } else {
                ProgWCC pr{cur, nxt, chg, nullptr, bs};
                launch_iter<ProgWCC, 1024>(geo, ctl, pr, *p, lds, s);
            }
        }
        // after the first block the final work goes out before the host reads the
        // changed flags (a power-law graph is settled by then), so a run that
        // settles there needs one synchronisation; otherwise it is redone at the end
        // (counting the streamed chunks twice is avoided: the count clears the lists)
        const bool speculate = kb == 0;
        if (speculate) finish_work(k);
        NXG_HIP(hipMemcpyAsync(hs.data(), w.stats.as<double>(), sizeof(double) * 4 * (k - kb),
                               hipMemcpyDeviceToHost, s));
        NXG_HIP(hipStreamSynchronize(s));
        for (int i = kb; i < k; ++i) {
            if (hs[4 * (i - kb) + 3] == 0.0) {
                fixed = true;
                break;
            }
            last_changed = i + 1;
        }
        finished = speculate && fixed;
    }
    if (!finished) finish_work(k);
    NXG_HIP(hipStreamSynchronize(s));
    float ms = 0.f;
    NXG_HIP(hipEventSynchronize(e1));
    NXG_HIP(hipEventElapsedTime(&ms, e0, e1));
    if (st) {
        memset(st, 0, sizeof(*st));
        st->iterations = std::min(k, last_changed + 1);
        st->converged = fixed ? 1 : 0;
        st->changed_rounds = last_changed;
        st->max_level = (int32_t)out3[2];
        st->reached_edges = (int64_t)out3[1];
        st->device_ms = ms;
        st->streamed_chunks = (int64_t)out3[0];
    }
    return fixed ? NXG_OK : NXG_ENOTCONV;
}


// ---------------------------------------------------------------------------
// SCC rounds (see ProgSCCF). Every kernel below takes vertices in internal
// ids; `ids` (NULL: the identity) gives a vertex's caller id.
// ---------------------------------------------------------------------------
// Block flags of a wave's 64 consecutive vertices from per-vertex predicates
// (blocks of 2^bs <= 64 vertices lie inside one wave, the wave's first vertex
// a multiple of 64): a block's first lane writes its flag, when that vertex is
// in the graph (in). Called by every lane of the wave.
__device__ inline void set_block_flags(uint8_t* __restrict__ chg, int64_t v, bool in, bool any, int bs) {
    const uint64_t m = __ballot(any);
    const int bl = 1 << bs, lane = lane_id();
    const int first = lane & ~(bl - 1);
    const uint64_t bm = (bl == 64 ? ~0ull : (1ull << bl) - 1ull) << first;
    if (lane == first && in) chg[v >> bs] = (m & bm) != 0;
}

// Round start: colours of the unassigned vertices (their caller ids; kInf for
// assigned ones) into both buffers; a block is flagged when it holds an
// unassigned vertex. Clears the count of vertices left.
__global__ __launch_bounds__(256) void k_scc_init_fwd(int32_t n, const int32_t* __restrict__ lab,
                                                      const int32_t* __restrict__ ids,
                                                      int32_t* __restrict__ c0, int32_t* __restrict__ c1,
                                                      uint8_t* __restrict__ chg, int bs,
                                                      unsigned long long* __restrict__ left) {
    const int64_t n64 = n, stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t v0 = (int64_t)blockIdx.x * blockDim.x; v0 < n64; v0 += stride) {
        const int64_t v = v0 + threadIdx.x;
        const bool in = v < n64;
        const bool open = in && lab[v] < 0;
        if (in) c0[v] = c1[v] = open ? (ids ? ids[v] : (int32_t)v) : kInf;
        set_block_flags(chg, v, in, open, bs);
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) *left = 0;
}

// Backward start: each colour's root joins (kInf - 1 - colour), every other vertex
// holds kInf; a block is flagged when it holds a root.
__global__ __launch_bounds__(256) void k_scc_init_bwd(int32_t n, const int32_t* __restrict__ lab,
                                                      const int32_t* __restrict__ ids,
                                                      const int32_t* __restrict__ col,
                                                      int32_t* __restrict__ q0, int32_t* __restrict__ q1,
                                                      uint8_t* __restrict__ chg, int bs) {
    const int64_t n64 = n, stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t v0 = (int64_t)blockIdx.x * blockDim.x; v0 < n64; v0 += stride) {
        const int64_t v = v0 + threadIdx.x;
        const bool in = v < n64;
        bool root = false;
        if (in) {
            const int32_t c = col[v];
            root = lab[v] < 0 && c == (ids ? ids[v] : (int32_t)v);
            q0[v] = q1[v] = root ? kInf - 1 - c : kInf;
        }
        set_block_flags(chg, v, in, root, bs);
    }
}

// Round end: joined vertices take their colour as label; the others are
// counted (one atomic per workgroup).
__global__ __launch_bounds__(256) void k_scc_assign(int32_t n, int32_t* __restrict__ lab,
                                                    const int32_t* __restrict__ col,
                                                    const int32_t* __restrict__ q,
                                                    unsigned long long* __restrict__ left) {
    __shared__ unsigned long long red[4];
    const int64_t n64 = n, stride = (int64_t)gridDim.x * blockDim.x;
    unsigned long long cnt = 0;
    for (int64_t v0 = (int64_t)blockIdx.x * blockDim.x; v0 < n64; v0 += stride) {
        const int64_t v = v0 + threadIdx.x;
        if (v < n64 && lab[v] < 0) {
            if (q[v] != kInf)
                lab[v] = col[v];
            else
                ++cnt;
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) cnt += __shfl_xor(cnt, off);
    if (lane_id() == 0) red[threadIdx.x >> 6] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned long long t = red[0] + red[1] + red[2] + red[3];
        if (t) atomicAdd(left, t);
    }
}

// One layout's state for taking an integer program to its fixed point with
// block activity, as the BFS/WCC runs do: both value buffers, the block flags
// and their prefix counts, the compacted chunk lists and the changed flags of
// one synchronisation block of passes.
struct ActiveSweep {
    Layout* L = nullptr;
    Plan* p = nullptr;
    Workspace w;
    int bs = 0, seg = 0, nseg = 0, block = 0;
    int64_t nb = 0;
    Geo geo;
    size_t lds = 0;
    uint8_t* chg() const { return w.blk.as<uint8_t>(); }
    unsigned long long* streamed() const { return w.bfsout.as<unsigned long long>(); }

    // vb: bytes of a value (and of an LDS accumulator)
    void init(nxg_dsss* g, Layout& Lr, int piece, int block_, hipStream_t s, size_t vb = 4) {
        ensure_chunk_ranges(Lr, s);
        L = &Lr;
        block = block_;
        p = get_plan(g, Lr, -piece, true, s);
        alloc_common(w, Lr, *p, vb, block, s, true);
        w.buf[0].alloc(vb * Lr.n, s);
        w.buf[1].alloc(vb * Lr.n, s);
        bs = std::min(6, Lr.t);
        nb = ((int64_t)Lr.n + (1 << bs) - 1) >> bs;
        seg = 4096;
        while ((nb + seg) / seg > 256) seg *= 2;
        nseg = (int)((nb + seg) / seg);
        w.blk.alloc((size_t)nb, s);
        w.bpre.alloc(sizeof(int32_t) * (size_t)(nb + 1), s);
        w.btot.alloc(sizeof(int32_t) * (size_t)nseg, s);
        w.clist.alloc(sizeof(int64_t) * std::max<int64_t>(Lr.n_chunks, 1), s);
        w.ccount.alloc(sizeof(int32_t) * Lr.n_tiles, s);
        w.bfsout.alloc(sizeof(unsigned long long), s);
        fill<int32_t>(w.ccount.as<int32_t>(), Lr.n_tiles, 0, s);
        fill<unsigned long long>(streamed(), 1, 0ull, s);
        geo = make_geo(Lr, *p, w, vb);
        geo.clist = w.clist.as<int64_t>();
        geo.ccount = w.ccount.as<int32_t>();
        geo.split_min = piece;
        lds = iter_lds(geo, Lr, vb);
    }

    // Passes from the values in buf[0] until one changes nothing, at most
    // `budget` of them in all (counted down). mk(cur, nxt, k) makes the program
    // of pass k (from 0). Returns the buffer that holds the fixed point; *changed = passes
    // that changed a value. A monotone program changes a value in at most
    // n + 1 passes; more means the device state is broken (error, no loop).
    template <class Prog, class Make>
    void* settle(Make mk, int64_t& budget, int64_t* changed, bool* ok, hipStream_t s) {
        std::vector<double> hs(4 * (size_t)block);
        int64_t k = 0;
        for (;;) {
            if (k > (int64_t)L->n + 1 + block)
                fail(NXG_EDEVICE, "a propagation did not settle within n + 1 passes");
            if (budget <= 0) {
                *ok = false;
                return w.buf[k & 1].p;
            }
            const int nb_ = (int)std::min<int64_t>(block, budget);
            for (int j = 0; j < nb_; ++j, ++k) {
                hipLaunchKernelGGL(k_blkscan, dim3(nseg), dim3(1024), 0, s, chg(), (const uint8_t*)nullptr,
                                   nb, seg, w.bpre.as<int32_t>(), (int32_t*)nullptr, w.btot.as<int32_t>(),
                                   (int32_t*)nullptr, w.ccount.as<int32_t>(), L->n_tiles, streamed(),
                                   w.stats.as<double>() + 4 * j + 3);
                NXG_CHECK_LAUNCH();
                if (L->n_chunks > 0) {
                    hipLaunchKernelGGL(k_compact, dim3(grid_for(L->n_chunks, 256, 4096)), dim3(256), 0, s,
                                       L->tile_chunk.as<int64_t>(), L->chunk_tile.as<int32_t>(), L->n_chunks,
                                       L->chunk_rng.as<int4>(), bs, seg, nseg, w.bpre.as<int32_t>(),
                                       w.btot.as<int32_t>(), (const int32_t*)nullptr, (const int32_t*)nullptr,
                                       w.clist.as<int64_t>(), w.ccount.as<int32_t>());
                    NXG_CHECK_LAUNCH();
                }
                Ctl ctl{w.stats.as<double>(), w.done.as<int32_t>(), j, 0.0};
                const Prog pr = mk(w.buf[k & 1].p, w.buf[(k + 1) & 1].p, k);
                launch_iter<Prog, 1024>(geo, ctl, pr, *p, lds, s);
            }
            budget -= nb_;
            NXG_HIP(hipMemcpyAsync(hs.data(), w.stats.as<double>(), sizeof(double) * 4 * nb_,
                                   hipMemcpyDeviceToHost, s));
            NXG_HIP(hipStreamSynchronize(s));
            for (int j = 0; j < nb_; ++j) {
                if (hs[4 * j + 3] == 0.0) {
                    // a pass that changes nothing leaves both buffers equal
                    return w.buf[k & 1].p;
                }
                ++*changed;
            }
        }
    }
};

struct SccCache : Cached {
    int piece = 0;
    ActiveSweep f, b;
    DevBuf lab, left;
};

nxg_status run_scc(nxg_dsss* g, const nxg_run_desc& d, hipStream_t s, nxg_run_stats* st) {
    if (!g->has_rev) fail(NXG_EINVAL, "SCC needs a build with NXG_BUILD_TRANSPOSE");
    if (d.dtype != NXG_I32) fail(NXG_EINVAL, "SCC needs dtype I32");
    if (d.batch != 1 && d.batch != 0) fail(NXG_EUNSUPPORTED, "SCC runs one problem per call");
    if (d.flags) fail(NXG_EINVAL, "SCC takes no run flags");
    if (((size_t)g->fwd.T + kSpill) * 4 > (size_t)lds_budget_bytes(g->device) || g->fwd.T > 65536)
        fail(NXG_EINVAL, "tile does not fit in LDS");
    const VMap vm = vmap_of(g);
    Layout& Lf = g->fwd;
    const int32_t n = Lf.n;
    const int cus = num_cus(g->device);
    int piece = env_int("NXG_PIECE_CHUNKS", 0);
    if (piece <= 0) piece = default_piece(Lf.n_chunks, Lf.C, (size_t)Lf.T * 4, cus);
    const int block = std::max(1, env_int("NXG_SYNC_BLOCK", 4));
    SccCache* c = nullptr;
    for (Cached* x : g->cached) {
        SccCache* m = dynamic_cast<SccCache*>(x);
        if (m && m->piece == piece && m->f.block == block) c = m;
    }
    if (!c) {
        c = new SccCache();
        g->cached.push_back(c);
        PendingEntry pend(g, c);
        c->piece = piece;
        c->f.init(g, g->fwd, piece, block, s);
        c->b.init(g, g->rev, piece, block, s);
        c->lab.alloc(sizeof(int32_t) * (size_t)n, s);
        c->left.alloc(sizeof(unsigned long long), s);
        pend.commit();
    } else {
        touch_cached(g, c);
        fill<unsigned long long>(c->f.streamed(), 1, 0ull, s);
        fill<unsigned long long>(c->b.streamed(), 1, 0ull, s);
    }
    int32_t* lab = c->lab.as<int32_t>();
    unsigned long long* left = c->left.as<unsigned long long>();
    const int32_t* ids = vm ? vm.n2o : nullptr;
    Events ev;
    NXG_HIP(hipEventRecord(ev.a, s));
    fill<int32_t>(lab, n, -1, s);
    int64_t budget = d.max_iters, changed = 0;
    int32_t rounds = 0;
    bool ok = true;
    unsigned long long h_left = (unsigned long long)n;
    while (h_left > 0 && ok) {
        ActiveSweep& F = c->f;
        ActiveSweep& B = c->b;
        hipLaunchKernelGGL(k_scc_init_fwd, dim3(grid_for(n)), dim3(256), 0, s, n, (const int32_t*)lab, ids,
                           F.w.buf[0].as<int32_t>(), F.w.buf[1].as<int32_t>(), F.chg(), F.bs, left);
        NXG_CHECK_LAUNCH();
        const int bsf = F.bs;
        int32_t* col = (int32_t*)F.settle<ProgSCCF>(
            [&](void* cu, void* nx, int64_t) {
                return ProgSCCF{(const int32_t*)cu, (int32_t*)nx, F.chg(), nullptr, bsf};
            },
            budget, &changed, &ok, s);
        if (!ok) break;
        hipLaunchKernelGGL(k_scc_init_bwd, dim3(grid_for(n)), dim3(256), 0, s, n, (const int32_t*)lab, ids,
                           (const int32_t*)col, B.w.buf[0].as<int32_t>(), B.w.buf[1].as<int32_t>(), B.chg(),
                           B.bs);
        NXG_CHECK_LAUNCH();
        const int bsb = B.bs;
        int32_t* q = (int32_t*)B.settle<ProgSCCB>(
            [&](void* cu, void* nx, int64_t) {
                return ProgSCCB{(const int32_t*)cu, (int32_t*)nx, B.chg(), nullptr, bsb, col};
            },
            budget, &changed, &ok, s);
        if (!ok) break;
        hipLaunchKernelGGL(k_scc_assign, dim3(grid_for(n)), dim3(256), 0, s, n, lab, (const int32_t*)col,
                           (const int32_t*)q, left);
        NXG_CHECK_LAUNCH();
        const unsigned long long before = h_left;
        NXG_HIP(hipMemcpyAsync(&h_left, left, sizeof(h_left), hipMemcpyDeviceToHost, s));
        NXG_HIP(hipStreamSynchronize(s));
        ++rounds;
        // the smallest unassigned caller id is its own colour's root, so a round
        // assigns at least its component
        if (h_left >= before) fail(NXG_EDEVICE, "SCC round assigned no vertex");
    }
    // the last passes' chunk lists into the streamed counts
    unsigned long long strm[2] = {0, 0};
    hipLaunchKernelGGL(k_count_streamed, dim3(1), dim3(1024), 0, s, c->f.w.ccount.as<int32_t>(), Lf.n_tiles,
                       c->f.streamed());
    NXG_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_count_streamed, dim3(1), dim3(1024), 0, s, c->b.w.ccount.as<int32_t>(),
                       g->rev.n_tiles, c->b.streamed());
    NXG_CHECK_LAUNCH();
    NXG_HIP(hipEventRecord(ev.b, s));
    // labels out in caller ids; a vertex dropped by degreeing is its own component
    if (vm)
        permute_rows<int32_t>(lab, vm.o2n, vm.n, 1, (int32_t*)d.d_values, s, 1, 0, 1);
    else {
        hipLaunchKernelGGL(k_copy<int32_t>, dim3(grid_for(n)), dim3(256), 0, s, (const int32_t*)lab,
                           (int32_t*)d.d_values, (int64_t)n);
        NXG_CHECK_LAUNCH();
    }
    NXG_HIP(hipMemcpyAsync(&strm[0], c->f.streamed(), sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
    NXG_HIP(hipMemcpyAsync(&strm[1], c->b.streamed(), sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
    NXG_HIP(hipStreamSynchronize(s));
    float ms = 0.f;
    NXG_HIP(hipEventSynchronize(ev.b));
    NXG_HIP(hipEventElapsedTime(&ms, ev.a, ev.b));
    if (st) {
        memset(st, 0, sizeof(*st));
        st->iterations = rounds;
        st->converged = ok ? 1 : 0;
        st->changed_rounds = (int32_t)std::min<int64_t>(changed, INT32_MAX);
        st->device_ms = ms;
        st->streamed_chunks = (int64_t)(strm[0] + strm[1]);
    }
    return ok ? NXG_OK : NXG_ENOTCONV;
}

// ---------------------------------------------------------------------------
// Several BFS at once (ProgMSBFS), one per root, B <= 64.
// ---------------------------------------------------------------------------
// Roots (caller ids) into the masks and levels: bit b at root b's internal id
// in both mask buffers, level 0, and its activity block flagged. A root that
// degreeing dropped (internal id -1) reaches nothing.
__global__ void k_msbfs_roots(int B, const int32_t* __restrict__ roots, const int32_t* __restrict__ o2n,
                              uint64_t* __restrict__ m0, uint64_t* __restrict__ m1,
                              int32_t* __restrict__ lev, uint8_t* __restrict__ chg, int bs) {
    const int b = threadIdx.x;
    if (b >= B) return;
    const int32_t r = o2n ? o2n[roots[b]] : roots[b];
    if (r < 0) return;
    atomicOr((unsigned long long*)&m0[r], 1ull << b);
    atomicOr((unsigned long long*)&m1[r], 1ull << b);
    lev[(int64_t)r * B + b] = 0;
    chg[r >> bs] = 1;
}

// Level 0 at each root's own row of the caller's output (for a root dropped by
// degreeing, the map-out filled its row with unreached).
__global__ void k_msbfs_root_rows(int B, const int32_t* __restrict__ roots, int32_t* __restrict__ out) {
    const int b = threadIdx.x;
    if (b < B) out[(int64_t)roots[b] * B + b] = 0;
}

// Edges reached over all searches: sum over v of |roots reaching v| * outdeg(v)
// (integer, one atomic per workgroup).
__global__ __launch_bounds__(256) void k_msbfs_reached(int32_t n, const uint64_t* __restrict__ m,
                                                       const int32_t* __restrict__ deg,
                                                       unsigned long long* __restrict__ total) {
    __shared__ unsigned long long red[4];
    unsigned long long c = 0;
    for (int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x; v < n; v += (int64_t)gridDim.x * 256)
        c += (unsigned long long)__popcll(m[v]) * (unsigned long long)deg[v];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off);
    if (lane_id() == 0) red[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned long long t = red[0] + red[1] + red[2] + red[3];
        if (t) atomicAdd(total, t);
    }
}

struct MsbfsCache : Cached {
    int piece = 0;
    ActiveSweep f;
    DevBuf lev, roots, reached;
    int32_t B = 0;
};

nxg_status run_msbfs(nxg_dsss* g, const nxg_run_desc& d, hipStream_t s, nxg_run_stats* st) {
    const int B = d.batch;
    if (B < 2 || B > 64) fail(NXG_EINVAL, "batched BFS takes 2 to 64 roots");
    if (d.dtype != NXG_I32) fail(NXG_EINVAL, "BFS needs dtype I32");
    if (!d.roots) fail(NXG_EINVAL, "BFS needs roots");
    if (d.flags) fail(NXG_EINVAL, "batched BFS takes no run flags");
    if (((size_t)g->fwd.T + kSpill) * 8 > (size_t)lds_budget_bytes(g->device))
        fail(NXG_EINVAL, "batched BFS keeps 8-byte root sets per destination in LDS; build with value_bytes = 8");
    const VMap vm = vmap_of(g);
    const int64_t n_out = vm ? vm.n : g->fwd.n;
    for (int b = 0; b < B; ++b)
        if (d.roots[b] < 0 || d.roots[b] >= n_out) fail(NXG_EINVAL, "BFS root outside [0, n)");
    Layout& L = g->fwd;
    const int32_t n = L.n;
    const int cus = num_cus(g->device);
    int piece = env_int("NXG_PIECE_CHUNKS", 0);
    if (piece <= 0) piece = default_piece(L.n_chunks, L.C, (size_t)L.T * 8, cus);
    const int block = std::max(1, env_int("NXG_SYNC_BLOCK", 4));
    MsbfsCache* c = nullptr;
    for (Cached* x : g->cached) {
        MsbfsCache* m = dynamic_cast<MsbfsCache*>(x);
        if (m && m->piece == piece && m->f.block == block && m->B == B) c = m;
    }
    if (!c) {
        c = new MsbfsCache();
        g->cached.push_back(c);
        PendingEntry pend(g, c);
        c->piece = piece;
        c->B = B;
        c->f.init(g, L, piece, block, s, 8);
        if (vm) c->lev.alloc(sizeof(int32_t) * (size_t)n * B, s);
        c->roots.alloc(sizeof(int32_t) * B, s);
        c->reached.alloc(sizeof(unsigned long long), s);
        pend.commit();
    } else {
        touch_cached(g, c);
        fill<unsigned long long>(c->f.streamed(), 1, 0ull, s);
    }
    ActiveSweep& F = c->f;
    int32_t* lev = vm ? c->lev.as<int32_t>() : (int32_t*)d.d_values;
    NXG_HIP(hipMemcpyAsync(c->roots.p, d.roots, sizeof(int32_t) * B, hipMemcpyHostToDevice, s));
    Events ev;
    NXG_HIP(hipEventRecord(ev.a, s));
    fill<uint64_t>(F.w.buf[0].as<uint64_t>(), n, 0ull, s);
    fill<uint64_t>(F.w.buf[1].as<uint64_t>(), n, 0ull, s);
    fill<int32_t>(lev, (int64_t)n * B, kInf, s);
    fill<uint8_t>(F.chg(), F.nb, (uint8_t)0, s);
    fill<unsigned long long>(c->reached.as<unsigned long long>(), 1, 0ull, s);
    hipLaunchKernelGGL(k_msbfs_roots, dim3(1), dim3(64), 0, s, B, (const int32_t*)c->roots.as<int32_t>(),
                       vm.o2n, F.w.buf[0].as<uint64_t>(), F.w.buf[1].as<uint64_t>(), lev, F.chg(), F.bs);
    NXG_CHECK_LAUNCH();
    const uint64_t full = B == 64 ? ~0ull : ((1ull << B) - 1ull);
    int64_t budget = d.max_iters, changed = 0;
    bool ok = true;
    const int bs = F.bs;
    uint64_t* fin = (uint64_t*)F.settle<ProgMSBFS>(
        [&](void* cu, void* nx, int64_t k) {
            return ProgMSBFS{(const uint64_t*)cu, (uint64_t*)nx, F.chg(), nullptr, bs, lev, B, (int32_t)(k + 1),
                             full};
        },
        budget, &changed, &ok, s);
    hipLaunchKernelGGL(k_count_streamed, dim3(1), dim3(1024), 0, s, F.w.ccount.as<int32_t>(), L.n_tiles,
                       F.streamed());
    NXG_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_msbfs_reached, dim3(grid_for(n, 256, 1024)), dim3(256), 0, s, n, (const uint64_t*)fin,
                       L.outdeg.as<int32_t>(), c->reached.as<unsigned long long>());
    NXG_CHECK_LAUNCH();
    NXG_HIP(hipEventRecord(ev.b, s));
    if (vm) {
        permute_rows<int32_t>(lev, vm.o2n, vm.n, B, (int32_t*)d.d_values, s, 1, kInf, 0);
        hipLaunchKernelGGL(k_msbfs_root_rows, dim3(1), dim3(64), 0, s, B, (const int32_t*)c->roots.as<int32_t>(),
                           (int32_t*)d.d_values);
        NXG_CHECK_LAUNCH();
    }
    unsigned long long out2[2] = {0, 0};
    NXG_HIP(hipMemcpyAsync(&out2[0], F.streamed(), sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
    NXG_HIP(hipMemcpyAsync(&out2[1], c->reached.p, sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
    NXG_HIP(hipStreamSynchronize(s));
    float ms = 0.f;
    NXG_HIP(hipEventSynchronize(ev.b));
    NXG_HIP(hipEventElapsedTime(&ms, ev.a, ev.b));
    if (st) {
        memset(st, 0, sizeof(*st));
        st->iterations = (int32_t)std::min<int64_t>(changed + 1, INT32_MAX);
        st->converged = ok ? 1 : 0;
        st->changed_rounds = (int32_t)changed;
        st->max_level = (int32_t)changed;  // round r sets level r
        st->reached_edges = (int64_t)out2[1];
        st->device_ms = ms;
        st->streamed_chunks = (int64_t)out2[0];
    }
    return ok ? NXG_OK : NXG_ENOTCONV;
}

nxg_status run_batched(nxg_dsss* g, const nxg_run_desc& d, hipStream_t s, nxg_run_stats* st) {
    const Layout& L = g->fwd;
    const int B = d.batch;
    if (B < 1 || B > 64) fail(NXG_EINVAL, "batch must be in [1, 64]");
    if (d.program != NXG_PAGERANK || d.dtype != NXG_F32)
        fail(NXG_EUNSUPPORTED, "batched runs support plain PageRank in FP32");
    if (d.d_teleport) fail(NXG_EUNSUPPORTED, "batched runs take seed vertices (d_seeds), not a dense teleport");
    if (d.flags & NXG_RUN_WARM_START) fail(NXG_EUNSUPPORTED, "batched runs start from the teleport vector");
    // the tile's [T, B] FP64 sums; at least the kernels' scalar reduction area
    // (48 x 64 doubles), so a narrow batch runs on a small tile too
    const size_t lds = std::max((size_t)L.T * B * 8, (size_t)(3 * 16) * 64 * 8);
    if (lds > (size_t)lds_budget_bytes(g->device))
        fail(NXG_EINVAL, "tile * batch * 8 bytes exceeds LDS; build with value_bytes = 8 * batch");
    const int cus = num_cus(g->device);
    int piece = env_int("NXG_PIECE_CHUNKS", 0);
    if (piece <= 0) piece = default_piece(L.n_chunks, L.C, (size_t)L.T * B * 8, cus);
    Plan* p = get_plan(g, L, piece, false, s);
    const int max_iters = d.max_iters;
    const bool capture = (d.flags & NXG_RUN_CAPTURE) != 0;
    if (capture && d.tol > 0) fail(NXG_EINVAL, "NXG_RUN_CAPTURE needs a fixed iteration count (tol <= 0)");
    if (capture && max_iters < 1) fail(NXG_EINVAL, "NXG_RUN_CAPTURE needs max_iters >= 1");
    // a captured run keeps its workspace (and graph) in the handle
    CapturedBatched* cap = nullptr;
    bool fresh = true;
    PendingEntry pend(g, nullptr);  // a new capture, until its graph is instantiated
    if (capture) {
        for (Cached* x : g->cached) {
            CapturedBatched* c = dynamic_cast<CapturedBatched*>(x);
            if (c && c->B == B && c->iters == max_iters && c->piece == piece && c->damping == d.damping &&
                c->values == d.d_values && c->seeds == d.d_seeds)
                cap = c;
        }
        fresh = cap == nullptr;
        if (!fresh) touch_cached(g, cap);
        if (fresh) {
            evict_captures<CapturedBatched>(g);
            cap = new CapturedBatched();
            g->cached.push_back(cap);
            pend.c = cap;
            cap->B = B;
            cap->iters = max_iters;
            cap->piece = piece;
            cap->damping = d.damping;
            cap->values = d.d_values;
            cap->seeds = d.d_seeds;
        }
    }
    Workspace wl;
    Workspace& w = cap ? cap->w : wl;
    const size_t nstat = (size_t)(max_iters + 2) * 3 * B;
    if (fresh) {
        // partial slots hold T*B doubles each
        const int64_t hub = (int64_t)std::max(p->n_slots, 1) * L.T * B;
        w.partial.alloc(sizeof(double) * hub, s);
        w.tile_s.alloc(sizeof(double) * 3 * B * (size_t)L.n_tiles, s);
        w.tile_flag.alloc(sizeof(int32_t) * L.n_tiles, s);
        w.stats.alloc(sizeof(double) * nstat, s);
        NXG_HIP(hipMemsetAsync(w.stats.p, 0, sizeof(double) * nstat, s));
        w.done.alloc(sizeof(int32_t), s);
        NXG_HIP(hipMemsetAsync(w.done.p, 0, sizeof(int32_t), s));
        w.buf[0].alloc(sizeof(float) * (size_t)L.n * B, s);
        w.buf[1].alloc(sizeof(float) * (size_t)L.n * B, s);
        w.bfsout.alloc(sizeof(unsigned long long) * kDangBlocks, s);  // dangling counts per workgroup
    }
    const int32_t* seeds = d.d_seeds;
    if (seeds) {
        // seeds index the vertex arrays (and the id map of a relabeled build)
        int32_t hseed[64];
        NXG_HIP(hipMemcpyAsync(hseed, seeds, sizeof(int32_t) * B, hipMemcpyDeviceToHost, s));
        NXG_HIP(hipStreamSynchronize(s));
        const int64_t n_out = g->relabeled ? (int64_t)g->n_caller : (int64_t)L.n;
        for (int b = 0; b < B; ++b)
            if (hseed[b] < 0 || hseed[b] >= n_out) fail(NXG_EINVAL, "seed vertex outside [0, n)");
    }
    const VMap vm = vmap_of(g);
    float* vals = (float*)d.d_values;
    if (vm) {
        // seeds to internal ids; the result rows come back through old2new
        if (seeds) {
            if (fresh) w.mseeds.alloc(sizeof(int32_t) * B, s);
            permute_rows<int32_t>(vm.o2n, seeds, B, 1, w.mseeds.as<int32_t>(), s);
            seeds = w.mseeds.as<int32_t>();
            int32_t hs2[64];
            NXG_HIP(hipMemcpyAsync(hs2, seeds, sizeof(int32_t) * B, hipMemcpyDeviceToHost, s));
            NXG_HIP(hipStreamSynchronize(s));
            for (int b = 0; b < B; ++b)
                if (hs2[b] < 0) fail(NXG_EINVAL, "seed vertex dropped by NXG_BUILD_DEGREE (it has no edges)");
        }
        if (fresh) w.mvals.alloc(sizeof(float) * (size_t)L.n * B, s);
        vals = w.mvals.as<float>();
    }
    auto start = [&](hipStream_t cs) {
        hipLaunchKernelGGL(k_init_batched, dim3(grid_for((int64_t)L.n * B, 256, 8192)), dim3(256), 0, cs,
                           L.n, B, L.outdeg.as<int32_t>(), seeds, w.buf[0].as<float>(), (double*)nullptr);
        NXG_CHECK_LAUNCH();
        if (!seeds) {
            hipLaunchKernelGGL(k_count_dangling, dim3(kDangBlocks), dim3(256), 0, cs, L.n,
                               L.outdeg.as<int32_t>(), w.bfsout.as<unsigned long long>());
            NXG_CHECK_LAUNCH();
        }
        hipLaunchKernelGGL(k_init_batched_delta, dim3(1), dim3(64), 0, cs, L.n, B, L.outdeg.as<int32_t>(),
                           seeds, (const unsigned long long*)w.bfsout.as<unsigned long long>(),
                           w.stats.as<double>());
        NXG_CHECK_LAUNCH();
    };
    Geo geo = make_geo(L, *p, w, 8);
    const int n_items = (int)p->h_items.size();
    const int n_fin = (int)p->h_fin.size();
    static size_t attr = 0;
    if (lds > attr) {
        NXG_HIP(hipFuncSetAttribute((const void*)k_iterate_batched<1024>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        NXG_HIP(hipFuncSetAttribute((const void*)k_finish_batched<1024>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        attr = lds;
    }
    // the scalar reduction: blocks of `per` tiles, then one block over the block sums
    const int rblocks = std::min(L.n_tiles, 256);
    const int rper = (L.n_tiles + rblocks - 1) / rblocks;
    if (fresh) w.part.alloc(sizeof(double) * 3 * B * (size_t)rblocks, s);
    auto one_iteration = [&](const BCtl& ctl, const float* cur, float* nxt, float* xout, hipStream_t cs) {
        if (n_items > 0) {
            hipLaunchKernelGGL(k_iterate_batched<1024>, dim3(n_items), dim3(1024), lds, cs, geo, ctl, cur,
                               nxt, xout, seeds, B, d.damping, w.tile_s.as<double>());
            NXG_CHECK_LAUNCH();
        }
        if (n_fin > 0) {
            hipLaunchKernelGGL(k_finish_batched<1024>, dim3(n_fin), dim3(1024), lds, cs, geo, ctl, cur, nxt,
                               xout, seeds, B, d.damping, w.tile_s.as<double>(), p->fin.as<Item>());
            NXG_CHECK_LAUNCH();
        }
        hipLaunchKernelGGL(k_reduce_batched1, dim3(rblocks), dim3(256), 0, cs, w.tile_s.as<double>(),
                           L.n_tiles, B, rper, ctl.done, w.part.as<double>());
        NXG_CHECK_LAUNCH();
        hipLaunchKernelGGL(k_reduce_batched2, dim3(1), dim3(256), 0, cs, w.part.as<double>(), rblocks, B,
                           ctl);
        NXG_CHECK_LAUNCH();
    };
    Events ev;
    hipEvent_t e0 = ev.a, e1 = ev.b;
    if (capture) {
        // record start, the fixed iterations and the id map once (no memset in
        // the graph: the workspace's counters were cleared at allocation and a
        // fixed-count run never sets the stop flag), then replay
        if (fresh) {
            NXG_HIP(hipStreamSynchronize(s));
            if (!g->capture_stream)
                NXG_HIP(hipStreamCreateWithFlags(&g->capture_stream, hipStreamNonBlocking));
            hipStream_t cs = g->capture_stream;
            NXG_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
            try {
                start(cs);
                for (int k = 0; k < max_iters; ++k) {
                    BCtl ctl{w.stats.as<double>(), w.done.as<int32_t>(), k, 0.0};
                    one_iteration(ctl, w.buf[k & 1].as<float>(), w.buf[(k + 1) & 1].as<float>(),
                                  k == max_iters - 1 ? vals : nullptr, cs);
                }
                if (vm) permute_rows<float>(vals, vm.o2n, vm.n, B, (float*)d.d_values, cs);
            } catch (...) {
                hipGraph_t dead = nullptr;
                (void)hipStreamEndCapture(cs, &dead);
                if (dead) (void)hipGraphDestroy(dead);
                throw;
            }
            NXG_HIP(hipStreamEndCapture(cs, &cap->graph));
            NXG_HIP(hipGraphInstantiate(&cap->exec, cap->graph, nullptr, nullptr, 0));
            pend.commit();
        }
        NXG_HIP(hipEventRecord(e0, s));
        NXG_HIP(hipGraphLaunch(cap->exec, s));
        NXG_HIP(hipEventRecord(e1, s));
        double resid = 0.0;
        if (st) {
            std::vector<double> hs(nstat);
            NXG_HIP(hipMemcpyAsync(hs.data(), w.stats.p, sizeof(double) * nstat, hipMemcpyDeviceToHost, s));
            NXG_HIP(hipStreamSynchronize(s));
            for (int b = 0; b < B; ++b)
                resid = std::max(resid, hs[(size_t)(max_iters - 1) * 3 * B + B + b]);
            float ms = 0.f;
            NXG_HIP(hipEventSynchronize(e1));
            NXG_HIP(hipEventElapsedTime(&ms, e0, e1));
            memset(st, 0, sizeof(*st));
            st->iterations = max_iters;
            st->residual = resid;
            st->device_ms = ms;
        }
        return NXG_OK;
    }
    start(s);
    NXG_HIP(hipEventRecord(e0, s));
    const int block = d.tol > 0 ? std::max(1, env_int("NXG_SYNC_BLOCK", 8)) : max_iters;
    int k = 0, done_h = 0;
    while (k < max_iters) {
        const int kend = std::min(max_iters, k + block);
        for (; k < kend; ++k) {
            BCtl ctl{w.stats.as<double>(), w.done.as<int32_t>(), k, d.tol};
            float* xout = (k == max_iters - 1) ? vals : nullptr;
            one_iteration(ctl, w.buf[k & 1].as<float>(), w.buf[(k + 1) & 1].as<float>(), xout, s);
        }
        if (d.tol > 0 && k < max_iters) {
            NXG_HIP(hipMemcpyAsync(&done_h, w.done.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
            NXG_HIP(hipStreamSynchronize(s));
            if (done_h) break;
        }
    }
    if (k < max_iters || max_iters == 0) {
        // emit x from the newest vector through the carry-over path
        NXG_HIP(hipMemsetAsync(w.done.p, 0xFF, sizeof(int32_t), s));
        BCtl ctl{w.stats.as<double>(), w.done.as<int32_t>(), k, d.tol};
        hipLaunchKernelGGL(k_iterate_batched<1024>, dim3(n_items), dim3(1024), lds, s, geo, ctl,
                           w.buf[k & 1].as<float>(), w.buf[(k + 1) & 1].as<float>(), vals, seeds, B,
                           d.damping, w.tile_s.as<double>());
        NXG_CHECK_LAUNCH();
    }
    if (vm) permute_rows<float>(vals, vm.o2n, vm.n, B, (float*)d.d_values, s);
    NXG_HIP(hipEventRecord(e1, s));
    std::vector<double> hs(nstat);
    NXG_HIP(hipMemcpyAsync(hs.data(), w.stats.p, sizeof(double) * nstat, hipMemcpyDeviceToHost, s));
    NXG_HIP(hipStreamSynchronize(s));
    int iters = k, conv_at = -1;
    double resid = 0.0;
    for (int i = 0; i < k; ++i) {
        double mx = 0.0;
        for (int b = 0; b < B; ++b) mx = std::max(mx, hs[(size_t)i * 3 * B + B + b]);
        resid = mx;
        if (d.tol > 0 && mx <= d.tol) {
            conv_at = i;
            break;
        }
    }
    if (conv_at >= 0) iters = conv_at + 1;
    float ms = 0.f;
    NXG_HIP(hipEventSynchronize(e1));
    NXG_HIP(hipEventElapsedTime(&ms, e0, e1));
    if (st) {
        memset(st, 0, sizeof(*st));
        st->iterations = iters;
        st->converged = conv_at >= 0;
        st->residual = resid;
        st->device_ms = ms;
    }
    return (d.tol > 0 && conv_at < 0) ? NXG_ENOTCONV : NXG_OK;
}


nxg_status run_multi(nxg_multi* mg, const nxg_run_desc& d, void* const* d_values, hipStream_t s,
                     nxg_run_stats* st) {
    if (d.program != NXG_PAGERANK || d.dtype != NXG_F32 || (d.batch != 1 && d.batch != 0))
        fail(NXG_EUNSUPPORTED, "the multi-graph launch runs plain FP32 PageRank");
    if (d.tol > 0) fail(NXG_EUNSUPPORTED, "the multi-graph launch runs a fixed number of iterations");
    if (d.flags & NXG_RUN_PERSISTENT)
        fail(NXG_EUNSUPPORTED, "the single persistent launch over all iterations is disabled: its "
                               "test did not finish on MI355X and the cause is not known");
    if (d.d_teleport || d.d_seeds || (d.flags & NXG_RUN_WARM_START))
        fail(NXG_EUNSUPPORTED, "the multi-graph launch uses the uniform teleport from x^0 = 1/n");
    if (!(d.damping >= 0.0 && d.damping < 1.0)) fail(NXG_EINVAL, "damping outside [0, 1)");
    if (!d_values) fail(NXG_EINVAL, "d_values is NULL");
    const int G = (int)mg->graphs.size();
    const int iters = d.max_iters;
    if (iters < 1) fail(NXG_EINVAL, "max_iters must be >= 1");
    for (int i = 0; i < G; ++i)
        if (!d_values[i]) fail(NXG_EINVAL, "d_values[" + std::to_string(i) + "] is NULL");
    const int device = mg->graphs[0]->device;
    const int cus = num_cus(device);
    int64_t chunks = 0;
    int maxT = 1;
    for (nxg_dsss* g : mg->graphs) {
        chunks += g->fwd.n_chunks;
        maxT = std::max(maxT, g->fwd.T);
    }
    size_t lds = ((size_t)maxT + kSpill) * 8;
    if (lds > (size_t)lds_budget_bytes(device)) fail(NXG_EINVAL, "a tile does not fit in LDS");
    int piece = env_int("NXG_PIECE_CHUNKS", 0);
    if (piece <= 0) {
        // half a CU's share: the items of many graphs vary more in size, and
        // smaller ones balance the end of each launch. The partial-size floor
        // is taken at the largest chunk (the graphs whose tiles are split)
        int maxC = 256;
        for (nxg_dsss* g : mg->graphs) maxC = std::max(maxC, g->fwd.C);
        piece = default_piece(chunks / 2, maxC, (size_t)maxT * 8, cus);
    }
    // per-graph plans, workspaces and descriptors, kept by the handle for the
    // next run with the same iteration count and piece size
    MultiCache* c = dynamic_cast<MultiCache*>(mg->run_cache);
    if (!c || c->iters != iters || c->piece != piece) {
        delete mg->run_cache;
        mg->run_cache = nullptr;
        std::unique_ptr<MultiCache> nc(new MultiCache());
        nc->iters = iters;
        nc->piece = piece;
        nc->ws.resize(G);
        nc->hdesc.resize(G);
        std::vector<Item> all_items;
        std::vector<int32_t> item_graph;
        std::vector<int64_t> item_words;
        std::vector<MultiFin> all_fin;
        for (int i = 0; i < G; ++i) {
            nxg_dsss* g = mg->graphs[i];
            const Layout& L = g->fwd;
            Plan* p = get_plan(g, L, piece, false, s);
            Workspace& w = nc->ws[i];
            alloc_common(w, L, *p, 8, iters, s, false);
            w.buf[0].alloc(sizeof(float) * (L.n), s);
            w.buf[1].alloc(sizeof(float) * (L.n), s);
            MultiGraph& m = nc->hdesc[i];
            m.geo = make_geo(L, *p, w, 8);
            lds = std::max(lds, iter_lds(m.geo, L, 8));
            m.stats = w.stats.as<double>();
            m.buf0 = w.buf[0].as<float>();
            m.buf1 = w.buf[1].as<float>();
            m.o2n = nullptr;
            if (g->relabeled) {
                w.mvals.alloc(sizeof(float) * L.n, s);
                m.xout = w.mvals.as<float>();
                m.o2n = g->old2new.as<int32_t>();
            }
            m.done0 = w.done.as<int32_t>();
            m.n_items = (int32_t)p->h_items.size();
            for (const Item& it : p->h_items) {
                all_items.push_back(it);
                item_graph.push_back(i);
                item_words.push_back((it.c1 - it.c0) * (int64_t)L.C);
            }
            for (const FinSeg& f : p->h_fseg) all_fin.push_back(MultiFin{i, f});
        }
        // heaviest items (in stream words) first over all graphs, so no heavy
        // item of a late graph starts when the GPU is draining
        std::vector<int32_t> ord(all_items.size());
        for (size_t x = 0; x < ord.size(); ++x) ord[x] = (int32_t)x;
        std::stable_sort(ord.begin(), ord.end(),
                         [&](int32_t a, int32_t b) { return item_words[a] > item_words[b]; });
        std::vector<Item> sorted_items(ord.size());
        std::vector<int32_t> sorted_graph(ord.size());
        for (size_t x = 0; x < ord.size(); ++x) {
            sorted_items[x] = all_items[ord[x]];
            sorted_graph[x] = item_graph[ord[x]];
        }
        nc->lds = lds;
        nc->per_iter = (int)sorted_items.size();
        nc->n_fin = (int)all_fin.size();
        nc->dfin.alloc(sizeof(MultiFin) * std::max<size_t>(all_fin.size(), 1), s);
        if (!all_fin.empty())
            NXG_HIP(hipMemcpyAsync(nc->dfin.p, all_fin.data(), sizeof(MultiFin) * all_fin.size(),
                                   hipMemcpyHostToDevice, s));
        nc->ditems.alloc(sizeof(Item) * std::max<size_t>(sorted_items.size(), 1), s);
        nc->dgraph.alloc(sizeof(int32_t) * std::max<size_t>(sorted_graph.size(), 1), s);
        nc->ddesc.alloc(sizeof(MultiGraph) * G, s);
        nc->dres.alloc(sizeof(double) * G, s);
        nc->dpart.alloc(sizeof(double) * G * kMultiBlocks, s);
        NXG_HIP(hipMemcpyAsync(nc->ditems.p, sorted_items.data(), sizeof(Item) * sorted_items.size(),
                               hipMemcpyHostToDevice, s));
        NXG_HIP(hipMemcpyAsync(nc->dgraph.p, sorted_graph.data(), sizeof(int32_t) * sorted_graph.size(),
                               hipMemcpyHostToDevice, s));
        NXG_HIP(hipStreamSynchronize(s));  // the host vectors above go out of scope
        c = nc.release();
        mg->run_cache = c;
    }
    lds = c->lds;
    // the caller's buffers of this run
    for (int i = 0; i < G; ++i) {
        MultiGraph& m = c->hdesc[i];
        m.user = (float*)d_values[i];
        if (!m.o2n) m.xout = m.user;
    }
    NXG_HIP(hipMemcpyAsync(c->ddesc.p, c->hdesc.data(), sizeof(MultiGraph) * G, hipMemcpyHostToDevice, s));
    static size_t attr = 0;
    if (lds > attr) {
        NXG_HIP(hipFuncSetAttribute((const void*)k_multi_iter<1024, false>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        NXG_HIP(hipFuncSetAttribute((const void*)k_multi_iter<1024, true>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        attr = lds;
    }
    const MultiGraph* ddesc = c->ddesc.as<MultiGraph>();
    auto enqueue = [&](hipStream_t cs) {
        hipLaunchKernelGGL(k_multi_init, dim3(G * kMultiBlocks), dim3(256), 0, cs, ddesc, c->dpart.as<double>());
        NXG_CHECK_LAUNCH();
        hipLaunchKernelGGL(k_multi_init_sum, dim3((G + 255) / 256), dim3(256), 0, cs, ddesc, G,
                           c->dpart.as<double>());
        NXG_CHECK_LAUNCH();
        for (int k = 0; k < iters; ++k) {
            if (mg->graphs[0]->fwd.order == NXG_ORDER_DST)
                hipLaunchKernelGGL((k_multi_iter<1024, true>), dim3(c->per_iter), dim3(1024), lds, cs, ddesc,
                                   c->dgraph.as<int32_t>(), c->ditems.as<Item>(), k, iters, d.damping);
            else
                hipLaunchKernelGGL((k_multi_iter<1024, false>), dim3(c->per_iter), dim3(1024), lds, cs, ddesc,
                                   c->dgraph.as<int32_t>(), c->ditems.as<Item>(), k, iters, d.damping);
            NXG_CHECK_LAUNCH();
            if (c->n_fin > 0) {
                hipLaunchKernelGGL(k_multi_finish<kFinWG>, dim3(c->n_fin), dim3(kFinWG),
                                   kFinSeg * sizeof(double), cs, ddesc, c->dfin.as<MultiFin>(), k, iters,
                                   d.damping);
                NXG_CHECK_LAUNCH();
            }
            hipLaunchKernelGGL(k_multi_reduce, dim3(G), dim3(1024), 0, cs, ddesc, k);
            NXG_CHECK_LAUNCH();
        }
        hipLaunchKernelGGL(k_multi_emit, dim3(G * kMultiBlocks), dim3(256), 0, cs, ddesc);
        NXG_CHECK_LAUNCH();
    };
    if ((d.flags & NXG_RUN_CAPTURE) && (!c->exec || c->cap_damping != d.damping)) {
        // record once on a private stream (the run has no memset: every
        // workspace value it reads is written earlier in the same run)
        c->drop_graph();
        NXG_HIP(hipStreamSynchronize(s));
        hipStream_t cs = nullptr;
        NXG_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
        hipError_t err = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
        if (err == hipSuccess) {
            try {
                enqueue(cs);
            } catch (...) {
                hipGraph_t dead = nullptr;
                (void)hipStreamEndCapture(cs, &dead);
                if (dead) (void)hipGraphDestroy(dead);
                (void)hipStreamDestroy(cs);
                throw;
            }
            err = hipStreamEndCapture(cs, &c->graph);
        }
        if (err == hipSuccess) err = hipGraphInstantiate(&c->exec, c->graph, nullptr, nullptr, 0);
        (void)hipStreamDestroy(cs);
        if (err != hipSuccess) {
            c->drop_graph();
            fail(NXG_EDEVICE, std::string("multi-graph capture: ") + hipGetErrorString(err));
        }
        c->cap_damping = d.damping;
    }
    Events ev;
    hipEvent_t e0 = ev.a, e1 = ev.b;
    NXG_HIP(hipEventRecord(e0, s));
    if (d.flags & NXG_RUN_CAPTURE)
        NXG_HIP(hipGraphLaunch(c->exec, s));
    else
        enqueue(s);
    NXG_HIP(hipEventRecord(e1, s));
    std::vector<double> res(G);
    if (st) {
        hipLaunchKernelGGL(k_multi_residuals, dim3(1), dim3(256), 0, s, ddesc, G, iters - 1, c->dres.as<double>());
        NXG_CHECK_LAUNCH();
        NXG_HIP(hipMemcpyAsync(res.data(), c->dres.p, sizeof(double) * G, hipMemcpyDeviceToHost, s));
    }
    NXG_HIP(hipStreamSynchronize(s));
    float ms = 0.f;
    NXG_HIP(hipEventSynchronize(e1));
    NXG_HIP(hipEventElapsedTime(&ms, e0, e1));
    if (st) {
        double worst = 0.0;
        for (double r : res) worst = std::max(worst, r);
        memset(st, 0, sizeof(*st));
        st->iterations = iters;
        st->residual = worst;
        st->device_ms = ms;
    }
    return NXG_OK;
}

nxg_status run_adjoint(nxg_dsss* g, const nxg_adjoint_desc& d, hipStream_t s, nxg_run_stats* st) {
    if (!g->has_rev || !g->fwd.has_weight || !g->fwd.has_perm || !g->rev.has_weight)
        fail(NXG_EINVAL, "the adjoint needs a build with weights, NXG_BUILD_TRANSPOSE and "
                         "NXG_BUILD_KEEP_PERM");
    if (!d.d_xstar || !d.d_gx) fail(NXG_EINVAL, "d_xstar / d_gx is NULL");
    if (!(d.damping >= 0.0 && d.damping < 1.0)) fail(NXG_EINVAL, "damping outside [0, 1)");
    if (d.max_iters < 1) fail(NXG_EINVAL, "max_iters must be >= 1");
    const Layout& R = g->rev;
    const Layout& F = g->fwd;
    if (((size_t)R.T + kSpill) * 8 > (size_t)lds_budget_bytes(g->device))
        fail(NXG_EINVAL, "destination tile does not fit in LDS; rebuild with value_bytes = 8");
    const int cus = num_cus(g->device);
    int piece = env_int("NXG_PIECE_CHUNKS", 0);
    if (piece <= 0) piece = default_piece(R.n_chunks, R.C, (size_t)R.T * 8, cus);
    Plan* p = get_plan(g, R, piece, false, s);
    Workspace w;
    const int max_iters = d.max_iters;
    alloc_common(w, R, *p, 8, max_iters, s, false);
    w.buf[0].alloc(sizeof(double) * (R.n), s);
    w.buf[1].alloc(sizeof(double) * (R.n), s);
    const int nb = grid_for(R.n, 256, 1024);
    w.part.alloc(sizeof(double) * nb, s);
    // a relabeled build works on x* and g in internal ids
    const VMap vm = vmap_of(g);
    const double* gx = d.d_gx;
    const double* xs = d.d_xstar;
    if (vm) {
        w.mgx.alloc(sizeof(double) * R.n, s);
        w.mxs.alloc(sizeof(double) * R.n, s);
        permute_rows<double>(gx, vm.n2o, R.n, 1, w.mgx.as<double>(), s);
        permute_rows<double>(xs, vm.n2o, R.n, 1, w.mxs.as<double>(), s);
        gx = w.mgx.as<double>();
        xs = w.mxs.as<double>();
    }
    hipLaunchKernelGGL(k_init_adj, dim3(nb), dim3(256), 0, s, R.n, gx, w.buf[0].as<double>(),
                       w.part.as<double>());
    NXG_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(64), 0, s, w.part.as<double>(), nb,
                       w.stats.as<double>());
    NXG_CHECK_LAUNCH();
    Geo geo = make_geo(R, *p, w, 8);
    geo.deg = F.outdeg.as<int32_t>();  // dangling set of the forward graph
    const size_t lds = iter_lds(geo, R, 8);
    const int n_items = (int)p->h_items.size();
    Events ev;
    hipEvent_t e0 = ev.a, e1 = ev.b;
    NXG_HIP(hipEventRecord(e0, s));
    const double tol = d.tol > 0 ? d.tol : 0.0;
    const int block = tol > 0 ? std::max(1, env_int("NXG_SYNC_BLOCK", 8)) : max_iters;
    const bool accel = tol > 0 && env_int("NXG_ADJOINT_EXTRAPOLATE", 1) != 0;
    int k = 0, done_h = 0, last_x = 0;
    double rh[4];
    while (k < max_iters) {
        const int kend = std::min(max_iters, k + block);
        for (; k < kend; ++k) {
            Ctl ctl{w.stats.as<double>(), w.done.as<int32_t>(), k, tol};
            ProgADJ pr{w.buf[k & 1].as<double>(), w.buf[(k + 1) & 1].as<double>(), gx, nullptr,
                       R.weight.as<float>(), d.damping};
            launch_iter<ProgADJ, 1024>(geo, ctl, pr, *p, lds, s);
        }
        if (tol > 0 && k < max_iters) {
            NXG_HIP(hipMemcpyAsync(&done_h, w.done.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
            if (accel && k >= 4)
                for (int i = 0; i < 3; ++i)
                    NXG_HIP(hipMemcpyAsync(&rh[i], w.stats.as<double>() + 4 * (k - 3 + i) + 1,
                                           sizeof(double), hipMemcpyDeviceToHost, s));
            NXG_HIP(hipStreamSynchronize(s));
            if (done_h) break;
            // The error of lambda = g + d M^T lambda decays as d^k along M^T's
            // dominant eigenvector (the all-ones vector for row-stochastic
            // weights) and much faster elsewhere. Once the step norms shrink at
            // a steady ratio rho, that mode is removed by one extrapolation
            // lambda += rho / (1 - rho) * (lambda_k - lambda_{k-1}); the
            // iteration then continues from there, and convergence is still
            // judged on plain steps.
            if (accel && k >= 4 && k - last_x >= 8) {
                const double r1 = rh[2] / rh[1], r2 = rh[1] / rh[0];
                if (rh[0] > 0 && rh[1] > 0 && r1 > 0.05 && r1 < 0.99 && std::fabs(r1 - r2) <= 0.01 * r1) {
                    const int nbx = grid_for(R.n, 256, 1024);
                    hipLaunchKernelGGL(k_extrapolate, dim3(nbx), dim3(256), 0, s, R.n,
                                       w.buf[k & 1].as<double>(), w.buf[(k + 1) & 1].as<double>(),
                                       r1 / (1.0 - r1), w.part.as<double>());
                    NXG_CHECK_LAUNCH();
                    hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(64), 0, s, w.part.as<double>(), nbx,
                                       w.stats.as<double>() + 4 * k);
                    NXG_CHECK_LAUNCH();
                    last_x = k;
                }
            }
        }
    }
    const double* lam = w.buf[k & 1].as<double>();
    if (vm) {
        if (d.d_lambda) permute_rows<double>(lam, vm.o2n, vm.n, 1, d.d_lambda, s);
        if (d.d_gt) permute_rows<double>(lam, vm.o2n, vm.n, 1, d.d_gt, s, 1.0 - d.damping);
    } else {
        if (d.d_lambda)
            hipLaunchKernelGGL(k_scale_copy, dim3(grid_for(R.n)), dim3(256), 0, s, lam, 1.0,
                               d.d_lambda, (int64_t)R.n);
        if (d.d_gt)
            hipLaunchKernelGGL(k_scale_copy, dim3(grid_for(R.n)), dim3(256), 0, s, lam,
                               1.0 - d.damping, d.d_gt, (int64_t)R.n);
    }
    NXG_CHECK_LAUNCH();
    if (d.d_gw && F.n_chunks > 0) {
        hipLaunchKernelGGL(k_edge_grad, dim3(grid_for(F.n_chunks * 64, 256, 16384)), dim3(256), 0, s,
                           F.words.as<uint32_t>(), F.chunk_row.as<int32_t>(),
                           F.tile_chunk.as<int64_t>(), F.n_tiles, F.n_chunks, F.C, F.I, F.L, F.t,
                           F.order == NXG_ORDER_SRC ? F.t : 0, F.order == NXG_ORDER_SRC ? 0 : F.L,
                           F.perm.as<int32_t>(), xs, lam, d.damping, d.d_gw);
        NXG_CHECK_LAUNCH();
    }
    NXG_HIP(hipEventRecord(e1, s));
    std::vector<double> hs(4 * (size_t)(max_iters + 2));
    NXG_HIP(hipMemcpyAsync(hs.data(), w.stats.p, sizeof(double) * hs.size(), hipMemcpyDeviceToHost, s));
    NXG_HIP(hipStreamSynchronize(s));
    int iters = k, conv_at = -1;
    for (int i = 0; i < k; ++i)
        if (tol > 0 && hs[4 * i + 1] <= tol * hs[4 * i + 2]) {
            conv_at = i;
            break;
        }
    if (conv_at >= 0) iters = conv_at + 1;
    float ms = 0.f;
    NXG_HIP(hipEventSynchronize(e1));
    NXG_HIP(hipEventElapsedTime(&ms, e0, e1));
    if (st) {
        memset(st, 0, sizeof(*st));
        st->iterations = iters;
        st->converged = conv_at >= 0;
        st->residual = iters > 0 ? hs[4 * (iters - 1) + 1] / std::max(hs[4 * (iters - 1) + 2], 1e-300) : 0.0;
        st->device_ms = ms;
    }
    return (tol > 0 && conv_at < 0) ? NXG_ENOTCONV : NXG_OK;
}

// Sets *bad when a weight the layout uses (the input index of a word) is not
// finite.
__global__ void k_check_used_weights(const int32_t* __restrict__ perm, int64_t n_words,
                                     const float* __restrict__ win, int32_t* __restrict__ bad) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_words;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t e = perm[i];
        if (e < 0) continue;
        if (!isfinite(win[e])) *bad = 1;
    }
}

void set_weights(nxg_dsss* g, const float* d_w, hipStream_t s) {
    if (g->fwd.host_stream) fail(NXG_EINVAL, "the weights of a HOST_STREAM handle are in host memory");
    for (Layout* L : {&g->fwd, &g->rev}) {
        if (L == &g->rev && !g->has_rev) continue;
        if (!L->has_weight || !L->has_perm)
            fail(NXG_EINVAL, "setting weights needs a build with weights and NXG_BUILD_KEEP_PERM");
    }
    // the new weights are checked before any is stored (finite)
    DevBuf bad;
    bad.alloc(sizeof(int32_t), s);
    fill<int32_t>(bad.as<int32_t>(), 1, 0, s);
    hipLaunchKernelGGL(k_check_used_weights, dim3(grid_for(g->fwd.n_words)), dim3(256), 0, s,
                       g->fwd.perm.as<int32_t>(), g->fwd.n_words, d_w, bad.as<int32_t>());
    NXG_CHECK_LAUNCH();
    int32_t hb = 0;
    NXG_HIP(hipMemcpyAsync(&hb, bad.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    NXG_HIP(hipStreamSynchronize(s));
    if (hb) fail(NXG_EINVAL, "edge weights must be finite");
    for (Layout* L : {&g->fwd, &g->rev}) {
        if (L == &g->rev && !g->has_rev) continue;
        hipLaunchKernelGGL(k_set_weights, dim3(grid_for(L->n_words)), dim3(256), 0, s,
                           L->perm.as<int32_t>(), L->n_words, d_w, L->weight.as<float>());
        NXG_CHECK_LAUNCH();
    }
}

}  // namespace

nxg_status pagerank_adjoint(nxg_dsss* g, const nxg_adjoint_desc& d, hipStream_t s, nxg_run_stats* st) {
    return run_adjoint(g, d, s, st);
}

nxg_status multi_run(nxg_multi* mg, const nxg_run_desc& d, void* const* d_values, hipStream_t s,
                     nxg_run_stats* st) {
    return run_multi(mg, d, d_values, s, st);
}

void dsss_set_weights(nxg_dsss* g, const float* d_w, hipStream_t s) { set_weights(g, d_w, s); }

int lds_budget_bytes(int device) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, device) != hipSuccess ||
        v <= 0)
        v = 65536;
    // headroom for the kernels' static shared variables
    return v - 1024;
}

// Sets *bad when a value is not finite (NaN or infinite).
template <typename V>
__global__ void k_check_finite(const V* __restrict__ x, int64_t n, int32_t* __restrict__ bad) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        if (!isfinite(x[i])) *bad = 1;
}

// A dense teleport vector (caller ids) must be finite (NXG_EINVAL); negative
// entries are accepted, as the iteration is linear in t. Synchronises the
// stream.
void check_teleport(nxg_dsss* g, const nxg_run_desc& d, hipStream_t s) {
    const VMap vm = vmap_of(g);
    const int64_t n = vm ? vm.n : g->fwd.n;
    DevBuf bad;
    bad.alloc(sizeof(int32_t), s);
    fill<int32_t>(bad.as<int32_t>(), 1, 0, s);
    if (d.dtype == NXG_F32)
        hipLaunchKernelGGL(k_check_finite<float>, dim3(grid_for(n)), dim3(256), 0, s,
                           (const float*)d.d_teleport, n, bad.as<int32_t>());
    else if (d.dtype == NXG_F64)
        hipLaunchKernelGGL(k_check_finite<double>, dim3(grid_for(n)), dim3(256), 0, s,
                           (const double*)d.d_teleport, n, bad.as<int32_t>());
    else
        return;  // the dtype is refused by the run itself
    NXG_CHECK_LAUNCH();
    int32_t hb = 0;
    NXG_HIP(hipMemcpyAsync(&hb, bad.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    NXG_HIP(hipStreamSynchronize(s));
    if (hb) fail(NXG_EINVAL, "teleport values must be finite");
}

nxg_status run_program(nxg_dsss* g, const nxg_run_desc& d, hipStream_t s, nxg_run_stats* st) {
    if (d.max_iters < 0) fail(NXG_EINVAL, "max_iters must be >= 0");
    if (!d.d_values) fail(NXG_EINVAL, "d_values is NULL");
    if (d.d_stats && ((d.program != NXG_PAGERANK && d.program != NXG_PAGERANK_WEIGHTED) || d.batch > 1 ||
                      d.d_seeds || (d.flags & NXG_RUN_SCATTER)))
        fail(NXG_EUNSUPPORTED, "d_stats is written by single-column PageRank runs only");
    if (g->fwd.host_stream &&
        ((d.program != NXG_PAGERANK && d.program != NXG_PAGERANK_WEIGHTED) || d.batch > 1 || d.d_seeds ||
         (d.flags & NXG_RUN_SCATTER)))
        fail(NXG_EINVAL, "a HOST_STREAM handle runs single-column PageRank only");
    if (g->fwd.pairs && (d.program != NXG_PAGERANK || d.batch > 1 || d.d_seeds || (d.flags & NXG_RUN_SCATTER)))
        fail(NXG_EINVAL, "a PAIRS handle runs plain single-column PageRank only");
    if ((d.flags & NXG_RUN_SCATTER) || (g->flags & NXG_BUILD_SCATTER)) {
        if (!(d.flags & NXG_RUN_SCATTER)) fail(NXG_EINVAL, "a NXG_BUILD_SCATTER layout runs only NXG_RUN_SCATTER PageRank");
        if (d.batch > 1 || d.d_seeds) fail(NXG_EUNSUPPORTED, "NXG_RUN_SCATTER runs one column");
        if (d.program != NXG_PAGERANK && d.program != NXG_PAGERANK_WEIGHTED)
            fail(NXG_EUNSUPPORTED, "NXG_RUN_SCATTER runs PageRank");
        if (!(d.damping >= 0.0 && d.damping < 1.0)) fail(NXG_EINVAL, "damping outside [0, 1)");
        if (d.d_teleport) check_teleport(g, d, s);
        if (d.dtype == NXG_F32) return run_scatter<float>(g, d, s, st);
        if (d.dtype == NXG_F64) return run_scatter<double>(g, d, s, st);
        fail(NXG_EINVAL, "PageRank needs dtype F32 or F64");
    }
    if ((d.flags & NXG_RUN_MPU) &&
        ((d.program != NXG_PAGERANK && d.program != NXG_PAGERANK_WEIGHTED) || d.batch > 1 || d.d_seeds))
        fail(NXG_EUNSUPPORTED, "NXG_RUN_MPU runs single-column PageRank");
    if (d.program == NXG_BFS && d.batch > 1 && !d.d_seeds) return run_msbfs(g, d, s, st);
    if (d.batch > 1 || d.d_seeds) {
        if (!(d.damping >= 0.0 && d.damping < 1.0)) fail(NXG_EINVAL, "damping outside [0, 1)");
        return run_batched(g, d, s, st);
    }
    if (d.batch != 1 && d.batch != 0) fail(NXG_EINVAL, "batch must be >= 1");
    switch (d.program) {
        case NXG_PAGERANK:
        case NXG_PAGERANK_WEIGHTED:
            if (!(d.damping >= 0.0 && d.damping < 1.0)) fail(NXG_EINVAL, "damping outside [0, 1)");
            if (d.d_teleport) check_teleport(g, d, s);
            if (d.flags & NXG_RUN_MPU) {
                if (d.dtype == NXG_F32) return run_pagerank_mpu<float>(g, d, s, st);
                if (d.dtype == NXG_F64) return run_pagerank_mpu<double>(g, d, s, st);
                fail(NXG_EINVAL, "PageRank needs dtype F32 or F64");
            }
            if (d.dtype == NXG_F32) return run_pagerank<float>(g, d, s, st);
            if (d.dtype == NXG_F64) return run_pagerank<double>(g, d, s, st);
            fail(NXG_EINVAL, "PageRank needs dtype F32 or F64");
        case NXG_BFS:
        case NXG_WCC:
            if (d.dtype != NXG_I32) fail(NXG_EINVAL, "BFS/WCC need dtype I32");
            return run_minprog(g, d, s, st);
        case NXG_SCC:
            return run_scc(g, d, s, st);
        default:
            fail(NXG_EINVAL, "unknown program");
    }
}

nxg_status run_pagerank_in(nxg_dsss* g, const nxg_run_desc& d, hipStream_t s, nxg_run_stats* st,
                           void* region, size_t cap, hipEvent_t e0, hipEvent_t e1) {
    if (d.max_iters < 0) fail(NXG_EINVAL, "max_iters must be >= 0");
    if (!d.d_values) fail(NXG_EINVAL, "d_values is NULL");
    if (d.program != NXG_PAGERANK && d.program != NXG_PAGERANK_WEIGHTED)
        fail(NXG_EUNSUPPORTED, "only PageRank runs without allocating");
    if (d.batch > 1 || d.d_seeds) fail(NXG_EUNSUPPORTED, "batched runs allocate; run them through nxg_run");
    if (d.batch != 1 && d.batch != 0) fail(NXG_EINVAL, "batch must be >= 1");
    if (d.flags & ~(uint32_t)NXG_RUN_WARM_START)
        fail(NXG_EINVAL, "only NXG_RUN_WARM_START is accepted without allocating");
    if ((g->flags & NXG_BUILD_SCATTER) || g->fwd.host_stream)
        fail(NXG_EINVAL, "SCATTER and HOST_STREAM handles cannot run without allocating");
    if (g->fwd.pairs && d.program != NXG_PAGERANK) fail(NXG_EINVAL, "a PAIRS handle runs plain PageRank only");
    if (!(d.damping >= 0.0 && d.damping < 1.0)) fail(NXG_EINVAL, "damping outside [0, 1)");
    Arena a;
    a.base = static_cast<unsigned char*>(region);
    a.cap = cap;
    a.e0 = e0;
    a.e1 = e1;
    if (d.dtype == NXG_F32) return run_pagerank<float>(g, d, s, st, &a);
    if (d.dtype == NXG_F64) return run_pagerank<double>(g, d, s, st, &a);
    fail(NXG_EINVAL, "PageRank needs dtype F32 or F64");
}

void prepare_pagerank_plan(nxg_dsss* g, hipStream_t s) {
    const Layout& L = g->fwd;
    if (L.host_stream || (g->flags & NXG_BUILD_SCATTER)) return;
    if (((size_t)L.T + kSpill) * sizeof(double) > (size_t)lds_budget_bytes(g->device)) return;
    int piece = env_int("NXG_PIECE_CHUNKS", 0);
    if (piece <= 0) piece = default_piece(L.n_chunks, L.C, (size_t)L.T * sizeof(double), num_cus(g->device));
    (void)get_plan(g, L, piece, false, s);
}

}  // namespace nxg
