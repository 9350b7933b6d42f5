// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <new>
#include <string>
#include <vector>

#include "nxgraph.h"

namespace nxg {

// ---------------------------------------------------------------------------
// Error plumbing: every entry point catches nxg::Error and turns it into a
// status plus a thread-local message.
// ---------------------------------------------------------------------------
struct Error {
    nxg_status status;
    std::string msg;
};

[[noreturn]] void fail(nxg_status s, const std::string& msg);
void set_last_error(const std::string& msg);

#define NXG_HIP(call)                                                              \
    do {                                                                           \
        hipError_t e_ = (call);                                                    \
        if (e_ != hipSuccess)                                                      \
            ::nxg::fail(NXG_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

#define NXG_CHECK_LAUNCH() NXG_HIP(hipGetLastError())

// Runs an entry point's body and turns what it throws into a status.
template <class F>
nxg_status guarded(F&& f) {
    try {
        set_last_error(std::string());
        return f();
    } catch (const Error& e) {
        set_last_error(e.msg);
        return e.status;
    } catch (const std::bad_alloc&) {
        set_last_error("host allocation failed");
        return NXG_ENOMEM;
    } catch (...) {
        set_last_error("unexpected internal error");
        return NXG_EDEVICE;
    }
}

// ---------------------------------------------------------------------------
// Device memory through the caller-settable allocator.
// ---------------------------------------------------------------------------
void* dev_alloc(size_t bytes, hipStream_t s);
void dev_free(void* p, size_t bytes, hipStream_t s);

// RAII owner of one device buffer.
struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    hipStream_t stream = nullptr;
    bool owned = true;  // false: a view of memory someone else owns (never freed here)
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    DevBuf(DevBuf&& o) noexcept { *this = std::move(o); }
    DevBuf& operator=(DevBuf&& o) noexcept {
        if (this != &o) {
            reset();
            p = o.p;
            bytes = o.bytes;
            stream = o.stream;
            owned = o.owned;
            o.p = nullptr;
            o.bytes = 0;
            o.owned = true;
        }
        return *this;
    }
    ~DevBuf() { reset(); }
    void alloc(size_t b, hipStream_t s) {
        reset();
        stream = s;
        bytes = b ? b : 16;
        p = dev_alloc(bytes, s);
    }
    // a view of `b` bytes at q (memory owned elsewhere)
    void borrow(void* q, size_t b) {
        reset();
        p = q;
        bytes = b;
        owned = false;
    }
    void reset() {
        if (p && owned) dev_free(p, bytes, stream);
        p = nullptr;
        bytes = 0;
        owned = true;
    }
    template <class T>
    T* as() const {
        return reinterpret_cast<T*>(p);
    }
};

// ---------------------------------------------------------------------------
// Physical DSSS layout.
//
// Destinations are cut into tiles of T vertices (T a power of two; tile tau
// owns [tau*T, (tau+1)*T)), independent of the interval size I: a tile's
// accumulators must fit in LDS, while I sets the source window each group
// gathers from. The edge stream lists tiles in increasing tau; inside a tile,
// the edges of source interval i come before those of interval i+1, and inside
// one (tile, i) group edges are sorted by destination, then source -- the
// paper's sub-shard order restricted to the tile. With T == I the stream is
// exactly the DSSS order. (order == NXG_ORDER_SRC sorts each group by source,
// then destination instead: the source-sorted ablation.)
//
// Each edge is one 32-bit word, bit 31 clear (needs L + t <= 31): in DSSS
// order bits [0, L) = src - i*I and bits [L, L+t) = dst - tile base; in the
// source-major order the two fields swap places. Each non-empty group is
// preceded by a marker word 0x80000000 | i. A tile's words are padded with
// 0xFFFFFFFF to a multiple of the chunk size C, so every chunk belongs to one
// tile; chunk_row[c] is the source interval in effect at the chunk's first
// word and chunk_tile[c] the chunk's tile.
// ---------------------------------------------------------------------------
// Pinned host memory (hipHostMalloc), freed with the owner.
struct HostBuf {
    void* p = nullptr;
    size_t bytes = 0;
    HostBuf() = default;
    HostBuf(const HostBuf&) = delete;
    HostBuf& operator=(const HostBuf&) = delete;
    ~HostBuf() { reset(); }
    void alloc(size_t b) {
        reset();
        bytes = b ? b : 16;
        if (hipHostMalloc(&p, bytes, hipHostMallocDefault) != hipSuccess) {
            p = nullptr;
            bytes = 0;
            fail(NXG_ENOMEM, "pinned host allocation failed");
        }
    }
    void reset() {
        if (p) (void)hipHostFree(p);
        p = nullptr;
        bytes = 0;
    }
    template <typename T>
    T* as() const {
        return static_cast<T*>(p);
    }
};

struct Layout {
    int32_t n = 0, I = 0, P = 0, L = 0;
    int32_t T = 0, t = 0, n_tiles = 0, C = 0, order = 0;
    int64_t m = 0, n_chunks = 0, n_words = 0, max_tile_edges = 0;
    DevBuf words;          // uint32 [n_words]
    DevBuf chunk_row;      // int32  [n_chunks]
    DevBuf chunk_tile;     // int32  [n_chunks]
    DevBuf chunk_src;      // int32  [n_chunks] pair layout: header source in effect at the
                           // chunk's first word
    DevBuf tile_chunk;     // int64  [n_tiles + 1] chunk index of each tile's first chunk
    DevBuf group_edge;     // int64  [n_tiles*P + 1] stream-order index of each group's first edge
    DevBuf group_word;     // int64  [n_tiles*P + 1] word position of each group's marker
    DevBuf perm;           // int32  [n_words] input index of the edge in that word, -1 otherwise
    DevBuf weight;         // float  [n_words] weight of the edge in that word, 0 otherwise
    DevBuf outdeg;         // int32  [n] out-degree in this (possibly reversed) graph
    DevBuf chunk_rng;      // int4   [n_chunks] {min src, max src, min dst, max dst} of the
                           // chunk's edges, made by the first BFS/WCC run
    std::vector<int64_t> h_tile_chunk;  // host copy of tile_chunk
    std::vector<int64_t> h_tile_edges;  // edges per tile (host)
    bool has_perm = false, has_weight = false;
    // NXG_BUILD_PAIRS (source order): besides plain edge words, a header word
    // 0x40000000 | s names a source field, and each later pair word
    // 0x20000000 | d | d' << 14 holds two destination fields of that source
    // (the edges of one source into one tile, two at a time)
    bool pairs = false;
    // NXG_BUILD_HOST_STREAM: words (and weights) live in pinned host memory
    bool host_stream = false;
    HostBuf h_words, h_weight;
};

// Item of work for the iteration kernels: one piece of one destination tile.
struct Item {
    int32_t tile;
    int32_t piece;
    int32_t npieces;
    int32_t slot;   // first partial-buffer slot of the tile (multi-piece tiles), else -1
    int64_t c0, c1; // chunk range [c0, c1)
};

// Something a handle keeps between runs (captured hipGraphs with their workspace).
struct Cached {
    virtual ~Cached() {}
};

// A vertex segment [v0, v0 + vlen) of a split tile, finished by one
// workgroup: it sums the tile's npieces hub slots (from `slot`) over the
// segment, applies the update and stores its scalars in scalar slot sslot.
struct FinSeg {
    int32_t tile, npieces, slot, v0, vlen, sslot;
};

struct Layout;
struct Plan {
    const Layout* layout = nullptr;
    bool whole_tiles = false;
    bool tile_order = false;  // items in stream order (host-streamed runs), not heaviest first
    int32_t piece_chunks = 0;
    std::vector<Item> h_items;
    DevBuf items;
    int32_t n_slots = 0;  // partial-buffer slots (one tile-sized array each)
    std::vector<Item> h_fin;  // piece 0 of every split tile (the finishing launch)
    DevBuf fin;
    std::vector<FinSeg> h_fseg;  // the split tiles cut into vertex segments
    DevBuf fseg;
};

}  // namespace nxg

struct nxg_dsss {
    int device = 0;
    int32_t value_bytes = 4;
    uint32_t flags = 0;
    nxg::Layout fwd;
    nxg::Layout rev;  // reversed graph (NXG_BUILD_TRANSPOSE)
    bool has_rev = false;
    // NXG_BUILD_RELABEL: both layouts use internal ids; new2old[k] is the caller
    // id of internal vertex k, old2new the inverse
    bool relabeled = false;
    nxg::DevBuf new2old, old2new;  // old2new[v] = -1 for a dropped id (NXG_BUILD_DEGREE)
    int32_t n_caller = 0;          // the caller's id range; fwd.n = kept vertices
    // cached iteration plans, keyed by piece size
    std::vector<nxg::Plan*> plans;
    // captured runs (hipGraph + workspace), see NXG_RUN_CAPTURE, recorded on a
    // private stream (the legacy default stream cannot be captured)
    std::vector<nxg::Cached*> cached;
    hipStream_t capture_stream = nullptr;
    ~nxg_dsss();
};

struct nxg_multi {
    std::vector<nxg_dsss*> graphs;
    nxg::Cached* run_cache = nullptr;  // workspaces of the last run (released first)
    ~nxg_multi() {
        delete run_cache;
        for (nxg_dsss* g : graphs) delete g;
    }
};

namespace nxg {
// builder entry (builder.hip)
// spread: with no tile given, keep at least one tile per compute unit (a graph
// that runs alone); false for the graphs of a multi-graph handle
void build_layout(const nxg_build_desc& d, bool reversed, hipStream_t s, Layout& out, bool spread = true);
void export_layout(const Layout& L, int64_t* d_offsets, int32_t* d_src, int32_t* d_dst,
                   int32_t* d_perm, hipStream_t s);
// validates the ids, orders the vertices by decreasing degree and renames the edges
// numbers the vertices internally (by decreasing out-degree when by_degree;
// without the ids that appear in no edge when drop) and renames the edges;
// returns the number of internal vertices
int32_t relabel_input(const nxg_build_desc& d, hipStream_t s, bool by_degree, bool drop,
                      DevBuf& new2old, DevBuf& old2new, DevBuf& src2, DevBuf& dst2);
// validated build of a whole handle, with the optional relabeling and transpose
// (capi.hip)
nxg_dsss* build_handle(const nxg_build_desc& d, hipStream_t s, bool spread = true);
// runtime entry (iterate.hip)
nxg_status run_program(nxg_dsss* g, const nxg_run_desc& d, hipStream_t s, nxg_run_stats* st);
// PageRank with its whole workspace carved out of the device region [region,
// region + cap) and the given timing events: allocates nothing (iterate.hip)
nxg_status run_pagerank_in(nxg_dsss* g, const nxg_run_desc& d, hipStream_t s, nxg_run_stats* st,
                           void* region, size_t cap, hipEvent_t e0, hipEvent_t e1);
// the iteration plan PageRank runs use by default, made at build time so that a
// run without allocation finds it (iterate.hip)
void prepare_pagerank_plan(nxg_dsss* g, hipStream_t s);
nxg_status pagerank_adjoint(nxg_dsss* g, const nxg_adjoint_desc& d, hipStream_t s, nxg_run_stats* st);
void dsss_set_weights(nxg_dsss* g, const float* d_w, hipStream_t s);
nxg_status tune(const nxg_build_desc& desc, int program, int dtype, int batch, hipStream_t s,
                nxg_tune_result* out);
nxg_status multi_run(nxg_multi* mg, const nxg_run_desc& d, void* const* d_values, hipStream_t s,
                     nxg_run_stats* st);
int lds_budget_bytes(int device);
// Chunks per work item when a run does not choose (see iterate.hip).
int default_piece(int64_t chunks, int C, size_t slot_bytes, int cus);
nxg_status copy_probe(int64_t bytes, int reps, hipStream_t s, double* gbps);
nxg_status read_probe(int64_t bytes, int reps, hipStream_t s, double* gbps);
}  // namespace nxg
