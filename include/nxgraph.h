/*
 * nxgraph.h -- C ABI of the MI355X (gfx950) DSSS graph-iteration library.
 *
 * The library stores a directed graph as Destination-Sorted Sub-Shards
 * (DSSS; Chi et al., "NXgraph", Sec. II-A and Sec. III-A): the vertex ids
 * [0, n) are cut into P equal intervals of size I (the last may be shorter);
 * sub-shard SS_{i.j} holds the edges whose source lies in interval i and whose
 * destination lies in interval j; inside a sub-shard edges are sorted by
 * destination, then by source. One iteration (Alg. 1, Alg. 5) streams every
 * sub-shard, gathers the source interval's values, reduces them by destination
 * into the destination interval and applies the vertex update of the chosen
 * program (PageRank, BFS, WCC).
 *
 * Conventions for every entry point:
 *  - Pointers named d_* are device pointers on the current HIP device; all
 *    others are host pointers. Sizes are element counts unless named *_bytes.
 *  - Vertex ids are 0-based int32 (the paper numbers vertices from 1).
 *  - Calls are asynchronous on the given stream unless they say they
 *    synchronise. Input buffers are borrowed for the duration of the call
 *    only; nothing is retained.
 *  - Every call returns an nxg_status. On failure a message is available
 *    from nxg_last_error() (thread-local) and no output handle is created.
 *    No C++ exception crosses this boundary.
 */
#ifndef NXGRAPH_H
#define NXGRAPH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define NXG_ABI_VERSION 9

typedef enum nxg_status {
    NXG_OK = 0,
    NXG_EINVAL = 1,       /* invalid argument: null pointer, size, id out of range, flags */
    NXG_ENOMEM = 2,       /* a device allocation failed; nothing was leaked */
    NXG_EDEVICE = 3,      /* the HIP runtime reported an error */
    NXG_ENOTCONV = 4,     /* tolerance not reached within max_iters; results are written */
    NXG_EUNSUPPORTED = 5  /* a valid request that this library does not implement */
} nxg_status;

typedef struct nxg_dsss nxg_dsss; /* opaque graph handle */

/* ------------------------------------------------------------------------- */
/* Library state                                                              */
/* ------------------------------------------------------------------------- */

/* Device allocator used for every buffer the library owns. alloc returns a
 * device pointer of at least `bytes` bytes (NULL = failure, reported as
 * NXG_ENOMEM) usable on `stream`; free releases it. Passing NULL for both
 * restores the default (hipMalloc / hipFree). Process-wide; set it before
 * creating handles and keep it until they are destroyed. */
typedef void* (*nxg_alloc_fn)(size_t bytes, void* stream, void* ctx);
typedef void (*nxg_free_fn)(void* ptr, size_t bytes, void* stream, void* ctx);
nxg_status nxg_set_allocator(nxg_alloc_fn alloc_fn, nxg_free_fn free_fn, void* ctx);

/* Message describing the last failure on the calling thread ("" if none). */
const char* nxg_last_error(void);

/* NXG_ABI_VERSION of the loaded library. */
int nxg_abi_version(void);

/* Attainable HBM bandwidth: times reps copies of a `bytes`-byte buffer (16-byte
 * non-temporal loads, plain stores) and returns read+written GB/s. The same
 * kernel, run under the FETCH_SIZE / WRITE_SIZE counters, calibrates them.
 * Synchronises the stream. */
nxg_status nxg_copy_probe(int64_t bytes, int32_t reps, void* stream, double* gbps);

/* Attainable read bandwidth: times reps passes of four-deep 16-byte
 * non-temporal loads over a `bytes`-byte buffer (nothing written back) and
 * returns read GB/s, the ceiling of an iteration that mostly reads.
 * NXG_EINVAL if bytes < 4096 or reps < 1. Synchronises the stream. */
nxg_status nxg_read_probe(int64_t bytes, int32_t reps, void* stream, double* gbps);

/* ------------------------------------------------------------------------- */
/* DSSS construction (Sec. III-A: intervals and sub-shards from an edge list)  */
/* ------------------------------------------------------------------------- */

#define NXG_BUILD_KEEP_PERM 0x1u  /* keep the map from stored edge to input edge index */
#define NXG_BUILD_TRANSPOSE 0x2u  /* also store the reversed graph (source-sorted view) */
#define NXG_BUILD_SYMMETRIZE 0x4u /* store E and reverse(E); implies NXG_BUILD_DEDUP */
#define NXG_BUILD_DEDUP 0x8u      /* store each distinct (src, dst) pair once */
#define NXG_BUILD_RELABEL 0x10u   /* number the vertices internally by decreasing
                                     out-degree (ties by id), so the most gathered
                                     source values are adjacent in memory; every
                                     run still takes and returns vertex data in
                                     the caller's ids (WCC labels stay the minimum
                                     caller id of the component) */
#define NXG_BUILD_SCATTER 0x20u   /* the coarse-grained, source-sorted layout the
                                     paper compares DSSS against (Sec. IV-B1,
                                     Table IV): one destination tile spanning all
                                     vertices and NXG_ORDER_SRC, so the stream is
                                     the whole edge list in (source, destination)
                                     order; I is capped at 2^(31 - ceil(log2 n))
                                     so both fields fit one word. Only
                                     NXG_RUN_SCATTER PageRank runs use it (the
                                     tile has no LDS bound); not combinable with
                                     NXG_BUILD_RELABEL, NXG_BUILD_TRANSPOSE or
                                     NXG_BUILD_DEGREE */
#define NXG_BUILD_DEGREE 0x40u    /* degreeing (Sec. III-A preprocessing): ids that
                                     appear in no edge are dropped and the others
                                     numbered densely in increasing id order (by
                                     decreasing out-degree with NXG_BUILD_RELABEL).
                                     The graph then has n_kept vertices: PageRank's
                                     uniform teleport and dangling share are
                                     1/n_kept, and a teleport vector counts only on
                                     kept ids. Runs still take and return vectors
                                     over the caller's n ids; dropped ids read as 0
                                     (PageRank, adjoint), INT32_MAX (BFS; a dropped
                                     root reaches only itself) and their own id
                                     (WCC). Batched seeds must be kept ids. Not for
                                     nxg_multi_build. */
#define NXG_BUILD_HOST_STREAM 0x80u /* the SPU schedule with the sub-shards on a
                                     slower tier (Sec. III-B1, Alg. 5): after the
                                     build the edge stream (and weights) moves to
                                     pinned host memory, and every iteration streams
                                     it through two device staging buffers, copies
                                     overlapped with the edge work, while the vertex
                                     data stays in device memory. Such a handle runs
                                     PageRank only (plain or weighted, F32 or F64,
                                     batch 1, no capture); the staging size is set by
                                     the environment variable NXG_STREAM_MB (default
                                     256 per buffer). Not combinable with
                                     NXG_BUILD_TRANSPOSE or NXG_BUILD_SCATTER, nor for
                                     nxg_multi_build; nxg_dsss_export and
                                     nxg_dsss_set_weights refuse such a handle. */

#define NXG_BUILD_SHUFFLE_SCHEDULE 0x200u /* debug: the work items of every run (tile
                                     pieces) and the finishing segments of split tiles
                                     are issued in a seeded random order instead of
                                     heaviest first. Results do not depend on the
                                     order (BFS/WCC bit-identical, PageRank equal up to
                                     the rounding of sums taken in another order):
                                     the sub-shards of one destination interval can be
                                     processed in any order (Sec. II-A) */
#define NXG_BUILD_PAIRS 0x100u    /* source-order sub-shards (NXG_ORDER_SRC) with the
                                     edges of one source into one destination tile
                                     packed two to a word: a header word names the
                                     source, then each pair word holds two
                                     destinations (one gather serves both); an
                                     unpaired edge keeps its plain word. Fewer words
                                     to stream than one per edge when sources have
                                     several edges per tile. Needs T <= 16384 and
                                     ceil(log2 I) + log2 T <= 29. Plain PageRank
                                     only (F32 or F64, batch 1, no weights, no
                                     NXG_RUN_SCATTER); BFS, WCC, batched and
                                     weighted runs, the adjoint and nxg_dsss_export
                                     refuse such a handle. Not combinable with
                                     NXG_BUILD_KEEP_PERM, NXG_BUILD_TRANSPOSE,
                                     NXG_BUILD_SYMMETRIZE, NXG_BUILD_SCATTER or
                                     NXG_BUILD_HOST_STREAM, nor with weights, nor
                                     for nxg_multi_build. */

/* Order of the edges inside one sub-shard. */
#define NXG_ORDER_DST 0 /* destination, then source: the DSSS order of Sec. III-A */
#define NXG_ORDER_SRC 1 /* source, then destination: the source-sorted sub-shard
                           the paper compares against (Sec. IV-B1); on this GPU it
                           lets the lanes of one gather read adjacent sources */

typedef struct nxg_build_desc {
    int32_t n;              /* vertices, in [1, 2^29) (NXG_EUNSUPPORTED above) */
    int64_t m;              /* input edges, >= 0 (< 2^31, and < 2^30 with SYMMETRIZE) */
    const int32_t* d_src;   /* [m] source ids in [0, n) */
    const int32_t* d_dst;   /* [m] destination ids in [0, n) */
    const float* d_weight;  /* [m] edge weights, or NULL (unweighted); each finite, else NXG_EINVAL
                               (checked on the device before the build; negative weights are
                               accepted: the iteration is linear in them) */
    int32_t interval;       /* I, interval size; P = ceil(n / I). 0 = planner's choice */
    int32_t tile;           /* destination tile size T, a power of two (tiles are the
                               vertex ranges [k*T, (k+1)*T), any T relative to I);
                               0 = planner's choice: the largest whose accumulators
                               fit in LDS, halved (not below 256) until there are at
                               least as many tiles as compute units (nxg_multi_build
                               keeps the largest: its graphs share launches) */
    int32_t chunk;          /* edge-stream words per work chunk, power of two in
                               [256, 65536]; 0 = planner's choice */
    int32_t value_bytes;    /* bytes of one destination accumulator the tile must hold
                               in LDS: 8 for PageRank (FP64 sums for FP32 and FP64
                               values), 4 for BFS/WCC (int32); 0 = 8 */
    uint32_t flags;         /* NXG_BUILD_* */
    int32_t order;          /* NXG_ORDER_DST (default) or NXG_ORDER_SRC */
} nxg_build_desc;

/* Builds the DSSS of the graph on `stream` and synchronises it once (to read
 * the device error word and the sizes). Ids outside [0, n) give NXG_EINVAL.
 * Weights require NXG_BUILD_KEEP_PERM semantics internally and are stored in
 * DSSS order; they may not be combined with NXG_BUILD_SYMMETRIZE. On success
 * *out owns every buffer; on failure *out is NULL. */
nxg_status nxg_dsss_build(const nxg_build_desc* desc, void* stream, nxg_dsss** out);

/* Releases every buffer of the handle. NULL is accepted. */
nxg_status nxg_dsss_destroy(nxg_dsss* g);

typedef struct nxg_dsss_info {
    int32_t n;           /* vertices */
    int64_t m;           /* stored edges (after DEDUP / SYMMETRIZE) */
    int32_t interval;    /* I */
    int32_t P;           /* number of intervals */
    int32_t tile;        /* destination tile size T */
    int32_t n_tiles;     /* destination tiles */
    int32_t chunk;       /* words per chunk */
    int64_t n_chunks;    /* chunks in the edge stream */
    int64_t n_words;     /* 32-bit words in the edge stream (edges + markers + padding) */
    int64_t device_bytes;/* bytes held on the device by the handle */
    int64_t max_tile_edges; /* edges of the heaviest destination tile */
    int32_t has_perm, has_weights, has_transpose;
    int32_t order;       /* NXG_ORDER_* */
    int32_t relabeled;   /* built with NXG_BUILD_RELABEL */
    int32_t n_kept;      /* vertices of the stored graph: n, or fewer with NXG_BUILD_DEGREE */
    int32_t pairs;       /* built with NXG_BUILD_PAIRS */
} nxg_dsss_info;

nxg_status nxg_dsss_info_get(const nxg_dsss* g, nxg_dsss_info* info);

/* Copies the stored graph back out, for structure checks. All outputs are
 * device buffers the caller owns; any may be NULL.
 *   d_offsets [P*P + 1]  first edge of SS_{i.j} at index j*P + i, in the order
 *                         of Sec. II-A (shards of increasing j, sub-shards of
 *                         increasing i) -- counts follow the paper's layout;
 *   d_src, d_dst [m]     edges in stream order: destination tile, then source
 *                         interval, then destination, then source (source,
 *                         then destination with NXG_ORDER_SRC). When the tile
 *                         equals the interval this is exactly the DSSS order
 *                         of Sec. II-A/III-A;
 *   d_perm [m]           input index of each stored edge (needs KEEP_PERM).
 * transposed != 0 exports the reversed graph instead (needs TRANSPOSE).
 * Synchronises the stream. */
nxg_status nxg_dsss_export(const nxg_dsss* g, int transposed, int64_t* d_offsets,
                           int32_t* d_src, int32_t* d_dst, int32_t* d_perm, void* stream);

/* Internal vertex numbering of a NXG_BUILD_RELABEL or NXG_BUILD_DEGREE build:
 * d_new2old[k] (device, [n_kept], caller-owned) receives the caller id of
 * internal vertex k. The ids that nxg_dsss_export returns are internal ids.
 * NXG_EINVAL if the handle was built with neither flag. Synchronises the stream. */
nxg_status nxg_dsss_vertex_map(const nxg_dsss* g, int32_t* d_new2old, void* stream);

/* ------------------------------------------------------------------------- */
/* Iterations (Alg. 1 update model, synchronous per Sec. II-B)                */
/* ------------------------------------------------------------------------- */

typedef enum nxg_program {
    NXG_PAGERANK = 0,          /* x' = d (W x + delta/n) + (1-d) t, W = 1/outdeg */
    NXG_PAGERANK_WEIGHTED = 1, /* same with the stored edge weights as W */
    NXG_BFS = 2,               /* Algs. 2-4: levels from a root, INT32_MAX = unreached */
    NXG_WCC = 3,               /* min-label propagation; needs a SYMMETRIZE build */
    NXG_SCC = 4                /* strongly connected components (named among the targeted
                                  queries of Sec. IV-D, no algorithm given there): d_values[v]
                                  = the smallest caller id of v's component. Needs a TRANSPOSE
                                  build (the backward step streams the reversed layout), dtype
                                  I32, batch 1, no run flags. Computed by colouring rounds:
                                  forward min-colour propagation over the unassigned vertices,
                                  then, per colour, backward reachability of the colour's root
                                  inside the colour; max_iters bounds the passes of all rounds
                                  together (NXG_ENOTCONV when they run out, d_values then
                                  unspecified). Stats: iterations = colouring rounds,
                                  changed_rounds = passes that changed a value,
                                  streamed_chunks = chunks streamed over both layouts */
} nxg_program;

typedef enum nxg_dtype { NXG_F32 = 0, NXG_F64 = 1, NXG_I32 = 2 } nxg_dtype;

#define NXG_RUN_WARM_START 0x1u /* d_values holds x^0 on entry (PageRank) */
#define NXG_RUN_PERSISTENT 0x2u /* nxg_multi_run: single persistent launch (switched off) */
#define NXG_RUN_CAPTURE 0x4u    /* PageRank, tol <= 0: record the launches of the run into a
                                   hipGraph kept by the handle (with its workspace) and replay
                                   it when a later run has the same program, dtype, iteration
                                   count, damping, flags, buffers and piece size. Batched
                                   runs too (same batch, seed and output buffers; the seeds
                                   are checked on the host at every call and read by the
                                   graph at every replay) */
#define NXG_RUN_SCATTER 0x8u    /* PageRank (plain or weighted, F32 or F64, batch 1) on a
                                   NXG_BUILD_SCATTER layout, coarse-grained: every edge adds
                                   its source's share to its destination with a device-scope
                                   FP64 atomic in global memory, the GPU form of the paper's
                                   lock-based source-sorted comparison (Sec. IV-B1). Same
                                   results as the DSSS runs up to the order of the additions;
                                   not combinable with NXG_RUN_CAPTURE */
#define NXG_RUN_MPU 0x10        /* single-column PageRank (plain or weighted, F32 or F64) with the
                                   mixed-phase update of Sec. III-B3 (Alg. 7), host memory as the
                                   slower tier: only the first Q source intervals keep their values
                                   in device memory, Q chosen from vertex_budget (each resident
                                   vertex costs two values and an 8-byte accumulator, plus one
                                   staged interval; the resident range is a whole number of
                                   intervals and tiles). The other intervals' values stay in pinned
                                   host memory, are staged one interval at a time while their row of
                                   sub-shards is processed, and sub-shards whose source and
                                   destination are both non-resident pass through shard hubs in
                                   host memory (dense, one tile-sized FP64 array per sub-shard).
                                   Q = P is the SPU, Q = 0 the DPU. Needs a build with natural ids
                                   (no RELABEL or DEGREE), a power-of-two interval, and no PAIRS,
                                   HOST_STREAM or SCATTER; not combinable with NXG_RUN_CAPTURE.
                                   d_values and d_teleport may be pinned host memory. The run
                                   stats report Q and the bytes moved to and from host memory */

typedef struct nxg_run_desc {
    nxg_program program;
    nxg_dtype dtype;        /* F32 or F64 for PageRank, I32 for BFS/WCC/SCC */
    int32_t batch;          /* B in [1, 64] value columns. B > 1 (or d_seeds set) runs batched
                               PageRank, FP32, values [n, B] row-major; the build needs
                               value_bytes >= 8 * B (FP64 sums per column in LDS).
                               NXG_BFS with B in [2, 64] runs B searches at once, one per
                               root (roots[B]): d_values [n, B] int32 levels, row-major; the
                               set of roots reaching a vertex is one 64-bit mask, so the
                               build needs value_bytes >= 8; stats: max_level and
                               changed_rounds over all searches, reached_edges summed */
    double damping;         /* d in [0, 1) */
    int32_t max_iters;      /* upper bound on iterations (>= 0) */
    double tol;             /* PageRank: stop when ||x^{k+1}-x^k||_1 <= tol (per column);
                               <= 0 runs exactly max_iters. BFS/WCC ignore it and stop
                               when a round changes nothing (bounded by max_iters). */
    const void* d_teleport; /* [n, B] row-major, dtype of the run; NULL = uniform 1/n. Each value
                               finite, else NXG_EINVAL: nxg_run checks a dense teleport on the
                               device before the run, which synchronises the stream
                               (nxg_run_noalloc does not check it). Negative entries are
                               accepted: the iteration is linear in t */
    const int32_t* roots;   /* BFS: host [B] root ids (caller ids, each in [0, n)) */
    void* d_values;         /* [n, B] output values (PageRank x, BFS level, WCC/SCC label) */
    uint32_t flags;         /* NXG_RUN_* */
    const int32_t* d_seeds; /* batched personalised PageRank: device [B] seed vertices;
                               column b teleports to seeds[b] (one-hot t). NULL = uniform */
    int32_t piece_chunks;   /* chunks per workgroup piece of a destination tile (0 = planner);
                               larger tiles are split, and a second launch sums the
                               pieces' partials in piece order (two phases) */
    double* d_stats;        /* single-column PageRank only (else NULL): device
                               [4 * max_iters] FP64 written on the stream at the end of
                               the run (also by every replay of a captured one), so
                               statistics need no host synchronisation. Entry 4k+0 is
                               the dangling mass entering iteration k (Alg. 1's
                               scalar), 4k+1 the residual ||x^{k+1} - x^k||_1, 4k+2
                               sum(x^{k+1}), 4k+3 unused (0); iterations after a
                               tolerance stop read 0. NULL = not written */
    int64_t vertex_budget;  /* NXG_RUN_MPU: device bytes for the run's vertex data; 0 = the
                               environment variable NXG_VERTEX_BUDGET_MB */
} nxg_run_desc;

typedef struct nxg_run_stats {
    int32_t iterations;     /* iterations (rounds) run */
    int32_t converged;      /* PageRank: tol reached; BFS/WCC: fixed point reached */
    double residual;        /* last ||x^{k+1}-x^k||_1 (max over columns) */
    int32_t max_level;      /* BFS: largest finite level (Alg. 4) */
    int32_t changed_rounds; /* BFS/WCC: rounds that changed at least one value */
    int64_t reached_edges;  /* BFS: sum of out-degrees of reached vertices */
    double device_ms;       /* time between the first and last launch, HIP events */
    int64_t streamed_chunks;/* BFS/WCC: chunks streamed, summed over the rounds. Sec. II-B
                               activity at the grain of 64-vertex blocks: a chunk is
                               streamed in a round when its source id range holds a block
                               changed in the previous round and, for BFS, its destination
                               id range holds a block with an unreached vertex; 0 for
                               other programs */
    int32_t resident_intervals; /* NXG_RUN_MPU: Q, the source intervals kept in device memory */
    int64_t host_read_bytes;    /* NXG_RUN_MPU: bytes read from host memory (staged intervals,
                                   shard hubs, old values of non-resident vertices) */
    int64_t host_write_bytes;   /* NXG_RUN_MPU: bytes written to host memory (shard hubs, new
                                   values of non-resident vertices) */
} nxg_run_stats;

/* Runs the program on the stored graph. With stats == NULL the call is fully
 * asynchronous (PageRank with tol <= 0 only); otherwise it synchronises the
 * stream and fills *stats. Returns NXG_ENOTCONV when tol > 0 was not reached
 * (values are still written). BFS and WCC runs keep their workspace (and the
 * per-chunk id ranges their activity test reads) in the handle from the first
 * run on, so such runs on one handle must not overlap. */
nxg_status nxg_run(nxg_dsss* g, const nxg_run_desc* desc, void* stream, nxg_run_stats* stats);

/* ------------------------------------------------------------------------- */
/* Runs without device allocation                                             */
/* ------------------------------------------------------------------------- */

/* For callers that cannot allocate device memory during a run (code under
 * stream capture, tight serving loops, harnesses that forbid allocation).
 * Same as nxg_run for single-column PageRank (NXG_PAGERANK or
 * NXG_PAGERANK_WEIGHTED, F32 or F64, batch 1, no seeds; flags 0 or
 * NXG_RUN_WARM_START), but the run's whole workspace -- value vectors, hub
 * partials, per-tile scalars, statistics, and on a relabeled build the
 * vectors in internal ids -- lives in one library-owned device array of
 * nxg_noalloc_scratch_bytes() bytes (64 MiB), and the call makes no device
 * allocation and no allocator callback. The caller still owns d_values and
 * d_teleport. Each device the library runs this on keeps its own array until
 * the process ends; its address on a device is looked up at the first call on
 * that device (which also creates the call's two timing events). Every call on
 * one device shares that device's array and leaves its contents there: calls
 * that overlap on one device race, so callers must serialise them (one stream,
 * or their own ordering). The handle must live on the current device
 * (NXG_EINVAL otherwise) and must have the iteration plan for the run's piece
 * size: nxg_dsss_build prepares the planner's (piece_chunks = 0); another
 * piece size needs one earlier nxg_run with it, else NXG_EINVAL. A run whose
 * workspace exceeds the array (about 2 * n * sizeof(value) plus hub partials,
 * statistics of 32 bytes per iteration and, relabeled, up to 2 more vectors)
 * is refused with NXG_EINVAL before anything is enqueued. SCATTER and
 * HOST_STREAM handles, NXG_RUN_CAPTURE and batched runs are refused.
 * Synchronises the stream at the end, like nxg_run. */
nxg_status nxg_run_noalloc(nxg_dsss* g, const nxg_run_desc* desc, void* stream, nxg_run_stats* stats);

/* Size in bytes of the per-device array nxg_run_noalloc works in. */
size_t nxg_noalloc_scratch_bytes(void);

/* ------------------------------------------------------------------------- */
/* Autotuning                                                                 */
/* ------------------------------------------------------------------------- */

typedef struct nxg_tune_result {
    int32_t interval;      /* best interval size I */
    int32_t tile;          /* best destination tile T */
    int32_t chunk;         /* best chunk size */
    int32_t order;         /* NXG_ORDER_* of the best layout */
    int32_t piece_chunks;  /* best nxg_run_desc.piece_chunks (0 = planner) */
    double ms_per_iter;    /* measured milliseconds per iteration */
    int32_t candidates;    /* candidates timed (0 when served from the cache) */
    int32_t relabel;       /* 1 if the best layout uses NXG_BUILD_RELABEL */
    int32_t pairs;         /* 1 if the best layout uses NXG_BUILD_PAIRS */
    int32_t width;         /* batched runs: columns per pass (build with value_bytes =
                              8 * width and run the batch in ceil(batch / width)
                              passes); 1 for single-column tuning */
} nxg_tune_result;

/* Times captured PageRank iterations (NXG_RUN_CAPTURE) of the graph in desc
 * under candidate layouts (vertex numbering x edge order inside a sub-shard,
 * then source interval x destination tile, then chunk and piece size, then,
 * for plain PageRank in source order, the pair encoding NXG_BUILD_PAIRS) and
 * returns the fastest. The paper picks the interval count from experience
 * (Sec. IV-B2); here it is measured. Results are cached per process and, when the
 * environment variable NXG_TUNE_CACHE names a file, appended to it and read
 * back, keyed by device, n, m, program, dtype, batch, value_bytes and flags.
 * Builds and runs on `stream` and synchronises it; never use under capture.
 * PageRank (plain or weighted), F32 or F64, batch 1; or batched personalised
 * PageRank (plain, F32, batch > 1): then the candidates are the vector width
 * (columns per pass: the batch up to 64, then 32 and 16) with the largest tile
 * its accumulators fit in LDS and half of it, then the source interval, then
 * edge order x vertex numbering, timed as uninterrupted 8-iteration batched
 * runs over ceil(batch / width) passes. */
nxg_status nxg_tune(const nxg_build_desc* desc, nxg_program program, nxg_dtype dtype,
                    int32_t batch, void* stream, nxg_tune_result* result);

/* ------------------------------------------------------------------------- */
/* Many graphs per launch                                                     */
/* ------------------------------------------------------------------------- */

typedef struct nxg_multi nxg_multi; /* opaque set of independent graphs */

/* Builds count independent graphs (descs[i] as for nxg_dsss_build). On failure
 * nothing is kept and *out is NULL. Synchronises the stream. */
nxg_status nxg_multi_build(int32_t count, const nxg_build_desc* descs, void* stream,
                           nxg_multi** out);

/* Runs desc->max_iters synchronous PageRank iterations (FP32 values, uniform
 * teleport, x^0 = 1/n, no tolerance stop) on every graph together: the edge
 * work of an iteration is ONE launch whose workgroups are the tile pieces of all
 * graphs, so small graphs fill the GPU together instead of one after another
 * (then one launch finishes the split tiles of all graphs and one reduces every
 * graph's scalars). d_values is a host array of count device pointers, graph
 * i's result [n_i] FP32. The handle keeps the run's workspaces for the next run
 * with the same iteration count; calls on one handle must not overlap.
 * NXG_RUN_PERSISTENT (one launch for all iterations, workgroups waiting on
 * per-graph iteration counters) returns NXG_EUNSUPPORTED: that variant did not
 * complete on MI355X and is switched off. Synchronises the stream. */
nxg_status nxg_multi_run(nxg_multi* mg, const nxg_run_desc* desc, void* const* d_values,
                         void* stream, nxg_run_stats* stats);

nxg_status nxg_multi_destroy(nxg_multi* mg); /* NULL accepted */

/* ------------------------------------------------------------------------- */
/* Weighted PageRank: new weights and the adjoint (gradient) pass             */
/* ------------------------------------------------------------------------- */

/* Replaces the stored edge weights with d_weight [m] (input edge order, FP32)
 * in the forward and, if present, the reversed graph. Needs a build with
 * weights and NXG_BUILD_KEEP_PERM. The weights the layout uses are checked
 * first (finite, else NXG_EINVAL and the stored weights stay), which
 * synchronises the stream; the update itself is asynchronous. */
nxg_status nxg_dsss_set_weights(nxg_dsss* g, const float* d_weight, void* stream);

typedef struct nxg_adjoint_desc {
    double damping;         /* d of the forward run */
    double tol;             /* stop when ||lambda^{k+1}-lambda^k||_1 <= tol * ||lambda^{k+1}||_1;
                               <= 0 runs exactly max_iters */
    int32_t max_iters;      /* >= 1 */
    const double* d_xstar;  /* [n] converged forward vector x* (FP64) */
    const double* d_gx;     /* [n] dL/dx* (FP64) */
    double* d_lambda;       /* [n] out: adjoint vector, or NULL */
    float* d_gw;            /* [m] out: dL/dw_e in input edge order, or NULL */
    double* d_gt;           /* [n] out: dL/dt = (1 - d) lambda, or NULL */
} nxg_adjoint_desc;

/* Gradient of L(x*) through the weighted-PageRank fixed point
 * x* = d (W^T x* + delta/n) + (1-d) t, with respect to the stored (given)
 * weights and the teleport vector, for dL/dx* = gx (the paper has no such
 * pass; it is the reverse-mode derivative of the forward iteration). The
 * adjoint lambda = gx + d (W lambda + 1_D sum(lambda)/n) is iterated over the
 * reversed graph -- each reduction runs by forward source, over out-edges --
 * then dL/dw_e = d x*[src_e] lambda[dst_e] and dL/dt = (1 - d) lambda. Needs a
 * build with weights, NXG_BUILD_TRANSPOSE and NXG_BUILD_KEEP_PERM and
 * value_bytes 8. Synchronises the stream; fills *stats if non-NULL. Returns
 * NXG_ENOTCONV (outputs still written) when tol was not reached. */
nxg_status nxg_pagerank_adjoint(nxg_dsss* g, const nxg_adjoint_desc* desc, void* stream,
                                nxg_run_stats* stats);

#ifdef __cplusplus
}
#endif

#endif /* NXGRAPH_H */
