// The C ABI (include/nxgraph.h): argument checks, the allocator hook, error
// text, and handle lifetime. Every entry point converts failures into a status.
#include <algorithm>
#include <cstring>
#include <new>

#include "nxg_internal.h"

namespace nxg {
namespace {
thread_local std::string g_last_error;
nxg_alloc_fn g_alloc = nullptr;
nxg_free_fn g_free = nullptr;
void* g_ctx = nullptr;
}  // namespace

void fail(nxg_status s, const std::string& msg) { throw Error{s, msg}; }
void set_last_error(const std::string& msg) { g_last_error = msg; }

void* dev_alloc(size_t bytes, hipStream_t s) {
    void* p = nullptr;
    if (g_alloc) {
        p = g_alloc(bytes, (void*)s, g_ctx);
    } else if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        p = nullptr;
    }
    if (!p) fail(NXG_ENOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed");
    return p;
}

void dev_free(void* p, size_t bytes, hipStream_t s) {
    if (!p) return;
    if (g_free)
        g_free(p, bytes, (void*)s, g_ctx);
    else
        (void)hipFree(p);
}

}  // namespace nxg

nxg_dsss::~nxg_dsss() {
    for (nxg::Cached* c : cached) delete c;
    for (nxg::Plan* p : plans) delete p;
    if (capture_stream) (void)hipStreamDestroy(capture_stream);
}

using namespace nxg;

extern "C" {

nxg_status nxg_set_allocator(nxg_alloc_fn alloc_fn, nxg_free_fn free_fn, void* ctx) {
    return guarded([&]() {
        if ((alloc_fn == nullptr) != (free_fn == nullptr))
            fail(NXG_EINVAL, "alloc_fn and free_fn must both be set or both be NULL");
        g_alloc = alloc_fn;
        g_free = free_fn;
        g_ctx = ctx;
        return NXG_OK;
    });
}

const char* nxg_last_error(void) { return g_last_error.c_str(); }

int nxg_abi_version(void) { return NXG_ABI_VERSION; }


nxg_status nxg_dsss_build(const nxg_build_desc* desc, void* stream, nxg_dsss** out) {
    return guarded([&]() {
        if (!out) fail(NXG_EINVAL, "out is NULL");
        *out = nullptr;
        if (!desc) fail(NXG_EINVAL, "desc is NULL");
        *out = build_handle(*desc, (hipStream_t)stream);
        return NXG_OK;
    });
}

nxg_status nxg_multi_build(int32_t count, const nxg_build_desc* descs, void* stream, nxg_multi** out) {
    return guarded([&]() {
        if (!out) fail(NXG_EINVAL, "out is NULL");
        *out = nullptr;
        if (count < 1 || !descs) fail(NXG_EINVAL, "count must be >= 1 and descs non-NULL");
        for (int32_t i = 0; i < count; ++i)
            if (descs[i].flags & (NXG_BUILD_DEGREE | NXG_BUILD_SCATTER | NXG_BUILD_HOST_STREAM |
                                  NXG_BUILD_PAIRS))
                fail(NXG_EUNSUPPORTED, "nxg_multi_build takes none of NXG_BUILD_DEGREE, NXG_BUILD_SCATTER, "
                                       "NXG_BUILD_HOST_STREAM, NXG_BUILD_PAIRS");
        nxg_multi* mg = new nxg_multi();
        try {
            for (int32_t i = 0; i < count; ++i)
                mg->graphs.push_back(build_handle(descs[i], (hipStream_t)stream, false));
        } catch (...) {
            delete mg;
            throw;
        }
        *out = mg;
        return NXG_OK;
    });
}

nxg_status nxg_multi_run(nxg_multi* mg, const nxg_run_desc* desc, void* const* d_values,
                         void* stream, nxg_run_stats* stats) {
    return guarded([&]() {
        if (!mg || !desc) fail(NXG_EINVAL, "NULL argument");
        return multi_run(mg, *desc, d_values, (hipStream_t)stream, stats);
    });
}

nxg_status nxg_multi_destroy(nxg_multi* mg) {
    return guarded([&]() {
        delete mg;
        return NXG_OK;
    });
}

}  // extern "C"

namespace nxg {
// Sets *bad when an edge weight is not finite (NaN or infinite).
__global__ void k_check_weights(const float* __restrict__ w, int64_t m, int32_t* __restrict__ bad) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
        const float v = w[i];
        if (!isfinite(v)) *bad = 1;
    }
}

// Edge weights must be finite (NXG_EINVAL otherwise); synchronises s.
void check_weights(const float* w, int64_t m, hipStream_t s) {
    if (m <= 0) return;
    DevBuf bad;
    bad.alloc(sizeof(int32_t), s);
    NXG_HIP(hipMemsetAsync(bad.p, 0, sizeof(int32_t), s));
    const int64_t blocks = std::min<int64_t>((m + 255) / 256, 4096);
    hipLaunchKernelGGL(k_check_weights, dim3((unsigned)blocks), dim3(256), 0, s, w, m, bad.as<int32_t>());
    NXG_CHECK_LAUNCH();
    int32_t hb = 0;
    NXG_HIP(hipMemcpyAsync(&hb, bad.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    NXG_HIP(hipStreamSynchronize(s));
    if (hb) fail(NXG_EINVAL, "edge weights must be finite");
}

nxg_dsss* build_handle(const nxg_build_desc& d, hipStream_t s, bool spread) {
    {
        if (d.n < 1) fail(NXG_EINVAL, "n must be >= 1");
        // gathers address the value arrays with 32-bit byte offsets (8-byte values)
        if (d.n >= (1 << 29)) fail(NXG_EUNSUPPORTED, "n must be below 2^29");
        if (d.m < 0) fail(NXG_EINVAL, "m must be >= 0");
        const bool sym = (d.flags & NXG_BUILD_SYMMETRIZE) != 0;
        if (d.m >= ((int64_t)1 << 31) || (sym && d.m >= ((int64_t)1 << 30)))
            fail(NXG_EINVAL, "too many edges");
        if (d.m > 0 && (!d.d_src || !d.d_dst)) fail(NXG_EINVAL, "d_src/d_dst is NULL");
        if (d.flags & ~(uint32_t)(NXG_BUILD_KEEP_PERM | NXG_BUILD_TRANSPOSE | NXG_BUILD_SYMMETRIZE |
                                  NXG_BUILD_DEDUP | NXG_BUILD_RELABEL | NXG_BUILD_SCATTER |
                                  NXG_BUILD_DEGREE | NXG_BUILD_HOST_STREAM | NXG_BUILD_PAIRS |
                                  NXG_BUILD_SHUFFLE_SCHEDULE))
            fail(NXG_EINVAL, "unknown build flag");
        if ((d.flags & NXG_BUILD_PAIRS) &&
            (d.d_weight || (d.flags & (NXG_BUILD_KEEP_PERM | NXG_BUILD_TRANSPOSE | NXG_BUILD_SYMMETRIZE |
                                       NXG_BUILD_SCATTER | NXG_BUILD_HOST_STREAM))))
            fail(NXG_EINVAL, "PAIRS cannot be combined with weights, KEEP_PERM, TRANSPOSE, SYMMETRIZE, "
                             "SCATTER or HOST_STREAM");
        if ((d.flags & NXG_BUILD_HOST_STREAM) && (d.flags & (NXG_BUILD_TRANSPOSE | NXG_BUILD_SCATTER)))
            fail(NXG_EINVAL, "HOST_STREAM cannot be combined with TRANSPOSE or SCATTER");
        if ((d.flags & NXG_BUILD_SCATTER) &&
            (d.flags & (NXG_BUILD_RELABEL | NXG_BUILD_TRANSPOSE | NXG_BUILD_DEGREE)))
            fail(NXG_EINVAL, "SCATTER cannot be combined with RELABEL, TRANSPOSE or DEGREE");
        if (sym && (d.d_weight || (d.flags & (NXG_BUILD_KEEP_PERM | NXG_BUILD_TRANSPOSE))))
            fail(NXG_EINVAL, "SYMMETRIZE cannot be combined with weights, KEEP_PERM or TRANSPOSE");
        if (d.interval < 0 || d.interval > d.n) fail(NXG_EINVAL, "interval outside [0, n]");
        if (d.d_weight) check_weights(d.d_weight, d.m, s);
        nxg_dsss* g = new nxg_dsss();
        try {
            NXG_HIP(hipGetDevice(&g->device));
            g->value_bytes = d.value_bytes ? d.value_bytes : 8;
            g->flags = d.flags;
            nxg_build_desc dd = d;
            DevBuf src2, dst2;
            g->n_caller = d.n;
            if (d.flags & (NXG_BUILD_RELABEL | NXG_BUILD_DEGREE)) {
                dd.n = relabel_input(d, s, (d.flags & NXG_BUILD_RELABEL) != 0,
                                     (d.flags & NXG_BUILD_DEGREE) != 0, g->new2old, g->old2new, src2, dst2);
                g->relabeled = true;
                dd.d_src = src2.as<int32_t>();
                dd.d_dst = dst2.as<int32_t>();
                if (dd.interval > dd.n) dd.interval = dd.n;
            }
            build_layout(dd, false, s, g->fwd, spread);
            if (d.flags & NXG_BUILD_HOST_STREAM) {
                // the edge stream (and weights) move to pinned host memory
                Layout& L = g->fwd;
                L.h_words.alloc(sizeof(uint32_t) * (size_t)L.n_words);
                NXG_HIP(hipMemcpyAsync(L.h_words.p, L.words.p, sizeof(uint32_t) * (size_t)L.n_words,
                                       hipMemcpyDeviceToHost, s));
                if (L.has_weight) {
                    L.h_weight.alloc(sizeof(float) * (size_t)L.n_words);
                    NXG_HIP(hipMemcpyAsync(L.h_weight.p, L.weight.p, sizeof(float) * (size_t)L.n_words,
                                           hipMemcpyDeviceToHost, s));
                }
                NXG_HIP(hipStreamSynchronize(s));
                L.words.reset();
                L.weight.reset();
                L.host_stream = true;
            }
            if (d.flags & NXG_BUILD_TRANSPOSE) {
                build_layout(dd, true, s, g->rev, spread);
                g->has_rev = true;
            }
            if (spread) prepare_pagerank_plan(g, s);
        } catch (...) {
            delete g;
            throw;
        }
        return g;
    }
}
}  // namespace nxg

extern "C" {

nxg_status nxg_dsss_destroy(nxg_dsss* g) {
    return guarded([&]() {
        delete g;
        return NXG_OK;
    });
}

nxg_status nxg_dsss_info_get(const nxg_dsss* g, nxg_dsss_info* info) {
    return guarded([&]() {
        if (!g || !info) fail(NXG_EINVAL, "NULL argument");
        const Layout& L = g->fwd;
        memset(info, 0, sizeof(*info));
        info->n = g->n_caller;
        info->n_kept = L.n;
        info->m = L.m;
        info->interval = L.I;
        info->P = L.P;
        info->tile = L.T;
        info->n_tiles = L.n_tiles;
        info->chunk = L.C;
        info->n_chunks = L.n_chunks;
        info->n_words = L.n_words;
        info->max_tile_edges = L.max_tile_edges;
        int64_t bytes = 0;
        for (const Layout* x : {&g->fwd, &g->rev}) {
            for (const DevBuf* b : {&x->words, &x->chunk_row, &x->chunk_tile, &x->tile_chunk,
                                    &x->group_edge, &x->group_word, &x->perm, &x->weight, &x->outdeg,
                                    &x->chunk_rng, &x->chunk_src})
                bytes += (int64_t)b->bytes;
        }
        bytes += (int64_t)(g->new2old.bytes + g->old2new.bytes);
        info->device_bytes = bytes;
        info->relabeled = g->relabeled ? 1 : 0;
        info->has_perm = L.has_perm;
        info->has_weights = L.has_weight;
        info->has_transpose = g->has_rev;
        info->order = L.order;
        info->pairs = L.pairs ? 1 : 0;
        return NXG_OK;
    });
}

nxg_status nxg_dsss_vertex_map(const nxg_dsss* g, int32_t* d_new2old, void* stream) {
    return guarded([&]() {
        if (!g || !d_new2old) fail(NXG_EINVAL, "NULL argument");
        if (!g->relabeled) fail(NXG_EINVAL, "the handle was built without NXG_BUILD_RELABEL or NXG_BUILD_DEGREE");
        hipStream_t s = (hipStream_t)stream;
        NXG_HIP(hipMemcpyAsync(d_new2old, g->new2old.p, sizeof(int32_t) * g->fwd.n,
                               hipMemcpyDeviceToDevice, s));
        NXG_HIP(hipStreamSynchronize(s));
        return NXG_OK;
    });
}

nxg_status nxg_dsss_export(const nxg_dsss* g, int transposed, int64_t* d_offsets, int32_t* d_src,
                           int32_t* d_dst, int32_t* d_perm, void* stream) {
    return guarded([&]() {
        if (!g) fail(NXG_EINVAL, "handle is NULL");
        if (transposed && !g->has_rev) fail(NXG_EINVAL, "handle has no transposed graph");
        if (!transposed && g->fwd.host_stream) fail(NXG_EINVAL, "the edge stream is in host memory (HOST_STREAM)");
        if (!transposed && g->fwd.pairs) fail(NXG_EINVAL, "a PAIRS layout cannot be exported");
        export_layout(transposed ? g->rev : g->fwd, d_offsets, d_src, d_dst, d_perm,
                      (hipStream_t)stream);
        return NXG_OK;
    });
}

nxg_status nxg_run(nxg_dsss* g, const nxg_run_desc* desc, void* stream, nxg_run_stats* stats) {
    return guarded([&]() {
        if (!g || !desc) fail(NXG_EINVAL, "NULL argument");
        return run_program(g, *desc, (hipStream_t)stream, stats);
    });
}

nxg_status nxg_copy_probe(int64_t bytes, int32_t reps, void* stream, double* gbps) {
    return guarded([&]() {
        if (!gbps) fail(NXG_EINVAL, "gbps is NULL");
        return copy_probe(bytes, reps, (hipStream_t)stream, gbps);
    });
}

nxg_status nxg_read_probe(int64_t bytes, int32_t reps, void* stream, double* gbps) {
    return guarded([&]() {
        if (!gbps) fail(NXG_EINVAL, "gbps is NULL");
        return read_probe(bytes, reps, (hipStream_t)stream, gbps);
    });
}

nxg_status nxg_tune(const nxg_build_desc* desc, nxg_program program, nxg_dtype dtype,
                    int32_t batch, void* stream, nxg_tune_result* result) {
    return guarded([&]() {
        if (!desc || !result) fail(NXG_EINVAL, "NULL argument");
        if (desc->n < 1 || desc->m < 0 || (desc->m > 0 && (!desc->d_src || !desc->d_dst)))
            fail(NXG_EINVAL, "invalid graph");
        return tune(*desc, program, dtype, batch, (hipStream_t)stream, result);
    });
}

nxg_status nxg_dsss_set_weights(nxg_dsss* g, const float* d_weight, void* stream) {
    return guarded([&]() {
        if (!g || !d_weight) fail(NXG_EINVAL, "NULL argument");
        dsss_set_weights(g, d_weight, (hipStream_t)stream);
        return NXG_OK;
    });
}

nxg_status nxg_pagerank_adjoint(nxg_dsss* g, const nxg_adjoint_desc* desc, void* stream,
                                nxg_run_stats* stats) {
    return guarded([&]() {
        if (!g || !desc) fail(NXG_EINVAL, "NULL argument");
        return pagerank_adjoint(g, *desc, (hipStream_t)stream, stats);
    });
}

}  // extern "C"
