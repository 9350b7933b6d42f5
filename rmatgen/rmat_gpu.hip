// Seeded synthetic inputs, device side: the same R-MAT edge keys as rmat_cpu.c,
// produced on the GPU for graphs too large to generate on the host, then sorted
// and de-duplicated with rocPRIM. Nothing here is part of the graph method; the
// output is an input edge list (sorted by (u, v), duplicates removed).
#include <hip/hip_runtime.h>
#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_select.hpp>
#include <stdint.h>

namespace {

constexpr uint32_t kM0 = 0xD2511F53u;
constexpr uint32_t kM1 = 0xCD9E8D57u;
constexpr uint32_t kW0 = 0x9E3779B9u;
constexpr uint32_t kW1 = 0xBB67AE85u;

__device__ inline void philox10(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += kW0;
            k1 += kW1;
        }
        uint32_t lo0 = kM0 * c[0], hi0 = __umulhi(kM0, c[0]);
        uint32_t lo1 = kM1 * c[2], hi1 = __umulhi(kM1, c[2]);
        uint32_t n0 = hi1 ^ c[1] ^ k0;
        uint32_t n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
    }
}

__global__ void rmat_keys_kernel(int scale, uint64_t seed, int64_t count, uint32_t thrA,
                                 uint32_t thrAB, uint32_t thrABC, uint64_t* __restrict__ keys) {
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count;
         e += (int64_t)gridDim.x * blockDim.x) {
        uint64_t k = (uint64_t)e;
        uint32_t u = 0, v = 0;
        uint32_t r[4] = {0, 0, 0, 0};
        for (int l = 0; l < scale; ++l) {
            if ((l & 3) == 0) {
                r[0] = (uint32_t)k;
                r[1] = (uint32_t)(k >> 32);
                r[2] = (uint32_t)(l >> 2);
                r[3] = 0u;
                philox10(r, k0, k1);
            }
            uint32_t x = r[l & 3];
            uint32_t q = x < thrA ? 0u : (x < thrAB ? 1u : (x < thrABC ? 2u : 3u));
            u = (u << 1) | (q >> 1);
            v = (v << 1) | (q & 1u);
        }
        keys[e] = ((uint64_t)u << 32) | (uint64_t)v;
    }
}

__global__ void split_kernel(const uint64_t* __restrict__ keys, const int64_t* __restrict__ m,
                             int32_t* __restrict__ src, int32_t* __restrict__ dst) {
    const int64_t mm = *m;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < mm;
         e += (int64_t)gridDim.x * blockDim.x) {
        uint64_t k = keys[e];
        src[e] = (int32_t)(k >> 32);
        dst[e] = (int32_t)(uint32_t)k;
    }
}

}  // namespace

extern "C" {

// Bytes of rocPRIM scratch needed to sort and de-duplicate `count` keys.
int rmatgen_gpu_tmp_bytes(int64_t count, int scale, size_t* bytes) {
    size_t a = 0, b = 0;
    uint64_t* nk = nullptr;
    int64_t* nc = nullptr;
    if (rocprim::radix_sort_keys(nullptr, a, nk, nk, (size_t)count, 0u,
                                 (unsigned)(32 + scale)) != hipSuccess)
        return 1;
    if (rocprim::unique(nullptr, b, nk, nk, nc, (size_t)count) != hipSuccess) return 1;
    *bytes = (a > b ? a : b) + 256;
    return 0;
}

// Generates `count` R-MAT keys, sorts them by (u, v), removes duplicates and splits
// the survivors into src/dst. Buffers are caller-owned device memory: keys_a and
// keys_b hold `count` uint64 each, src/dst hold `count` int32 each, tmp holds
// rmatgen_gpu_tmp_bytes bytes, d_m one int64. Synchronises the stream once and
// returns the edge count through *m_out. Returns 0 on success.
int rmatgen_gpu_edges(int scale, int64_t count, uint64_t seed, uint32_t thrA, uint32_t thrAB,
                      uint32_t thrABC, uint64_t* keys_a, uint64_t* keys_b, void* tmp,
                      size_t tmp_bytes, int64_t* d_m, int32_t* src, int32_t* dst,
                      int64_t* m_out, hipStream_t stream) {
    if (scale < 1 || scale > 31 || count < 0) return 1;
    if (count == 0) {
        *m_out = 0;
        return 0;
    }
    const int threads = 256;
    int64_t want = (count + threads - 1) / threads;
    int blocks = (int)(want < 65536 ? want : 65536);
    hipLaunchKernelGGL(rmat_keys_kernel, dim3(blocks), dim3(threads), 0, stream, scale, seed,
                       count, thrA, thrAB, thrABC, keys_a);
    if (hipGetLastError() != hipSuccess) return 2;
    size_t sz = tmp_bytes;
    if (rocprim::radix_sort_keys(tmp, sz, keys_a, keys_b, (size_t)count, 0u,
                                 (unsigned)(32 + scale), stream) != hipSuccess)
        return 3;
    sz = tmp_bytes;
    if (rocprim::unique(tmp, sz, keys_b, keys_a, d_m, (size_t)count, rocprim::equal_to<uint64_t>(),
                        stream) != hipSuccess)
        return 4;
    hipLaunchKernelGGL(split_kernel, dim3(blocks), dim3(threads), 0, stream, keys_a, d_m, src,
                       dst);
    if (hipGetLastError() != hipSuccess) return 5;
    if (hipMemcpyAsync(m_out, d_m, sizeof(int64_t), hipMemcpyDeviceToHost, stream) != hipSuccess)
        return 6;
    if (hipStreamSynchronize(stream) != hipSuccess) return 7;
    return 0;
}

}  // extern "C"
