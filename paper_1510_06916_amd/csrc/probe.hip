// Attainable HBM bandwidth on this device: a streaming copy (also the kernel
// that calibrates the FETCH_SIZE / WRITE_SIZE counters) and a read-only
// stream, the ceiling of an iteration that mostly reads.
#include <hip/hip_runtime.h>

#include "nxg_internal.h"

namespace nxg {
namespace {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void k_copy_probe(const u32x4* __restrict__ a, u32x4* __restrict__ b,
                                                    int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        b[i] = __builtin_nontemporal_load(a + i);
}

// Four independent 16-byte non-temporal loads per thread in flight; the XOR
// of everything read is stored only if it equals a value it cannot take for
// the buffer's fill, so the loads stay live without a store per element.
__global__ __launch_bounds__(256) void k_read_probe(const u32x4* __restrict__ a, int64_t n,
                                                    uint32_t* __restrict__ sink) {
    constexpr int kU = 4;
    const int64_t stride = (int64_t)gridDim.x * 256;
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    u32x4 acc = {0u, 0u, 0u, 0u};
    for (; i + (kU - 1) * stride < n; i += kU * stride) {
        u32x4 v[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) v[u] = __builtin_nontemporal_load(a + i + u * stride);
#pragma unroll
        for (int u = 0; u < kU; ++u) acc ^= v[u];
    }
    for (; i < n; i += stride) acc ^= a[i];
    if ((acc.x ^ acc.y ^ acc.z ^ acc.w) == 0x5A5A5A5Au) sink[0] = 1u;
}

int probe_grid() {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
        cus = 256;
    return cus * 16;
}

}  // namespace

nxg_status copy_probe(int64_t bytes, int reps, hipStream_t s, double* gbps) {
    if (bytes < 4096 || reps < 1) fail(NXG_EINVAL, "copy probe needs bytes >= 4096 and reps >= 1");
    const int64_t n = bytes / 16;
    DevBuf a, b;
    a.alloc(n * 16, s);
    b.alloc(n * 16, s);
    NXG_HIP(hipMemsetAsync(a.p, 1, n * 16, s));
    const int grid = probe_grid();
    hipLaunchKernelGGL(k_copy_probe, dim3(grid), dim3(256), 0, s, a.as<u32x4>(), b.as<u32x4>(), n);
    NXG_CHECK_LAUNCH();
    hipEvent_t e0 = nullptr, e1 = nullptr;
    NXG_HIP(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        fail(NXG_EDEVICE, "hipEventCreate failed");
    }
    float ms = 0.f;
    hipError_t err = hipEventRecord(e0, s);
    for (int r = 0; r < reps && err == hipSuccess; ++r) {
        hipLaunchKernelGGL(k_copy_probe, dim3(grid), dim3(256), 0, s, a.as<u32x4>(), b.as<u32x4>(), n);
        err = hipGetLastError();
    }
    if (err == hipSuccess) err = hipEventRecord(e1, s);
    if (err == hipSuccess) err = hipEventSynchronize(e1);
    if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (err != hipSuccess) fail(NXG_EDEVICE, std::string("copy probe: ") + hipGetErrorString(err));
    *gbps = 2.0 * n * 16 * reps / (ms * 1e-3) / 1e9;
    return NXG_OK;
}

nxg_status read_probe(int64_t bytes, int reps, hipStream_t s, double* gbps) {
    if (bytes < 4096 || reps < 1) fail(NXG_EINVAL, "read probe needs bytes >= 4096 and reps >= 1");
    const int64_t n = bytes / 16;
    DevBuf a, sink;
    a.alloc(n * 16, s);
    sink.alloc(sizeof(uint32_t), s);
    NXG_HIP(hipMemsetAsync(a.p, 1, n * 16, s));
    const int grid = probe_grid();
    hipLaunchKernelGGL(k_read_probe, dim3(grid), dim3(256), 0, s, a.as<u32x4>(), n, sink.as<uint32_t>());
    NXG_CHECK_LAUNCH();
    hipEvent_t e0 = nullptr, e1 = nullptr;
    NXG_HIP(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        fail(NXG_EDEVICE, "hipEventCreate failed");
    }
    float ms = 0.f;
    hipError_t err = hipEventRecord(e0, s);
    for (int r = 0; r < reps && err == hipSuccess; ++r) {
        hipLaunchKernelGGL(k_read_probe, dim3(grid), dim3(256), 0, s, a.as<u32x4>(), n, sink.as<uint32_t>());
        err = hipGetLastError();
    }
    if (err == hipSuccess) err = hipEventRecord(e1, s);
    if (err == hipSuccess) err = hipEventSynchronize(e1);
    if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (err != hipSuccess) fail(NXG_EDEVICE, std::string("read probe: ") + hipGetErrorString(err));
    *gbps = (double)n * 16 * reps / (ms * 1e-3) / 1e9;
    return NXG_OK;
}

}  // namespace nxg
