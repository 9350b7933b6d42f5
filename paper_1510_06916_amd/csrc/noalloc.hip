// PageRank without any device allocation (nxg_run_noalloc), for callers that
// cannot allocate: code under stream capture, tight serving loops.
//
// The run's whole workspace -- the two value vectors, the hub partials of
// split tiles, the per-tile scalars, the per-iteration statistics and, for a
// relabeled build, the vectors in internal ids -- is carved out of one
// file-scope device array of kScratchBytes. Each device holds its own copy of
// the array (for the life of the process); its address on a device is looked
// up once, with that device current, and every later call on the device uses
// that address. Calls that overlap on one device share the array and race.
#include <mutex>

#include "nxg_internal.h"

namespace {

constexpr size_t kScratchBytes = (size_t)64 << 20;
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

// Per device: the array's device address and the run's two timing events,
// made at the first call on that device.
struct DeviceScratch {
    void* ptr = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
};
DeviceScratch g_scratch[kMaxDevices];
std::mutex g_scratch_mu;

const DeviceScratch& scratch_on(int dev) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (dev < 0 || dev >= kMaxDevices) nxg::fail(NXG_EINVAL, "device index out of range");
    DeviceScratch& d = g_scratch[dev];
    if (!d.ptr) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            nxg::fail(NXG_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        if (!d.e0) NXG_HIP(hipEventCreate(&d.e0));
        if (!d.e1) NXG_HIP(hipEventCreate(&d.e1));
        d.ptr = p;
    }
    return d;
}

}  // namespace

extern "C" {

size_t nxg_noalloc_scratch_bytes(void) { return kScratchBytes; }

nxg_status nxg_run_noalloc(nxg_dsss* g, const nxg_run_desc* desc, void* stream, nxg_run_stats* stats) {
    return nxg::guarded([&]() {
        if (!g || !desc) nxg::fail(NXG_EINVAL, "NULL argument");
        int dev = -1;
        NXG_HIP(hipGetDevice(&dev));
        if (dev != g->device) nxg::fail(NXG_EINVAL, "the handle lives on another device than the current one");
        const DeviceScratch& d = scratch_on(dev);
        return nxg::run_pagerank_in(g, *desc, (hipStream_t)stream, stats, d.ptr, kScratchBytes, d.e0, d.e1);
    });
}

}  // extern "C"
