// alm2map for callers that cannot allocate device memory: the workspace is a
// fixed device array of the library instead of a caller buffer.
#include <mutex>

#include "sht_internal.h"

// The workspace of sht_alm2map_noalloc.  In host code the name is a stand-in
// only: its device address comes from hipGetSymbolAddress, once per device.
static __device__ __align__(256) unsigned char scratch[SHT_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_scratch[kMaxDevices];   // device address of `scratch` on each device

// Device address of the array on `dev`, the current device (looked up on the
// first call there; nullptr on failure).
void *scratch_on(int dev)
{
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_scratch[dev]) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return nullptr;
        g_scratch[dev] = ptr;
    }
    return g_scratch[dev];
}

}  // namespace

extern "C" sht_status sht_alm2map_noalloc(sht_plan_t p, const double *alm, double *map,
                                          void *stream)
{
    sht_status s = sht::check_plan_device(p);
    if (s != SHT_OK) return s;
    if (!alm || !map) return SHT_ERR_INVALID_ARG;
    if (sht::forward_workspace(p) > (size_t)SHT_NOALLOC_SCRATCH_BYTES) return SHT_ERR_WORKSPACE;
    if (p->device < 0 || p->device >= kMaxDevices) return SHT_ERR_UNSUPPORTED;
    void *ws = scratch_on(p->device);
    if (!ws) return SHT_ERR_HIP;
    return sht::forward_transform(p, alm, map, ws, (hipStream_t)stream);
}
