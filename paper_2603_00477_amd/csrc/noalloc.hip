// Allocation-free run: the intermediate grid of multi-pass runs lives in a
// file-scope device array instead of memory the plan allocates.
//
// For callers that cannot allocate device memory (code under HIP graph
// capture, tight serving loops, harnesses that forbid hipMalloc).  The array
// exists once per GPU for the life of the process; every call on a GPU uses
// that GPU's copy, so calls that overlap on one GPU race.  A pass overwrites
// every element it writes before any later pass reads it, so the array needs
// no clearing between calls.
//
// The array's name is a host-side stand-in in host code: its device address
// is looked up once per device with hipGetSymbolAddress and only that address
// is handed to kernels.

#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "internal.h"

namespace {

static __device__ __align__(256) unsigned char scratch[STENCIL_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;

std::mutex g_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up on the first
// call per device, with that device current).
hipError_t scratch_address(int dev, void **out)
{
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!ptr) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

}  // namespace

extern "C" int stencil_run_noalloc(stencil_plan_t plan, const void *in, void *out, int64_t steps,
                                   void *stream)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return stl::fail(STENCIL_ERR_HIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices)
        return stl::fail(STENCIL_ERR_UNSUPPORTED, "stencil_run_noalloc: device index out of range");
    void *ptr = nullptr;
    e = scratch_address(dev, &ptr);
    if (e != hipSuccess)
        return stl::fail(STENCIL_ERR_HIP, std::string("hipGetSymbolAddress: ") + hipGetErrorString(e));
    return stl::run_without_allocation(plan, in, out, steps, (hipStream_t)stream, ptr,
                                       (size_t)STENCIL_NOALLOC_SCRATCH_BYTES);
}
