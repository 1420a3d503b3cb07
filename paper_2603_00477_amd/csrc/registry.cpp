// Registry of all kernel tables and the staging of batched job tables.
#include <hip/hip_runtime.h>

#include <cstring>

#include "internal.h"

namespace stl {

hipError_t BatchStaging::begin(hipStream_t stream)
{
    (void)stream;
    if (pending_) {
        hipError_t e = hipEventSynchronize(done_);
        if (e != hipSuccess) return e;
        pending_ = false;
    }
    used_ = 0;
    return hipSuccess;
}

hipError_t BatchStaging::grow(size_t need, hipStream_t stream)
{
    // regions handed out in this call may still be read by queued kernels
    hipError_t e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return e;
    size_t cap = cap_ ? cap_ : (size_t)1 << 16;
    while (cap < need) cap *= 2;
    uint8_t *h = nullptr, *d = nullptr;
    e = hipHostMalloc((void **)&h, cap, hipHostMallocDefault);
    if (e != hipSuccess) return e;
    e = hipMalloc((void **)&d, cap);
    if (e != hipSuccess) {
        (void)hipHostFree(h);
        return e;
    }
    if (host_) (void)hipHostFree(host_);
    if (dev_) (void)hipFree(dev_);
    host_ = h;
    dev_ = d;
    cap_ = cap;
    used_ = 0;
    return hipSuccess;
}

hipError_t BatchStaging::put(const void *host, size_t bytes, void **dev, hipStream_t stream)
{
    const size_t off = (used_ + 255) & ~(size_t)255;
    if (off + bytes > cap_) {
        hipError_t e = grow(off + bytes > 2 * cap_ ? off + bytes : 2 * cap_, stream);
        if (e != hipSuccess) return e;
        return put(host, bytes, dev, stream);
    }
    std::memcpy(host_ + off, host, bytes);
    hipError_t e = hipMemcpyAsync(dev_ + off, host_ + off, bytes, hipMemcpyHostToDevice, stream);
    if (e != hipSuccess) return e;
    used_ = off + bytes;
    *dev = dev_ + off;
    return hipSuccess;
}

hipError_t BatchStaging::end(hipStream_t stream)
{
    if (!done_) {
        hipError_t e = hipEventCreateWithFlags(&done_, hipEventDisableTiming);
        if (e != hipSuccess) return e;
    }
    hipError_t e = hipEventRecord(done_, stream);
    if (e == hipSuccess) pending_ = true;
    return e;
}

BatchStaging::~BatchStaging()
{
    // process teardown: the runtime may already be gone, errors are ignored
    if (host_) (void)hipHostFree(host_);
    if (dev_) (void)hipFree(dev_);
    if (done_) (void)hipEventDestroy(done_);
}


std::vector<const std::vector<KernelEntry> *> all_kernel_tables()
{
    return {&valu2d_table_f64(),  &valu2d_table_f32(),  &valu2d_table_bf16(),
            &valu2d_table_f16(),  &valu2d_table_x3(),   &valu3d_kernels(),    &mfma2d_table_f64(),
            &mfma2d_table_f32(),  &mfma2d_table_bf16(), &mfma2d_table_f16(),
            &mfma2d_table_x3(),   &mfma3d_table_f64(),  &mfma3d_table_f32(),    &generic_kernels()};
}
}  // namespace stl
