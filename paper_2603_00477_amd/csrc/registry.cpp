// Registry of all kernel tables and the staging of batched job tables.
#include <hip/hip_runtime.h>

#include <cstring>

#include "internal.h"

namespace stl {

hipError_t BatchStaging::begin(hipStream_t stream)
{
    (void)stream;
    cur_ = (cur_ + 1) % kSlots;
    Slot &s = slots_[cur_];
    if (s.pending) {
        // the batch that last used this slot may still read its tables
        hipError_t e = hipEventSynchronize(s.done);
        if (e != hipSuccess) return e;
        s.pending = false;
    }
    // buffers the slot outgrew during that batch are no longer referenced
    for (auto &old : s.retired) {
        (void)hipHostFree(old.first);
        (void)hipFree(old.second);
    }
    s.retired.clear();
    s.used = 0;
    return hipSuccess;
}

hipError_t BatchStaging::grow(Slot &s, size_t need)
{
    // Regions of this slot handed out earlier in the same batch call stay
    // valid: kernels already queued, and launches of this call not yet
    // issued, may read them.  The old buffers are retired, not freed, and
    // released by the next begin() on this slot, after the slot's event has
    // shown that the whole batch finished.
    size_t cap = s.cap ? s.cap : (size_t)1 << 16;
    while (cap < need) cap *= 2;
    uint8_t *h = nullptr, *d = nullptr;
    hipError_t e = hipHostMalloc((void **)&h, cap, hipHostMallocDefault);
    if (e != hipSuccess) return e;
    e = hipMalloc((void **)&d, cap);
    if (e != hipSuccess) {
        (void)hipHostFree(h);
        return e;
    }
    if (s.host || s.dev) s.retired.emplace_back(s.host, s.dev);
    s.host = h;
    s.dev = d;
    s.cap = cap;
    s.used = 0;
    return hipSuccess;
}

hipError_t BatchStaging::put(const void *host, size_t bytes, void **dev, hipStream_t stream)
{
    Slot &s = slots_[cur_];
    const size_t off = (s.used + 255) & ~(size_t)255;
    if (off + bytes > s.cap) {
        hipError_t e = grow(s, bytes > 2 * s.cap ? bytes : 2 * s.cap);
        if (e != hipSuccess) return e;
        return put(host, bytes, dev, stream);
    }
    std::memcpy(s.host + off, host, bytes);
    hipError_t e = hipMemcpyAsync(s.dev + off, s.host + off, bytes, hipMemcpyHostToDevice, stream);
    if (e != hipSuccess) return e;
    s.used = off + bytes;
    *dev = s.dev + off;
    return hipSuccess;
}

hipError_t BatchStaging::end(hipStream_t stream)
{
    Slot &s = slots_[cur_];
    if (!s.done) {
        hipError_t e = hipEventCreateWithFlags(&s.done, hipEventDisableTiming);
        if (e != hipSuccess) return e;
    }
    hipError_t e = hipEventRecord(s.done, stream);
    if (e == hipSuccess) s.pending = true;
    return e;
}

BatchStaging::~BatchStaging()
{
    // process teardown: the runtime may already be gone, errors are ignored
    for (Slot &s : slots_) {
        for (auto &old : s.retired) {
            (void)hipHostFree(old.first);
            (void)hipFree(old.second);
        }
        if (s.host) (void)hipHostFree(s.host);
        if (s.dev) (void)hipFree(s.dev);
        if (s.done) (void)hipEventDestroy(s.done);
    }
}


hipError_t stage_job_table(BatchStaging *stage, const void *jobs, size_t job_bytes,
                           const std::vector<int> &start, void **djobs, void **dstart, hipStream_t stream)
{
    const size_t jb = (job_bytes + 255) & ~(size_t)255;
    std::vector<uint8_t> blob(jb + start.size() * sizeof(int));
    std::memcpy(blob.data(), jobs, job_bytes);
    std::memcpy(blob.data() + jb, start.data(), start.size() * sizeof(int));
    void *d = nullptr;
    hipError_t e = stage->put(blob.data(), blob.size(), &d, stream);
    if (e != hipSuccess) return e;
    *djobs = d;
    *dstart = static_cast<uint8_t *>(d) + jb;
    return hipSuccess;
}

std::vector<const std::vector<KernelEntry> *> all_kernel_tables()
{
    return {&valu2d_table_f64(),   &valu2d_table_f32(),  &valu2d_table_bf16(), &valu2d_table_f16(),
            &valu2d_table_x3(),    &valu3d_fused_kernels(), &valu3d_kernels(),    &valu3d_box_kernels(), &valu2d_table_cases(),
            &mfma2d_table_cases(), &mfma3d_table_cases(), &mfma2d_table_f64(),  &mfma2d_table_f32(),
            &mfma2d_table_bf16(),  &mfma2d_table_f16(),  &mfma2d_table_x3(),    &mfma3d_table_f64(),
            &mfma3d_table_f32(),   &mfma2d_table_sparse(), &mfma2d_table_seq(),
            &generic_kernels()};
}
}  // namespace stl
