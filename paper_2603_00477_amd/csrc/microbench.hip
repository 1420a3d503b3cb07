// Measured ceilings of the roofline model: HBM copy bandwidth and the peak
// rates of the instructions the two kernel families issue.
//
// Each probe runs one kernel over the whole chip and times it with HIP events
// on the given stream (the call blocks).  The FMA probes run 8 independent
// dependency chains per lane so that issue, not latency, limits them.

#include <hip/hip_runtime.h>

#include <cstdint>

#include "internal.h"
#include "mfma2d_impl.h"

namespace stl {
namespace {

__global__ __launch_bounds__(256) void mb_copy(const uint4 *__restrict__ a, uint4 *__restrict__ b, size_t n)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        b[i] = a[i];
}

template <typename F>
__global__ __launch_bounds__(256) void mb_fma(F *out, int iters, F seed)
{
    F x[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) x[c] = seed + (F)(threadIdx.x + c);
    const F m = (F)0.999, a = (F)1e-3;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int c = 0; c < 8; ++c) x[c] = fma_c(x[c], m, a);
    }
    F s = 0;
#pragma unroll
    for (int c = 0; c < 8; ++c) s += x[c];
    if (s == (F)-1) out[threadIdx.x] = s;  // keeps the chains live
}

// FP32 FMA chains whose multiplier is a scalar register (SGPR = 1) or a
// vector register (SGPR = 0), as the stencil kernels' weights are.
template <int SGPR>
__global__ __launch_bounds__(256) void mb_fma32_operand(float *out, int iters, const float *w)
{
    float x[16], y[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) {
        x[c] = (float)(threadIdx.x + c) * 1e-3f;
        y[c] = (float)((threadIdx.x & 7) + c + 1) * 0.5f;
    }
    float m = w[0];
    if constexpr (SGPR == 0) m = m + (float)threadIdx.x * 1e-9f;  // per-lane: a vector register
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int c = 0; c < 16; ++c) x[c] = fma_c(m, y[c], x[c]);
    }
    float s = 0;
#pragma unroll
    for (int c = 0; c < 16; ++c) s += x[c];
    if (s == -1.f) out[threadIdx.x] = s;
}

template <int DT>
__global__ __launch_bounds__(256) void mb_mfma(float *out, int iters)
{
    using MT = MfmaTypes<DT>;
    using FR = typename MT::FR;
    using ACC = typename MT::ACC;
    FR a, b;
    if constexpr (sizeof(FR) == 8 || sizeof(FR) == 4) {
        a = (FR)(threadIdx.x * 1e-3);
        b = (FR)(1.0 - threadIdx.x * 1e-4);
    } else {
        for (int e = 0; e < 8; ++e) {
            a[e] = (typename MT::OP)(threadIdx.x * 1e-3f);
            b[e] = (typename MT::OP)(1.0f);
        }
    }
    ACC c0 = ACC{}, c1 = ACC{}, c2 = ACC{}, c3 = ACC{};
    for (int i = 0; i < iters; ++i) {
        c0 = mfma16(a, b, c0);
        c1 = mfma16(a, b, c1);
        c2 = mfma16(a, b, c2);
        c3 = mfma16(a, b, c3);
    }
    const float s = (float)(c0[0] + c1[1] + c2[2] + c3[3]);
    if (s == -1.f) out[threadIdx.x] = s;
}

}  // namespace
}  // namespace stl

using namespace stl;

extern "C" int stencil_microbench(int kind, void *buf, int64_t bytes, void *stream_v, double *result)
{
    if (!result || kind < 0 || kind > 7) return fail(STENCIL_ERR_INVALID_ARG, "stencil_microbench: bad kind");
    if (kind == 0 && (!buf || bytes < 2 * 4096 || bytes % 32))
        return fail(STENCIL_ERR_INVALID_ARG, "stencil_microbench: copy needs an even buffer of >= 8 KiB");
    hipStream_t stream = (hipStream_t)stream_v;
    const int cus = device_cu_count();
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return fail(STENCIL_ERR_HIP, "stencil_microbench: hipEventCreate");
    float *sink = nullptr;
    if (hipMalloc(&sink, 256 * sizeof(double)) != hipSuccess) {
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        return fail(STENCIL_ERR_OOM, "stencil_microbench: sink");
    }
    if (hipMemset(sink, 0, 256 * sizeof(double)) != hipSuccess) {  // the FMA kinds 6/7 read w[0] from it
        (void)hipFree(sink);
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        return fail(STENCIL_ERR_HIP, "stencil_microbench: memset");
    }
    const int grid = cus * 8;
    const int iters = 4096;
    double work = 0;
    auto launch = [&]() {
        switch (kind) {
        case 0: {
            const size_t n = (size_t)bytes / 2 / sizeof(uint4);
            const uint4 *a = static_cast<const uint4 *>(buf);
            uint4 *b = static_cast<uint4 *>(buf) + n;
            hipLaunchKernelGGL(mb_copy, dim3(cus * 16), dim3(256), 0, stream, a, b, n);
            work = 2.0 * n * sizeof(uint4);
            break;
        }
        case 1:
            hipLaunchKernelGGL(mb_fma<double>, dim3(grid), dim3(256), 0, stream, (double *)sink, iters, 1.0);
            work = 2.0 * 8 * iters * (double)grid * 256;
            break;
        case 2:
            hipLaunchKernelGGL(mb_fma<float>, dim3(grid), dim3(256), 0, stream, sink, iters, 1.0f);
            work = 2.0 * 8 * iters * (double)grid * 256;
            break;
        case 3:
            hipLaunchKernelGGL(mb_mfma<STENCIL_F64>, dim3(grid), dim3(256), 0, stream, sink, iters);
            work = 4.0 * iters * 2.0 * 16 * 16 * 4 * (double)grid * 4;
            break;
        case 4:
            hipLaunchKernelGGL(mb_mfma<STENCIL_F32>, dim3(grid), dim3(256), 0, stream, sink, iters);
            work = 4.0 * iters * 2.0 * 16 * 16 * 4 * (double)grid * 4;
            break;
        case 6:
        case 7:
            if (kind == 6)
                hipLaunchKernelGGL(mb_fma32_operand<1>, dim3(grid), dim3(256), 0, stream, sink, iters,
                                   (const float *)sink);
            else
                hipLaunchKernelGGL(mb_fma32_operand<0>, dim3(grid), dim3(256), 0, stream, sink, iters,
                                   (const float *)sink);
            work = 2.0 * 16 * iters * (double)grid * 256;
            break;
        case 5:
            hipLaunchKernelGGL(mb_mfma<STENCIL_BF16>, dim3(grid), dim3(256), 0, stream, sink, iters);
            work = 4.0 * iters * 2.0 * 16 * 16 * 32 * (double)grid * 4;
            break;
        }
    };
    launch();  // warm-up
    float ms = 0;
    hipError_t e = hipEventRecord(e0, stream);
    for (int rep = 0; rep < 5 && e == hipSuccess; ++rep) launch();
    if (e == hipSuccess) e = hipEventRecord(e1, stream);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    (void)hipFree(sink);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e != hipSuccess) return fail(STENCIL_ERR_HIP, std::string("stencil_microbench: ") + hipGetErrorString(e));
    *result = work * 5 / (ms * 1e-3);  // bytes/s (copy) or flop/s
    return STENCIL_OK;
}
