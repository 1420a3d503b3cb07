// Direct single-step kernel for patterns without a specialised variant.
//
// One thread per output point of the output box; it sums the K weighted
// neighbours in canonical order straight from global memory (cached), with the
// boundary rule applied per neighbour.  Used for radii or dimensionalities the
// streaming kernels are not instantiated for; a pass of T steps becomes T
// launches of this kernel.

#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include "internal.h"
#include "valu_common.h"

namespace stl {
namespace {

constexpr int kGenericMaxK = 343;  // box r = 3 in 3D; the argument block stays under 4 KiB

template <typename TC>
struct GenericArgs {
    const void *src;
    void *dst;
    int n[3];
    int lo[3], hi[3];
    int d, K, periodic;
    TC h;
    TC w[kGenericMaxK];
    int8_t off[kGenericMaxK][3];
};

template <typename TS, typename TC>
__global__ __launch_bounds__(256) void generic_kernel(GenericArgs<TC> a)
{
    const int e0 = a.hi[0] - a.lo[0], e1 = a.hi[1] - a.lo[1], e2 = a.hi[2] - a.lo[2];
    const int64_t total = (int64_t)e0 * e1 * e2;
    const TS *src = static_cast<const TS *>(a.src);
    TS *dst = static_cast<TS *>(a.dst);
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int x2 = a.lo[2] + (int)(idx % e2);
        const int x1 = a.lo[1] + (int)((idx / e2) % e1);
        const int x0 = a.lo[0] + (int)(idx / ((int64_t)e1 * e2));
        TC acc = TC(0);
        for (int k = 0; k < a.K; ++k) {
            int y0 = x0 + a.off[k][0], y1 = x1 + a.off[k][1], y2 = x2 + a.off[k][2];
            TC v;
            const bool in = y0 >= 0 && y0 < a.n[0] && y1 >= 0 && y1 < a.n[1] && y2 >= 0 && y2 < a.n[2];
            if (in || a.periodic) {
                y0 = wrap(y0, a.n[0]);
                y1 = wrap(y1, a.n[1]);
                y2 = wrap(y2, a.n[2]);
                v = to_compute<TC>(src[((int64_t)y0 * a.n[1] + y1) * a.n[2] + y2]);
            } else {
                v = a.h;
            }
            acc = fma_c(a.w[k], v, acc);
        }
        dst[((int64_t)x0 * a.n[1] + x1) * a.n[2] + x2] = to_storage<TS>(acc);
    }
}

template <typename TS, typename TC>
hipError_t launch_generic(const PassArgs &p, hipStream_t stream)
{
    if (p.steps != 1 || p.K > kGenericMaxK) return hipErrorNotSupported;
    GenericArgs<TC> a;
    a.src = p.src;
    a.dst = p.dst;
    a.d = p.d;
    a.K = p.K;
    a.periodic = p.boundary == STENCIL_PERIODIC;
    a.h = (TC)p.halo;
    // view a 2D grid as 1 x n0 x n1
    const int sh = 3 - p.d;
    for (int i = 0; i < 3; ++i) {
        const int j = i - sh;
        a.n[i] = j < 0 ? 1 : (int)p.dims[j];
        a.lo[i] = j < 0 ? 0 : p.region_lo[j];
        a.hi[i] = j < 0 ? 1 : p.region_hi[j];
    }
    for (int k = 0; k < p.K; ++k) {
        a.w[k] = (TC)p.w[k];
        for (int i = 0; i < 3; ++i) a.off[k][i] = 0;
    }
    for (int k = 0; k < p.K; ++k)
        for (int i = 0; i < p.d; ++i) a.off[k][i + sh] = (int8_t)p.offs[k * p.d + i];
    const int64_t total = (int64_t)(a.hi[0] - a.lo[0]) * (a.hi[1] - a.lo[1]) * (a.hi[2] - a.lo[2]);
    if (total <= 0) return hipSuccess;
    int64_t blocks = (total + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL((generic_kernel<TS, TC>), dim3((unsigned)blocks), dim3(256), 0, stream, a);
    return hipGetLastError();
}

}  // namespace

const std::vector<KernelEntry> &generic_kernels()
{
    static const std::vector<KernelEntry> table = {
        {STENCIL_PATH_VALU, STENCIL_F64, -1, 2, -1, 1, &launch_generic<double, double>, nullptr},
        {STENCIL_PATH_VALU, STENCIL_F64, -1, 3, -1, 1, &launch_generic<double, double>, nullptr},
        {STENCIL_PATH_VALU, STENCIL_F32, -1, 2, -1, 1, &launch_generic<float, float>, nullptr},
        {STENCIL_PATH_VALU, STENCIL_F32, -1, 3, -1, 1, &launch_generic<float, float>, nullptr},
        {STENCIL_PATH_VALU, STENCIL_BF16, -1, 2, -1, 1, &launch_generic<__hip_bfloat16, float>, nullptr},
        {STENCIL_PATH_VALU, STENCIL_BF16, -1, 3, -1, 1, &launch_generic<__hip_bfloat16, float>, nullptr},
        {STENCIL_PATH_VALU, STENCIL_F16, -1, 2, -1, 1, &launch_generic<__half, float>, nullptr},
        {STENCIL_PATH_VALU, STENCIL_F16, -1, 3, -1, 1, &launch_generic<__half, float>, nullptr},
    };
    return table;
}

}  // namespace stl
