// VALU 2D kernel instances beyond r <= 3, T <= 4: the paper's evaluation
// patterns (Sec. "Experiments": 2D radii 1, 3, 7; Table 3 fusion depths up to
// 7; the arithmetic-intensity-versus-depth study of Box-2D1R and Star-2D1R).
#include "valu2d_impl.h"

#define V2_DEEP(TS, TC, DT, SH) \
    V2(TS, TC, DT, SH, 1, 5), V2(TS, TC, DT, SH, 1, 6), V2(TS, TC, DT, SH, 1, 7), V2(TS, TC, DT, SH, 1, 8)

namespace stl {
const std::vector<KernelEntry> &valu2d_table_cases()
{
    static const std::vector<KernelEntry> table = {
        V2_DEEP(double, double, STENCIL_F64, STENCIL_BOX), V2_DEEP(double, double, STENCIL_F64, STENCIL_STAR),
        V2_DEEP(float, float, STENCIL_F32, STENCIL_BOX),   V2_DEEP(float, float, STENCIL_F32, STENCIL_STAR),
        // r = 7: box weights streamed from the kernel-argument block (225 of
        // them), the float64 star's 29 in scalar registers
        V2(double, double, STENCIL_F64, STENCIL_BOX, 7, 1), V2(float, float, STENCIL_F32, STENCIL_BOX, 7, 1),
        V2(float, float, STENCIL_F32, STENCIL_STAR, 7, 1), V2(double, double, STENCIL_F64, STENCIL_STAR, 7, 1),
    };
    return table;
}
}  // namespace stl
