// MFMA 2D kernel instances with composite radius 7: the paper's Table 3
// cases Box-2D1R fused 7 deep and Box-2D7R (Sec. "Analytical Criteria
// Verification"), and the 16-bit Box-2D1R fused 7 deep, the dense side of
// the dense-versus-sparse comparison of Table 4; star composites of radius 7.
#include "mfma2d_impl.h"

namespace stl {
const std::vector<KernelEntry> &mfma2d_table_cases()
{
    static const std::vector<KernelEntry> table = {
        M2(STENCIL_F32, STENCIL_BOX, 1, 7), M2(STENCIL_F32, STENCIL_BOX, 7, 1),
        M2(STENCIL_F64, STENCIL_BOX, 1, 7), M2(STENCIL_F64, STENCIL_BOX, 7, 1),
        M2(STENCIL_BF16, STENCIL_BOX, 1, 7), M2(STENCIL_F16, STENCIL_BOX, 1, 7),
        // the paper's star patterns of radius 7 (Sec. "Experiments")
        M2(STENCIL_F32, STENCIL_STAR, 7, 1), M2(STENCIL_F64, STENCIL_STAR, 7, 1),
        M2(STENCIL_F32, STENCIL_STAR, 1, 7), M2(STENCIL_F64, STENCIL_STAR, 1, 7),
    };
    return table;
}
}  // namespace stl
