// MFMA 2D kernel instances with composite radius 7: the paper's Table 3
// cases Box-2D1R fused 7 deep and Box-2D7R (Sec. "Analytical Criteria
// Verification").
#include "mfma2d_impl.h"

namespace stl {
const std::vector<KernelEntry> &mfma2d_table_cases()
{
    static const std::vector<KernelEntry> table = {
        M2(STENCIL_F32, STENCIL_BOX, 1, 7), M2(STENCIL_F32, STENCIL_BOX, 7, 1),
        M2(STENCIL_F64, STENCIL_BOX, 1, 7), M2(STENCIL_F64, STENCIL_BOX, 7, 1),
    };
    return table;
}
}  // namespace stl
