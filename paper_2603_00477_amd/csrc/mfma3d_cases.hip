// MFMA 3D kernel instance with composite radius 7: the paper's Table 3 case
// Box-3D1R fused 7 deep, float (Sec. "Analytical Criteria Verification").
// Periodic grids only: no fused VALU kernel of that depth exists for the
// Dirichlet band fix-up.
#include "mfma3d_impl.h"

namespace stl {
const std::vector<KernelEntry> &mfma3d_table_cases()
{
    static const std::vector<KernelEntry> table = {M3(STENCIL_F32, STENCIL_BOX, 1, 7)};
    return table;
}
}  // namespace stl
