// VALU 2D kernel instances: float storage, double arithmetic.
#include "valu2d_impl.h"

namespace stl {
const std::vector<KernelEntry> &valu2d_table_x3()
{
    static const std::vector<KernelEntry> table = {V2_S(float, double, STENCIL_F32_BF16X3)};
    return table;
}
}  // namespace stl
