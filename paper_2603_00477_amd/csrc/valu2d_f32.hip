// VALU 2D kernel instances: float storage, float arithmetic.
#include "valu2d_impl.h"

namespace stl {
const std::vector<KernelEntry> &valu2d_table_f32()
{
    static const std::vector<KernelEntry> table = {V2_S(float, float, STENCIL_F32)};
    return table;
}
}  // namespace stl
