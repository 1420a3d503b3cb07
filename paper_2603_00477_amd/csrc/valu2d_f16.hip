// VALU 2D kernel instances: __half storage, float arithmetic.
#include "valu2d_impl.h"

namespace stl {
const std::vector<KernelEntry> &valu2d_table_f16()
{
    static const std::vector<KernelEntry> table = {V2_S(__half, float, STENCIL_F16)};
    return table;
}
}  // namespace stl
