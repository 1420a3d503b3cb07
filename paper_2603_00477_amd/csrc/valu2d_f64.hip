// VALU 2D kernel instances: double storage, double arithmetic.
#include "valu2d_impl.h"

namespace stl {
const std::vector<KernelEntry> &valu2d_table_f64()
{
    static const std::vector<KernelEntry> table = {V2_S(double, double, STENCIL_F64)};
    return table;
}
}  // namespace stl
