// VALU 2D kernel instances: __hip_bfloat16 storage, float arithmetic.
#include "valu2d_impl.h"

namespace stl {
const std::vector<KernelEntry> &valu2d_table_bf16()
{
    static const std::vector<KernelEntry> table = {V2_S(__hip_bfloat16, float, STENCIL_BF16)};
    return table;
}
}  // namespace stl
