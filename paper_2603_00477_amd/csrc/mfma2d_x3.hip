// MFMA 2D kernel instances for x3 storage.
#include "mfma2d_impl.h"

namespace stl {
const std::vector<KernelEntry> &mfma2d_table_x3()
{
    static const std::vector<KernelEntry> table = {M2_S(STENCIL_F32_BF16X3)};
    return table;
}
}  // namespace stl
