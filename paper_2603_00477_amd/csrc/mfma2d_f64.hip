// MFMA 2D kernel instances for f64 storage.
#include "mfma2d_impl.h"

namespace stl {
const std::vector<KernelEntry> &mfma2d_table_f64()
{
    static const std::vector<KernelEntry> table = {M2_S(STENCIL_F64)};
    return table;
}
}  // namespace stl
