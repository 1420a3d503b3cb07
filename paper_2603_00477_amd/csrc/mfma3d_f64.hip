// MFMA 3D kernel instances for f64 storage.
#include "mfma3d_impl.h"

namespace stl {
const std::vector<KernelEntry> &mfma3d_table_f64()
{
    static const std::vector<KernelEntry> table = {M3_S(STENCIL_F64)};
    return table;
}
}  // namespace stl
