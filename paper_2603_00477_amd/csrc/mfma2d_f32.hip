// MFMA 2D kernel instances for f32 storage.
#include "mfma2d_impl.h"

namespace stl {
const std::vector<KernelEntry> &mfma2d_table_f32()
{
    static const std::vector<KernelEntry> table = {M2_S(STENCIL_F32)};
    return table;
}
}  // namespace stl
