// MFMA 3D kernel instances for f32 storage.
#include "mfma3d_impl.h"

namespace stl {
const std::vector<KernelEntry> &mfma3d_table_f32()
{
    static const std::vector<KernelEntry> table = {M3_S(STENCIL_F32)};
    return table;
}
}  // namespace stl
