// MFMA 2D kernel instances for bf16 storage.
#include "mfma2d_impl.h"

namespace stl {
const std::vector<KernelEntry> &mfma2d_table_bf16()
{
    static const std::vector<KernelEntry> table = {M2_S(STENCIL_BF16)};
    return table;
}
}  // namespace stl
