// MFMA 2D kernel instances on 2:4 structured-sparse instructions: bf16 and
// f16 storage, float32 accumulation, composite radius <= 7.
#include "mfma2d_impl.h"

namespace stl {
const std::vector<KernelEntry> &mfma2d_table_sparse()
{
    static const std::vector<KernelEntry> table = {
        M2SP_S(STENCIL_BF16, STENCIL_BOX), M2SP_S(STENCIL_BF16, STENCIL_STAR),
        M2SP_S(STENCIL_F16, STENCIL_BOX), M2SP_S(STENCIL_F16, STENCIL_STAR)};
    return table;
}
}  // namespace stl
