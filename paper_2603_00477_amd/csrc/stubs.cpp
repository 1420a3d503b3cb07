// Registries of kernel families that are not built yet.
#include "internal.h"

namespace stl {
const std::vector<KernelEntry> &mfma2d_kernels()
{
    static const std::vector<KernelEntry> t;
    return t;
}
const std::vector<KernelEntry> &mfma3d_kernels()
{
    static const std::vector<KernelEntry> t;
    return t;
}
void mfma_build_fragments(int, int, int, const double *, int, int, std::vector<uint8_t> *hi,
                          std::vector<uint8_t> *lo)
{
    hi->clear();
    lo->clear();
}
}  // namespace stl
