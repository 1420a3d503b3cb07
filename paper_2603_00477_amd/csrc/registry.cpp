// Registry of all kernel tables, and tables of families not built yet.
#include "internal.h"

namespace stl {
const std::vector<KernelEntry> &mfma3d_kernels()
{
    static const std::vector<KernelEntry> t;
    return t;
}

std::vector<const std::vector<KernelEntry> *> all_kernel_tables()
{
    return {&valu2d_table_f64(),  &valu2d_table_f32(),  &valu2d_table_bf16(),
            &valu2d_table_f16(),  &valu2d_table_x3(),   &valu3d_kernels(),    &mfma2d_table_f64(),
            &mfma2d_table_f32(),  &mfma2d_table_bf16(), &mfma2d_table_f16(),
            &mfma2d_table_x3(),   &mfma3d_kernels(),    &generic_kernels()};
}
}  // namespace stl
