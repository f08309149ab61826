// segmented scan kernels for bf16 inputs: one instantiation per operator and
// compiled tile shape (kept in its own unit so the build runs in parallel).
#include "scan_kernel.hpp"

namespace lscan {

void register_bf16_seg_kernels(KernelTable& t)
{
    fill_row<AddBF16, kModeSegmented>(t, kBF16Add);
    fill_row<AddBF16Comp, kModeSegmented>(t, kBF16AddComp);
    fill_row<MaxBF16, kModeSegmented>(t, kBF16Max);
    fill_row<MinBF16, kModeSegmented>(t, kBF16Min);
}

}  // namespace lscan
