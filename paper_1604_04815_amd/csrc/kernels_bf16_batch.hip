// batched (many-array) scan kernels for bf16 inputs: one instantiation per operator and
// compiled tile shape (kept in its own unit so the build runs in parallel).
#include "scan_kernel.hpp"

namespace lscan {

void register_bf16_batch_kernels(KernelTable& t)
{
    fill_row<AddBF16, kModeBatched>(t, kBF16Add);
    fill_row<AddBF16Comp, kModeBatched>(t, kBF16AddComp);
    fill_row<MaxBF16, kModeBatched>(t, kBF16Max);
    fill_row<MinBF16, kModeBatched>(t, kBF16Min);
}

}  // namespace lscan
