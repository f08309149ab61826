// plain scan kernels for bf16 inputs: one instantiation per operator and
// compiled tile shape (kept in its own unit so the build runs in parallel).
#include "scan_kernel.hpp"

namespace lscan {

void register_bf16_kernels(KernelTable& t)
{
    fill_row<AddBF16, kModePlain>(t, kBF16Add);
    fill_row<AddBF16Comp, kModePlain>(t, kBF16AddComp);
    fill_row<MaxBF16, kModePlain>(t, kBF16Max);
    fill_row<MinBF16, kModePlain>(t, kBF16Min);
}

}  // namespace lscan
