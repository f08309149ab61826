// batched (many-array) scan kernels for i64 inputs: one instantiation per operator and
// compiled tile shape (kept in its own unit so the build runs in parallel).
#include "scan_kernel.hpp"

namespace lscan {

void register_i64_batch_kernels(KernelTable& t)
{
    fill_row<AddI64, kModeBatched>(t, kI64Add);
    fill_row<MaxI64, kModeBatched>(t, kI64Max);
    fill_row<MinI64, kModeBatched>(t, kI64Min);
}

}  // namespace lscan
