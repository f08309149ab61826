// plain scan kernels for i32 inputs: one instantiation per operator and
// compiled tile shape (kept in its own unit so the build runs in parallel).
#include "scan_kernel.hpp"

namespace lscan {

void register_i32_kernels(KernelTable& t)
{
    fill_row<AddI32, kModePlain>(t, kI32Add);
    fill_row<MaxI32, kModePlain>(t, kI32Max);
    fill_row<MinI32, kModePlain>(t, kI32Min);
}

}  // namespace lscan
