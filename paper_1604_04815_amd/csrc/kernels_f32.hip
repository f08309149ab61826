// plain scan kernels for f32 inputs: one instantiation per operator and
// compiled tile shape (kept in its own unit so the build runs in parallel).
#include "scan_kernel.hpp"

namespace lscan {

void register_f32_kernels(KernelTable& t)
{
    fill_row<AddF32, kModePlain>(t, kF32Add);
    fill_row<AddF32Comp, kModePlain>(t, kF32AddComp);
    fill_row<MaxF32, kModePlain>(t, kF32Max);
    fill_row<MinF32, kModePlain>(t, kF32Min);
}

}  // namespace lscan
