// running argmax / argmin kernels (plain scans): int32, int64 and float32
// keys, every compiled tile shape.
#include "scan_kernel.hpp"

namespace lscan {

void register_arg_kernels(KernelTable& t)
{
    fill_row<ArgMaxI32, kModePlain>(t, kI32ArgMax);
    fill_row<ArgMinI32, kModePlain>(t, kI32ArgMin);
    fill_row<ArgMaxI64, kModePlain>(t, kI64ArgMax);
    fill_row<ArgMinI64, kModePlain>(t, kI64ArgMin);
    fill_row<ArgMaxF32, kModePlain>(t, kF32ArgMax);
    fill_row<ArgMinF32, kModePlain>(t, kF32ArgMin);
}

}  // namespace lscan
