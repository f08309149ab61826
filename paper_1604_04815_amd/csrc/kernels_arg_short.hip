// running argmax / argmin kernels with a 32-bit index (arrays of fewer than
// 2^31 elements): int32, int64 and float32 keys, every compiled tile shape.
#include "scan_kernel.hpp"

namespace lscan {

void register_arg_short_kernels(KernelTable& t)
{
    static_assert(kI32ArgMaxS - kI32ArgMax == kArgShortOffset && kF32ArgMinS - kF32ArgMin == kArgShortOffset,
                  "short-index rows follow the wide ones");
    fill_row<ArgMaxI32S, kModePlain>(t, kI32ArgMaxS);
    fill_row<ArgMinI32S, kModePlain>(t, kI32ArgMinS);
    fill_row<ArgMaxI64S, kModePlain>(t, kI64ArgMaxS);
    fill_row<ArgMinI64S, kModePlain>(t, kI64ArgMinS);
    fill_row<ArgMaxF32S, kModePlain>(t, kF32ArgMaxS);
    fill_row<ArgMinF32S, kModePlain>(t, kF32ArgMinS);
}

}  // namespace lscan
