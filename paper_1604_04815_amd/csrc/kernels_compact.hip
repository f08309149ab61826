// stream-compaction kernels: 4-byte items (int32 and float32 bits) and 8-byte
// items (int64), every compiled tile shape.  The compaction rows of the
// kernel table use the add opcodes of the item width.
#include "compact_kernel.hpp"

namespace lscan {

void register_compact_kernels(KernelTable& t)
{
    fill_compact_row<uint32_t>(t, kI32Add);
    fill_compact_row<uint64_t>(t, kI64Add);
}

}  // namespace lscan
