// kernel_table.hpp -- what the host runtime knows about each compiled scan
// kernel.  Shared by the runtime and the kernel instantiation units only.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lscan {

// One array of a batched launch (device-side descriptor).  Array r owns data
// blocks [first_block, first_block + ceil((n + max(phase, 0)) / L)); the table ends with a
// sentinel whose first_block is the total block count M.
struct BatchArray {
    const void* x;
    void* y;
    int64_t n;
    int64_t first_block;
    int64_t phase;    // -1: element path; else x sits this many elements past a vector
                      // boundary and the array's blocks cover n + phase positions
    int64_t stage_y;  // 1: y sits at another phase than x; rows read as vectors are
                      // written through the LDS stage as aligned vectors
};

// Kernel flavours: one array; one array cut into segments by offsets (heads
// inside blocks); many arrays, each starting on a block boundary; stream
// compaction (a scan of keep flags driving a scatter).
enum ScanMode : int { kModePlain = 0, kModeSegmented = 1, kModeBatched = 2, kModeCompact = 3 };
constexpr int kNumModes = 4;

// Arguments of one persistent scan launch.
struct ScanArgs {
    const void* x;            // input, n elements
    void* y;                  // output, n elements (may equal x)
    int64_t n;                // N
    int64_t num_blocks;       // M = ceil(N / L)
    const int64_t* offsets;   // segmented: S + 1 offsets (device), else null
    int64_t num_segments;     // S
    const BatchArray* arrays; // batched: num_arrays + 1 descriptors (device), else null
    int64_t num_arrays;
    uint64_t* slots;          // M * slot_words flag words (epoch tag | data)
    uint32_t* ctrl;           // [0] last epoch tag, [1] exit counter, [2] timeout flag,
                              // [3] tag of the last launch that gave up a wait,
                              // [4] residency arrivals, [5] residency failure, [6] residency exits
    uint64_t spin_limit;      // wall-clock ticks one wait may last
    int32_t exclusive;        // 1: exclusive scan
    int32_t vec_ok;           // 1: full blocks read x with full-width vectors
    int32_t phase;            // plain and segmented scans: x sits this many elements past a vector
                              // boundary (the block grid is shifted by it; 0 when aligned)
    int32_t store_vec;        // plain and segmented scans: 1 when y sits at the same phase, so full
                              // blocks also write vectors directly (else through an LDS stage, or
                              // element by element for 32-byte output vectors)
    int32_t residency_check;  // 1: only test that all workgroups are resident at once, then exit
    int32_t chain;            // 1: the paper's prefix chain (block i waits for P(i - 1))
    uint32_t* status_host;    // optional host-visible word that also receives the timeout flag
    const uint8_t* keep;      // compaction: one keep byte per item (null: keep non-zero items)
    int64_t* count;           // compaction: receives the number of kept items (device)
    const int64_t* seg_first; // segmented: M + 1 entries, the first segment whose offset is at
                              // or past block i's start (null: the kernel searches the offsets)
};

using LaunchFn = hipError_t (*)(const ScanArgs&, int grid, hipStream_t);

// Segmented scans: fill a.seg_first (M + 1 entries) from the offsets for
// blocks of tile_elems elements, before the scan on the same stream.
hipError_t launch_segment_table(const ScanArgs& a, int64_t tile_elems, hipStream_t stream);

// Layout tag of KernelEntry and ScanArgs: a kernel instantiated by a
// caller's library (lscan_custom.hpp) is refused unless it was built with
// the same layout as the runtime.  High half: a fixed mark; then the size
// of ScanArgs; low nibble: a revision for same-size layout changes.
constexpr uint32_t kKernelAbiMark = 0x4C530000u;
constexpr uint32_t kKernelAbi = kKernelAbiMark | (uint32_t(sizeof(ScanArgs)) << 4) | 3u;
static_assert(sizeof(ScanArgs) < 4096, "the size of ScanArgs fits the tag");

struct KernelEntry {
    uint32_t abi;             // kKernelAbi of the headers the kernel was built with
    const void* func;         // the __global__ function (occupancy queries)
    LaunchFn launch;
    int32_t block_threads;    // T
    int32_t vectors_per_lane; // vector loads per lane per data block
    int32_t elems_per_vec;    // elements per lane per vector load
    int32_t slot_words;       // 64-bit flag words per data block
    int32_t in_bytes;         // sizeof input element
    int32_t out_bytes;        // sizeof output element
    int64_t tile_elems;       // L
};

// Operator codes (dtype x operator x precision).
enum OpCode : int {
    kI32Add = 0, kI32Max, kI32Min,
    kI64Add, kI64Max, kI64Min,
    kF32Add, kF32AddComp, kF32Max, kF32Min,
    kBF16Add, kBF16AddComp, kBF16Max, kBF16Min,
    kI32ArgMax, kI32ArgMin, kI64ArgMax, kI64ArgMin, kF32ArgMax, kF32ArgMin,  // plain scans only
    // the same with a 32-bit index, for arrays of fewer than 2^31 elements
    kI32ArgMaxS, kI32ArgMinS, kI64ArgMaxS, kI64ArgMinS, kF32ArgMaxS, kF32ArgMinS,
    kNumOpCodes
};

// Compiled tile shapes (T, vectors per lane).
constexpr int kNumShapes = 10;
constexpr int kArgShortOffset = 6;  // kI32ArgMaxS - kI32ArgMax
constexpr int kShapeThreads[kNumShapes] = {256, 512, 512, 256, 1024, 1024, 512, 256, 256, 1024};
constexpr int kShapeVectors[kNumShapes] = {8, 8, 4, 16, 4, 2, 2, 4, 2, 1};

// table[mode][opcode][shape]
using KernelTable = KernelEntry[kNumModes][kNumOpCodes][kNumShapes];

void register_i32_kernels(KernelTable& t);
void register_i64_kernels(KernelTable& t);
void register_f32_kernels(KernelTable& t);
void register_bf16_kernels(KernelTable& t);
void register_i32_seg_kernels(KernelTable& t);
void register_i64_seg_kernels(KernelTable& t);
void register_f32_seg_kernels(KernelTable& t);
void register_bf16_seg_kernels(KernelTable& t);
void register_i32_batch_kernels(KernelTable& t);
void register_i64_batch_kernels(KernelTable& t);
void register_f32_batch_kernels(KernelTable& t);
void register_bf16_batch_kernels(KernelTable& t);
void register_compact_kernels(KernelTable& t);
void register_arg_kernels(KernelTable& t);
void register_arg_short_kernels(KernelTable& t);

}  // namespace lscan
