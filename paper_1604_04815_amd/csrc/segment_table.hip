// segment_table.hip -- the first segment of every data block of a segmented
// scan, computed for all blocks at once before the scan (one thread per block,
// a binary search through the offsets each), so that the scan reads two table
// entries per block instead of running a chain of dependent searches.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernel_table.hpp"

namespace lscan {

namespace {

constexpr int kTableThreads = 256;

// first[i] = the first k in [0, S) with off[k] >= i * L - ph (S if none),
// for i = 0 .. M: block i starts i * L positions after a grid that begins
// ph elements before x.
__global__ void __launch_bounds__(kTableThreads)
segment_table_kernel(const int64_t* off, int64_t S, int64_t L, int64_t M, int64_t ph, int64_t* first)
{
    const int64_t i = int64_t(blockIdx.x) * kTableThreads + threadIdx.x;
    if (i > M) return;
    const int64_t v = i * L - ph;
    int64_t lo = 0, hi = S;
    while (lo < hi) {
        const int64_t mid = lo + ((hi - lo) >> 1);
        if (off[mid] < v)
            lo = mid + 1;
        else
            hi = mid;
    }
    first[i] = lo;
}

}  // namespace

hipError_t launch_segment_table(const ScanArgs& a, int64_t tile_elems, hipStream_t stream)
{
    const int64_t entries = a.num_blocks + 1;
    const int64_t grid = (entries + kTableThreads - 1) / kTableThreads;
    (void)hipGetLastError();
    hipLaunchKernelGGL(segment_table_kernel, dim3(unsigned(grid)), dim3(kTableThreads), 0, stream, a.offsets,
                       a.num_segments, tile_elems, a.num_blocks, int64_t(a.phase), const_cast<int64_t*>(a.seg_first));
    return hipGetLastError();
}

}  // namespace lscan
