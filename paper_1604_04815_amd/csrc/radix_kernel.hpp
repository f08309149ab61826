// radix_kernel.hpp -- arguments of the digit-count kernel (the first half of
// lscan_radix_offsets; the second half is the exclusive scan of its counts).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lscan {

struct RadixArgs {
    const void* keys;      // n keys of key_bytes (unsigned bit patterns)
    int64_t n;
    int64_t block_items;   // keys per block
    int64_t num_blocks;    // M = ceil(n / block_items)
    int64_t group;         // blocks per workgroup (G)
    int64_t* counts;       // 2^bits x M, digit-major
    int32_t key_bytes;     // 4 or 8
    int32_t shift;         // digit = (key >> shift) & (2^bits - 1)
    int32_t bits;          // 1 .. 8
    int32_t vec_ok;        // keys 16-byte aligned and block_items a multiple of 16 / key_bytes
};

// Enqueue the digit-count kernel; G * 2^bits * 4 bytes of LDS per workgroup.
hipError_t launch_digit_counts(const RadixArgs& a, hipStream_t stream);

}  // namespace lscan
