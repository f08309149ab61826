// radix_kernel.hip -- digit counts for the digit offsets of one radix-sort
// pass (a consumer of the scan; the paper names sorting among the uses of
// the scan, Section 1).
//
// The keys are cut into blocks of block_items; count[d][b] is the number of
// keys of block b whose digit (key >> shift) & (2^bits - 1) is d.  Written in
// digit-major order, the exclusive +-scan of that matrix is the digit
// offsets: where block b's first key of digit d lands in a stable partition
// of the keys by digit.  The runtime runs this kernel and then the plain
// single-pass scan (exclusive, int64) over the matrix in place.
//
// One workgroup takes G consecutive blocks: per block, each wave counts into
// its own LDS histogram (LDS atomics), the wave histograms are summed into
// the workgroup's G x 2^bits table, and at the end the table leaves in
// digit-major order, G consecutive counts per digit.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "radix_kernel.hpp"

namespace lscan {

namespace {

constexpr int kHistThreads = 256;
constexpr int kHistWaves = kHistThreads / 64;
constexpr int kMaxDigits = 256;

typedef uint32_t u32x4v __attribute__((ext_vector_type(4)));

template <class K>
__device__ __forceinline__ uint32_t digit_of(K key, int shift, uint32_t mask)
{
    return uint32_t(uint64_t(key) >> shift) & mask;
}

template <class K>
__global__ void __launch_bounds__(kHistThreads) digit_count_kernel(RadixArgs a)
{
    __shared__ uint32_t s_wave_hist[kHistWaves][kMaxDigits];
    extern __shared__ uint32_t s_table[];  // [G][digits]

    const int tid = threadIdx.x;
    const int wave = tid >> 6;
    const int digits = 1 << a.bits;
    const uint32_t mask = uint32_t(digits - 1);
    const int64_t b0 = int64_t(blockIdx.x) * a.group;
    const int64_t gcount = (a.num_blocks - b0 < a.group) ? (a.num_blocks - b0) : a.group;
    const K* keys = static_cast<const K*>(a.keys);
    constexpr int E = 16 / int(sizeof(K));

    for (int d = tid; d < kHistWaves * kMaxDigits; d += kHistThreads) (&s_wave_hist[0][0])[d] = 0;
    __syncthreads();

    for (int64_t g = 0; g < gcount; ++g) {
        const int64_t lo = (b0 + g) * a.block_items;
        const int64_t hi = (lo + a.block_items < a.n) ? lo + a.block_items : a.n;
        uint32_t* hist = s_wave_hist[wave];
        int64_t p = lo;
        if (a.vec_ok) {  // 16-byte vectors over the aligned body of the block
            const int64_t v_end = lo + ((hi - lo) / E) * E;
            const int64_t stride = int64_t(kHistThreads) * E;
            int64_t q = lo + int64_t(tid) * E;
            // four vectors in flight per thread before their counts go to LDS
            for (; q + 3 * stride < v_end; q += 4 * stride) {
                u32x4v w[4];
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    w[u] = __builtin_nontemporal_load(reinterpret_cast<const u32x4v*>(keys + q + u * stride));
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    K k[E];
                    __builtin_memcpy(k, &w[u], 16);
#pragma unroll
                    for (int e = 0; e < E; ++e) atomicAdd(&hist[digit_of(k[e], a.shift, mask)], 1u);
                }
            }
            for (; q < v_end; q += stride) {
                u32x4v w = __builtin_nontemporal_load(reinterpret_cast<const u32x4v*>(keys + q));
                K k[E];
                __builtin_memcpy(k, &w, 16);
#pragma unroll
                for (int e = 0; e < E; ++e) atomicAdd(&hist[digit_of(k[e], a.shift, mask)], 1u);
            }
            p = v_end;
        }
        for (int64_t q = p + tid; q < hi; q += kHistThreads) atomicAdd(&hist[digit_of(keys[q], a.shift, mask)], 1u);
        __syncthreads();
        for (int d = tid; d < digits; d += kHistThreads) {
            uint32_t c = 0;
#pragma unroll
            for (int w = 0; w < kHistWaves; ++w) {
                c += s_wave_hist[w][d];
                s_wave_hist[w][d] = 0;
            }
            s_table[g * digits + d] = c;
        }
        __syncthreads();
    }

    // digit-major: for each digit, the G counts of this group's blocks
    for (int64_t t = tid; t < int64_t(digits) * gcount; t += kHistThreads) {
        const int64_t d = t / gcount, g = t - d * gcount;
        a.counts[d * a.num_blocks + b0 + g] = int64_t(s_table[g * digits + d]);
    }
}

}  // namespace

hipError_t launch_digit_counts(const RadixArgs& a, hipStream_t stream)
{
    const int64_t groups = (a.num_blocks + a.group - 1) / a.group;
    const size_t table_bytes = size_t(a.group) * size_t(1 << a.bits) * sizeof(uint32_t);
    (void)hipGetLastError();
    if (a.key_bytes == 4)
        hipLaunchKernelGGL(digit_count_kernel<uint32_t>, dim3(unsigned(groups)), dim3(kHistThreads), table_bytes,
                           stream, a);
    else
        hipLaunchKernelGGL(digit_count_kernel<uint64_t>, dim3(unsigned(groups)), dim3(kHistThreads), table_bytes,
                           stream, a);
    return hipGetLastError();
}

}  // namespace lscan
