// scan_kernel.hpp -- the persistent single-pass scan kernel for gfx950.
//
// Method (paper, Section 4, restated for CDNA4):
//   * The input is cut into M data blocks of L = T * R * E elements.  A fixed
//     grid of B resident workgroups takes the blocks round-robin: block i is
//     processed by workgroup i mod B, in increasing i (Section 4, cyclic
//     distribution; no atomic ticket decides the order).
//   * Per block, each lane loads R vectors of E consecutive elements; wave w
//     owns R consecutive "rows" of 64 * E elements, so every vector load of a
//     wave reads one contiguous span (coalesced, each x read once).
//   * Intra-wave local scan (Algorithm 2): a sequential scan of each lane's E
//     elements, a wave64 cross-lane scan of the lane totals per row (DPP, in
//     place of warp shuffles), and the rows chained through their totals.
//   * Intra-block local scan (Algorithm 3): wave totals go through LDS; wave
//     0 folds them into the block aggregate A(i); every wave folds the totals
//     of the waves before it.
//   * Inter-block communication (Algorithm 4), re-designed: A(i) is published
//     at once in a flag slot (epoch tag and data in one 64-bit word per 32
//     data bits, written with a device-scope atomic store, so one store is
//     one indivisible update, as the paper requires of its (u, v) pair).  A
//     workgroup already holds P(i - B), the inclusive prefix through its own
//     previous block, so it obtains
//         P(i - 1) = P(i - B) (+) A(i - B + 1) (+) ... (+) A(i - 1)
//     from the aggregates of the B - 1 blocks in between, read 64 slots per
//     wave load, without waiting for any other workgroup's prefix.  The
//     serial prefix chain of the paper (one cross-workgroup hop per block)
//     becomes one hop per block plus a chain of M / B steps that stays inside
//     each workgroup, and the association is fixed, so float results are
//     deterministic for a given (T, R, B).  The paper's chain itself is
//     kept as a launch option (ScanArgs::chain): block i waits for the
//     inclusive prefix P(i - 1) that block i - 1 published, then publishes
//     P(i).
//   * Software pipeline: a block's prefix is resolved one round late.  Each
//     step loads and scans block i and publishes A(i) before it waits for
//     anything, then folds the window of the previous block i - B (whose
//     aggregates were published a round earlier) and stores block i - B;
//     block i waits in registers as block-local values.  The flag words of
//     that window were copied into LDS at the end of the previous step, so
//     their round trip through the memory system overlaps a whole step, and
//     the next full block of the workgroup is prefetched into LDS while the
//     current one is scanned.  The last step, which only drains the pending
//     block, is a separate instantiation so that inside the loop every load
//     is consumed on every path.
//   * Intra-block global scan (Algorithm 5): each element becomes
//     (P(i - 1) (+) (wave prefix (+) row prefix (+) lane prefix)) (+) its
//     in-lane scan value -- the block prefix joins each lane-row once, then
//     its elements -- and is stored once, coalesced.
//
// Forward progress: all B workgroups must be resident at once (Section 5.1
// notes the deadlock otherwise); the host caps B by the occupancy limit and
// by a co-residency test run in this kernel (check_residency).  A wait that
// outlasts spin_limit raises a timeout flag and the workgroup stops; the
// others see the launch's tag in the abort word and stop waiting too, so
// every wave always exits.
#pragma once

#include <type_traits>

#include "kernel_table.hpp"
#include "scan_ops.hpp"

namespace lscan {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

// Streaming vector access (non-temporal: each byte is touched once).
template <class T, int E>
__device__ __forceinline__ void load_vector(const T* p, T (&out)[E])
{
    constexpr int kBytes = int(sizeof(T)) * E;
    static_assert(kBytes == 16 || kBytes == 8, "16- or 8-byte vectors");
    if constexpr (kBytes == 16) {
        u32x4 w = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(p));
        __builtin_memcpy(out, &w, 16);
    } else {
        u32x2 w = __builtin_nontemporal_load(reinterpret_cast<const u32x2*>(p));
        __builtin_memcpy(out, &w, 8);
    }
}

template <class T, int E>
__device__ __forceinline__ void store_vector(T* p, const T (&v)[E])
{
    constexpr int kBytes = int(sizeof(T)) * E;
    static_assert(kBytes == 16 || kBytes == 32, "16- or 32-byte output vectors");
    u32x4 w[kBytes / 16];
    __builtin_memcpy(w, v, kBytes);
#pragma unroll
    for (int h = 0; h < kBytes / 16; ++h) __builtin_nontemporal_store(w[h], reinterpret_cast<u32x4*>(p) + h);
}

// Lanes of one wave exchange values through LDS: every lane's LDS writes
// before this point are visible to every lane's reads after it.  The wave
// barrier alone orders only the instructions; the wavefront-scope fences
// order the memory accesses themselves.
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ---------------------------------------------------------------------------
// Next-block prefetch into LDS.  gfx950 loads 16 bytes per lane from global
// memory straight into LDS (lane l's bytes land at M0 + 16 * l), with no
// register held while the load is in flight.  The load is issued from inline
// assembly so that the compiler, which does not track which LDS bytes such a
// load writes, does not wait for it before every later LDS read; the kernel
// places the waits itself: all vector memory operations drained (vmcnt(0))
// before the prefetched rows are read, and the reads completed (lgkmcnt(0))
// before the next prefetch overwrites them.  No VGPR is written by the load,
// and the address registers are read when it issues.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t lds_address(const void* p)
{
    return static_cast<uint32_t>(reinterpret_cast<uintptr_t>((const __attribute__((address_space(3))) char*)p));
}
__device__ __forceinline__ void lds_load16(const void* g, uint32_t lds_byte)
{
    const uint32_t m0 = __builtin_amdgcn_readfirstlane(lds_byte);
    asm volatile("s_mov_b32 m0, %1\n\tglobal_load_lds_dwordx4 %0, off nt" ::"v"(g), "s"(m0) : "memory");
}

// The same load with the cache policy of agent-scope atomic loads (sc1): flag
// words published by workgroups on other XCDs are read from where those
// writes land, never from a stale line of this XCD's L2.
__device__ __forceinline__ void lds_load16_coherent(const void* g, uint32_t lds_byte)
{
    const uint32_t m0 = __builtin_amdgcn_readfirstlane(lds_byte);
    asm volatile("s_mov_b32 m0, %1\n\tglobal_load_lds_dwordx4 %0, off sc1" ::"v"(g), "s"(m0) : "memory");
}

__device__ __forceinline__ void vmem_drain() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }
// Wait until at most N vector memory operations of the wave are outstanding.
// They complete in issue order, so with N stores issued after a prefetch this
// waits for the prefetch (and everything before it) but not for those stores.
template <int N>
__device__ __forceinline__ void vmem_wait_keep()
{
    static_assert(N >= 0 && N < 64, "vmcnt range");
    asm volatile("s_waitcnt vmcnt(%0)" ::"n"(N) : "memory");
}
// Make the compiler complete the loads that produced v here (it must have
// the value in registers before the empty statement), so that its waits
// for them stay on the path that issued them.
template <class T, int N>
__device__ __forceinline__ void complete_loads(T (&v)[N])
{
    static_assert(sizeof(T) * N == 16 || sizeof(T) * N == 8, "one 8- or 16-byte lane vector");
    if constexpr (sizeof(T) * N == 16) {
        u32x4 w;
        __builtin_memcpy(&w, v, 16);
        asm volatile("" : "+v"(w));
        __builtin_memcpy(v, &w, 16);
    } else {
        u32x2 w;
        __builtin_memcpy(&w, v, 8);
        asm volatile("" : "+v"(w));
        __builtin_memcpy(v, &w, 8);
    }
}
__device__ __forceinline__ void lds_reads_drain() { asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory"); }

// ---------------------------------------------------------------------------
// Lane-blocked rows.  Operators whose combine is expensive (the compensated
// sums) give each lane R consecutive 16-byte vectors of the block instead of
// one vector per wave-row: a lane then scans R * E consecutive elements in
// registers and the wave needs one cross-lane scan per block instead of one
// per row.  The loads still read whole 1 KiB spans (into LDS), and the
// outputs go back through LDS to leave as 1 KiB spans too.  Within a wave's
// LDS rows, chunk c (16 bytes, in memory order) sits in slot lds_slot(c): a
// permutation inside each aligned group of 64 chunks under which the
// lane-blocked accesses (chunks 4l .. 4l + 3 of lane l) and the striped ones
// (chunk 64r + l) both run without bank conflicts (measured: 16-byte reads
// are served 16 lanes at a time, writes 8 at a time; the blocked accesses
// without the permutation take 4 times the LDS cycles).  lds_chunk inverts it.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int lds_slot(int c)
{
    return c ^ (((c >> 4) & 1) | (((c >> 3) & 1) << 1) | (((c >> 5) & 1) << 3));
}
__device__ __forceinline__ int lds_chunk(int s)
{
    return s ^ (((s >> 4) & 1) | ((((s >> 3) ^ (s >> 5)) & 1) << 1) | (((s >> 5) & 1) << 3));
}
// The lane id as a value the compiler cannot see through: slots computed from
// it where they are used are not hoisted out of the block loop, where they
// would hold registers across it (the compensated kernels at 1024 x 4 spilled
// them, and every reload inside the loop then waited for the prefetch too).
__device__ __forceinline__ int opaque_lane()
{
    int l = static_cast<int>(threadIdx.x & 63u);
    asm volatile("" : "+v"(l));
    return l;
}

// Segmented scans of sums take lane-blocked rows too (a zero input word, which
// partial blocks hold outside the array, lifts to the identity of a sum).
template <class Op>
struct blocked_segmented : std::false_type {};
template <>
struct blocked_segmented<AddI32> : std::true_type {};
template <>
struct blocked_segmented<AddI64> : std::true_type {};
template <>
struct blocked_segmented<AddF32> : std::true_type {};
template <>
struct blocked_segmented<AddF32Comp> : std::true_type {};
template <class F>
struct blocked_segmented<FromBF16<F>> : blocked_segmented<F> {};

// ---------------------------------------------------------------------------
// Flag slots: one 64-bit word per 32 bits of payload, (tag << 32) | data.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t slot_load(const uint64_t* p)
{
    return __hip_atomic_load(const_cast<uint64_t*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void slot_store(uint64_t* p, uint64_t w)
{
    __hip_atomic_store(p, w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Lanes 0 .. W-1 each publish one word of the (wave-uniform) value v.
template <class V>
__device__ __forceinline__ void publish_slot(uint64_t* slot, const V& v, uint32_t tag, int lane)
{
    constexpr int W = sizeof(V) / 4;
    uint32_t w[W];
    __builtin_memcpy(w, &v, sizeof(V));
    if (lane < W) {
        uint32_t mine = w[0];
#pragma unroll
        for (int k = 1; k < W; ++k) mine = (lane == k) ? w[k] : mine;
        slot_store(slot + lane, (uint64_t(tag) << 32) | mine);
    }
}

// Re-read a flag word until it carries this launch's tag, or give up
// (ok = false) after `limit` wall-clock ticks or as soon as another
// workgroup of this launch has given up (*abort_word == tag), so one timeout
// does not turn into a cascade of waits for values that never come.
__device__ __forceinline__ uint64_t await_word(const uint64_t* p, uint64_t w, uint32_t tag,
                                               uint64_t limit, const uint32_t* abort_word, bool& ok)
{
    if (uint32_t(w >> 32) == tag || !ok) return w;
    const uint64_t t0 = wall_clock64();
    do {
        __builtin_amdgcn_s_sleep(1);
        w = slot_load(p);
        if (uint32_t(w >> 32) == tag) return w;
        if (__hip_atomic_load(const_cast<uint32_t*>(abort_word), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == tag)
            break;
    } while (wall_clock64() - t0 < limit);
    ok = false;
    return w;
}

// Fold of the aggregates in slots [lo, lo + cnt) in index order, read by one
// wave: 64 consecutive slots per load round, each round reduced with the
// cross-lane scan (a fixed tree), rounds folded left to right.
// first(j, k) gives the first reading of word k of window slot j (the
// flag word itself, or a copy fetched earlier); words not yet published are
// re-read from the slots.  QC rounds of 64 slots are read at once (8 KiB of
// flag words from global memory, 4 KiB from an LDS copy).
template <class Op, int QC, class First>
__device__ typename Op::V window_fold_from(First first, const uint64_t* slots, int64_t lo, int64_t cnt,
                                           uint32_t tag, uint64_t limit, const uint32_t* abort_word, int lane,
                                           bool& ok)
{
    using V = typename Op::V;
    constexpr int W = sizeof(V) / 4;
    V acc = Op::identity();
    for (int64_t q0 = 0; q0 < cnt; q0 += 64 * QC) {
        uint64_t w[QC][W];
#pragma unroll
        for (int q = 0; q < QC; ++q) {
            const int64_t j = q0 + 64 * q + lane;
#pragma unroll
            for (int k = 0; k < W; ++k) w[q][k] = (j < cnt) ? first(j, k) : (uint64_t(tag) << 32);
        }
#pragma unroll
        for (int q = 0; q < QC; ++q) {
            const int64_t j = q0 + 64 * q + lane;
            if (j < cnt) {
#pragma unroll
                for (int k = 0; k < W; ++k)
                    w[q][k] = await_word(slots + (lo + j) * W + k, w[q][k], tag, limit, abort_word, ok);
            }
        }
#pragma unroll
        for (int q = 0; q < QC; ++q) {
            if (q0 + 64 * q < cnt) {
                const int64_t j = q0 + 64 * q + lane;
                V v = Op::identity();
                if (j < cnt) {
                    uint32_t d[W];
#pragma unroll
                    for (int k = 0; k < W; ++k) d[k] = uint32_t(w[q][k]);
                    __builtin_memcpy(&v, d, sizeof(V));
                }
                const V s = wave_inclusive_scan<Op>(v);
                acc = Op::combine(acc, read_lane(s, 63));
            }
        }
    }
    return acc;
}
template <class Op>
__device__ typename Op::V window_fold(const uint64_t* slots, int64_t lo, int64_t cnt, uint32_t tag,
                                      uint64_t limit, const uint32_t* abort_word, int lane, bool& ok)
{
    constexpr int W = sizeof(typename Op::V) / 4;
    constexpr int QC = (W == 1) ? 8 : (W == 2) ? 4 : 2;
    auto first = [&](int64_t j, int k) { return slot_load(slots + (lo + j) * W + k); };
    return window_fold_from<Op, QC>(first, slots, lo, cnt, tag, limit, abort_word, lane, ok);
}

// Wave-wide copy of the flag words of slots [lo, lo + cnt) (W words each)
// into LDS at lds_base, in 16-byte loads from the aligned chunk that holds the
// first word (every chunk read lies inside the slot array: it starts 16-byte
// aligned and holds, right after the window, the slot of the block the window
// belongs to).  *shift receives the first word's index in the copy.  Issues
// nothing and returns false when the window needs more than max_chunks loads'
// worth of chunks or the slots are not 16-byte aligned.
template <int W>
__device__ __forceinline__ bool fetch_window_flags(const uint64_t* slots, int64_t lo, int64_t cnt, uint32_t lds_base,
                                                   int64_t max_chunks, int lane, int& shift)
{
    const uintptr_t ab = reinterpret_cast<uintptr_t>(slots + lo * W);
    const int sh = int((ab & 15u) >> 3);
    const int64_t chunks = (int64_t(sh) * 8 + cnt * (W * 8) + 15) >> 4;
    if ((reinterpret_cast<uintptr_t>(slots) & 15u) != 0 || chunks > max_chunks) return false;
    const char* c0 = reinterpret_cast<const char*>(ab - uintptr_t(sh) * 8);
    lds_reads_drain();  // the previous window's words are read
    for (int64_t d = 0; d * 64 < chunks; ++d) {
        const int64_t c = (d * 64 + lane < chunks) ? d * 64 + lane : chunks - 1;
        lds_load16_coherent(c0 + c * 16, lds_base + uint32_t(d) * 1024u);
    }
    shift = sh;
    return true;
}

// The paper's hand-off (Algorithm 4): wait for the inclusive prefix that the
// previous block published in its slot.  Lanes 0 .. W-1 each wait for one
// word; the value is assembled from their lanes.
template <class Op>
__device__ __forceinline__ typename Op::V chain_prefix(const uint64_t* slot, uint32_t tag, uint64_t limit,
                                                       const uint32_t* abort_word, int lane, bool& ok)
{
    using V = typename Op::V;
    constexpr int W = sizeof(V) / 4;
    uint64_t w = uint64_t(tag) << 32;
    if (lane < W) {
        w = slot_load(slot + lane);
        w = await_word(slot + lane, w, tag, limit, abort_word, ok);
    }
    uint32_t d[W];
#pragma unroll
    for (int k = 0; k < W; ++k) d[k] = __builtin_amdgcn_readlane(uint32_t(w), k);
    V v;
    __builtin_memcpy(&v, d, sizeof(V));
    return v;
}

// Read-only data reached through the constant address space: wave-uniform
// loads from it go through the scalar cache and do not queue behind the
// vector loads of the data.
typedef const int64_t __attribute__((address_space(4))) CInt64;
typedef const BatchArray __attribute__((address_space(4))) CBatchArray;

// Up to this many segment heads in a block are matched by a wave-uniform loop;
// more take a per-lane binary search.
constexpr int64_t kFewHeads = 32;

// First index k in [lo, hi) with off[k] >= v, or hi.
__device__ __forceinline__ int64_t lower_bound_i64(const int64_t* off, int64_t lo, int64_t hi, int64_t v)
{
    while (lo < hi) {
        const int64_t mid = lo + ((hi - lo) >> 1);
        if (off[mid] < v)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

// Co-residency test run by the host once per (kernel, grid): every
// workgroup counts itself in and waits, for at most `limit` ticks, until all
// gridDim.x have arrived.  Any workgroup that stops waiting before that sets
// the failure word, so the host learns whether the grid fits on the device
// at once -- the condition the persistent scan needs to make progress.  All
// waves of the workgroup stay alive (at the barrier) until the wait ends, so
// the test occupies exactly what a real launch occupies.  The last workgroup
// out clears the counters.
__device__ __forceinline__ void check_residency(uint32_t* ctrl, uint64_t limit)
{
    const uint32_t grid = gridDim.x;
    if (threadIdx.x == 0) {
        uint32_t seen = __hip_atomic_fetch_add(ctrl + 4, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + 1u;
        if (seen < grid) {
            const uint64_t t0 = wall_clock64();
            do {
                __builtin_amdgcn_s_sleep(2);
                seen = __hip_atomic_load(ctrl + 4, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            } while (seen < grid && wall_clock64() - t0 < limit);
        }
        if (seen < grid) __hip_atomic_store(ctrl + 5, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint32_t out = __hip_atomic_fetch_add(ctrl + 6, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (out == grid - 1u) {
            __hip_atomic_store(ctrl + 4, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(ctrl + 6, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// Operators of each kernel flavour: ElemOp scans the elements of a block,
// BlkOp combines block aggregates and prefixes.  Segmented scans carry head
// flags at both levels; batched scans only at block level, because every
// array starts on a block boundary.
template <class BaseOp, int MODE>
struct ModeOps {
    using ElemOp = BaseOp;
    using BlkOp = BaseOp;
};
template <class BaseOp>
struct ModeOps<BaseOp, kModeSegmented> {
    using ElemOp = Seg<BaseOp>;
    using BlkOp = Seg<BaseOp>;
};
template <class BaseOp>
struct ModeOps<BaseOp, kModeBatched> {
    using ElemOp = BaseOp;
    using BlkOp = Seg<BaseOp>;
};

// Batches of int32 arrays run 512 x 8 with two workgroups per CU, so four
// waves per SIMD: those kernels' registers are held to the 128 that allows
// (the y stage of arrays at another phase would otherwise take them to 129;
// the other types spill at this bound and run other shapes).
template <class BaseOp, int T, int R, int MODE>
constexpr int kMinWavesPerSimd = (MODE == kModeBatched && T == 512 && R == 8 &&
                                  std::is_same<typename BaseOp::In, int32_t>::value &&
                                  sizeof(typename BaseOp::V) == 4) ? 4 : 1;

template <class BaseOp, int T, int R, int MODE>
__global__ void __launch_bounds__(T, (kMinWavesPerSimd<BaseOp, T, R, MODE>)) scan_kernel(ScanArgs a)
{
    using EOp = typename ModeOps<BaseOp, MODE>::ElemOp;
    using BOp = typename ModeOps<BaseOp, MODE>::BlkOp;
    using V = typename EOp::V;    // element-level scan value
    using VB = typename BOp::V;   // block-level value (aggregates, prefixes)
    using In = typename BaseOp::In;
    using Out = typename BaseOp::Out;
    constexpr int E = BaseOp::E;
    constexpr int NWAVE = T / 64;
    constexpr int W = sizeof(VB) / 4;
    constexpr int ROW = 64 * E;                  // elements per wave-row
    constexpr int64_t L = int64_t(T) * R * E;    // elements per data block
    static_assert(T % 64 == 0 && NWAVE <= 16, "wave64 workgroups of up to 1024 threads");
    static_assert(R <= 32, "one bit per row");

    if (a.residency_check) {
        check_residency(a.ctrl, a.spin_limit);
        return;
    }

    // 32-byte lane outputs (int64 indices of 16-byte key vectors): each wave
    // passes its row through LDS, so that every store instruction writes one
    // contiguous 1 KiB span instead of 16 bytes at a 32-byte stride (which
    // left lines half-written per instruction: 1.14x the output bytes reached
    // HBM)
    constexpr bool kStage32 = E * sizeof(Out) == 32;
    __shared__ __attribute__((aligned(16))) u32x4 s_out32[kStage32 ? NWAVE : 1][kStage32 ? 128 : 1];
    // plain and segmented scans: the next full block of the workgroup is
    // prefetched into LDS (each wave its own R rows, a byte image of them)
    // while the current block is scanned, so a workgroup's loads stay in
    // flight through its compute.  Each 16-byte LDS load of a wave moves one
    // 1 KiB span: one row of 16-byte lane vectors, or two rows of 8-byte ones
    // (bf16), read back from LDS one lane vector at a time.  (Batched scans
    // load as before: with arrays of a few blocks, a workgroup's next block
    // usually lies in another array and is often partial, and the prefetch
    // measured slower, 4096 arrays: 4.87 -> 4.64 TB/s.)
    constexpr int kVecBytes = E * int(sizeof(In));  // one lane-row of input
    constexpr bool kPrefetch = (MODE == kModePlain || MODE == kModeSegmented) &&
                               (kVecBytes == 16 || (kVecBytes == 8 && R % 2 == 0));
    constexpr int kPfOps = R * kVecBytes / 16;        // 16-byte LDS loads per lane and block
    constexpr int kChunkElems = 16 / int(sizeof(In)); // elements per 16-byte chunk
    __shared__ __attribute__((aligned(16))) u32x4 s_pf[kPrefetch ? T * kPfOps : 1];
    // lane-blocked rows (lds_slot): plain scans of the operators that ask for them.
    // Lane l's first element sits kLaneElems after lane l - 1's, and its rows
    // kRowStep apart; s_tr turns each wave's outputs back into 1 KiB spans
    constexpr bool kBlocked = kPrefetch && E * sizeof(Out) == 16 &&
                              ((MODE == kModePlain && blocked_lanes<BaseOp>::value) ||
                               (MODE == kModeSegmented && blocked_segmented<BaseOp>::value));
    constexpr int64_t kLaneElems = kBlocked ? int64_t(R) * E : E;
    constexpr int64_t kRowStep = kBlocked ? E : ROW;
    __shared__ __attribute__((aligned(16))) u32x4 s_tr[kBlocked ? T * R : 1];
    // arrays whose y sits at another alignment phase than x: each wave stages
    // one output row here to write it as aligned vectors
    constexpr bool kStageY = E * sizeof(Out) == 16;
    // the rows written as vectors stage the wave's span of them (a wave's rows are
    // contiguous, and so are the rows of a partial batched block that lie inside
    // its array) and write it after the last row: one LDS round trip and two
    // partial vectors per block instead of per row (lane-blocked kernels, whose
    // LDS holds the transpose, stage row by row)
    constexpr bool kStageSpan = kStageY && !kBlocked;
    __shared__ __attribute__((aligned(16))) Out s_ystage[kStageY ? NWAVE : 1][kStageY ? (kStageSpan ? R * ROW : ROW) + E : 1];
    __shared__ V s_wave_total[2][NWAVE];
    __shared__ VB s_block_prefix[2];
    __shared__ int s_abort[2];

    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int64_t B = gridDim.x;
    const uint32_t tag = __hip_atomic_load(a.ctrl, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + 1u;

    // The block scanned in the previous iteration waits, in registers, for
    // its prefix: it is resolved (window fold) and stored one iteration
    // later, while the loads of the next block are in flight, and by then
    // the aggregates it needs were published a round earlier.
    bool have_pend = false;
    int64_t p_i = 0, p_n = 0, p_lane0 = 0, p_ph = 0;
    uint32_t p_vrow = 0;
    bool p_svec = true;
    Out* p_y = nullptr;
    bool p_full = false;
    uint32_t p_block_head = 0;
    uint32_t p_head[R];
    // the in-lane inclusive scan values of each row and, per row, the local
    // prefix of the lane (waves, rows and lanes before it); segmented scans
    // keep each value's head flag as a bit of p_seen (a head lies at or
    // before it inside the lane's vector)
    using PV = typename BaseOp::V;
    PV pe[kBlocked ? 1 : R][E];
    In p_raw[kBlocked ? R : 1][E];  // lane-blocked rows: the raw inputs
    uint32_t p_seen[R];
    V p_lp[R];
    VB p_agg = BOp::identity();         // wave 0: the pending block's aggregate
    VB carry = BOp::identity();         // wave 0: P(j - B) for the pending block j

    // the prefetch: this wave's LDS rows, and whether they hold the block to scan next
    const uint32_t pf_lds = kPrefetch ? lds_address(&s_pf[0]) + uint32_t(wave) * kPfOps * 1024u : 0u;
    // the 16-byte LDS loads need 16-byte aligned chunks: a grid origin of 8-byte
    // vectors that is not (bf16 input 8 bytes past a 16-byte boundary) has its
    // full blocks loaded straight into registers instead
    const bool pf_ok = kPrefetch && (kVecBytes == 16 ||
                                     ((reinterpret_cast<uintptr_t>(a.x) - uintptr_t(a.phase) * sizeof(In)) & 15u) == 0);
    bool pf_have = false;
    // the previous step wrote its pending block with at least R vector stores per
    // wave, all issued after the prefetch that the next step waits for
    bool pf_then_stores = false;
    // The flag words of the window that the next step folds, copied into LDS by
    // wave 0 at the end of a step (so the round trip to them, about 2 us under a
    // full memory load, overlaps a whole step); windows of up to 8 KiB.
    constexpr int kFlagChunks = 512;
    __shared__ __attribute__((aligned(16))) u32x4 s_flags[kFlagChunks];
    const uint32_t flags_lds = lds_address(&s_flags[0]);
    bool flags_have = false;  // wave 0: s_flags holds the pending block's window
    int flags_shift = 0;      // the window's first word is word flags_shift of s_flags
    auto flags_fetch = [&](int64_t lo, int64_t cnt) -> bool {
        return fetch_window_flags<W>(a.slots, lo, cnt, flags_lds, kFlagChunks, lane, flags_shift);
    };
    auto prefetch = [&](const In* xg, int64_t t0) {  // xg: the array's grid origin, t0: the block's first position
        // load d puts chunk 64d + l of the wave's rows in slot 64d + l (lane-blocked
        // rows: chunk 64d + lds_chunk(l))
        const int src = kBlocked ? lds_chunk(lane) : lane;
        const In* xs = xg + t0 + int64_t(wave) * (R * ROW) + int64_t(src) * kChunkElems;
#pragma unroll
        for (int d = 0; d < kPfOps; ++d) lds_load16(xs + int64_t(d) * (64 * kChunkElems), pf_lds + uint32_t(d) * 1024u);
    };

    int parity = 0;
    // Batched scans: the array of a block is found by a wave-uniform search
    // through the scalar cache (the table is read-only during the launch)
    // from this workgroup's previous array (a workgroup's blocks only move
    // forward), one step ahead, so the data loads never wait for it.
    int64_t arr_lo = 0;
    BatchArray next_d;
    next_d.x = nullptr;
    next_d.y = nullptr;
    next_d.n = 0;
    next_d.first_block = 0;
    next_d.phase = 0;
    next_d.stage_y = 0;
    auto find_array = [&](int64_t blk) {
        const CBatchArray* arr = (const CBatchArray*)(a.arrays);
        int64_t lo = arr_lo, hi = a.num_arrays;
        while (hi - lo > 1) {
            const int64_t mid = (lo + hi) >> 1;
            if (arr[mid].first_block <= blk)
                lo = mid;
            else
                hi = mid;
        }
        arr_lo = lo;
        next_d.x = arr[lo].x;  // field by field: no copy constructor binds the constant address space
        next_d.y = arr[lo].y;
        next_d.n = arr[lo].n;
        next_d.first_block = arr[lo].first_block;
        next_d.phase = arr[lo].phase;
        next_d.stage_y = arr[lo].stage_y;
    };
    if constexpr (MODE == kModeBatched) {
        if (int64_t(blockIdx.x) < a.num_blocks) find_array(blockIdx.x);
    }
    // Block i read with full vectors (every position inside its array): its grid
    // origin and first position.  Batched scans take block i's array from
    // next_d, which the lookup one step ahead has filled.
    auto full_src = [&](int64_t i, const In*& xg, int64_t& t0) -> bool {
        if constexpr (MODE == kModeBatched) {
            const int64_t ph = next_d.phase;
            if (ph < 0) return false;
            xg = static_cast<const In*>(next_d.x) - ph;
            t0 = (i - next_d.first_block) * L;
            return t0 + L <= next_d.n + ph && t0 >= ph;
        } else {
            xg = static_cast<const In*>(a.x) - a.phase;
            t0 = i * L;
            return pf_ok && a.vec_ok != 0 && t0 + L <= a.n + a.phase && t0 >= a.phase;
        }
    };
    if constexpr (kPrefetch) {
        const In* xg;
        int64_t t0;
        if (int64_t(blockIdx.x) < a.num_blocks && full_src(blockIdx.x, xg, t0)) {
            prefetch(xg, t0);
            pf_have = true;
        }
    }
    // One pipeline step: load and scan block i (when have_new) while the pending
    // block is resolved and stored.  The step that only drains the last
    // pending block is a separate instantiation, so inside the main loop every
    // load issued is consumed on every path and the compiler never has to
    // drain the previous step's stores before the next loads go out.
    // Returns false if the pending block's window timed out.
    auto step = [&](auto new_tag, int64_t i) -> bool {
        constexpr bool have_new = decltype(new_tag)::value;

        // -- 1. where the new block lives, and its loads (issued first)
        const In* x = nullptr;
        Out* y = nullptr;
        int64_t n = 0, tile0 = 0, lane0 = 0;
        int64_t ph = 0;  // alignment phase: the block grid starts ph positions before x
        bool full = false;
        bool svec = true;  // full blocks store vectors (y at the grid's phase)
        uint32_t vrow = 0;  // batched partial blocks: the wave's rows that lie wholly inside the array
        uint32_t block_head = 0;
        uint32_t head[R];
#pragma unroll
        for (int r = 0; r < R; ++r) head[r] = 0;
        In raw[R][E];
        if (have_new) {
            bool vec_ok;
            if constexpr (MODE == kModeBatched) {
                // the array of block i was looked up one step ahead (next_d);
                // the host decided its path and phase
                const BatchArray d = next_d;
                vec_ok = d.phase >= 0;
                ph = vec_ok ? d.phase : 0;
                x = static_cast<const In*>(d.x) - ph;
                y = static_cast<Out*>(d.y) - ph;
                n = d.n + ph;
                tile0 = (i - d.first_block) * L;
                block_head = (tile0 == 0) ? 1u : 0u;
                svec = d.stage_y == 0;
            } else {
                // arrays that start ph elements past a vector boundary run in
                // virtual positions v = index + ph, so that every block but
                // the first (whose first ph positions hold nothing) is read
                // and written with whole vectors (plain and segmented scans;
                // segment offsets move with the grid)
                ph = a.phase;
                x = static_cast<const In*>(a.x) - ph;
                y = static_cast<Out*>(a.y) - ph;
                n = a.n + ph;
                tile0 = i * L;
                vec_ok = a.vec_ok != 0;
                svec = a.store_vec != 0;
            }
            lane0 = tile0 + int64_t(wave) * (R * ROW) + int64_t(lane) * kLaneElems;
            full = vec_ok && (tile0 + L <= n) && (tile0 >= ph);
            if (full) {
                if (kPrefetch && pf_ok) {
                    // a full block arrives through LDS: prefetched during the previous
                    // step (or, after a partial block, loaded that way now), so no
                    // data load of the compiler's own is ever pending past this point
                    if (pf_have && pf_then_stores) {
                        vmem_wait_keep<R>();
                    } else {
                        if (!pf_have) prefetch(x, tile0);
                        vmem_drain();
                    }
                    const u32x4* pw = &s_pf[wave * kPfOps * 64];  // this wave's rows
                    if constexpr (kBlocked) {  // the lane's kPfOps consecutive chunks
                        const int lb = opaque_lane() * kPfOps;
                        u32x4 w[kPfOps];
#pragma unroll
                        for (int h = 0; h < kPfOps; ++h) w[h] = pw[lds_slot(lb + h)];
                        static_assert(sizeof(w) == sizeof(raw), "the lane's rows");
                        __builtin_memcpy(raw, w, sizeof(raw));
                    } else if constexpr (kVecBytes == 16) {
#pragma unroll
                        for (int r = 0; r < R; ++r) {
                            const u32x4 w = pw[r * 64 + lane];
                            __builtin_memcpy(raw[r], &w, 16);
                        }
                    } else {  // 8-byte lane vectors: row r of lane l is 8-byte unit 64r + l
                        const u32x2* pw8 = reinterpret_cast<const u32x2*>(pw);
#pragma unroll
                        for (int r = 0; r < R; ++r) {
                            const u32x2 w = pw8[r * 64 + lane];
                            __builtin_memcpy(raw[r], &w, 8);
                        }
                    }
                    lds_reads_drain();  // the rows are read before the next prefetch overwrites them
                } else {
#pragma unroll
                    for (int r = 0; r < R; ++r) load_vector<In, E>(x + lane0 + int64_t(r) * kRowStep, raw[r]);
                    // (kernels that prefetch: completed here, off the path of the LDS reads)
                    if constexpr (kPrefetch) {
#pragma unroll
                        for (int r = 0; r < R; ++r) complete_loads(raw[r]);
                    }
                }
            } else if (MODE == kModeBatched && vec_ok) {
                // an array's first or last block: whole rows of the wave (a
                // wave-uniform choice) still move as vectors
                const int64_t row0 = tile0 + int64_t(wave) * (R * ROW);
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const int64_t rs = row0 + int64_t(r) * ROW;
                    if (rs >= ph && rs + ROW <= n) {
                        load_vector<In, E>(x + lane0 + int64_t(r) * ROW, raw[r]);
                        vrow |= 1u << r;
                    }
                }
            }
            if constexpr (kPrefetch) pf_have = false;
            if constexpr (MODE == kModeBatched) {  // while the loads are in flight: the next block's array
                if (i + B < a.num_blocks) find_array(i + B);
            }
            if constexpr (MODE == kModeSegmented) {  // segment heads inside this lane's vectors
                // Found while the data loads are in flight.  The block's range
                // of offsets comes from the table of first segments per block
                // that a small kernel writes before the scan (else from two
                // interleaved wave-uniform binary searches through the scalar
                // cache); a few heads are then matched against every lane's
                // vectors, many by a per-lane search.
                const CInt64* off = (const CInt64*)(a.offsets);
                const int64_t S = a.num_segments;
                int64_t s_lo, s_hi;
                // offsets count from x, block positions from ph before it
                if (a.seg_first) {  // the table written just before this launch: two scalar loads
                    const CInt64* first = (const CInt64*)(a.seg_first);
                    s_lo = first[i];
                    s_hi = first[i + 1];
                } else {
                    int64_t lo1 = 0, hi1 = S, lo2 = 0, hi2 = S;
                    while (lo1 < hi1 || lo2 < hi2) {
                        const bool a1 = lo1 < hi1, a2 = lo2 < hi2;
                        const int64_t m1 = a1 ? lo1 + ((hi1 - lo1) >> 1) : 0;
                        const int64_t m2 = a2 ? lo2 + ((hi2 - lo2) >> 1) : 0;
                        const int64_t v1 = off[m1], v2 = off[m2];
                        if (a1) {
                            if (v1 + ph < tile0) lo1 = m1 + 1; else hi1 = m1;
                        }
                        if (a2) {
                            if (v2 + ph < tile0 + L) lo2 = m2 + 1; else hi2 = m2;
                        }
                    }
                    s_lo = lo1;
                    s_hi = lo2;
                }
                if (s_hi - s_lo <= kFewHeads) {
                    for (int64_t k = s_lo; k < s_hi; ++k) {
                        const int64_t rel = off[k] + ph - lane0;
#pragma unroll
                        for (int r = 0; r < R; ++r) {
                            const int64_t d = rel - int64_t(r) * kRowStep;
                            if (uint64_t(d) < uint64_t(E)) head[r] |= 1u << uint32_t(d);
                        }
                    }
                } else {
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        const int64_t p = lane0 + int64_t(r) * kRowStep;
                        int64_t k = lower_bound_i64(a.offsets, s_lo, s_hi, p - ph);
                        uint32_t h = 0;
                        for (; k < s_hi; ++k) {
                            const int64_t o = a.offsets[k] + ph;
                            if (o >= p + E) break;
                            h |= 1u << uint32_t(o - p);
                        }
                        head[r] = h;
                    }
                }
            }
        }

        // -- 2. inter-block communication for the pending block (wave 0).  Kernels
        //       that prefetch run it after the new block's aggregate is out (so no
        //       workgroup waits on this one's waits), on flag words copied into LDS
        //       a step earlier; the others run it while their data loads are in
        //       flight, on flag words read then.
        auto resolve_pending = [&](bool pf_now) {
            if (have_pend && wave == 0) {
                const int64_t j = p_i;
                bool ok = true;
                VB prefix;  // P(j - 1)
                if (a.chain) {
                    // the paper's chain: P(j - 1) from block j - 1's slot, then P(j) published
                    prefix = (j == 0) ? BOp::identity() : chain_prefix<BOp>(a.slots + (j - 1) * W, tag, a.spin_limit,
                                                                            a.ctrl + 3, lane, ok);
                    publish_slot(a.slots + j * W, BOp::combine(prefix, p_agg), tag, lane);
                } else {
                    const int64_t cnt = (j < B - 1) ? j : (B - 1);
                    VB win;
                    if (flags_have) {
                        // the copy made at the end of the previous step is complete once
                        // no more than the operations issued after it are outstanding that
                        // this step may still have in flight: its kPfOps prefetch loads and the
                        // new block's aggregate (data loads of this step were waited for)
                        const bool published = have_new;
                        if (pf_now && published)
                            vmem_wait_keep<kPfOps + 1>();
                        else if (pf_now)
                            vmem_wait_keep<kPfOps>();
                        else if (published)
                            vmem_wait_keep<1>();
                        else
                            vmem_drain();
                        const uint64_t* fw = reinterpret_cast<const uint64_t*>(&s_flags[0]) + flags_shift;
                        auto first = [&](int64_t q, int k) { return fw[q * W + k]; };
                        constexpr int QC = (W == 1) ? 4 : (W == 2) ? 2 : 1;
                        win = window_fold_from<BOp, QC>(first, a.slots, j - cnt, cnt, tag, a.spin_limit, a.ctrl + 3,
                                                        lane, ok);
                    } else {
                        win = window_fold<BOp>(a.slots, j - cnt, cnt, tag, a.spin_limit, a.ctrl + 3, lane, ok);
                    }
                    prefix = BOp::combine(carry, win);
                    carry = BOp::combine(prefix, p_agg);  // P(j)
                }
                const bool abort = __ballot(!ok) != 0;
                if (lane == 0) {
                    s_block_prefix[parity] = prefix;
                    s_abort[parity] = abort ? 1 : 0;
                    if (abort) {
                        __hip_atomic_store(a.ctrl + 2, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        __hip_atomic_store(a.ctrl + 3, tag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        if (a.status_host)
                            __hip_atomic_store(a.status_host, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                    }
                }
            }
        };
        if constexpr (!kPrefetch) resolve_pending(false);

        // the next full block of this workgroup goes out into LDS now, after every
        // wait of this step on data: vector memory operations complete in issue
        // order, so a later wait on a load of the compiler's own would also wait
        // for the prefetch
        // (after a partial block, only once its own loads are done: below)
        bool pf_late = false;
        bool pf_now = false;  // kPfOps prefetch loads per wave issued in this step
        if constexpr (kPrefetch) {
            const In* xg;
            int64_t t0;
            if (have_new && i + B < a.num_blocks && full_src(i + B, xg, t0)) {
                if (full) {
                    prefetch(xg, t0);
                    pf_have = true;
                    pf_now = true;
                } else {
                    pf_late = true;
                }
            }
        }

        // -- 3. intra-wave local scan of the new block: in-lane, then across lanes per row
        V e[R][E];
        V lane_prefix[R];
        V row_prefix[R];
        if (have_new) {
            if (full) {
                // (lane-blocked rows keep the raw inputs: lifted below)
#pragma unroll
                for (int r = 0; r < R && !kBlocked; ++r)
#pragma unroll
                    for (int k = 0; k < E; ++k) {
                        if constexpr (MODE == kModeSegmented)
                            e[r][k] = EOp::make(lift_elem<BaseOp>(raw[r][k], lane0 + int64_t(r) * kRowStep + k - ph),
                                                (head[r] >> k) & 1u);
                        else
                            e[r][k] = lift_elem<BaseOp>(raw[r][k], lane0 + int64_t(r) * kRowStep + k - ph);
                    }
            } else {
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    // prefetching kernels complete this row's loads here, inside the
                    // partial-block path, so that the waits the compiler places for
                    // them never land on the path of full blocks (nor wait for a prefetch)
                    if constexpr (MODE == kModeBatched) {
                        if ((vrow >> r) & 1u) {  // a whole row, read as vectors in stage 1
                            if constexpr (kPrefetch) complete_loads(raw[r]);
#pragma unroll
                            for (int k = 0; k < E; ++k)
                                e[r][k] = lift_elem<BaseOp>(raw[r][k], lane0 + int64_t(r) * ROW + k - ph);
                            continue;
                        }
                    }
                    In xv[E];
#pragma unroll
                    for (int k = 0; k < E; ++k) {
                        const int64_t p = lane0 + int64_t(r) * kRowStep + k;
                        xv[k] = (p < n && p >= ph) ? x[p] : In{};
                    }
                    if constexpr (kPrefetch) complete_loads(xv);
                    if constexpr (kBlocked) {  // a zero input word lifts to the identity
#pragma unroll
                        for (int k = 0; k < E; ++k) raw[r][k] = xv[k];
                        continue;
                    }
#pragma unroll
                    for (int k = 0; k < E; ++k) {
                        const int64_t p = lane0 + int64_t(r) * kRowStep + k;
                        if (p < n && p >= ph) {
                            if constexpr (MODE == kModeSegmented)
                                e[r][k] = EOp::make(lift_elem<BaseOp>(xv[k], p - ph), (head[r] >> k) & 1u);
                            else
                                e[r][k] = lift_elem<BaseOp>(xv[k], p - ph);
                        } else {
                            e[r][k] = EOp::identity();
                        }
                    }
                }
            }
            if constexpr (kPrefetch) {
                if (pf_late) {  // the partial block's loads are done: the next block goes out now
                    const In* xg;
                    int64_t t0;
                    full_src(i + B, xg, t0);
                    prefetch(xg, t0);
                    pf_have = true;
                    pf_now = true;
                }
            }
            if constexpr (!kBlocked) {
#pragma unroll
                for (int r = 0; r < R; ++r)
#pragma unroll
                    for (int k = 1; k < E; ++k) e[r][k] = EOp::combine(e[r][k - 1], e[r][k]);
            }
            if constexpr (kBlocked) {
                // the lane's rows are consecutive: their totals (the scan inside
                // each row is redone from the raw inputs at the fix-up, which keeps
                // the pending block in half the registers), their running totals,
                // then one cross-lane scan of the lane totals.  lane_prefix[0] holds
                // the lanes before this one, lane_prefix[r] (r > 0) this lane's rows
                // before r
                V run = EOp::identity();
                auto lifted = [&](int r, int k) -> V {
                    const auto v = lift_elem<BaseOp>(raw[r][k], lane0 + int64_t(r) * kRowStep + k - ph);
                    if constexpr (MODE == kModeSegmented)
                        return EOp::make(v, (head[r] >> k) & 1u);
                    else
                        return v;
                };
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    V t = lifted(r, 0);
#pragma unroll
                    for (int k = 1; k < E; ++k) t = EOp::combine(t, lifted(r, k));
                    if (r == 0) {
                        run = t;
                    } else {
                        lane_prefix[r] = run;
                        run = EOp::combine(run, t);
                    }
                }
                const V sc = wave_inclusive_scan<EOp>(run);
                lane_prefix[0] = wave_shift_right<EOp>(sc);
                const V wave_total = read_lane(sc, 63);
                if (lane == 0) s_wave_total[parity][wave] = wave_total;
            } else {
                V row_total[R];
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const V sc = wave_inclusive_scan<EOp>(e[r][E - 1]);
                    row_total[r] = read_lane(sc, 63);
                    lane_prefix[r] = wave_shift_right<EOp>(sc);
                }
                row_prefix[0] = EOp::identity();
#pragma unroll
                for (int r = 1; r < R; ++r) row_prefix[r] = EOp::combine(row_prefix[r - 1], row_total[r - 1]);
                // -- intra-block local scan: wave totals through LDS
                if (lane == 0) s_wave_total[parity][wave] = EOp::combine(row_prefix[R - 1], row_total[R - 1]);
            }
        }

        __syncthreads();  // wave totals of the new block (and, without the prefetch, the pending block's prefix) are visible

        // -- 4. the new block's aggregate (published by wave 0) and its block-local
        //       scan: wave prefix, row prefix and lane prefix folded into each value,
        //       so only the block prefix is left for the fix-up
        V wave_prefix = EOp::identity();
        VB agg = BOp::identity();
        if (have_new) {
            for (int w = 0; w < wave; ++w) wave_prefix = EOp::combine(wave_prefix, s_wave_total[parity][w]);
            if (wave == 0) {
                V agg_e = s_wave_total[parity][0];
#pragma unroll
                for (int w = 1; w < NWAVE; ++w) agg_e = EOp::combine(agg_e, s_wave_total[parity][w]);
                if constexpr (MODE == kModeBatched)
                    agg = BOp::make(agg_e, block_head);
                else
                    agg = agg_e;
                if (!a.chain) publish_slot(a.slots + i * W, agg, tag, lane);
            }
        }

        if constexpr (kPrefetch) {
            resolve_pending(pf_now);
            __syncthreads();  // the pending block's prefix is visible
        }
        if (have_pend && s_abort[parity]) return false;

        // -- 5. intra-block global scan and one coalesced store per vector, for the pending block:
        //       the block prefix joins each row's lane prefix once, then each element
        //       (inclusive or exclusive is chosen once per block: the flag is uniform,
        //       and every element's output is then one finish with fixed operands)
        auto fix_up = [&](auto excl_tag) {
            constexpr bool EXCL = decltype(excl_tag)::value;
            V prefix;
            if constexpr (MODE == kModeBatched)  // the first block of an array starts from the identity
                prefix = p_block_head ? EOp::identity() : s_block_prefix[parity].v;
            else
                prefix = s_block_prefix[parity];
            // lane-blocked rows: the lane's first chunk, and its slot in a striped row
            const int tb = kBlocked ? opaque_lane() * R : 0;
            const int ts = kBlocked ? lds_slot(opaque_lane()) : 0;
            // staged full blocks: the wave span's offset from the aligned vector below it
            const int32_t span_shift =
                kStageSpan ? int32_t((reinterpret_cast<uintptr_t>(p_y + (p_lane0 - int64_t(lane) * E)) % 16) / sizeof(Out))
                           : 0;
            // one row of outputs (lane vector r, first position p) to y
            auto store_row = [&](int r, const Out (&out)[E], int64_t p) __attribute__((always_inline)) {
                // rows read as vectors (a full block, or a whole row of an array's
                // first or last block) are written as vectors too
                const bool vec_row = p_full || ((p_vrow >> r) & 1u);
                if (kStage32 && vec_row && p_svec) {
                    // lane l's 32 bytes are 16-byte chunks 2l and 2l + 1 of the row;
                    // store k writes chunks 64k .. 64k + 63, one per lane.  Chunk c
                    // sits in slot (c & ~7) | ((c + (c >> 3)) & 7): a rotation inside
                    // each group of 8 slots, so that 8 consecutive lanes touch 8
                    // different 16-byte slots both when writing chunks 2l (or 2l + 1)
                    // and when reading chunks c = 64k + l.  Measured bank-conflict
                    // cycles per launch (int32 2^28): 16.8M without the rotation, 8.4M
                    // with it, 25.2M with the same rotation over groups of 16
                    auto slot = [](int c) { return (c & ~7) | ((c + (c >> 3)) & 7); };
                    u32x4 w[2];
                    __builtin_memcpy(w, out, 32);
                    u32x4* stage = s_out32[kStage32 ? wave : 0];
                    stage[slot(2 * lane)] = w[0];
                    stage[slot(2 * lane + 1)] = w[1];
                    wave_lds_sync();  // lanes read what other lanes wrote
                    u32x4* dst = reinterpret_cast<u32x4*>(p_y + (p - int64_t(lane) * E));  // the row's first output
#pragma unroll
                    for (int h = 0; h < 2; ++h)
                        __builtin_nontemporal_store(stage[slot(64 * h + lane)], dst + 64 * h + lane);
                    wave_lds_sync();  // the next row's stage writes come after every lane's reads
                } else if (vec_row && p_svec) {
                    store_vector<Out, E>(p_y + p, out);
                } else if (kStageSpan && vec_row) {  // staged here, written after the last row
                    Out* stage = s_ystage[kStageY ? wave : 0];
#pragma unroll
                    for (int k = 0; k < E; ++k) stage[span_shift + r * ROW + lane * E + k] = out[k];
                } else if (kStageY && vec_row) {
                    // y at another phase than the grid: stage the wave's row
                    // at its offset from the aligned vector below it, then
                    // write whole aligned vectors (and the partial vectors at
                    // both ends element by element)
                    Out* stage = s_ystage[kStageY ? wave : 0];
                    Out* row_y = p_y + (p - int64_t(lane) * E);  // the wave-row's first output
                    const int32_t shift = int32_t((reinterpret_cast<uintptr_t>(row_y) % 16) / sizeof(Out));
#pragma unroll
                    for (int k = 0; k < E; ++k) stage[shift + lane * E + k] = out[k];
                    wave_lds_sync();  // lanes read what other lanes wrote
                    Out* dst = row_y - shift;
                    const int32_t span = shift + ROW;  // staged outputs occupy [shift, span)
                    for (int32_t c = lane * E; c < span; c += 64 * E) {
                        if (c >= shift && c + E <= span) {
                            Out v[E];
#pragma unroll
                            for (int k = 0; k < E; ++k) v[k] = stage[c + k];
                            store_vector<Out, E>(dst + c, v);
                        } else {
#pragma unroll
                            for (int k = 0; k < E; ++k)
                                if (c + k >= shift && c + k < span) dst[c + k] = stage[c + k];
                        }
                    }
                    wave_lds_sync();  // the next row's stage writes come after every lane's reads
                } else {
#pragma unroll
                    for (int k = 0; k < E; ++k)
                        if (p + k < p_n && p + k >= p_ph) p_y[p + k] = out[k];
                }
            };
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const V q = EOp::combine(prefix, p_lp[r]);  // everything before this lane's vector
                V ev[E];
#pragma unroll
                for (int k = 0; k < E; ++k) {
                    if constexpr (kBlocked) {  // the in-row scan, again from the raw inputs
                        const auto xv = lift_elem<BaseOp>(p_raw[r][k], p_lane0 + int64_t(r) * kRowStep + k - p_ph);
                        V xk;
                        if constexpr (MODE == kModeSegmented)
                            xk = EOp::make(xv, (p_head[r] >> k) & 1u);
                        else
                            xk = xv;
                        ev[k] = (k == 0) ? xk : EOp::combine(ev[k - 1], xk);
                    } else if constexpr (MODE == kModeSegmented) {
                        ev[k] = EOp::make(pe[r][k], (p_seen[r] >> k) & 1u);
                    } else {
                        ev[k] = pe[r][k];
                    }
                }
                Out out[E];
#pragma unroll
                for (int k = 0; k < E; ++k) {
                    if constexpr (MODE == kModeSegmented) {
                        // a head inside the lane's vector at or before the element: its value alone
                        if constexpr (!EXCL) {
                            out[k] = ev[k].f ? BaseOp::lower(ev[k].v) : finish_of<BaseOp>(q.v, ev[k].v);
                        } else if (k == 0) {
                            out[k] = (p_head[r] & 1u) ? BaseOp::lower(BaseOp::identity()) : BaseOp::lower(q.v);
                        } else {
                            out[k] = ((p_head[r] >> k) & 1u) ? BaseOp::lower(BaseOp::identity())
                                     : ev[k - 1].f          ? BaseOp::lower(ev[k - 1].v)
                                                            : finish_of<BaseOp>(q.v, ev[k - 1].v);
                        }
                    } else {
                        if constexpr (!EXCL)
                            out[k] = finish_of<BaseOp>(q, ev[k]);
                        else
                            out[k] = (k == 0) ? BaseOp::lower(q) : finish_of<BaseOp>(q, ev[k - 1]);
                    }
                }
                if constexpr (kBlocked) {  // through LDS: lane-blocked in, striped out
                    u32x4 w;
                    __builtin_memcpy(&w, out, 16);
                    s_tr[wave * R * 64 + lds_slot(tb + r)] = w;
                } else {
                    store_row(r, out, p_lane0 + int64_t(r) * ROW);
                }
            }
            if constexpr (kStageSpan) {
                const uint32_t vmask = p_full ? ((R == 32) ? ~0u : ((1u << R) - 1u)) : p_vrow;
                if (!p_svec && vmask != 0) {  // the staged rows: aligned vectors, partial ones at both ends
                    wave_lds_sync();  // lanes read what other lanes wrote
                    const Out* stage = s_ystage[kStageY ? wave : 0];
                    Out* dst = p_y + (p_lane0 - int64_t(lane) * E) - span_shift;
                    // staged outputs occupy [lo, hi): rows r0 .. r1, shifted by span_shift
                    const int32_t r0 = __builtin_ctz(vmask), r1 = 31 - __builtin_clz(vmask);
                    const int32_t lo = span_shift + r0 * ROW, hi = span_shift + (r1 + 1) * ROW;
                    for (int32_t c = r0 * ROW + lane * E; c < hi; c += 64 * E) {
                        if (c >= lo && c + E <= hi) {
                            Out v[E];
#pragma unroll
                            for (int k = 0; k < E; ++k) v[k] = stage[c + k];
                            store_vector<Out, E>(dst + c, v);
                        } else {
#pragma unroll
                            for (int k = 0; k < E; ++k)
                                if (c + k >= lo && c + k < hi) dst[c + k] = stage[c + k];
                        }
                    }
                    wave_lds_sync();  // the next block's stage writes come after every lane's reads
                }
            }
            if constexpr (kBlocked) {
                wave_lds_sync();  // lanes read what other lanes wrote
                if (p_full && !p_svec) {
                    // y at another phase than the grid: aligned output vector k holds the
                    // wave's outputs k*E - shift .. k*E - shift + E - 1, taken from
                    // staged chunks k - 1 and k (the partial vectors at both ends of the
                    // wave's span element by element)
                    static_assert(E * sizeof(Out) == 16, "16-byte output chunks");
                    const u32x4* tw = &s_tr[wave * R * 64];
                    Out* wave_y = p_y + (p_lane0 - int64_t(lane) * kLaneElems);
                    const int32_t shift = int32_t((reinterpret_cast<uintptr_t>(wave_y) % 16) / sizeof(Out));
                    Out* dst = wave_y - shift;
                    constexpr int32_t kWaveOut = R * 64 * E;
                    auto staged = [&](int32_t c, Out (&o)[E]) {
                        const u32x4 w = tw[(c & ~63) | lds_slot(c & 63)];
                        __builtin_memcpy(o, &w, 16);
                    };
                    for (int32_t k = lane; k <= R * 64; k += 64) {
                        Out prev[E] = {}, cur[E] = {};
                        if (k > 0) staged(k - 1, prev);
                        if (k < R * 64) staged(k, cur);
                        Out v[E];
#pragma unroll
                        for (int sh = 0; sh < E; ++sh) {  // shift is wave-uniform
                            if (shift == sh) {
#pragma unroll
                                for (int j = 0; j < E; ++j) {
                                    if (j < sh)
                                        v[j] = prev[E - sh + j];
                                    else
                                        v[j] = cur[j - sh];
                                }
                            }
                        }
                        const int32_t first = k * E - shift;  // wave output index of v[0]
                        if (first >= 0 && first + E <= kWaveOut) {
                            store_vector<Out, E>(dst + k * E, v);
                        } else {
#pragma unroll
                            for (int j = 0; j < E; ++j)
                                if (first + j >= 0 && first + j < kWaveOut) dst[k * E + j] = v[j];
                        }
                    }
                } else {
                    const int64_t p0 = p_lane0 - int64_t(lane) * (kLaneElems - E);  // striped: lane l's vector of row r
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        const u32x4 w = s_tr[wave * R * 64 + r * 64 + ts];  // chunk 64r + l
                        Out out[E];
                        __builtin_memcpy(out, &w, 16);
                        store_row(r, out, p0 + int64_t(r) * ROW);
                    }
                }
                wave_lds_sync();  // the next block's writes come after every lane's reads
            }
        };
        if (have_pend) {
            if (a.exclusive)
                fix_up(std::true_type{});
            else
                fix_up(std::false_type{});
        }
        // full blocks with y at the grid's phase leave through one vector store per
        // row (two for 32-byte lane outputs), after any prefetch of this step
        pf_then_stores = have_pend && p_full && p_svec;
        // the window of the new block, for the next step's fold
        if (kPrefetch && wave == 0) {
            flags_have = false;
            if (have_new && !a.chain) {
                const int64_t cnt = (i < B - 1) ? i : (B - 1);
                if (cnt > 0) flags_have = flags_fetch(i - cnt, cnt);
            }
        }

        // -- 6. the new block becomes the pending one
        have_pend = have_new;
        if (have_new) {
            p_i = i;
            p_n = n;
            p_ph = ph;
            p_vrow = vrow;
            p_svec = svec;
            p_lane0 = lane0;
            p_y = y;
            p_full = full;
            p_block_head = block_head;
            p_agg = agg;
            V wl = EOp::identity();
            if constexpr (kBlocked) wl = EOp::combine(wave_prefix, lane_prefix[0]);  // waves and lanes before
#pragma unroll
            for (int r = 0; r < R; ++r) {
                p_head[r] = head[r];
                // local prefix of this lane's row: waves before, rows before, lanes before
                if constexpr (kBlocked)
                    p_lp[r] = (r == 0) ? wl : EOp::combine(wl, lane_prefix[r]);
                else
                    p_lp[r] = EOp::combine(EOp::combine(wave_prefix, row_prefix[r]), lane_prefix[r]);
                if constexpr (kBlocked) {
#pragma unroll
                    for (int k = 0; k < E; ++k) p_raw[r][k] = raw[r][k];
                } else if constexpr (MODE == kModeSegmented) {
                    uint32_t seen = 0;
#pragma unroll
                    for (int k = 0; k < E; ++k) {
                        pe[r][k] = e[r][k].v;
                        seen |= (e[r][k].f ? 1u : 0u) << k;
                    }
                    p_seen[r] = seen;
                } else {
#pragma unroll
                    for (int k = 0; k < E; ++k) pe[r][k] = e[r][k];
                }
            }
        }
        return true;
    };

    int64_t i = blockIdx.x;
    bool live = true;
    for (; i < a.num_blocks; i += B, parity ^= 1)
        if (!(live = step(std::true_type{}, i))) break;
    if (live && have_pend) step(std::false_type{}, i);
    vmem_drain();  // no load into LDS outlives the workgroup

    // Every workgroup counts itself out; the last one advances the epoch so
    // the next launch on this workspace uses a fresh tag (no memset needed).
    if (threadIdx.x == 0) {
        const uint32_t prev = __hip_atomic_fetch_add(a.ctrl + 1, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (prev == uint32_t(gridDim.x) - 1u) {
            __hip_atomic_store(a.ctrl + 1, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(a.ctrl, tag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// ---------------------------------------------------------------------------
// Registration helpers used by the instantiation units.
// ---------------------------------------------------------------------------
template <class BaseOp, int MODE, int T, int R>
hipError_t launch_scan(const ScanArgs& a, int grid, hipStream_t stream)
{
    (void)hipGetLastError();  // a stale error from earlier work must not be read as this launch's
    hipLaunchKernelGGL((scan_kernel<BaseOp, T, R, MODE>), dim3(grid), dim3(T), 0, stream, a);
    return hipGetLastError();
}

template <class BaseOp, int MODE, int S>
KernelEntry make_entry()
{
    constexpr int T = kShapeThreads[S];
    constexpr int R = kShapeVectors[S];
    using BOp = typename ModeOps<BaseOp, MODE>::BlkOp;
    KernelEntry k;
    k.abi = kKernelAbi;
    k.func = reinterpret_cast<const void*>(&scan_kernel<BaseOp, T, R, MODE>);
    k.launch = &launch_scan<BaseOp, MODE, T, R>;
    k.block_threads = T;
    k.vectors_per_lane = R;
    k.elems_per_vec = BaseOp::E;
    k.slot_words = int(sizeof(typename BOp::V) / 4);
    k.in_bytes = int(sizeof(typename BaseOp::In));
    k.out_bytes = int(sizeof(typename BaseOp::Out));
    k.tile_elems = int64_t(T) * R * BaseOp::E;
    return k;
}

template <class BaseOp, int MODE>
void fill_row(KernelTable& t, int opcode)
{
    KernelEntry* row = t[MODE][opcode];
    row[0] = make_entry<BaseOp, MODE, 0>();
    row[1] = make_entry<BaseOp, MODE, 1>();
    row[2] = make_entry<BaseOp, MODE, 2>();
    row[3] = make_entry<BaseOp, MODE, 3>();
    row[4] = make_entry<BaseOp, MODE, 4>();
    row[5] = make_entry<BaseOp, MODE, 5>();
    row[6] = make_entry<BaseOp, MODE, 6>();
    row[7] = make_entry<BaseOp, MODE, 7>();
    row[8] = make_entry<BaseOp, MODE, 8>();
    row[9] = make_entry<BaseOp, MODE, 9>();
    static_assert(kNumShapes == 10, "one entry per compiled shape");
}

}  // namespace lscan
