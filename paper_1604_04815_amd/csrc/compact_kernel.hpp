// compact_kernel.hpp -- stream compaction on the persistent single-pass scan.
//
// Compaction is the selection that a +-scan of 0/1 flags drives, one of the
// uses of the scan the paper lists (Section 1): every x[i] whose keep flag is
// set goes to out[c_i], where c_i is the number of kept elements before i
// (the exclusive scan of the flags).  The kernel is the scan of
// scan_kernel.hpp with the flags as its input and a scatter as its fix-up:
//   * data blocks of L = T * R * E elements, taken cyclically by B resident
//     workgroups (Section 4); each lane holds R vectors of E elements of x
//     and the E keep bytes beside each, read once, coalesced (the flags of a
//     wave's rows are one span, read in 16-byte chunks per lane and handed
//     to their lanes through LDS);
//   * per lane and row the kept elements are counted (popcount of the
//     flags); the counts are scanned across the wave (DPP), across rows and
//     across waves (LDS), giving each lane-row the number of kept elements
//     of the block before it, and the block count A(i) (Algorithms 2-3);
//   * A(i) is published in an epoch-tagged 64-bit slot pair; the block's
//     starting position P(i - 1) comes one round later from the workgroup's
//     own previous P(i - B) and the B - 1 counts in between (the window
//     hand-off of the scan), so the count carried between blocks is 64-bit;
//   * the pending block then writes each kept element to its position; the
//     kept elements of a wave-row land in one contiguous range of out, so
//     each wave stages the row in LDS at its offsets from the aligned vector
//     below the range and writes it as whole aligned 16-byte vectors (items
//     one by one only in the partial vectors at both ends).
// The workgroup that resolves the last block writes the total count.
#pragma once

#include "scan_kernel.hpp"

namespace lscan {

// Element payloads: 4-byte (int32, float32 bits) and 8-byte (int64) items,
// moved as raw bits.
template <class T>
struct CompactItem {
    using In = T;
    static constexpr int E = 16 / int(sizeof(T));  // items per 16-byte vector
};

// The E keep bytes of one lane-row (in LDS) as a bit mask (bit k: item k is kept).
template <int E>
__device__ __forceinline__ uint32_t keep_bits(const uint8_t* k)
{
    if constexpr (E == 4) {
        const uint32_t w = *reinterpret_cast<const uint32_t*>(k);
        return ((w & 0xffu) ? 1u : 0u) | ((w & 0xff00u) ? 2u : 0u) | ((w & 0xff0000u) ? 4u : 0u) |
               ((w & 0xff000000u) ? 8u : 0u);
    } else {
        const uint16_t w = *reinterpret_cast<const uint16_t*>(k);
        return ((w & 0xffu) ? 1u : 0u) | ((w & 0xff00u) ? 2u : 0u);
    }
}

// Flag bytes a lane reads per load: the wave's R rows of flags are one
// contiguous span of R * 64 * E bytes, read in chunks of up to 16 bytes per
// lane (full-width loads even though each lane-row needs only E bytes).
template <int C> struct FlagWord;
template <> struct FlagWord<16> { using type = u32x4; };
template <> struct FlagWord<8> { using type = u32x2; };
template <> struct FlagWord<4> { using type = uint32_t; };
template <> struct FlagWord<2> { using type = uint16_t; };

template <int R, int E>
struct FlagChunks {
    static constexpr int C = (R * E >= 16) ? 16 : R * E;  // bytes per lane per load
    static constexpr int N = (R * E) / C;                 // loads per lane
    using Word = typename FlagWord<C>::type;
};

template <class T, int TT, int R>
__global__ void __launch_bounds__(TT) compact_kernel(ScanArgs a)
{
    using Item = CompactItem<T>;
    using EOp = AddI32;  // counts inside a block (at most L)
    using BOp = AddI64;  // counts carried between blocks
    using VB = int64_t;
    constexpr int E = Item::E;
    constexpr int NWAVE = TT / 64;
    constexpr int W = sizeof(VB) / 4;
    constexpr int ROW = 64 * E;
    constexpr int64_t L = int64_t(TT) * R * E;
    static_assert(TT % 64 == 0 && NWAVE <= 16, "wave64 workgroups of up to 1024 threads");

    if (a.residency_check) {
        check_residency(a.ctrl, a.spin_limit);
        return;
    }

    __shared__ int32_t s_wave_total[2][NWAVE];
    __shared__ VB s_block_prefix[2];
    __shared__ int s_abort[2];
    // per wave: one row of kept items, laid out as in out (shifted by the
    // row's misalignment), so that it leaves in aligned 16-byte vectors
    __shared__ __attribute__((aligned(16))) T s_stage[NWAVE][ROW + E];
    // per wave: the keep bytes of its R rows, as read from memory
    __shared__ __attribute__((aligned(16))) uint8_t s_flags[NWAVE][R * ROW];
    using FC = FlagChunks<R, E>;
    static_assert(FC::N * FC::C == R * E, "flag chunks tile the wave's flag span");

    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int64_t B = gridDim.x;
    const uint32_t tag = __hip_atomic_load(a.ctrl, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + 1u;
    const T* x = static_cast<const T*>(a.x);
    T* out = static_cast<T*>(a.y);
    const uint8_t* keep = a.keep;
    const int64_t n = a.n;

    // pending block: its items, keep masks, and per row the kept count of the
    // block before the wave-row, before the lane inside it, and in the row
    bool have_pend = false;
    int64_t p_i = 0;
    T p_x[R][E];
    uint32_t p_bits[R];
    int32_t p_row0[R];
    int32_t p_lane[R];
    int32_t p_rowcnt[R];
    const bool out_vec = (reinterpret_cast<uintptr_t>(out) % 16) == 0;
    VB p_agg = 0;    // wave 0: kept items in the pending block
    VB carry = 0;    // wave 0: kept items before block (pending - B + 1)

    // The next full block of the workgroup is prefetched into LDS while the
    // current one is counted and scattered, as in the scan: its items (each
    // wave its R rows of 1 KiB) and its keep bytes (straight into the wave's
    // flag span, which has the layout a 16-byte-per-lane LDS load writes).
    // Shapes whose flag chunks are narrower than 16 bytes load as before.
    constexpr bool kPrefetch = FC::C == 16;
    __shared__ __attribute__((aligned(16))) u32x4 s_pfx[kPrefetch ? TT * R : 1];
    const uint32_t pfx_lds = kPrefetch ? lds_address(&s_pfx[0]) + uint32_t(wave) * R * 1024u : 0u;
    const uint32_t pff_lds = kPrefetch ? lds_address(&s_flags[wave][0]) : 0u;
    bool pf_have = false;
    auto full_block = [&](int64_t i) -> bool { return a.vec_ok && ((i + 1) * L <= n); };
    auto prefetch = [&](int64_t i) {
        const int64_t w0 = i * L + int64_t(wave) * (R * ROW);
        const T* xs = x + w0 + int64_t(lane) * E;
#pragma unroll
        for (int r = 0; r < R; ++r) lds_load16(xs + int64_t(r) * ROW, pfx_lds + uint32_t(r) * 1024u);
        if (keep) {
            const uint8_t* kw = keep + w0 + lane * FC::C;
#pragma unroll
            for (int q = 0; q < FC::N; ++q) lds_load16(kw + q * 64 * FC::C, pff_lds + uint32_t(q) * 1024u);
        }
    };
    if constexpr (kPrefetch) {
        if (int64_t(blockIdx.x) < a.num_blocks && full_block(blockIdx.x)) {
            prefetch(blockIdx.x);
            pf_have = true;
        }
    }

    int parity = 0;
    auto step = [&](auto new_tag, int64_t i) -> bool {
        constexpr bool have_new = decltype(new_tag)::value;

        // -- 1. loads of the new block
        const int64_t tile0 = i * L;
        const int64_t lane0 = tile0 + int64_t(wave) * (R * ROW) + int64_t(lane) * E;
        const bool full = have_new && a.vec_ok && (tile0 + L <= n);
        T raw[R][E];
        uint32_t bits[R];
        typename FC::Word fw[FC::N];
        if constexpr (kPrefetch) {
            // a full block arrives through LDS (prefetched during the previous
            // step, or loaded that way now after a partial block)
            if (have_new && full) {
                if (!pf_have) prefetch(i);
                vmem_drain();
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const u32x4 w = s_pfx[(wave * R + r) * 64 + lane];
                    __builtin_memcpy(raw[r], &w, 16);
                }
                if (keep) {
#pragma unroll
                    for (int r = 0; r < R; ++r) bits[r] = keep_bits<E>(s_flags[wave] + r * ROW + lane * E);
                }
                lds_reads_drain();  // read before the next prefetch overwrites them
            }
            if (have_new) pf_have = false;
        } else if (have_new && full) {
#pragma unroll
            for (int r = 0; r < R; ++r) load_vector<T, E>(x + lane0 + int64_t(r) * ROW, raw[r]);
            if (keep) {
                const uint8_t* kw = keep + tile0 + int64_t(wave) * (R * ROW) + lane * FC::C;
#pragma unroll
                for (int q = 0; q < FC::N; ++q)
                    fw[q] = __builtin_nontemporal_load(reinterpret_cast<const typename FC::Word*>(kw + q * 64 * FC::C));
            }
        }

        // -- 2. the window of the pending block (wave 0): its start P(j - 1)
        if (have_pend && wave == 0) {
            const int64_t j = p_i;
            bool ok = true;
            const int64_t cnt = (j < B - 1) ? j : (B - 1);
            const VB win = window_fold<BOp>(a.slots, j - cnt, cnt, tag, a.spin_limit, a.ctrl + 3, lane, ok);
            const VB prefix = carry + win;
            carry = prefix + p_agg;  // P(j)
            const bool abort = __ballot(!ok) != 0;
            if (lane == 0) {
                s_block_prefix[parity] = prefix;
                s_abort[parity] = abort ? 1 : 0;
                if (abort) {
                    __hip_atomic_store(a.ctrl + 2, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    __hip_atomic_store(a.ctrl + 3, tag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    if (a.status_host)
                        __hip_atomic_store(a.status_host, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                } else if (j == a.num_blocks - 1) {
                    *a.count = carry;  // the total kept
                }
            }
        }

        // the next full block goes out into LDS after every wait of this step on
        // data or flag words (waits complete in issue order)
        // (after a partial block, only once its own loads are done: below)
        bool pf_late = false;
        if constexpr (kPrefetch) {
            if (have_new && i + B < a.num_blocks && full_block(i + B)) {
                if (full) {
                    prefetch(i + B);
                    pf_have = true;
                } else {
                    pf_late = true;
                }
            }
        }

        // -- 3. counts of the new block: per lane-row, across the wave, across rows
        int32_t lane_prefix[R];
        int32_t row_prefix[R];
        int32_t row_total[R];
        if (have_new) {
            if (!full) {  // the tail block, or unaligned pointers: item by item
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    uint32_t kv[E];
#pragma unroll
                    for (int k = 0; k < E; ++k) {
                        const int64_t p = lane0 + int64_t(r) * ROW + k;
                        raw[r][k] = (p < n) ? x[p] : T(0);
                        kv[k] = (p < n && keep) ? uint32_t(keep[p]) : 0u;
                    }
                    // with the prefetch: the row's loads complete inside this partial-block
                    // path, so the compiler's waits for them stay off full blocks
                    if constexpr (kPrefetch) {
                        complete_loads(raw[r]);
#pragma unroll
                        for (int k = 0; k < E; ++k) asm volatile("" : "+v"(kv[k]));
                    }
                    uint32_t m = 0;
#pragma unroll
                    for (int k = 0; k < E; ++k) {
                        const int64_t p = lane0 + int64_t(r) * ROW + k;
                        if (p < n && (keep ? (kv[k] != 0) : (raw[r][k] != T(0)))) m |= 1u << k;
                    }
                    bits[r] = m;
                }
            } else if (!keep) {
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    uint32_t m = 0;
#pragma unroll
                    for (int k = 0; k < E; ++k) m |= (raw[r][k] != T(0) ? 1u : 0u) << k;
                    bits[r] = m;
                }
            } else if constexpr (!kPrefetch) {  // the flag span through LDS: each lane then takes its rows' E bytes
                uint8_t* sf = s_flags[wave];
#pragma unroll
                for (int q = 0; q < FC::N; ++q)
                    *reinterpret_cast<typename FC::Word*>(sf + q * 64 * FC::C + lane * FC::C) = fw[q];
                wave_lds_sync();
#pragma unroll
                for (int r = 0; r < R; ++r) bits[r] = keep_bits<E>(sf + r * ROW + lane * E);
                wave_lds_sync();
            }
            if constexpr (kPrefetch) {
                if (pf_late) {  // the partial block's loads are done: the next block goes out now
                    prefetch(i + B);
                    pf_have = true;
                }
            }
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int32_t sc = wave_inclusive_scan<EOp>(int32_t(__builtin_popcount(bits[r])));
                row_total[r] = read_lane(sc, 63);
                lane_prefix[r] = wave_shift_right<EOp>(sc);
            }
            row_prefix[0] = 0;
#pragma unroll
            for (int r = 1; r < R; ++r) row_prefix[r] = row_prefix[r - 1] + row_total[r - 1];
            if (lane == 0) s_wave_total[parity][wave] = row_prefix[R - 1] + row_total[R - 1];
        }

        __syncthreads();  // wave totals of the new block and the pending block's start are visible
        if (have_pend && s_abort[parity]) return false;

        // -- 4. the new block's count (published by wave 0) and each wave's offset in it
        int32_t wave_prefix = 0;
        VB agg = 0;
        if (have_new) {
            for (int w = 0; w < wave; ++w) wave_prefix += s_wave_total[parity][w];
            if (wave == 0) {
                int32_t total = 0;
#pragma unroll
                for (int w = 0; w < NWAVE; ++w) total += s_wave_total[parity][w];
                agg = total;
                publish_slot(a.slots + i * W, agg, tag, lane);
            }
        }

        // -- 5. the pending block's kept items to out
        if (have_pend) {
            const VB base = s_block_prefix[parity];
            T* stage = s_stage[wave];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int64_t g0 = base + p_row0[r];  // first position of this wave-row's items
                const uint32_t m = p_bits[r];
                if (!out_vec) {  // out not 16-byte aligned: item by item
                    int32_t before = 0;
#pragma unroll
                    for (int k = 0; k < E; ++k) {
                        if ((m >> k) & 1u) out[g0 + p_lane[r] + before] = p_x[r][k];
                        before += int32_t((m >> k) & 1u);
                    }
                    continue;
                }
                // stage the row's kept items at their offsets from the aligned
                // vector below g0, then write whole aligned vectors (and the
                // partial vectors at both ends item by item)
                const int32_t shift = int32_t(g0 & int64_t(E - 1));
                int32_t at = shift + p_lane[r];
#pragma unroll
                for (int k = 0; k < E; ++k) {
                    if ((m >> k) & 1u) stage[at] = p_x[r][k];
                    at += int32_t((m >> k) & 1u);
                }
                wave_lds_sync();
                const int32_t span = shift + p_rowcnt[r];  // staged items occupy [shift, span)
                T* dst = out + (g0 - shift);
                for (int32_t c = lane * E; c < span; c += 64 * E) {
                    if (c >= shift && c + E <= span) {
                        T v[E];
                        __builtin_memcpy(v, stage + c, 16);
                        u32x4 w;
                        __builtin_memcpy(&w, v, 16);
                        *reinterpret_cast<u32x4*>(dst + c) = w;
                    } else {
#pragma unroll
                        for (int k = 0; k < E; ++k)
                            if (c + k >= shift && c + k < span) dst[c + k] = stage[c + k];
                    }
                }
                wave_lds_sync();
            }
        }

        // -- 6. the new block becomes the pending one
        have_pend = have_new;
        if (have_new) {
            p_i = i;
            p_agg = agg;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                p_bits[r] = bits[r];
                p_row0[r] = wave_prefix + row_prefix[r];
                p_lane[r] = lane_prefix[r];
                p_rowcnt[r] = row_total[r];
#pragma unroll
                for (int k = 0; k < E; ++k) p_x[r][k] = raw[r][k];
            }
        }
        return true;
    };

    int64_t i = blockIdx.x;
    bool live = true;
    for (; i < a.num_blocks; i += B, parity ^= 1)
        if (!(live = step(std::true_type{}, i))) break;
    if (live && have_pend) step(std::false_type{}, i);
    if constexpr (kPrefetch) vmem_drain();  // no LDS load outlives the workgroup

    // count out; the last workgroup advances the epoch (as in the scan)
    if (threadIdx.x == 0) {
        const uint32_t prev = __hip_atomic_fetch_add(a.ctrl + 1, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (prev == uint32_t(gridDim.x) - 1u) {
            __hip_atomic_store(a.ctrl + 1, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(a.ctrl, tag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

template <class T, int TT, int R>
hipError_t launch_compact(const ScanArgs& a, int grid, hipStream_t stream)
{
    (void)hipGetLastError();
    hipLaunchKernelGGL((compact_kernel<T, TT, R>), dim3(grid), dim3(TT), 0, stream, a);
    return hipGetLastError();
}

template <class T, int S>
KernelEntry make_compact_entry()
{
    constexpr int TT = kShapeThreads[S];
    constexpr int R = kShapeVectors[S];
    KernelEntry k;
    k.abi = kKernelAbi;
    k.func = reinterpret_cast<const void*>(&compact_kernel<T, TT, R>);
    k.launch = &launch_compact<T, TT, R>;
    k.block_threads = TT;
    k.vectors_per_lane = R;
    k.elems_per_vec = CompactItem<T>::E;
    k.slot_words = 2;
    k.in_bytes = int(sizeof(T));
    k.out_bytes = int(sizeof(T));
    k.tile_elems = int64_t(TT) * R * CompactItem<T>::E;
    return k;
}

template <class T>
void fill_compact_row(KernelTable& t, int opcode)
{
    KernelEntry* row = t[kModeCompact][opcode];
    row[0] = make_compact_entry<T, 0>();
    row[1] = make_compact_entry<T, 1>();
    row[2] = make_compact_entry<T, 2>();
    row[3] = make_compact_entry<T, 3>();
    row[4] = make_compact_entry<T, 4>();
    row[5] = make_compact_entry<T, 5>();
    row[6] = make_compact_entry<T, 6>();
    row[7] = make_compact_entry<T, 7>();
    row[8] = make_compact_entry<T, 8>();
    row[9] = make_compact_entry<T, 9>();
    static_assert(kNumShapes == 10, "one entry per compiled shape");
}

}  // namespace lscan
