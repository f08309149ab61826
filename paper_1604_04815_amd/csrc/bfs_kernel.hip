// bfs_kernel.hip -- breadth-first search as a persistent grid of workgroups
// that talk to each other only through epoch-tagged flag words: the paper's
// inter-block hand-off (Section 4.3) used for the graph search it names as
// the next application of that hand-off (Section 6), in place of the atomic
// queue-tail counter that level-synchronous GPU searches usually use.
//
// One launch runs the whole search, level by level (top-down expansion):
//   * The frontier of a level is a queue of the vertices found at the level
//     before that have at least one edge, with the exclusive prefix of their
//     degrees beside it, so the level's edges have flat ranks 0 .. D - 1.
//     The ranks are cut into chunks of kBfsChunkEdges; chunk c is taken by
//     workgroup c mod B, in increasing c (the cyclic distribution of the
//     scan).  Every chunk has the same number of edges, however skewed the
//     degrees: a hub's edges spread over many chunks.
//   * Per chunk, the workgroup loads the frontier vertices its ranks fall in
//     (a table written while the frontier was built gives the first one),
//     maps each rank to its vertex by a search in LDS, and claims every
//     endpoint not yet discovered by setting its bit in the visited bitmap
//     with an atomic or: the lane that flips the bit wins.  The winners are the
//     vertices of the next level that this chunk discovered; those with
//     edges are kept in LDS with their degrees (a chunk discovers at most
//     one vertex per edge, so they always fit).
//   * Where they go in the next frontier is a scan over chunks: the chunk
//     publishes (vertices, edges) packed in one 64-bit value in its flag
//     words at once, obtains its offsets from its own previous chunk's
//     running total and the values of the chunks in between (the window
//     fold of the scan), and writes its vertices, their edge offsets and
//     the next level's chunk table there.  No shared tail counter.
//   * A level ends with a grid barrier built from the same flag words: each
//     workgroup publishes its sums under the level's tag, workgroup 0 adds
//     them up and publishes the totals, which every workgroup waits for.
//     The next frontier's writes are released before the arrival and
//     acquired after the release word, at agent scope.
//   * Every flag word carries the tag of its level, so nothing is cleared
//     between levels or launches; the host hands each launch a fresh range
//     of tags.  Every wait is bounded and honours the abort word, so a grid
//     that is not co-resident ends with a timeout instead of hanging.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bfs_kernel.hpp"
#include "scan_kernel.hpp"  // flag words, bounded waits, window fold, co-residency test

namespace lscan {

namespace {

constexpr int kWaves = kBfsThreads / 64;
constexpr int K = kBfsChunkEdges;
constexpr int kPer = K / kBfsThreads;  // edges per thread per chunk
constexpr int64_t kCountMask = (int64_t(1) << kBfsCountBits) - 1;
constexpr int kBarrierWords = 4;
constexpr int kGatherPer = kBfsMaxGrid / kBfsThreads;  // arrivals gathered per thread of workgroup 0
constexpr int kGatherBatch = 1;
constexpr int kFoldBatch = 1;  // chunk values in flight per thread in the window sum

struct BfsShared {
    int64_t eo[K + 2];       // edge offsets of the chunk's vertices; eo[n] is a sentinel
    int64_t shift[K + 1];    // row start - edge offset: edge index = rank + shift
    int32_t u[K + 1];        // the chunk's vertices
    int32_t stage[2][K];     // discovered vertices that have edges: the chunk being
                             // claimed and the one waiting to be placed
    int64_t wave_tot[kWaves];
    uint64_t found_e;        // edges of the staged vertices
    uint32_t found;          // staged vertices
    uint32_t found_all;      // vertices this workgroup discovered in the current level
    uint32_t bad;            // malformed entries this workgroup met
    int32_t ok;
    int64_t p_n, p_e;        // the chunk's offsets in the next frontier
    int64_t res[kBarrierWords];
    int64_t gather[kWaves][4];
};

__device__ __forceinline__ uint32_t lanes_before(uint64_t mask)
{
    return __builtin_amdgcn_mbcnt_hi(uint32_t(mask >> 32), __builtin_amdgcn_mbcnt_lo(uint32_t(mask), 0u));
}

__device__ __forceinline__ void give_up(const BfsArgs& a, uint32_t tag)
{
    __hip_atomic_store(a.abort_word, tag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(a.timeout_flag, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Degree of v with *beg its first edge, or -1 if its row range is not
// inside [0, E].
__device__ __forceinline__ int64_t row_range(const BfsArgs& a, int64_t v, int64_t* beg)
{
    const int64_t b0 = a.row[v], b1 = a.row[v + 1];
    *beg = b0;
    return (b0 >= 0 && b1 >= b0 && b1 <= a.ne) ? b1 - b0 : -1;
}

// Exclusive +-scan of one int64 per thread over the workgroup; *total gets
// the sum.  Ends with the workgroup synchronised.
__device__ __forceinline__ int64_t block_exclusive_sum(int64_t v, BfsShared& s, int64_t* total)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t inc = wave_inclusive_scan<AddI64>(v);
    if (lane == 63) s.wave_tot[wave] = inc;
    __syncthreads();
    int64_t before = 0, all = 0;
#pragma unroll
    for (int k = 0; k < kWaves; ++k) {
        const int64_t t = s.wave_tot[k];
        before += (k < wave) ? t : 0;
        all += t;
    }
    *total = all;
    __syncthreads();
    return before + inc - v;
}

// The chunk vertex that owns flat edge rank r: the last k < n with eo[k] <= r.
__device__ __forceinline__ int owner_of(const BfsShared& s, int n, int64_t r)
{
    int lo = 0, hi = n;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (s.eo[mid] <= r)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

// Sum of the packed values of chunks [lo, lo + cnt) (cnt < kBfsMaxGrid),
// read by the whole workgroup: every load in flight before the first wait,
// so the window costs one round trip.  Integer sums, so the order of the
// additions does not matter.  `ok` (every thread's) turns false if a wait
// gave up.  Ends with the workgroup synchronised.
__device__ __forceinline__ int64_t block_window_sum(const BfsArgs& a, BfsShared& s, int64_t lo, int64_t cnt,
                                                    uint32_t tag, bool& ok)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int64_t sum = 0;
    for (int i0 = 0; i0 < kGatherPer; i0 += kFoldBatch) {
        if (threadIdx.x + int64_t(i0) * kBfsThreads >= cnt) break;
        uint64_t w[kFoldBatch][2];
#pragma unroll
        for (int i = 0; i < kFoldBatch; ++i) {
            const int64_t j = threadIdx.x + int64_t(i0 + i) * kBfsThreads;
#pragma unroll
            for (int k = 0; k < 2; ++k)
                w[i][k] = (j < cnt) ? slot_load(a.slots + 2 * (lo + j) + k) : (uint64_t(tag) << 32);
        }
#pragma unroll
        for (int i = 0; i < kFoldBatch; ++i) {
            const int64_t j = threadIdx.x + int64_t(i0 + i) * kBfsThreads;
            if (j < cnt) {
#pragma unroll
                for (int k = 0; k < 2; ++k)
                    w[i][k] = await_word(a.slots + 2 * (lo + j) + k, w[i][k], tag, a.spin_limit, a.abort_word, ok);
                sum += int64_t(uint64_t(uint32_t(w[i][0])) | (uint64_t(uint32_t(w[i][1])) << 32));
            }
        }
    }
    const bool wave_ok = __ballot(!ok) == 0;
    sum = read_lane(wave_inclusive_scan<AddI64>(sum), 63);
    if (lane == 0) {
        s.gather[wave][0] = sum;
        s.gather[wave][3] = wave_ok ? 1 : 0;
    }
    __syncthreads();
    int64_t all = 0;
    bool all_ok = true;
#pragma unroll
    for (int k = 0; k < kWaves; ++k) {
        all += s.gather[k][0];
        all_ok = all_ok && s.gather[k][3] != 0;
    }
    ok = all_ok;
    __syncthreads();
    return all;
}

// Grid barrier over flag words.  Every workgroup publishes the four 32-bit
// values v[] (thread 0's) under `tag`; workgroup 0 adds them up over the
// grid (word 1 and 2 are the low and high halves of one 64-bit value) and
// publishes the sums, which every workgroup reads into s.res.  Writes made
// before the call are visible to every workgroup after it.  Returns false
// if a wait gave up.
__device__ bool grid_barrier(const BfsArgs& a, BfsShared& s, uint32_t tag, const uint32_t (&v)[kBarrierWords])
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    static_assert(kGatherPer * kBfsThreads >= kBfsMaxGrid, "workgroup 0 gathers the whole grid");
    // The workgroup barrier orders every wave's frontier writes before
    // thread 0's agent-scope release below, which makes them visible to the
    // whole device (a release is cumulative over what happens before it).
    __syncthreads();
    if (threadIdx.x == 0) {
        __hip_atomic_store(a.partial + blockIdx.x, int64_t(s.bad), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
#pragma unroll
        for (int k = 0; k < kBarrierWords; ++k)
            slot_store(a.arrive + kBarrierWords * blockIdx.x + k, (uint64_t(tag) << 32) | v[k]);
    }
    if (blockIdx.x == 0) {
        // every thread of workgroup 0 gathers up to kGatherPer workgroups'
        // arrivals, kGatherBatch of them in flight before the first wait
        bool ok = true;
        int64_t n = 0, e = 0, found = 0;
        for (int i0 = 0; i0 < kGatherPer; i0 += kGatherBatch) {
            if (threadIdx.x + int64_t(i0) * kBfsThreads >= int64_t(gridDim.x)) break;
            uint64_t w[kGatherBatch][kBarrierWords];
#pragma unroll
            for (int i = 0; i < kGatherBatch; ++i) {
                const int64_t j = threadIdx.x + int64_t(i0 + i) * kBfsThreads;
#pragma unroll
                for (int k = 0; k < kBarrierWords; ++k)
                    w[i][k] = (j < int64_t(gridDim.x)) ? slot_load(a.arrive + kBarrierWords * j + k)
                                                       : (uint64_t(tag) << 32);
            }
#pragma unroll
            for (int i = 0; i < kGatherBatch; ++i) {
                const int64_t j = threadIdx.x + int64_t(i0 + i) * kBfsThreads;
                if (j < int64_t(gridDim.x)) {
#pragma unroll
                    for (int k = 0; k < kBarrierWords; ++k)
                        w[i][k] = await_word(a.arrive + kBarrierWords * j + k, w[i][k], tag, a.spin_limit,
                                             a.abort_word, ok);
                }
                n += uint32_t(w[i][0]);
                e += int64_t(uint64_t(uint32_t(w[i][1])) | (uint64_t(uint32_t(w[i][2])) << 32));
                found += uint32_t(w[i][3]);
            }
        }
        // workgroup sums: waves through LDS
        const bool wave_ok = __ballot(!ok) == 0;
        n = read_lane(wave_inclusive_scan<AddI64>(n), 63);
        e = read_lane(wave_inclusive_scan<AddI64>(e), 63);
        found = read_lane(wave_inclusive_scan<AddI64>(found), 63);
        if (lane == 0) {
            s.gather[wave][0] = n;
            s.gather[wave][1] = e;
            s.gather[wave][2] = found;
            s.gather[wave][3] = wave_ok ? 1 : 0;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            bool all_ok = true;
            n = e = found = 0;
#pragma unroll
            for (int k = 0; k < kWaves; ++k) {
                n += s.gather[k][0];
                e += s.gather[k][1];
                found += s.gather[k][2];
                all_ok = all_ok && s.gather[k][3] != 0;
            }
            if (all_ok) {
                __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");
                const uint32_t out[kBarrierWords] = {uint32_t(n), uint32_t(uint64_t(e)), uint32_t(uint64_t(e) >> 32),
                                                     uint32_t(found)};
#pragma unroll
                for (int k = 0; k < kBarrierWords; ++k) slot_store(a.go + k, (uint64_t(tag) << 32) | out[k]);
            } else {
                give_up(a, tag);
            }
        }
    }
    if (threadIdx.x == 0) {
        bool ok = true;
        uint64_t w[kBarrierWords];
#pragma unroll
        for (int k = 0; k < kBarrierWords; ++k) {
            w[k] = slot_load(a.go + k);
            w[k] = await_word(a.go + k, w[k], tag, a.spin_limit, a.abort_word, ok);
        }
        if (!ok) give_up(a, tag);
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        s.ok = ok ? 1 : 0;
        s.res[0] = uint32_t(w[0]);
        s.res[1] = int64_t(uint64_t(uint32_t(w[1])) | (uint64_t(uint32_t(w[2])) << 32));
        s.res[2] = 0;
        s.res[3] = uint32_t(w[3]);
    }
    __syncthreads();
    return s.ok != 0;
}

__global__ void __launch_bounds__(kBfsThreads) bfs_kernel(BfsArgs a)
{
    if (a.residency_check) {
        check_residency(a.ctrl, a.spin_limit);
        return;
    }
    __shared__ BfsShared s;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t B = gridDim.x, wg = blockIdx.x;
    const int64_t V = a.nv;

    // Initial state: nothing visited but the source; the first frontier is
    // the source if it has edges.  Every
    // workgroup also counts the places where the row offsets decrease: rows
    // that overlap would break the bound of the chunk tables, so such a
    // graph is not searched.
    int64_t src_beg = 0;
    const int64_t src_deg = row_range(a, a.src, &src_beg);
    uint32_t decreasing = 0;
    for (int64_t v = wg * kBfsThreads + tid; v < V; v += B * kBfsThreads) {
        const bool is_src = (v == a.src);
        if ((v & 31) == 0) a.visited[v >> 5] = ((a.src >> 5) == (v >> 5)) ? (1u << (a.src & 31)) : 0u;
        a.level[v] = is_src ? 0 : -1;
        if (a.parent) a.parent[v] = is_src ? a.src : -1;
        decreasing += (a.row[v] > a.row[v + 1]) ? 1u : 0u;
    }
    const int64_t d0 = (src_deg > 0) ? src_deg : 0;
    if (wg == 0 && tid == 0 && d0 > 0) {
        a.queue[0][0] = a.src;
        a.edge_off[0][0] = 0;
        a.edge_shift[0][0] = src_beg;
    }
    for (int64_t b = wg * kBfsThreads + tid; b * K < d0 && b < a.chunk_cap; b += B * kBfsThreads)
        a.chunk_first[0][b] = 0;
    if (tid == 0) {
        s.bad = (wg == 0 && src_deg < 0) ? 1u : 0u;
        s.found_all = 0;
        s.found = 0;
    }
    __syncthreads();
    if (decreasing) atomicAdd(&s.found, decreasing);
    __syncthreads();

    uint32_t tag = a.base_tag + 1u;
    uint32_t v0[kBarrierWords] = {0u, 0u, 0u, s.found};
    bool ok = grid_barrier(a, s, tag, v0);
    const int64_t bad_rows = s.res[3];
    if (ok && bad_rows > 0) {
        // not searched: nothing reached, the decreasing steps reported
        if (wg == 0 && tid == 0) {
            a.level[a.src] = -1;
            if (a.parent) a.parent[a.src] = -1;
            if (a.stats) {
                a.stats[0] = 0;
                a.stats[1] = 0;
                a.stats[2] = 0;
                a.stats[3] = bad_rows;
            }
        }
        return;
    }

    int64_t f = (d0 > 0) ? 1 : 0, D = d0;
    int64_t levels = 1, reached = 1, scanned = 0;
    int32_t lev = 0;
    while (ok && f > 0) {
        ++tag;
        const int q = lev & 1;
        const int32_t* cur = a.queue[q];
        const int64_t* cur_eo = a.edge_off[q];
        const int64_t* cur_sh = a.edge_shift[q];
        const int32_t* cur_cf = a.chunk_first[q];
        int32_t* nxt = a.queue[q ^ 1];
        int64_t* nxt_eo = a.edge_off[q ^ 1];
        int64_t* nxt_sh = a.edge_shift[q ^ 1];
        int32_t* nxt_cf = a.chunk_first[q ^ 1];
        const int64_t nc = (D + K - 1) / K;
        if (nc > a.chunk_cap) break;  // cannot happen with non-decreasing rows (memory guard)
        scanned += D;
        int64_t run_n = 0, run_e = 0;    // offsets through this workgroup's previous chunk
        int64_t mine_n = 0, mine_e = 0;  // what this workgroup placed in this level
        if (tid == 0) s.found_all = 0;
        // Software pipeline: the iteration that claims chunk c places this
        // workgroup's previous chunk c - B, whose window of counts was
        // published about a round earlier, so placing rarely waits.
        int64_t prev_c = -1, prev_n = 0, prev_e = 0;
        int sb = 0;  // stage buffer of the chunk being claimed
        for (int64_t c = wg;; c += B) {
            const bool have = c < nc;
            int64_t A_n = 0, A_e = 0;  // the claimed chunk's staged vertices and their edges
            if (have) {
                // (a) the chunk's frontier vertices
                const int64_t r_lo = c * K;
                const int64_t r_hi = (D - r_lo < K) ? D : r_lo + K;
                int64_t k0 = cur_cf[c];
                int64_t kend = (c + 1 < nc) ? int64_t(cur_cf[c + 1]) : f - 1;
                k0 = (k0 < 0) ? 0 : (k0 >= f ? f - 1 : k0);  // memory guards: the table is consistent
                kend = (kend < k0) ? k0 : (kend >= f ? f - 1 : kend);
                if (kend - k0 > K) kend = k0 + K;
                const int n = int(kend - k0 + 1);
                for (int j = tid; j < n; j += kBfsThreads) {
                    s.eo[j] = cur_eo[k0 + j];
                    s.shift[j] = cur_sh[k0 + j];
                    s.u[j] = cur[k0 + j];
                }
                if (tid == 0) {
                    s.eo[n] = INT64_MAX;
                    s.found = 0;
                    s.found_e = 0;
                }
                __syncthreads();

                // (b) map each rank to its edge and vertex, then claim every
                //     endpoint not yet visited; stage the winners that have edges
                int64_t e[kPer];
                int32_t u[kPer];
                bool act[kPer];
#pragma unroll
                for (int p = 0; p < kPer; ++p) {
                    const int64_t r = r_lo + int64_t(p) * kBfsThreads + tid;
                    act[p] = false;
                    e[p] = 0;
                    u[p] = -1;
                    if (r < r_hi) {
                        const int kk = owner_of(s, n, r);
                        e[p] = r + s.shift[kk];
                        u[p] = s.u[kk];
                        act[p] = (e[p] >= 0 && e[p] < a.ne);
                        if (!act[p]) atomicAdd(&s.bad, 1u);
                    }
                }
                int32_t v[kPer];
#pragma unroll
                for (int p = 0; p < kPer; ++p) v[p] = act[p] ? a.col[e[p]] : -1;
                uint32_t bits[kPer];
#pragma unroll
                for (int p = 0; p < kPer; ++p) {
                    if (act[p] && uint32_t(v[p]) >= uint32_t(V)) {
                        atomicAdd(&s.bad, 1u);
                        act[p] = false;
                    }
                    bits[p] = act[p] ? a.visited[v[p] >> 5] : ~0u;  // a stale clear bit only costs an atomic
                }
                bool win[kPer];
#pragma unroll
                for (int p = 0; p < kPer; ++p) {
                    const uint32_t mask = 1u << (v[p] & 31);
                    win[p] = false;
                    if (act[p] && !(bits[p] & mask))
                        win[p] = !(atomicOr(a.visited + (v[p] >> 5), mask) & mask);
                }
                int64_t dv[kPer];
#pragma unroll
                for (int p = 0; p < kPer; ++p) {
                    dv[p] = 0;
                    if (win[p]) {
                        a.level[v[p]] = lev + 1;
                        if (a.parent) a.parent[v[p]] = u[p];
                        int64_t beg;
                        dv[p] = row_range(a, v[p], &beg);
                        if (dv[p] < 0) {
                            atomicAdd(&s.bad, 1u);
                            dv[p] = 0;
                        }
                    }
                }
#pragma unroll
                for (int p = 0; p < kPer; ++p) {
                    const bool keep = win[p] && dv[p] > 0;
                    const uint64_t m_all = __ballot(win[p]);
                    const uint64_t m = __ballot(keep);
                    uint32_t base = 0;
                    if (lane == 0) {
                        if (m_all) atomicAdd(&s.found_all, uint32_t(__popcll(m_all)));
                        if (m) base = atomicAdd(&s.found, uint32_t(__popcll(m)));
                    }
                    base = __builtin_amdgcn_readlane(base, 0);
                    if (keep) {
                        const uint32_t pos = base + lanes_before(m);  // < K: one discovery per edge at most
                        s.stage[sb][pos] = v[p];
                        atomicAdd(reinterpret_cast<unsigned long long*>(&s.found_e), (unsigned long long)dv[p]);
                    }
                }
                __syncthreads();
                A_n = s.found;
                A_e = int64_t(s.found_e);

                // (c) publish (edges, vertices) packed, at once
                if (wave == 0) publish_slot(a.slots + 2 * c, (A_e << kBfsCountBits) | A_n, tag, lane);
                mine_n += A_n;
                mine_e += A_e;
                if (prev_c < 0) {
                    prev_c = c;
                    prev_n = A_n;
                    prev_e = A_e;
                    sb ^= 1;
                    continue;
                }
            }
            if (prev_c < 0) break;  // no chunks in this level

            // (d) place the previous chunk: offsets = own running total + the
            //     values of the chunks in between; then its vertices, their
            //     edge offsets and first edges, and the next level's chunk
            //     table entries that fall in their edge ranges
            {
                const int32_t* st = s.stage[sb ^ 1];  // where the previous chunk was staged
                int32_t vl[kPer];
                int64_t bl[kPer], dl[kPer];
                int64_t dsum = 0;
#pragma unroll
                for (int t = 0; t < kPer; ++t) {  // loads in flight during the window wait
                    const int j = tid * kPer + t;
                    vl[t] = -1;
                    bl[t] = 0;
                    dl[t] = 0;
                    if (j < prev_n) {
                        vl[t] = st[j];
                        bl[t] = a.row[vl[t]];
                        dl[t] = a.row[vl[t] + 1] - bl[t];
                    }
                }
                const int64_t lo = (prev_c - B + 1 > 0) ? prev_c - B + 1 : 0;
                bool good = true;
                const int64_t between = block_window_sum(a, s, lo, prev_c - lo, tag, good);
                if (!good) {
                    if (tid == 0) give_up(a, tag);
                    ok = false;
                    break;
                }
                const int64_t p_n = run_n + (between & kCountMask);
                const int64_t p_e = run_e + (between >> kBfsCountBits);
                run_n = p_n + prev_n;
                run_e = p_e + prev_e;
#pragma unroll
                for (int t = 0; t < kPer; ++t) dsum += dl[t];
                int64_t tot = 0;
                int64_t eoff = p_e + block_exclusive_sum(dsum, s, &tot);
#pragma unroll
                for (int t = 0; t < kPer; ++t) {
                    const int j = tid * kPer + t;
                    if (j < prev_n) {
                        const int64_t pos = p_n + j;
                        if (pos < V) {
                            nxt[pos] = vl[t];
                            nxt_eo[pos] = eoff;
                            nxt_sh[pos] = bl[t] - eoff;
                            for (int64_t b = (eoff + K - 1) / K; b * K < eoff + dl[t] && b < a.chunk_cap; ++b)
                                nxt_cf[b] = int32_t(pos);
                        }
                        eoff += dl[t];
                    }
                }
            }
            if (!have) break;
            prev_c = c;
            prev_n = A_n;
            prev_e = A_e;
            sb ^= 1;
        }
        if (!ok) break;
        // (e) the level barrier: the next frontier's size and edges
        const uint32_t vb[kBarrierWords] = {uint32_t(mine_n), uint32_t(uint64_t(mine_e)),
                                            uint32_t(uint64_t(mine_e) >> 32), s.found_all};
        ok = grid_barrier(a, s, tag, vb);
        if (!ok) break;
        f = s.res[0];
        D = s.res[1];
        if (f > V) f = V;  // cannot happen: each vertex is claimed once (memory guard)
        if (s.res[3] > 0) {
            ++levels;
            reached += s.res[3];
        }
        ++lev;
    }

    if (ok && wg == 0 && tid == 0 && a.stats) {
        int64_t bad = 0;
        for (int64_t j = 0; j < B; ++j)
            bad += __hip_atomic_load(a.partial + j, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        a.stats[0] = levels;
        a.stats[1] = reached;
        a.stats[2] = scanned;
        a.stats[3] = bad;
    }
}

}  // namespace

hipError_t launch_bfs(const BfsArgs& a, int grid, hipStream_t stream)
{
    (void)hipGetLastError();
    hipLaunchKernelGGL(bfs_kernel, dim3(unsigned(grid)), dim3(kBfsThreads), 0, stream, a);
    return hipGetLastError();
}

const void* bfs_kernel_func() { return reinterpret_cast<const void*>(&bfs_kernel); }

}  // namespace lscan
