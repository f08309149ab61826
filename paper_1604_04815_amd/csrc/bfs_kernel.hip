// bfs_kernel.hip -- breadth-first search as a persistent grid of workgroups
// that talk to each other only through epoch-tagged flag words: the paper's
// inter-block hand-off (Section 4.3) used for the graph search it names as
// the next application of that hand-off (Section 6), in place of the atomic
// queue-tail counter that level-synchronous GPU searches usually use.
//
// One launch runs the whole search, level by level (top-down expansion):
//   * The frontier of level l is a queue of f vertices, cut into chunks of
//     kBfsChunk vertices.  Chunk c is taken by workgroup c mod B, in
//     increasing c (the cyclic distribution of the scan).
//   * Per chunk, the workgroup lays the chunk's edges out flat (an exclusive
//     scan of the degrees in LDS), walks them with one edge per thread, and
//     claims every endpoint not yet discovered with a compare-and-swap of
//     the vertex's claim word from "none" to the edge index.  The winners --
//     the vertices of level l + 1 that this chunk discovered -- are counted
//     and kept in LDS.
//   * Where the discoveries go in the next frontier is a scan over chunks:
//     the chunk publishes its count A(c) in its flag word at once, then
//     obtains its offset from the counts of the B - 1 chunks before it and
//     its own previous chunk's running total (the window fold of the scan),
//     and writes its discoveries there.  No shared tail counter is bumped.
//   * A level ends with a grid barrier built from the same flag words: each
//     workgroup publishes (tag, vertices it placed); workgroup 0 gathers
//     them, and publishes (tag, size of the next frontier), which every
//     workgroup waits for.  The next frontier's writes are released before
//     the arrival and acquired after the release word, at agent scope.
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
constexpr int kUnroll = 4;  // edges per thread in flight at once
constexpr uint64_t kUnclaimed = ~uint64_t(0);

struct BfsShared {
    int64_t off[kBfsChunk + 1];  // exclusive prefix of the chunk's degrees; off[n] = edges of the chunk
    int64_t beg[kBfsChunk];      // first edge of each chunk vertex
    int32_t u[kBfsChunk];        // the chunk's vertices
    int32_t stage[kBfsStage];    // vertices the chunk discovered (first kBfsStage of them)
    int64_t wave_tot[kWaves];
    uint32_t wave_cnt[kWaves];
    uint32_t found;              // discoveries of the chunk
    uint32_t bad;                // malformed row or column entries seen by this workgroup
    int32_t prefix;              // the chunk's offset in the next frontier
    int32_t result;              // a barrier's result for the whole workgroup (-1: gave up)
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

// The chunk vertex that owns flat edge rank r: the last k < n with off[k] <= r.
__device__ __forceinline__ int owner_of(const BfsShared& s, int n, int64_t r)
{
    int lo = 0, hi = n;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (s.off[mid] <= r)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

// Grid barrier over flag words.  Every workgroup publishes `mine` under
// `tag`; workgroup 0 sums the B arrivals and publishes the sum, which every
// workgroup returns (-1 if a wait gave up).  Writes made before the call are
// visible to every workgroup after it.
__device__ int32_t grid_barrier(const BfsArgs& a, BfsShared& s, uint32_t tag, uint32_t mine, int64_t edges)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");  // this wave's frontier writes
    __syncthreads();
    if (threadIdx.x == 0) {
        __hip_atomic_store(a.partial + 2 * blockIdx.x, edges, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(a.partial + 2 * blockIdx.x + 1, int64_t(s.bad), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        slot_store(a.arrive + blockIdx.x, (uint64_t(tag) << 32) | mine);
    }
    if (blockIdx.x == 0 && wave == 0) {
        bool ok = true;
        uint32_t sum = 0;
        for (int64_t j = lane; j < int64_t(gridDim.x); j += 64) {
            uint64_t w = slot_load(a.arrive + j);
            w = await_word(a.arrive + j, w, tag, a.spin_limit, a.abort_word, ok);
            sum += uint32_t(w);
        }
        const bool all_ok = __ballot(!ok) == 0;
        sum = uint32_t(read_lane(wave_inclusive_scan<AddI32>(int32_t(sum)), 63));
        if (lane == 0) {
            if (all_ok) {
                __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");
                slot_store(a.go, (uint64_t(tag) << 32) | sum);
            } else {
                give_up(a, tag);
            }
        }
    }
    if (threadIdx.x == 0) {
        bool ok = true;
        uint64_t w = slot_load(a.go);
        w = await_word(a.go, w, tag, a.spin_limit, a.abort_word, ok);
        if (!ok) give_up(a, tag);
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        s.result = ok ? int32_t(uint32_t(w)) : -1;
    }
    __syncthreads();
    return s.result;
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

    // Initial state: nothing claimed but the source (whose claim names no edge).
    for (int64_t v = wg * kBfsThreads + tid; v < V; v += B * kBfsThreads) {
        const bool is_src = (v == a.src);
        a.claim[v] = is_src ? uint64_t(a.ne) : kUnclaimed;
        a.level[v] = is_src ? 0 : -1;
        if (a.parent) a.parent[v] = is_src ? a.src : -1;
    }
    if (wg == 0 && tid == 0) a.queue0[0] = a.src;
    if (tid == 0) s.bad = 0;

    int64_t edges = 0;  // edges this workgroup scanned (thread 0's count)
    uint32_t tag = a.base_tag + 1u;
    int32_t f = (grid_barrier(a, s, tag, 0u, 0) < 0) ? -1 : 1;
    int64_t reached = 1;
    int32_t lev = 0;

    while (f > 0) {
        ++tag;
        const int32_t* cur = (lev & 1) ? a.queue1 : a.queue0;
        int32_t* nxt = (lev & 1) ? a.queue0 : a.queue1;
        const int64_t nc = (int64_t(f) + kBfsChunk - 1) / kBfsChunk;
        int32_t run = 0;     // discoveries of chunks 0 .. (this workgroup's previous chunk)
        uint32_t mine = 0;   // discoveries this workgroup placed in this level
        bool ok = true;
        for (int64_t c = wg; c < nc; c += B) {
            // (a) the chunk's vertices, their edge ranges, flat edge ranks
            const int n = int((int64_t(f) - c * kBfsChunk < kBfsChunk) ? int64_t(f) - c * kBfsChunk : kBfsChunk);
            int64_t deg = 0, b0 = 0;
            int32_t u = -1;
            if (tid < n) {
                u = cur[c * kBfsChunk + tid];
                if (uint32_t(u) < uint32_t(V)) {
                    b0 = a.row[u];
                    const int64_t b1 = a.row[u + 1];
                    if (b0 >= 0 && b1 >= b0 && b1 <= a.ne)
                        deg = b1 - b0;
                    else
                        atomicAdd(&s.bad, 1u);
                }
            }
            int64_t D = 0;
            const int64_t off = block_exclusive_sum(deg, s, &D);
            if (tid < n) {
                s.off[tid] = off;
                s.beg[tid] = b0;
                s.u[tid] = u;
            }
            if (tid == 0) {
                s.off[n] = D;
                s.found = 0;
                edges += D;
            }
            __syncthreads();

            // (b) claim every endpoint not yet discovered; stage the winners
            for (int64_t r0 = 0; r0 < D; r0 += int64_t(kBfsThreads) * kUnroll) {
                int k[kUnroll];
                int64_t e[kUnroll];
                int32_t v[kUnroll];
#pragma unroll
                for (int q = 0; q < kUnroll; ++q) {
                    const int64_t r = r0 + int64_t(q) * kBfsThreads + tid;
                    k[q] = -1;
                    e[q] = 0;
                    if (r < D) {
                        k[q] = owner_of(s, n, r);
                        e[q] = s.beg[k[q]] + (r - s.off[k[q]]);
                    }
                }
#pragma unroll
                for (int q = 0; q < kUnroll; ++q) v[q] = (k[q] >= 0) ? a.col[e[q]] : -1;
                uint64_t cl[kUnroll];
#pragma unroll
                for (int q = 0; q < kUnroll; ++q) {
                    const bool valid = (k[q] >= 0) && uint32_t(v[q]) < uint32_t(V);
                    if (k[q] >= 0 && !valid) atomicAdd(&s.bad, 1u);
                    if (!valid) k[q] = -1;
                    cl[q] = (k[q] >= 0) ? a.claim[v[q]] : 0;  // a stale "none" only costs a failed swap
                }
#pragma unroll
                for (int q = 0; q < kUnroll; ++q) {
                    bool win = false;
                    if (k[q] >= 0 && cl[q] == kUnclaimed) {
                        win = atomicCAS(reinterpret_cast<unsigned long long*>(a.claim + v[q]),
                                        (unsigned long long)kUnclaimed, (unsigned long long)e[q]) ==
                              (unsigned long long)kUnclaimed;
                        if (win) {
                            a.level[v[q]] = lev + 1;
                            if (a.parent) a.parent[v[q]] = s.u[k[q]];
                        }
                    }
                    const uint64_t m = __ballot(win);
                    uint32_t base = 0;
                    if (lane == 0 && m != 0) base = atomicAdd(&s.found, uint32_t(__popcll(m)));
                    base = __builtin_amdgcn_readlane(base, 0);
                    const uint32_t pos = base + lanes_before(m);
                    if (win && pos < uint32_t(kBfsStage)) s.stage[pos] = v[q];
                }
            }
            __syncthreads();
            const uint32_t A = s.found;

            // (c) publish A(c); offset = own previous running total + the
            //     counts of the chunks in between (window fold)
            if (wave == 0) {
                if (lane == 0) slot_store(a.slots + c, (uint64_t(tag) << 32) | A);
                const int64_t lo = (c - B + 1 > 0) ? c - B + 1 : 0;
                bool good = true;
                const int32_t between = window_fold<AddI32>(a.slots, lo, c - lo, tag, a.spin_limit, a.abort_word,
                                                            lane, good);
                const bool all_good = __ballot(!good) == 0;
                if (lane == 0) {
                    s.prefix = all_good ? run + between : -1;
                    if (!all_good) give_up(a, tag);
                }
            }
            __syncthreads();
            const int32_t p = s.prefix;
            if (p < 0) {
                ok = false;
                break;
            }
            run = p + int32_t(A);
            mine += A;

            // (d) place the discoveries at p .. p + A - 1
            if (A <= uint32_t(kBfsStage)) {
                for (uint32_t q = tid; q < A; q += kBfsThreads)
                    if (int64_t(p) + q < V) nxt[p + q] = s.stage[q];
            } else {
                // more than LDS holds: walk the edges again and emit those
                // whose claim names them (this chunk's winners, in rank order)
                int64_t placed = p;
                for (int64_t r0 = 0; r0 < D; r0 += kBfsThreads) {
                    const int64_t r = r0 + tid;
                    bool win = false;
                    int32_t v = -1;
                    if (r < D) {
                        const int k = owner_of(s, n, r);
                        const int64_t e = s.beg[k] + (r - s.off[k]);
                        v = a.col[e];
                        if (uint32_t(v) < uint32_t(V))
                            win = __hip_atomic_load(a.claim + v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ==
                                  uint64_t(e);
                    }
                    const uint64_t m = __ballot(win);
                    if (lane == 0) s.wave_cnt[wave] = uint32_t(__popcll(m));
                    __syncthreads();
                    uint32_t before = 0, all = 0;
#pragma unroll
                    for (int w = 0; w < kWaves; ++w) {
                        const uint32_t t = s.wave_cnt[w];
                        before += (w < wave) ? t : 0;
                        all += t;
                    }
                    const int64_t pos = placed + before + lanes_before(m);
                    if (win && pos < V) nxt[pos] = v;
                    placed += all;
                    __syncthreads();
                }
            }
            __syncthreads();  // LDS is reused by the next chunk
        }
        if (!ok) {
            f = -1;
            break;
        }
        // (e) the level barrier: the next frontier's size
        f = grid_barrier(a, s, tag, mine, edges);
        if (f > 0) {
            if (int64_t(f) > V) f = int32_t(V);  // cannot happen: each vertex is claimed once
            reached += f;
        }
        ++lev;
    }

    if (f == 0 && wg == 0 && tid == 0 && a.stats) {
        int64_t all_edges = 0, all_bad = 0;
        for (int64_t j = 0; j < B; ++j) {
            all_edges += __hip_atomic_load(a.partial + 2 * j, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            all_bad += __hip_atomic_load(a.partial + 2 * j + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        a.stats[0] = lev;
        a.stats[1] = reached;
        a.stats[2] = all_edges;
        a.stats[3] = all_bad;
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
