// copy_ceiling.hip -- streaming copies that bound what the scan can move.
//
// The scan reads every input byte once and writes every output byte once
// (paper, Section 1, contribution (i)), so a copy of the same bytes is its
// practical ceiling.  Two structures are measured beside it:
//   * persistent cyclic: the scan's own structure without the hand-off --
//     a fixed grid of resident workgroups takes tiles round-robin (tile i
//     on workgroup i mod B, Section 4), each lane moves the same 16-byte
//     non-temporal vectors as the scan (wave w owns R consecutive 1 KiB
//     rows of the tile), and the loads of tile i are issued before the
//     stores of tile i - B, which waited in registers (the scan's one-round
//     pipeline);
//   * persistent cyclic with strips: the same grid and pipeline, but row r of
//     a tile is row r of wave 0, then of wave 1, ... (a wave's rows are T * 16
//     bytes apart), so the r-th load of the whole workgroup reads one
//     contiguous span of T * 16 bytes -- the best persistent structure found
//     on MI355X (the scan keeps each wave's rows contiguous: its in-lane and
//     cross-lane steps measured faster that way);
//   * flat grid: one tile per workgroup, as many workgroups as tiles,
//     dispatched by the hardware (no forward-progress requirement, no
//     hand-off possible without an atomic ticket).
// Built into its own library; only the benchmark loads it.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

namespace {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

template <int T, int R, bool STRIPS>
__global__ void __launch_bounds__(T) copy_persistent(const u32x4* __restrict__ x, u32x4* __restrict__ y,
                                                     int64_t nvec)
{
    constexpr int64_t TILE = int64_t(T) * R;  // vectors per tile
    constexpr int64_t RSTEP = STRIPS ? T : 64;  // vectors from one of a lane's rows to the next
    const int64_t B = gridDim.x;
    const int64_t M = (nvec + TILE - 1) / TILE;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t lane0 = (STRIPS ? int64_t(wave) * 64 : int64_t(wave) * R * 64) + lane;  // row 0 of this lane
    u32x4 pend[R];
    int64_t pb = -1;
    for (int64_t b = blockIdx.x;; b += B) {
        const bool have = b < M;
        u32x4 v[R];
        if (have) {
            const int64_t base = b * TILE + lane0;
            if ((b + 1) * TILE <= nvec) {
#pragma unroll
                for (int r = 0; r < R; ++r) v[r] = __builtin_nontemporal_load(x + base + int64_t(r) * RSTEP);
            } else {
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const int64_t q = base + int64_t(r) * RSTEP;
                    v[r] = q < nvec ? x[q] : u32x4{0u, 0u, 0u, 0u};
                }
            }
        }
        if (pb >= 0) {
            const int64_t base = pb * TILE + lane0;
            if ((pb + 1) * TILE <= nvec) {
#pragma unroll
                for (int r = 0; r < R; ++r) __builtin_nontemporal_store(pend[r], y + base + int64_t(r) * RSTEP);
            } else {
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const int64_t q = base + int64_t(r) * RSTEP;
                    if (q < nvec) y[q] = pend[r];
                }
            }
        }
        if (!have) break;
#pragma unroll
        for (int r = 0; r < R; ++r) pend[r] = v[r];
        pb = b;
    }
}

template <int T, int R>
__global__ void __launch_bounds__(T) copy_flat(const u32x4* __restrict__ x, u32x4* __restrict__ y, int64_t nvec)
{
    constexpr int64_t TILE = int64_t(T) * R;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t base = int64_t(blockIdx.x) * TILE + int64_t(wave) * R * 64 + lane;
    u32x4 v[R];
    if ((int64_t(blockIdx.x) + 1) * TILE <= nvec) {
#pragma unroll
        for (int r = 0; r < R; ++r) v[r] = __builtin_nontemporal_load(x + base + int64_t(r) * 64);
#pragma unroll
        for (int r = 0; r < R; ++r) __builtin_nontemporal_store(v[r], y + base + int64_t(r) * 64);
    } else {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int64_t q = base + int64_t(r) * 64;
            if (q < nvec) y[q] = x[q];
        }
    }
}

typedef void (*CopyFn)(const u32x4*, u32x4*, int64_t);

struct Shape {
    int threads, vectors;
    CopyFn persistent, flat, strips;
};

#define LSCAN_COPY_SHAPE(T, R) {T, R, copy_persistent<T, R, false>, copy_flat<T, R>, copy_persistent<T, R, true>}
const Shape kShapes[] = {
    LSCAN_COPY_SHAPE(256, 1), LSCAN_COPY_SHAPE(256, 4), LSCAN_COPY_SHAPE(256, 8),
    LSCAN_COPY_SHAPE(256, 16), LSCAN_COPY_SHAPE(512, 8), LSCAN_COPY_SHAPE(1024, 4),
};
#undef LSCAN_COPY_SHAPE

}  // namespace

extern "C" {

// Copy `bytes` (a multiple of 16; x and y 16-byte aligned, not overlapping)
// from x to y on `stream`.  structure 0: flat grid; 1: persistent cyclic
// grid of groups_per_cu workgroups per CU (capped by the occupancy limit and
// by the number of tiles), each wave's rows contiguous; 2: the same grid
// with strips (rows across waves).  *grid_out receives the grid.  Returns 0,
// or -1 for bad arguments / an uncompiled shape, -4 for a HIP error.
int ceiling_copy(const void* x, void* y, int64_t bytes, int structure, int threads, int vectors,
                 int groups_per_cu, void* stream, int* grid_out)
{
    if (!x || !y || bytes < 0 || bytes % 16 || reinterpret_cast<uintptr_t>(x) % 16 ||
        reinterpret_cast<uintptr_t>(y) % 16 || structure < 0 || structure > 2)
        return -1;
    const Shape* sh = nullptr;
    for (const Shape& s : kShapes)
        if (s.threads == threads && s.vectors == vectors) sh = &s;
    if (!sh) return -1;
    const int64_t nvec = bytes / 16;
    if (nvec == 0) return 0;
    const int64_t tile = int64_t(threads) * vectors;
    const int64_t M = (nvec + tile - 1) / tile;
    int64_t grid = M;
    CopyFn fn = sh->flat;
    if (structure != 0) {
        int dev = 0, cus = 0, occ = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(
                &occ, reinterpret_cast<const void*>(structure == 1 ? sh->persistent : sh->strips), threads, 0) !=
                hipSuccess)
            return -4;
        if (groups_per_cu < 1) return -1;
        grid = std::min<int64_t>(M, int64_t(std::min(groups_per_cu, occ)) * cus);
        fn = structure == 1 ? sh->persistent : sh->strips;
    } else if (grid > int64_t(INT32_MAX)) {
        return -1;
    }
    (void)hipGetLastError();
    hipLaunchKernelGGL(fn, dim3(unsigned(grid)), dim3(threads), 0, static_cast<hipStream_t>(stream),
                       static_cast<const u32x4*>(x), static_cast<u32x4*>(y), nvec);
    if (hipGetLastError() != hipSuccess) return -4;
    if (grid_out) *grid_out = int(grid);
    return 0;
}

}  // extern "C"
