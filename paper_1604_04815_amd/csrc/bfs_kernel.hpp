// bfs_kernel.hpp -- arguments of the breadth-first search kernel: one
// persistent launch runs a whole search, level by level, with every
// hand-off between workgroups made through epoch-tagged flag words.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lscan {

constexpr int kBfsThreads = 256;
// Edges of the frontier taken by one workgroup at a time (four per thread).
// A chunk discovers at most this many vertices, so its discoveries always
// fit in LDS.
constexpr int kBfsChunkEdges = 4 * kBfsThreads;
// Largest grid: a window of grid - 1 chunk counts (at most kBfsChunkEdges
// each) must fit the 21-bit count field of a packed flag value.
constexpr int kBfsMaxGrid = 2048;
constexpr int kBfsCountBits = 21;

struct BfsArgs {
    const int64_t* row;      // V + 1 row offsets (compressed rows)
    const int32_t* col;      // E column indices
    int64_t nv;              // V (< 2^31)
    int64_t ne;              // E (< 2^42)
    int32_t src;             // source vertex
    int32_t* level;          // V: level of each vertex, -1 unreached
    int32_t* parent;         // V or null: a BFS-tree parent (src for src, -1 unreached)
    int64_t* stats;          // 4 or null: levels, vertices reached, edges scanned, bad entries
    uint32_t* visited;       // ceil(V / 32): one bit per vertex, set by the vertex's claim
    int32_t* queue[2];       // V each: frontier vertices (those with at least one edge)
    int64_t* edge_off[2];    // V each: exclusive prefix of the frontier's degrees
    int64_t* edge_shift[2];  // V each: first edge of the vertex minus its edge offset
    int32_t* chunk_first[2]; // ceil(E / chunk) + 1 each: frontier index holding each chunk's first edge
    int64_t chunk_cap;       // entries of each chunk_first array (ceil(E / chunk) + 1)
    uint64_t* slots;         // 2 * chunk_cap flag words: packed per-chunk (edges << 21 | vertices)
    uint64_t* arrive;        // 4 * grid words: level barrier arrivals
                             // (vertices queued, their edges lo, hi, vertices found)
    int64_t* partial;        // grid: malformed entries seen by each workgroup
    uint64_t* go;            // 4 words: barrier release (the four sums)
    uint32_t* abort_word;    // tag of a wait that gave up (every waiter stops)
    uint32_t* timeout_flag;  // raised to 1 when a wait gives up
    uint32_t* ctrl;          // co-residency test words [4..6]
    uint64_t spin_limit;     // wall-clock ticks one wait may last
    uint32_t base_tag;       // tags base_tag + 1 .. base_tag + V + 2 belong to this launch
    int32_t residency_check; // 1: only test that the grid is resident at once
};

// Enqueue the search (or its co-residency test) with `grid` workgroups.
hipError_t launch_bfs(const BfsArgs& a, int grid, hipStream_t stream);

// The kernel function, for occupancy queries.
const void* bfs_kernel_func();

}  // namespace lscan
