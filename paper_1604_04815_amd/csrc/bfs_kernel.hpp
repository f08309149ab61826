// bfs_kernel.hpp -- arguments of the breadth-first search kernel: one
// persistent launch runs a whole search, level by level, with every
// hand-off between workgroups made through epoch-tagged flag words.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lscan {

// Vertices of the frontier taken by one workgroup at a time (one per thread).
constexpr int kBfsThreads = 256;
constexpr int kBfsChunk = kBfsThreads;
// Vertices a chunk may discover and still keep in LDS; more are found again
// by a second walk over the chunk's edges.
constexpr int kBfsStage = 2048;

struct BfsArgs {
    const int64_t* row;      // V + 1 row offsets (compressed rows)
    const int32_t* col;      // E column indices
    int64_t nv;              // V (< 2^31)
    int64_t ne;              // E
    int32_t src;             // source vertex
    int32_t* level;          // V: level of each vertex, -1 unreached
    int32_t* parent;         // V or null: a BFS-tree parent (src for src, -1 unreached)
    int64_t* stats;          // 4 or null: levels, vertices reached, edges scanned, bad entries
    uint64_t* claim;         // V: edge index that discovered the vertex (all ones: not yet)
    int32_t* queue0;         // V: frontier of even levels
    int32_t* queue1;         // V: frontier of odd levels
    uint64_t* slots;         // ceil(V / chunk) flag words: per-chunk discovery counts
    uint64_t* arrive;        // grid words: level barrier arrivals (tag | vertices found)
    int64_t* partial;        // grid entries: edges scanned by each workgroup so far
    uint64_t* go;            // 1 word: barrier release (tag | next frontier size)
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
