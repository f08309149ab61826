/*
 * lscan.h -- C ABI of a single-pass, device-wide scan for AMD MI355X (gfx950).
 *
 * Operation (paper, Section 1): given a binary associative operator (+) and
 * x_0 .. x_{N-1}, the inclusive scan writes y_j = x_0 (+) ... (+) x_j and the
 * exclusive scan writes y_j = x_0 (+) ... (+) x_{j-1}, with y_0 = e, the
 * identity of (+).  The device method follows Section 4 of the paper: the
 * input is cut into M data blocks of L elements, a fixed set of B resident
 * workgroups takes the blocks round-robin (block i -> workgroup i mod B),
 * each block is scanned in registers (per-lane values, wave-wide cross-lane
 * scan, cross-wave pass through LDS), and block prefixes travel between
 * workgroups through flag words in device memory, so every x is read once
 * and every y written once in one kernel launch.
 *
 * Types and operators:
 *   LSCAN_I32, LSCAN_I64 : add (wraps modulo 2^32 / 2^64), max, min; exact.
 *   LSCAN_F32            : add (rounded; see LSCAN_F_COMPENSATED), max, min
 *                          (IEEE 754 totalOrder on non-NaN values, -0 < +0;
 *                          exact).  Output float32.
 *   LSCAN_BF16           : input bfloat16 (2-byte bit patterns), widened
 *                          exactly to float32; the scan runs in float32 and
 *                          the output is float32.
 * Identities: add 0; max: INT_MIN / -inf; min: INT_MAX / +inf.
 *
 * Pointers: x, y and offsets are DEVICE pointers owned by the caller, who
 * keeps them valid until the work completes (stream order).  x and y must be
 * aligned to their element size.  Full blocks use 16-byte vectors when x
 * sits on a vector boundary (16 bytes; 8 for bf16) and y on 16 bytes, or
 * when x and y sit the same number of elements past such boundaries (the
 * block grid is then shifted by that many elements).  Plain and segmented
 * scans whose y sits at another phase than x still read vectors and write
 * aligned vectors staged through LDS; batched arrays in that case move
 * every element on its own (slower).
 * y == x (in place) is allowed when input and output types are equal
 * (Section 4.5 of the paper: every element is read once before it is written
 * once); any other overlap is rejected.  Streams are hipStream_t passed as
 * void* (NULL = the null stream).  Calls are asynchronous: they validate,
 * enqueue one kernel launch and return.
 *
 * Errors are negative lscan_status values; arguments are checked before any
 * device work, so a rejected call has no effect.  HIP failures map to
 * LSCAN_ERR_DEVICE (the HIP code is kept per thread, see
 * lscan_last_device_error).  A workgroup that waits too long for a block
 * prefix (a forward-progress failure) stops, and the next lscan_check on
 * that stream reports LSCAN_ERR_TIMEOUT.
 *
 * Thread safety: every entry point may be called from any thread.  Each
 * (device, stream) pair owns its own flag workspace, so launches on one
 * stream are ordered and launches on different streams never share flags.
 * A scan's persistent grid fills the device, and two such grids running at
 * once on different streams could each hold part of it and wait for
 * workgroups that cannot become resident.  So a launch on a stream other
 * than the device's previous one first waits, on the device, for that
 * previous launch (hipStreamWaitEvent; launches on one stream pay nothing,
 * and the first switch to a second stream synchronizes the device once).
 * Graph replays and the request server's launches are not part of this
 * order: do not run them on a device at the same time as other scans.
 *
 * Graph capture: every call that enqueues device work, except
 * lscan_graph_launch, refuses a stream that
 * is being captured into a HIP graph (LSCAN_ERR_UNSUPPORTED, nothing
 * enqueued).  A kernel captured from such a call would keep pointers into
 * the stream's flag workspace, which a later call may free or regrow, and
 * its replays would escape the host's count of flag epochs.  To replay
 * scans, capture them with lscan_graph_create_*: those graphs own their
 * workspace.
 *
 * Besides the scans (plain, exclusive, segmented, batched, graph-captured,
 * served), the same persistent machinery gives: stream compaction
 * (lscan_compact), radix-sort digit offsets (lscan_radix_offsets),
 * breadth-first search with workgroups handing frontier offsets to each
 * other (lscan_bfs), and scans with a caller's own operator built from
 * lscan_custom.hpp (lscan_scan_custom).  These take part in the same
 * cross-stream order and honour the same watchdog (lscan_set_watchdog_us).
 */
#ifndef LSCAN_H
#define LSCAN_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LSCAN_I32 = 0,
    LSCAN_I64 = 1,
    LSCAN_F32 = 2,
    LSCAN_BF16 = 3 /* input only; the output is float32 */
} lscan_dtype;

/* LSCAN_ARGMAX / LSCAN_ARGMIN: running argmax / argmin, a pair operator on
 * (value, index): y[j] is the int64 index of the largest / smallest element
 * of the prefix, the earliest among equal values (float32 under totalOrder,
 * so -0 < +0); the exclusive form gives -1 for the empty prefix.  Keys
 * LSCAN_I32, LSCAN_I64, LSCAN_F32; plain inclusive / exclusive scans only
 * (segmented, batched, served, compensated and bf16: LSCAN_ERR_UNSUPPORTED).
 * y holds n int64 and may not overlap x. */
typedef enum {
    LSCAN_ADD = 0,
    LSCAN_MAX = 1,
    LSCAN_MIN = 2,
    LSCAN_ARGMAX = 3,
    LSCAN_ARGMIN = 4
} lscan_op;

/* flags */
#define LSCAN_F_COMPENSATED 0x1u /* F32/BF16 add: carry a TwoSum error term */
/* LSCAN_F_DETERMINISTIC asks for a fixed association of the float sums; it
 * is accepted everywhere and always met: both hand-offs fold in a fixed
 * order, so one tile shape and grid give the same bits on every run. */
#define LSCAN_F_DETERMINISTIC 0x2u
#define LSCAN_F_EXCLUSIVE 0x4u   /* lscan_segmented only: exclusive scan */
/* LSCAN_F_INDEX64: running argmax / argmin only -- run the kernels that
 * carry a 64-bit index whatever n is.  Arrays of fewer than 2^31 elements
 * normally take kernels with a 32-bit index (smaller values, faster), larger
 * ones always take the 64-bit kernels; the result is the same.  With any
 * other operator: LSCAN_ERR_INVALID_ARG. */
#define LSCAN_F_INDEX64 0x8u

typedef int32_t lscan_status;
#define LSCAN_OK 0
#define LSCAN_PENDING 1
#define LSCAN_ERR_INVALID_ARG (-1)
#define LSCAN_ERR_UNSUPPORTED (-2)
#define LSCAN_ERR_NO_MEMORY (-3)
#define LSCAN_ERR_DEVICE (-4)
#define LSCAN_ERR_AGAIN (-5)
#define LSCAN_ERR_TIMEOUT (-6)
#define LSCAN_ERR_NOT_FOUND (-7)

/*
 * lscan_inclusive -- y_j = x_0 (+) ... (+) x_j for j < n (paper Section 1;
 * device method of Section 4).
 *   x      device pointer, n elements of dt
 *   y      device pointer, n elements of the output type (F32 for BF16)
 *   n      element count, n >= 0; n == 0 is a no-op returning LSCAN_OK
 *   flags  0 or LSCAN_F_COMPENSATED (F32/BF16 with LSCAN_ADD only, else
 *          LSCAN_ERR_UNSUPPORTED), optionally | LSCAN_F_DETERMINISTIC
 * Float add results depend on the association fixed by the launch
 * parameters; for a fixed parameter set they are deterministic.
 */
lscan_status lscan_inclusive(const void *x, void *y, int64_t n, lscan_dtype dt,
                             lscan_op op, uint32_t flags, void *stream);

/*
 * lscan_exclusive -- y_0 = e, y_j = x_0 (+) ... (+) x_{j-1} (paper Section 1,
 * the variant it notes can be derived from the inclusive scan).  Arguments
 * as lscan_inclusive.
 */
lscan_status lscan_exclusive(const void *x, void *y, int64_t n, lscan_dtype dt,
                             lscan_op op, uint32_t flags, void *stream);

/*
 * lscan_inclusive_noalloc -- lscan_inclusive for callers that cannot
 * allocate device memory (tight serving loops, harnesses that forbid
 * hipMalloc): same arguments, same kernels, same results bit for bit, but
 * no allocation of any kind.  The flag words live in a static device array
 * of the library (4 MiB of flag slots plus 256 bytes of control words, held
 * by every GPU the library runs on until the process ends); the first call
 * on a device looks up that device's copy and clears it, the first call of
 * each kernel shape runs its co-residency test once on the same words.
 *   Limit: the blocks of the scan (n / tile size, the tile of the kernel the
 *   call selects) times its flag words per block must fit the 2^19 slots:
 *   add / max / min scans of any type up to about 2^33 elements, running
 *   argmax / argmin up to about 1.4e9.  Larger n: LSCAN_ERR_NO_MEMORY,
 *   decided on the host before any device work.
 *   Sharing: every call on one GPU uses that GPU's one array, and it keeps
 *   the last call's contents (flag words carry launch tags, so they need no
 *   clearing between calls).  Calls that overlap on one GPU -- on two
 *   streams or threads at once, or at the same time as any other scan of
 *   this library -- race on those words and may deadlock; order them.  A
 *   stream being captured is refused (LSCAN_ERR_UNSUPPORTED), as for
 *   lscan_inclusive.  A timed-out launch is reported by the next
 *   lscan_check on any stream of the device.
 */
lscan_status lscan_inclusive_noalloc(const void *x, void *y, int64_t n,
                                     lscan_dtype dt, lscan_op op,
                                     uint32_t flags, void *stream);

/*
 * lscan_segmented -- the scan of Section 1 applied independently to each
 * segment x[offsets[s], offsets[s+1]), s < num_segments, in ONE persistent
 * launch (the segmented operator on (head flag, value) pairs, which is
 * associative, so the block method of Section 4 applies unchanged).
 *   offsets  DEVICE pointer to num_segments + 1 non-decreasing int64 values
 *            with offsets[0] == 0; empty segments are allowed; n is
 *            offsets[num_segments], which the caller passes as n_total
 *   flags    LSCAN_F_EXCLUSIVE for the exclusive form, LSCAN_F_COMPENSATED
 *            as above
 * The offsets are not validated on the device (that would need a device
 * read); malformed offsets give unspecified values in y but stay in bounds:
 * every access is limited to [0, n_total).
 */
lscan_status lscan_segmented(const void *x, void *y, int64_t n_total,
                             const int64_t *offsets, int64_t num_segments,
                             lscan_dtype dt, lscan_op op, uint32_t flags,
                             void *stream);

/*
 * lscan_batched -- the scan of Section 1 applied independently to each of
 * `count` arrays in ONE persistent launch (batching for serving).  Each array
 * occupies whole data blocks of its own, so the block method of Section 4
 * runs unchanged inside an array and the prefix hand-off between blocks uses
 * the segmented operator, restarting at the first block of every array.
 *   arrays  HOST pointer to `count` descriptors; each x / y is a DEVICE
 *           pointer with the element-alignment and in-place rules above
 *           (the vector rule above applies per array); arrays
 *           must not overlap each other (not checked); n == 0 is allowed
 *   flags   LSCAN_F_EXCLUSIVE, LSCAN_F_COMPENSATED as above
 * The descriptor table is copied to the device before the launch; the host
 * table may be reused as soon as the call returns.
 */
typedef struct {
    const void *x;
    void *y;
    int64_t n;
} lscan_array;

lscan_status lscan_batched(const lscan_array *arrays, int64_t count,
                           lscan_dtype dt, lscan_op op, uint32_t flags,
                           void *stream);

/*
 * Launch parameters (the paper's T, K and B of Section 5.1, chosen by
 * measurement here):
 *   block_threads     T: threads per workgroup (multiple of 64)
 *   vectors_per_lane  16-byte input vectors each lane holds per data block
 *                     (so K = vectors_per_lane * 16 / sizeof(input))
 *   groups_per_cu     resident workgroups per compute unit; B = this times
 *                     the CU count, capped by the occupancy limit and by M
 *   handoff           how a block obtains the prefix of the blocks before it
 *                     (Section 4.3, Algorithm 4):
 *                     LSCAN_HANDOFF_WINDOW (0, default): every block publishes
 *                       its aggregate; block i folds its workgroup's previous
 *                       inclusive prefix P(i-B) with the aggregates of blocks
 *                       i-B+1 .. i-1 in a fixed order;
 *                     LSCAN_HANDOFF_CHAIN (1): the paper's chain: block i
 *                       waits for the inclusive prefix published by block
 *                       i-1 and publishes its own, so the M blocks form one
 *                       serial chain of flag hand-offs (the paper-faithful
 *                       baseline; slow on a device with 8 separate L2s);
 *                     other values are invalid (LSCAN_ERR_INVALID_ARG).
 *                     Both give the same integer / max / min results; float
 *                     sums differ only in association.
 * The persistent grid needs all B workgroups resident at once (paper,
 * Section 5.1).  Before the first launch of a (kernel, groups_per_cu) pair
 * on a device, the library runs that kernel once in a test mode in which
 * every workgroup only waits (at most 20 ms) for all B to arrive; if they do
 * not, it lowers groups_per_cu and tests again, and it caches the answer.
 * The test synchronizes the stream, so the first call of a shape must not be
 * made while the stream is being captured into a graph
 * (LSCAN_ERR_UNSUPPORTED).
 */
#define LSCAN_HANDOFF_WINDOW 0
#define LSCAN_HANDOFF_CHAIN 1

typedef struct {
    int32_t block_threads;
    int32_t vectors_per_lane;
    int32_t groups_per_cu;
    int32_t handoff;
} lscan_params;

/* Number of compiled (block_threads, vectors_per_lane) tile shapes, and the
 * shape with index idx (groups_per_cu is returned as 0). */
int32_t lscan_num_tile_shapes(void);
lscan_status lscan_tile_shape(int32_t idx, lscan_params *out);

/* Kernel kinds for lscan_get_params / lscan_set_params (for
 * LSCAN_KIND_COMPACT only the item width of dt matters: op and flags are
 * ignored). */
#define LSCAN_KIND_PLAIN 0
#define LSCAN_KIND_SEGMENTED 1
#define LSCAN_KIND_BATCHED 2
#define LSCAN_KIND_COMPACT 3

/* Default parameters for (dt, op, flags & LSCAN_F_COMPENSATED) and a kernel
 * kind; set replaces them (e.g. from an autotuner).  The defaults are those
 * of large arrays: while an operator's parameters are the library's own,
 * plain add / max / min scans of at most 32 MiB of input run smaller tiles of
 * 1024- or 512-thread workgroups (they finish sooner when the array cannot
 * fill the device); other parameters, once set, apply to every size. */
lscan_status lscan_get_params(lscan_dtype dt, lscan_op op, uint32_t flags,
                              int32_t kind, lscan_params *out);
lscan_status lscan_set_params(lscan_dtype dt, lscan_op op, uint32_t flags,
                              int32_t kind, const lscan_params *p);

/* As lscan_inclusive / lscan_exclusive / lscan_segmented with explicit
 * parameters (p == NULL: the defaults).  exclusive selects the form for the
 * plain scan. */
lscan_status lscan_scan_with_params(const void *x, void *y, int64_t n,
                                    lscan_dtype dt, lscan_op op,
                                    uint32_t flags, int32_t exclusive,
                                    const lscan_params *p, void *stream);
lscan_status lscan_segmented_with_params(const void *x, void *y,
                                         int64_t n_total,
                                         const int64_t *offsets,
                                         int64_t num_segments, lscan_dtype dt,
                                         lscan_op op, uint32_t flags,
                                         const lscan_params *p, void *stream);

lscan_status lscan_batched_with_params(const lscan_array *arrays,
                                       int64_t count, lscan_dtype dt,
                                       lscan_op op, uint32_t flags,
                                       const lscan_params *p, void *stream);

/*
 * Stream compaction, the selection a +-scan of 0/1 flags drives (the paper
 * lists sorting and graph algorithms among the uses of the scan, Section 1):
 * every x[i] whose keep[i] is non-zero -- or, with keep == NULL, whose bits
 * are not all zero (so -0.0f is kept) -- is written, in index order, to out,
 * and the number written to *count.  One persistent launch on the scan's
 * machinery: the flags are counted and scanned per block, block counts are
 * handed forward through the flag slots, and each block scatters its kept
 * items to out[number kept before them].
 *   x      device pointer, n items of dt (LSCAN_I32, LSCAN_F32: 4 bytes,
 *          moved as bits; LSCAN_I64: 8 bytes; LSCAN_BF16:
 *          LSCAN_ERR_UNSUPPORTED)
 *   keep   device pointer to n bytes, or NULL
 *   out    device pointer with room for n items; only out[0, *count) is
 *          written; out may not overlap x, keep or count
 *          (LSCAN_ERR_INVALID_ARG)
 *   count  device pointer to one int64_t, 8-byte aligned; written by the
 *          launch (n == 0: set to 0 by a memset on the stream)
 * Results are exact (no arithmetic on the items).  lscan_compact_with_params
 * takes a tile shape and groups per CU as the scans do (handoff must be
 * LSCAN_HANDOFF_WINDOW, else LSCAN_ERR_UNSUPPORTED).
 */
lscan_status lscan_compact(const void *x, const uint8_t *keep, void *out,
                           int64_t *count, int64_t n, lscan_dtype dt,
                           void *stream);
lscan_status lscan_compact_with_params(const void *x, const uint8_t *keep,
                                       void *out, int64_t *count, int64_t n,
                                       lscan_dtype dt, const lscan_params *p,
                                       void *stream);

/*
 * Digit offsets of one radix-sort pass, the other scan consumer (sorting is
 * among the uses of the scan in Section 1): keys (unsigned bit patterns of
 * 4 bytes for LSCAN_I32 / LSCAN_F32, 8 bytes for LSCAN_I64; LSCAN_BF16:
 * LSCAN_ERR_UNSUPPORTED) are cut into M = ceil(n / block_items) blocks, and
 *   offsets[d * M + b] = (keys whose digit is below d)
 *                      + (keys of digit d in blocks before b),
 * digit = (key >> shift) & (2^bits - 1): where block b's first key of digit d
 * goes in a stable partition by digit.  A digit-count kernel writes the
 * counts digit-major into offsets, then the single-pass exclusive scan
 * (int64 add) turns them into offsets in place.
 *   bits         1 .. 8; shift >= 0 and shift + bits <= key width
 *   block_items  >= 1
 *   offsets      device array of 2^bits * M int64, 8-byte aligned, not
 *                overlapping keys; n == 0 writes nothing
 */
lscan_status lscan_radix_offsets(const void *keys, int64_t n, lscan_dtype dt,
                                 int32_t shift, int32_t bits,
                                 int64_t block_items, int64_t *offsets,
                                 void *stream);

/*
 * Scan with a user-defined associative operator.  The paper writes its
 * method as templates over the element type and operator and supports only
 * built-in scalar types (Section 6); here any trivially copyable value type
 * works.  The kernel is the library's persistent
 * single-pass scan instantiated for the caller's operator in the caller's own
 * HIP translation unit through include/lscan_custom.hpp, which returns a
 * handle (a pointer to a static description of the kernel; it stays valid
 * while that code object is loaded).  The library runs it like its own
 * kernels: per-stream flag workspace, co-residency test per (kernel, grid),
 * ordering across streams, the window or chain hand-off.
 *   kernel  handle from lscan_custom::kernel<Op, T, R>(); the operator must
 *           be associative; it need not be commutative (the earlier operand
 *           is always on the left)
 *   x, y    device arrays of n elements of the operator's In and Out types;
 *           aligned to min(sizeof, 16) bytes; y == x allowed when In and Out
 *           have the same size, other overlaps are invalid
 *   flags   0, LSCAN_F_EXCLUSIVE and/or LSCAN_F_DETERMINISTIC
 *   p       null or groups_per_cu / handoff (a tile shape: the kernel fixes
 *           it, LSCAN_ERR_UNSUPPORTED)
 * Every handle carries a tag of the kernel-argument layout of the headers it
 * was built with: a handle built against headers of another layout is
 * refused with LSCAN_ERR_UNSUPPORTED before any device work; a null handle,
 * or one that lscan_custom.hpp did not make, is LSCAN_ERR_INVALID_ARG.
 */
typedef struct lscan_custom_kernel lscan_custom_kernel;
lscan_status lscan_scan_custom(const lscan_custom_kernel *kernel,
                               const void *x, void *y, int64_t n,
                               uint32_t flags, const lscan_params *p,
                               void *stream);

/*
 * Breadth-first search on the device, the graph search that Section 6 names
 * as the next use of the paper's inter-block hand-off (Section 4.3): one
 * persistent launch runs the whole search.  The edges of each level's
 * frontier are cut into equal chunks taken cyclically by a co-resident
 * grid; each chunk claims the undiscovered endpoints of its edges (an
 * atomic or on a visited bitmap: the lane that sets a vertex's bit finds
 * it), publishes how many
 * vertices and edges it found in epoch-tagged flag words, and obtains where
 * they go in the next frontier from the values published before it (the
 * window fold of the scan) -- no shared queue-tail counter.  Levels end
 * with a grid barrier made of the same flag words.
 *   row_offsets  device array of num_vertices + 1 int64, 8-byte aligned:
 *                the edges of vertex u are cols[row_offsets[u] ..
 *                row_offsets[u + 1]) (a directed graph in compressed rows);
 *                expected non-decreasing: where it decreases anywhere the
 *                graph is not searched (every level and parent -1, stats
 *                {0, 0, 0, number of decreasing steps})
 *   cols         device array of num_edges int32 (may be null if
 *                num_edges == 0); num_edges < 2^42
 *   num_vertices 0 .. 2^31 - 2; 0 does nothing (stats, if given, zeroed)
 *   source       0 .. num_vertices - 1
 *   levels       device array of num_vertices int32 (output): the number of
 *                edges on a shortest path from source, -1 if unreachable;
 *                unique, so exact
 *   parents      device array of num_vertices int32 (output), or null: a
 *                breadth-first tree -- parents[source] = source, for every
 *                other reached v an edge parents[v] -> v with
 *                levels[parents[v]] = levels[v] - 1, -1 if unreached
 *                (which parent is chosen is not fixed: any valid one)
 *   stats        device array of 4 int64 (output), or null: number of levels,
 *                vertices reached, edges scanned (the out-degrees of the
 *                reached vertices), malformed entries met (a reached vertex
 *                whose row range is not inside [0, num_edges], or a column
 *                outside [0, num_vertices) in such a row; those are
 *                skipped, never dereferenced)
 * Outputs may not overlap the inputs or each other.  The library keeps a
 * per-stream workspace of about 40 bytes per vertex and 24 bytes per 1024
 * edges.  Not capturable into a HIP graph (LSCAN_ERR_UNSUPPORTED while the
 * stream captures: each launch takes fresh flag tags from the host).  A wait
 * that outlasts the watchdog stops the whole grid; the next lscan_check on
 * the stream reports LSCAN_ERR_TIMEOUT and the outputs are undefined.
 * lscan_bfs_with_params honours groups_per_cu only (a tile shape or the
 * chain hand-off: LSCAN_ERR_UNSUPPORTED).
 */
lscan_status lscan_bfs(const int64_t *row_offsets, const int32_t *cols,
                       int64_t num_vertices, int64_t num_edges, int32_t source,
                       int32_t *levels, int32_t *parents, int64_t *stats,
                       void *stream);
lscan_status lscan_bfs_with_params(const int64_t *row_offsets,
                                   const int32_t *cols, int64_t num_vertices,
                                   int64_t num_edges, int32_t source,
                                   int32_t *levels, int32_t *parents,
                                   int64_t *stats, const lscan_params *p,
                                   void *stream);

/*
 * Graph-captured launches.  lscan_graph_create_* prepares one plain,
 * segmented or batched launch (workspace, co-residency test, descriptor
 * upload, all on a
 * private stream, synchronously) and captures it into a hipGraph that owns
 * its own flag workspace; lscan_graph_launch replays it on `stream`.  The
 * device pointers are fixed at creation: the caller changes the DATA in x /
 * offsets between replays, not the pointers.  Replays of one graph must be
 * ordered on one stream (they share the graph's flags); the flag epoch lives
 * in device memory and is advanced by the kernel itself, so replays need no
 * reset.  lscan_graph_check synchronizes `stream` and reports a timed-out
 * replay; lscan_graph_destroy synchronizes the device and frees the graph.
 */
typedef struct lscan_graph lscan_graph;
/* One plain scan of n elements (Section 1): inclusive, or exclusive with
 * LSCAN_F_EXCLUSIVE in flags; the other flags, types, operators and pointer
 * rules are those of lscan_inclusive.  n == 0 (nothing to capture) is
 * LSCAN_ERR_INVALID_ARG. */
lscan_status lscan_graph_create_scan(const void *x, void *y, int64_t n,
                                     lscan_dtype dt, lscan_op op,
                                     uint32_t flags, const lscan_params *p,
                                     lscan_graph **out);
lscan_status lscan_graph_create_segmented(const void *x, void *y,
                                          int64_t n_total,
                                          const int64_t *offsets,
                                          int64_t num_segments,
                                          lscan_dtype dt, lscan_op op,
                                          uint32_t flags,
                                          const lscan_params *p,
                                          lscan_graph **out);
lscan_status lscan_graph_create_batched(const lscan_array *arrays,
                                        int64_t count, lscan_dtype dt,
                                        lscan_op op, uint32_t flags,
                                        const lscan_params *p,
                                        lscan_graph **out);
lscan_status lscan_graph_launch(lscan_graph *g, void *stream);
lscan_status lscan_graph_check(lscan_graph *g, void *stream);
lscan_status lscan_graph_destroy(lscan_graph *g);

/*
 * Request server (continuous batching).  Requests are submitted one at a
 * time and polled by ticket; a scheduler thread groups pending requests with
 * the same (dtype, operator, flags) into one lscan_batched launch whenever
 * one of num_streams stream slots is free, so requests that arrive while
 * others run are launched as soon as a slot and budget allow, and batches on
 * different streams run on the device at the same time.
 *   Admission: a request holds n * (sizeof input + sizeof output) bytes of
 *   the HBM budget from launch to completion.  submit returns
 *   LSCAN_ERR_NO_MEMORY if one request exceeds the whole budget and
 *   LSCAN_ERR_AGAIN if max_queue requests are already pending.  Requests are
 *   launched oldest first: the oldest pending request fixes each batch's
 *   key, later requests of that key join it in submit order while the budget
 *   allows, and a request that does not fit waits (nothing of its key
 *   overtakes it).
 *   Ownership: x and y are device pointers owned by the caller and must stay
 *   valid until lscan_poll / lscan_wait returns a final status.
 *   Co-residency: the batches of stream i launch g_i workgroups per CU and
 *   the g_i sum to at most 3, so the persistent grids of all streams fit on
 *   the device together; groups_per_cu > 0 gives every stream that many
 *   (num_streams * groups_per_cu <= 3), groups_per_cu == 0 splits 3 among
 *   the streams, larger shares first (2 + 1 for two streams).  A batch goes
 *   to the free stream with the largest share.
 *   Large requests: a request of at least solo_bytes is never grouped; when
 *   it is the oldest it waits until no batch runs, then runs alone as a
 *   plain full-device scan (lscan_inclusive / lscan_exclusive with the
 *   default parameters), and nothing else launches until it completes.  The
 *   largest requests set the tail latency, and they get the fastest kernel.
 *   Scheduling happens in the thread that makes it possible -- lscan_submit
 *   or the completion of a batch -- so an arrival that finds a free stream
 *   is launched before lscan_submit returns.
 * lscan_poll returns LSCAN_PENDING (result partly filled) or the final
 * status, and forgets a ticket once it has reported its final status;
 * lscan_wait blocks until then.  lscan_server_destroy finishes every
 * submitted request first.  All timestamps are steady-clock nanoseconds.
 */
typedef struct {
    int32_t device;
    int32_t num_streams;       /* concurrent batches, 1..3 (default 2) */
    uint64_t hbm_budget_bytes; /* bytes of requests in flight (default 32 GiB) */
    int32_t max_queue;         /* pending requests (default 65536) */
    int32_t max_batch;         /* arrays per launch (default 4096) */
    int32_t groups_per_cu;     /* per stream; 0 = split 3 (default 0) */
    int32_t reserved;
    uint64_t solo_bytes;       /* requests this large run alone (0 = 64 MiB) */
} lscan_server_config;

typedef struct {
    lscan_dtype dt;
    lscan_op op;
    uint32_t flags; /* LSCAN_F_EXCLUSIVE, LSCAN_F_COMPENSATED */
    int32_t reserved;
    int64_t n;
    const void *x;  /* device */
    void *y;        /* device */
} lscan_request;

typedef struct {
    lscan_status status; /* LSCAN_PENDING, LSCAN_OK or an error */
    int32_t batch_size;  /* requests in the launch that carried it */
    uint64_t batch_id;
    uint64_t t_submit_ns, t_admit_ns, t_launch_ns, t_done_ns;
} lscan_result;

typedef struct {
    uint64_t submitted, completed, failed, batches;
    uint64_t bytes_in_flight, peak_bytes_in_flight;
    int64_t pending;
} lscan_server_stats;

typedef struct lscan_server lscan_server;
lscan_status lscan_server_default_config(lscan_server_config *cfg);
lscan_status lscan_server_create(const lscan_server_config *cfg,
                                 lscan_server **out);
lscan_status lscan_submit(lscan_server *s, const lscan_request *r,
                          uint64_t *ticket);
lscan_status lscan_poll(lscan_server *s, uint64_t ticket, lscan_result *out);
lscan_status lscan_wait(lscan_server *s, uint64_t ticket, lscan_result *out);
lscan_status lscan_server_get_stats(lscan_server *s, lscan_server_stats *out);
lscan_status lscan_server_destroy(lscan_server *s);

/*
 * Watchdog of every wait between workgroups (scan prefixes, compaction
 * counts, search offsets and level barriers): a wait that lasts longer than
 * `us` microseconds of the device's constant clock gives up, the grid stops
 * (each waiter sees the abort word) and the next lscan_check on the stream
 * reports LSCAN_ERR_TIMEOUT; the outputs of that launch are undefined.
 * Applies to launches made after the call, on every device (a captured
 * graph keeps the value it was captured with).  Default 2,000,000 (2 s).
 * 0 gives up at the first wait not already satisfied -- a way to exercise
 * the timeout path.  us outside [0, 3.6e9]: LSCAN_ERR_INVALID_ARG.
 */
lscan_status lscan_set_watchdog_us(int64_t us);
int64_t lscan_get_watchdog_us(void);

/* Shape of the last launch made by the calling thread. */
typedef struct {
    int64_t n;             /* elements */
    int64_t num_blocks;    /* M */
    int64_t tile_elems;    /* L */
    int32_t grid;          /* B */
    int32_t block_threads; /* T */
    int32_t slot_words;    /* 64-bit flag words per data block */
    int32_t vector_path;   /* 1: full blocks read and write vectors; 2: they
                              read vectors and write y, which sits at another
                              alignment phase than x, through an LDS stage;
                              0: elements */
    int32_t groups_per_cu; /* workgroups per CU of the launch */
    int32_t occupancy;     /* workgroups per CU the occupancy query allows */
} lscan_launch_info;
lscan_status lscan_last_launch(lscan_launch_info *out);

/* Wait for the stream and report LSCAN_ERR_TIMEOUT if a launch on it stopped
 * waiting for a block prefix since the previous check (the flag is then
 * cleared), else LSCAN_OK. */
lscan_status lscan_check(void *stream);

/* Release every flag workspace of the calling thread's current device
 * (synchronizes the device first). */
lscan_status lscan_release_workspaces(void);

/* Text of a status code; the HIP error of the last LSCAN_ERR_DEVICE on the
 * calling thread (0 if none). */
const char *lscan_status_string(lscan_status s);
int32_t lscan_last_device_error(void);

#ifdef __cplusplus
}
#endif

#endif /* LSCAN_H */
