/*
 * lscan_oracle.c -- sequential CPU reference for the device-wide scan.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or
 * calls this file: only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header or constant with the
 * HIP library; it is plain C written from the problem statement of the paper
 * (Section 1: inclusive scan y_j = x_0 (+) ... (+) x_j, exclusive scan
 * y_j = x_0 (+) ... (+) x_{j-1}).
 *
 * Every scan here is one left fold over the input in index order, which is
 * the definition itself.  The method of the paper (Section 4) only splits
 * this fold into data blocks and re-associates it; for the exact operators
 * (integer add modulo 2^w, integer max/min, float max/min under totalOrder)
 * any association gives the same bits, so the fold is the exact answer.
 * Float add is re-associated by every parallel scan, so for it the oracle
 * returns the exact prefix sums computed in FP64 with Neumaier compensation,
 * plus the running sum of magnitudes A_j = sum_{i<=j} |x_i| that scales the
 * accepted error.
 *
 * Readings of points the paper leaves open (each is listed in the design
 * notes of the repository):
 *   - identity element e of each operator (the paper writes a literal 0,
 *     which is only right for add): add -> 0, max -> the smallest value,
 *     min -> the largest value; for floats -inf / +inf;
 *   - integer overflow wraps modulo 2^w (two's complement);
 *   - float max/min follow IEEE 754 totalOrder restricted to non-NaN values
 *     (so -0 < +0); NaN inputs are outside the contract;
 *   - bf16 inputs are widened exactly to f32 (the 16 bits become the high
 *     half of the f32 word) and the scan is an f32 scan of those values;
 *   - segmented scan = the plain scan applied to each segment
 *     x[off[s], off[s+1]) independently; empty segments are allowed.
 *
 * Build: gcc -O2 -std=c11 -ffp-contract=off -fPIC -shared
 * (no -ffast-math: the compensated FP64 fold needs strict IEEE order).
 */
#include <math.h>
#include <stdint.h>
#include <string.h>

enum { OR_I32 = 0, OR_I64 = 1, OR_F32 = 2, OR_BF16 = 3 };
enum { OR_ADD = 0, OR_MAX = 1, OR_MIN = 2 };
enum { OR_OK = 0, OR_BAD_ARG = -1 };

/* ------------------------------------------------------------------ */
/* integer scans (exact)                                               */
/* ------------------------------------------------------------------ */

int oracle_scan_i32(const int32_t *x, int32_t *y, int64_t n, int op,
                    int exclusive)
{
    if (n < 0 || op < OR_ADD || op > OR_MIN) return OR_BAD_ARG;
    int32_t acc = (op == OR_ADD) ? 0 : (op == OR_MAX) ? INT32_MIN : INT32_MAX;
    for (int64_t j = 0; j < n; ++j) {
        int32_t v = x[j];          /* read before the write: y may be x */
        if (exclusive) y[j] = acc;
        if (op == OR_ADD)
            acc = (int32_t)((uint32_t)acc + (uint32_t)v);   /* mod 2^32 */
        else if (op == OR_MAX)
            acc = (v > acc) ? v : acc;
        else
            acc = (v < acc) ? v : acc;
        if (!exclusive) y[j] = acc;
    }
    return OR_OK;
}

int oracle_scan_i64(const int64_t *x, int64_t *y, int64_t n, int op,
                    int exclusive)
{
    if (n < 0 || op < OR_ADD || op > OR_MIN) return OR_BAD_ARG;
    int64_t acc = (op == OR_ADD) ? 0 : (op == OR_MAX) ? INT64_MIN : INT64_MAX;
    for (int64_t j = 0; j < n; ++j) {
        int64_t v = x[j];
        if (exclusive) y[j] = acc;
        if (op == OR_ADD)
            acc = (int64_t)((uint64_t)acc + (uint64_t)v);   /* mod 2^64 */
        else if (op == OR_MAX)
            acc = (v > acc) ? v : acc;
        else
            acc = (v < acc) ? v : acc;
        if (!exclusive) y[j] = acc;
    }
    return OR_OK;
}

/* ------------------------------------------------------------------ */
/* float max / min under IEEE 754 totalOrder (non-NaN), exact          */
/* ------------------------------------------------------------------ */

/* a precedes b in totalOrder: numeric order, and -0 before +0. */
static int total_less(float a, float b)
{
    if (a < b) return 1;
    if (a > b) return 0;
    /* a == b numerically: only the two zeros can still differ */
    return signbit(a) && !signbit(b);
}

static float widen_bf16(uint16_t h)
{
    uint32_t bits = (uint32_t)h << 16;
    float f;
    memcpy(&f, &bits, sizeof f);
    return f;
}

static void fold_order(float v, float *acc, int op)
{
    if (op == OR_MAX) {
        if (total_less(*acc, v)) *acc = v;
    } else {
        if (total_less(v, *acc)) *acc = v;
    }
}

int oracle_scan_f32_order(const float *x, float *y, int64_t n, int op,
                          int exclusive)
{
    if (n < 0 || (op != OR_MAX && op != OR_MIN)) return OR_BAD_ARG;
    float acc = (op == OR_MAX) ? -INFINITY : INFINITY;
    for (int64_t j = 0; j < n; ++j) {
        float v = x[j];
        if (exclusive) y[j] = acc;
        fold_order(v, &acc, op);
        if (!exclusive) y[j] = acc;
    }
    return OR_OK;
}

int oracle_scan_bf16_order(const uint16_t *x, float *y, int64_t n, int op,
                           int exclusive)
{
    if (n < 0 || (op != OR_MAX && op != OR_MIN)) return OR_BAD_ARG;
    float acc = (op == OR_MAX) ? -INFINITY : INFINITY;
    for (int64_t j = 0; j < n; ++j) {
        float v = widen_bf16(x[j]);
        if (exclusive) y[j] = acc;
        fold_order(v, &acc, op);
        if (!exclusive) y[j] = acc;
    }
    return OR_OK;
}

/* ------------------------------------------------------------------ */
/* float add: exact prefix sums in FP64 (Neumaier), and A_j = sum |x_i| */
/* ------------------------------------------------------------------ */

/* One Neumaier step: (s, c) accumulates v; s + c is the running sum. */
static void neumaier_add(double *s, double *c, double v)
{
    double t = *s + v;
    if (fabs(*s) >= fabs(v))
        *c += (*s - t) + v;
    else
        *c += (v - t) + *s;
    *s = t;
}

int oracle_scan_f32_add(const float *x, double *y64, double *absum,
                        int64_t n, int exclusive)
{
    if (n < 0) return OR_BAD_ARG;
    double s = 0.0, c = 0.0, a = 0.0;
    for (int64_t j = 0; j < n; ++j) {
        double v = (double)x[j];
        if (exclusive) {
            y64[j] = s + c;
            if (absum) absum[j] = a;
        }
        neumaier_add(&s, &c, v);
        a += fabs(v);
        if (!exclusive) {
            y64[j] = s + c;
            if (absum) absum[j] = a;
        }
    }
    return OR_OK;
}

int oracle_scan_bf16_add(const uint16_t *x, double *y64, double *absum,
                         int64_t n, int exclusive)
{
    if (n < 0) return OR_BAD_ARG;
    double s = 0.0, c = 0.0, a = 0.0;
    for (int64_t j = 0; j < n; ++j) {
        double v = (double)widen_bf16(x[j]);
        if (exclusive) {
            y64[j] = s + c;
            if (absum) absum[j] = a;
        }
        neumaier_add(&s, &c, v);
        a += fabs(v);
        if (!exclusive) {
            y64[j] = s + c;
            if (absum) absum[j] = a;
        }
    }
    return OR_OK;
}

/* ------------------------------------------------------------------ */
/* generic entry points                                                */
/* ------------------------------------------------------------------ */

/*
 * oracle_scan: one scan of n elements.
 *   dtype OR_I32 / OR_I64: y has the input type, exact.
 *   dtype OR_F32 / OR_BF16 with OR_MAX / OR_MIN: y is float[n], exact.
 *   dtype OR_F32 / OR_BF16 with OR_ADD: y is double[n] (exact prefix sums
 *     to FP64 rounding) and absum, if not NULL, receives A_j.
 * Returns OR_OK or OR_BAD_ARG.
 */
int oracle_scan(const void *x, void *y, double *absum, int64_t n, int dtype,
                int op, int exclusive)
{
    if (n < 0) return OR_BAD_ARG;
    switch (dtype) {
    case OR_I32:
        return oracle_scan_i32((const int32_t *)x, (int32_t *)y, n, op,
                               exclusive);
    case OR_I64:
        return oracle_scan_i64((const int64_t *)x, (int64_t *)y, n, op,
                               exclusive);
    case OR_F32:
        if (op == OR_ADD)
            return oracle_scan_f32_add((const float *)x, (double *)y, absum,
                                       n, exclusive);
        return oracle_scan_f32_order((const float *)x, (float *)y, n, op,
                                     exclusive);
    case OR_BF16:
        if (op == OR_ADD)
            return oracle_scan_bf16_add((const uint16_t *)x, (double *)y,
                                        absum, n, exclusive);
        return oracle_scan_bf16_order((const uint16_t *)x, (float *)y, n, op,
                                      exclusive);
    default:
        return OR_BAD_ARG;
    }
}

static int64_t in_size(int dtype)
{
    return dtype == OR_I64 ? 8 : dtype == OR_BF16 ? 2 : 4;
}

static int64_t out_size(int dtype, int op)
{
    if (dtype == OR_I64) return 8;
    if (dtype == OR_I32) return 4;
    return op == OR_ADD ? 8 : 4;   /* float add -> double reference */
}

/*
 * oracle_segscan: the plain scan applied to every segment
 * x[off[s], off[s+1]), s = 0 .. num_segments-1.  off has num_segments + 1
 * non-decreasing entries with off[0] = 0; elements past off[num_segments]
 * are not touched.  Layout of y and absum as in oracle_scan.
 */
int oracle_segscan(const void *x, void *y, double *absum, const int64_t *off,
                   int64_t num_segments, int dtype, int op, int exclusive)
{
    if (num_segments < 0) return OR_BAD_ARG;
    if (num_segments > 0 && off[0] != 0) return OR_BAD_ARG;
    int64_t isz = in_size(dtype), osz = out_size(dtype, op);
    for (int64_t s = 0; s < num_segments; ++s) {
        int64_t lo = off[s], hi = off[s + 1];
        if (hi < lo) return OR_BAD_ARG;
        int rc = oracle_scan((const char *)x + lo * isz, (char *)y + lo * osz,
                             absum ? absum + lo : NULL, hi - lo, dtype, op,
                             exclusive);
        if (rc != OR_OK) return rc;
    }
    return OR_OK;
}

/* ------------------------------------------------------------------ */
/* stream compaction (a consumer of the scan)                          */
/* ------------------------------------------------------------------ */

/*
 * oracle_compact: the selection that a +-scan of 0/1 flags drives, one of
 * the uses of the scan the paper lists (Section 1: sorting, graph
 * algorithms): every element x[i] of elem_size bytes whose keep[i] is not
 * zero -- or, with keep == NULL, whose bytes are not all zero -- is copied,
 * in index order, to out.  Returns the number copied, or -1 for bad
 * arguments.  The position of a kept x[i] in out is the number of kept
 * elements before it, i.e. the exclusive +-scan of the flags at i.
 */
int64_t oracle_compact(const void *x, const uint8_t *keep, int64_t n,
                       int elem_size, void *out)
{
    if (n < 0 || (elem_size != 2 && elem_size != 4 && elem_size != 8))
        return -1;
    const unsigned char *src = (const unsigned char *)x;
    unsigned char *dst = (unsigned char *)out;
    int64_t count = 0;
    for (int64_t i = 0; i < n; ++i) {
        const unsigned char *e = src + i * elem_size;
        int take = 0;
        if (keep) {
            take = keep[i] != 0;
        } else {
            for (int b = 0; b < elem_size; ++b) take |= e[b] != 0;
        }
        if (take) {
            memcpy(dst + count * elem_size, e, (size_t)elem_size);
            ++count;
        }
    }
    return count;
}

/*
 * oracle_radix_offsets: the digit offsets of one radix-sort pass, the other
 * scan consumer named with sorting in the paper's introduction (Section 1).
 * The keys (key_bytes = 4 or 8, unsigned bit patterns) are cut into blocks
 * of block_items; digit(k) = (k >> shift) & (2^bits - 1).  For digit d and
 * block b, out[d * M + b] (M = number of blocks) is the number of keys whose
 * digit is smaller than d, plus the number of keys with digit d in blocks
 * before b: where block b's first key of digit d goes in a stable
 * partition by digit.  Returns M, or -1 for bad arguments.
 */
int64_t oracle_radix_offsets(const void *keys, int64_t n, int key_bytes,
                             int shift, int bits, int64_t block_items,
                             int64_t *out)
{
    if (n < 0 || (key_bytes != 4 && key_bytes != 8) || bits < 1 || bits > 8 ||
        shift < 0 || shift + bits > 8 * key_bytes || block_items < 1)
        return -1;
    const int64_t m = (n + block_items - 1) / block_items;
    const int64_t nd = (int64_t)1 << bits;
    const uint64_t mask = (uint64_t)nd - 1;
    for (int64_t i = 0; i < nd * m; ++i) out[i] = 0;
    /* counts per (digit, block) */
    for (int64_t i = 0; i < n; ++i) {
        uint64_t k = (key_bytes == 4) ? (uint64_t)((const uint32_t *)keys)[i]
                                      : ((const uint64_t *)keys)[i];
        int64_t d = (int64_t)((k >> shift) & mask);
        out[d * m + i / block_items] += 1;
    }
    /* exclusive running sum in digit-major order */
    int64_t acc = 0;
    for (int64_t i = 0; i < nd * m; ++i) {
        int64_t c = out[i];
        out[i] = acc;
        acc += c;
    }
    return m;
}

/* ------------------------------------------------------------------ */
/* argmax / argmin scans (a pair operator: value and index)            */
/* ------------------------------------------------------------------ */

/*
 * oracle_argscan: y[j] = the index of the largest (want_max) or smallest
 * element of x[0..j] (inclusive) or x[0..j-1] (exclusive; -1 for j = 0),
 * the earliest index among equal values.  dtype OR_I32, OR_I64 or OR_F32
 * (float order: IEEE totalOrder restricted to non-NaN values, as for max /
 * min above).  One left fold, keeping (best value, its index).
 */
int oracle_argscan(const void *x, int64_t *y, int64_t n, int dtype,
                   int want_max, int exclusive)
{
    if (n < 0 || (dtype != OR_I32 && dtype != OR_I64 && dtype != OR_F32))
        return OR_BAD_ARG;
    int64_t best = -1;
    for (int64_t j = 0; j < n; ++j) {
        if (exclusive) y[j] = best;
        int better;
        if (best < 0) {
            better = 1;
        } else if (dtype == OR_I32) {
            int32_t v = ((const int32_t *)x)[j], b = ((const int32_t *)x)[best];
            better = want_max ? (v > b) : (v < b);
        } else if (dtype == OR_I64) {
            int64_t v = ((const int64_t *)x)[j], b = ((const int64_t *)x)[best];
            better = want_max ? (v > b) : (v < b);
        } else {
            float v = ((const float *)x)[j], b = ((const float *)x)[best];
            better = want_max ? total_less(b, v) : total_less(v, b);
        }
        if (better) best = j;
        if (!exclusive) y[j] = best;
    }
    return OR_OK;
}

/* ------------------------------------------------------------------ */
/* a non-commutative operator: composition of affine maps mod 2^32     */
/* ------------------------------------------------------------------ */

/*
 * oracle_affine_scan: the scan of Section 1 with (+) the composition of
 * affine maps x -> a*x + b over 32-bit unsigned integers (mod 2^32), the
 * earlier map applied first:
 *     (a1, b1) (+) (a2, b2) = (a2 * a1, a2 * b1 + b2),   e = (1, 0).
 * Maps are stored as interleaved pairs ab[2j] = a_j, ab[2j + 1] = b_j; the
 * output holds the composed prefixes in the same layout.  Its b half is the
 * linear recurrence h_j = a_j * h_{j-1} + b_j with h_{-1} = 0.  One left fold.
 */
int oracle_affine_scan(const uint32_t *ab, uint32_t *out, int64_t n,
                       int exclusive)
{
    if (n < 0)
        return OR_BAD_ARG;
    uint32_t pa = 1u, pb = 0u; /* the identity map */
    for (int64_t j = 0; j < n; ++j) {
        const uint32_t a = ab[2 * j], b = ab[2 * j + 1];
        if (exclusive) {
            out[2 * j] = pa;
            out[2 * j + 1] = pb;
        }
        pb = a * pb + b; /* apply the prefix, then map j */
        pa = a * pa;
        if (!exclusive) {
            out[2 * j] = pa;
            out[2 * j + 1] = pb;
        }
    }
    return OR_OK;
}

/* ------------------------------------------------------------------ */
/* breadth-first search levels (device-level messaging between blocks) */
/* ------------------------------------------------------------------ */

/*
 * oracle_bfs_levels: the breadth-first search that the paper names as the
 * next use of its inter-block hand-off (Section 6): level[v] is the number
 * of edges on a shortest path from src to v in the directed graph given in
 * compressed rows (row_ptr[num_vertices + 1], col[row_ptr[V]]), or -1 if v
 * is unreachable.  A plain queue, vertices visited in FIFO order.  Returns
 * the number of levels (the largest level + 1), or -1 for bad arguments.
 * queue must hold num_vertices entries.
 */
int64_t oracle_bfs_levels(const int64_t *row_ptr, const int32_t *col,
                          int64_t num_vertices, int64_t src, int32_t *level,
                          int32_t *queue)
{
    if (num_vertices < 0 || (num_vertices > 0 && (src < 0 || src >= num_vertices)))
        return -1;
    for (int64_t v = 0; v < num_vertices; ++v) level[v] = -1;
    if (num_vertices == 0) return 0;
    int64_t head = 0, tail = 0, depth = 0;
    level[src] = 0;
    queue[tail++] = (int32_t)src;
    while (head < tail) {
        int32_t u = queue[head++];
        if (level[u] + 1 > depth) depth = level[u] + 1;
        for (int64_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
            int32_t v = col[e];
            if (v < 0 || v >= num_vertices) return -1;
            if (level[v] < 0) {
                level[v] = level[u] + 1;
                queue[tail++] = v;
            }
        }
    }
    return depth;
}
