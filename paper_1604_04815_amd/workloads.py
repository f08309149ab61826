"""Seeded synthetic inputs for the scan workloads.

This module only draws numbers: it holds none of the scan arithmetic, so the
HIP path and the CPU oracle can both be fed from it without sharing any part
of the method.  Every generator takes an explicit seed and uses numpy's PCG64.

The paper evaluates on synthetic arrays of 32M..512M elements with the add
operator and four scalar types (Section 5); it states no value distribution,
so the distributions below are this library's own choice, one per workload:

* ``uniform_int``: integers uniform in ``[lo, hi]`` (both ends included).
* ``full_range_int32``: uniform over all int32 values.
* ``signed_lognormal_f32``: ``sign * lognormal(mu=0, sigma=2)``, sign +-1
  with probability 1/2, rounded to float32.
* ``bf16_unit``: the upper 16 bits (truncation) of float32 uniform [0, 1).
* ``segment_offsets``: lengths ``floor(exp(U * ln(max_len + 1)))`` (log-
  uniform in ``[1, max_len]``), returned as int64 offsets with ``off[0]=0``.
* ``request_trace``: Poisson arrivals with log-uniform sizes, dtype and op
  drawn uniformly.
"""
from __future__ import annotations

import numpy as np

BASE_SEED = 1604


def seed_for(config: int, trial: int = 0) -> int:
    """Seed of a workload: 1604 + 100*config + trial."""
    return BASE_SEED + 100 * int(config) + int(trial)


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def uniform_int(n: int, lo: int, hi: int, seed: int, dtype=np.int32) -> np.ndarray:
    """n integers uniform in [lo, hi] (inclusive) of the given dtype."""
    return rng(seed).integers(lo, hi, size=int(n), dtype=dtype, endpoint=True)


def full_range_int32(n: int, seed: int) -> np.ndarray:
    return rng(seed).integers(-(2 ** 31), 2 ** 31, size=int(n), dtype=np.int64).astype(np.int32)


def int64_half_open(n: int, lo: int, hi: int, seed: int) -> np.ndarray:
    """n int64 uniform in [lo, hi)."""
    return rng(seed).integers(lo, hi, size=int(n), dtype=np.int64)


def signed_lognormal_f32(n: int, seed: int, sigma: float = 2.0) -> np.ndarray:
    g = rng(seed)
    mag = g.lognormal(mean=0.0, sigma=sigma, size=int(n))
    sign = g.choice(np.array([-1.0, 1.0]), size=int(n))
    return (mag * sign).astype(np.float32)


def uniform01_f32(n: int, seed: int) -> np.ndarray:
    return rng(seed).random(int(n), dtype=np.float32)


def bf16_unit(n: int, seed: int) -> np.ndarray:
    """bf16 bit patterns (uint16): truncation of float32 uniform [0, 1)."""
    f = rng(seed).random(int(n), dtype=np.float32)
    return (f.view(np.uint32) >> 16).astype(np.uint16)


def f32_from_bf16_bits(h: np.ndarray) -> np.ndarray:
    """Reinterpret bf16 bit patterns as float32 (exact widening)."""
    return (h.astype(np.uint32) << 16).view(np.float32)


def segment_offsets(num_segments: int, max_len: int, seed: int, min_len: int = 1) -> np.ndarray:
    """int64 offsets (num_segments + 1 entries) of log-uniform segment lengths."""
    u = rng(seed).random(int(num_segments))
    lens = np.floor(np.exp(u * np.log(max_len + 1.0))).astype(np.int64)
    lens = np.clip(lens, min_len, max_len)
    off = np.zeros(num_segments + 1, dtype=np.int64)
    np.cumsum(lens, out=off[1:])
    return off


def values_for(dtype: str, op: str, n: int, seed: int) -> np.ndarray:
    """Inputs of one request or array, following the per-type recipes.

    int32 add: uniform [-1000, 1000]; int32 max/min: full int32 range;
    int64: uniform [-2^31, 2^31); float32: signed lognormal(0, 2);
    bfloat16: truncated uniform [0, 1) (uint16 bit patterns).
    """
    if dtype == "int32":
        if op == "add":
            return uniform_int(n, -1000, 1000, seed)
        return full_range_int32(n, seed)
    if dtype == "int64":
        return int64_half_open(n, -(2 ** 31), 2 ** 31, seed)
    if dtype == "float32":
        return signed_lognormal_f32(n, seed)
    if dtype == "bfloat16":
        return bf16_unit(n, seed)
    raise ValueError(dtype)


def request_trace(rate_hz: float, duration_s: float, seed: int,
                  log2_min: int = 10, log2_max: int = 26,
                  dtypes=("int32", "int64", "float32"), ops=("add", "max")):
    """Poisson arrival times and request shapes.

    Returns a list of dicts with keys ``t`` (arrival, seconds), ``n``,
    ``dtype``, ``op`` and ``seed`` (for the request's values).
    """
    g = rng(seed)
    out = []
    t = 0.0
    k = 0
    while True:
        t += g.exponential(1.0 / rate_hz)
        if t >= duration_s:
            break
        u = g.random()
        n = int(np.floor(2.0 ** (log2_min + (log2_max - log2_min) * u)))
        out.append({
            "t": t,
            "n": n,
            "dtype": dtypes[int(g.integers(0, len(dtypes)))],
            "op": ops[int(g.integers(0, len(ops)))],
            "seed": int(seed * 1000003 + k) % (2 ** 63),
        })
        k += 1
    return out


# ---------------------------------------------------------------------------
# Graphs for the breadth-first search
# ---------------------------------------------------------------------------
#
# ``rmat_edges`` draws a Kronecker (R-MAT) edge list with the quadrant
# probabilities of the Graph500 generator (A, B, C, D = 0.57, 0.19, 0.19,
# 0.05): each of the ``scale`` bit levels of an edge picks one quadrant; the
# vertex labels are then permuted at random, so degree does not follow the
# label.  ``csr_from_edges`` lays an edge list out in compressed rows
# (optionally with every edge in both directions); self loops and repeated
# edges are kept, as the generator makes them.

RMAT_ABC = (0.57, 0.19, 0.19)


def rmat_edges(scale: int, edge_factor: int, seed: int, abc=RMAT_ABC) -> tuple[np.ndarray, np.ndarray]:
    """edge_factor * 2^scale directed edges (src, dst) as int32 arrays over
    2^scale vertices."""
    a, b, c = abc
    g = rng(seed)
    m = int(edge_factor) << int(scale)
    src = np.zeros(m, dtype=np.int32)
    dst = np.zeros(m, dtype=np.int32)
    for level in range(int(scale)):
        r = g.random(m, dtype=np.float32)
        down = r >= np.float32(a + b)                                          # quadrants C, D
        right = (r >= np.float32(a)) & ~down | (r >= np.float32(a + b + c))    # quadrants B, D
        src |= down.astype(np.int32) << level
        dst |= right.astype(np.int32) << level
    perm = g.permutation(1 << int(scale)).astype(np.int32)
    return perm[src], perm[dst]


def csr_from_edges(src: np.ndarray, dst: np.ndarray, num_vertices: int,
                   symmetric: bool = True) -> tuple[np.ndarray, np.ndarray]:
    """(row_offsets int64[V + 1], cols int32[E]) of the edge list, rows in
    vertex order, each row's columns sorted."""
    src = np.asarray(src, dtype=np.int64)
    dst = np.asarray(dst, dtype=np.int64)
    if symmetric:
        src, dst = np.concatenate([src, dst]), np.concatenate([dst, src])
    order = np.argsort(src * int(num_vertices) + dst, kind="stable")
    cols = dst[order].astype(np.int32)
    counts = np.bincount(src, minlength=int(num_vertices)).astype(np.int64)
    row = np.zeros(int(num_vertices) + 1, dtype=np.int64)
    np.cumsum(counts, out=row[1:])
    return row, cols


def uniform_random_edges(num_vertices: int, num_edges: int, seed: int) -> tuple[np.ndarray, np.ndarray]:
    """num_edges directed edges with both ends uniform over the vertices."""
    g = rng(seed)
    return (g.integers(0, num_vertices, num_edges, dtype=np.int32),
            g.integers(0, num_vertices, num_edges, dtype=np.int32))


def rmat_csr_torch(scale: int, edge_factor: int, seed: int, device="cuda", abc=RMAT_ABC):
    """The recipe of ``rmat_edges`` + ``csr_from_edges(symmetric=True)``
    drawn with torch's generator on ``device`` (seconds instead of minutes at
    2^22 vertices; a different random stream than the numpy version).
    Returns (row_offsets int64[V + 1], cols int32[E]) on ``device``."""
    import torch

    a, b, c = abc
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    m = int(edge_factor) << int(scale)
    nv = 1 << int(scale)
    src = torch.zeros(m, dtype=torch.int64, device=device)
    dst = torch.zeros(m, dtype=torch.int64, device=device)
    for level in range(int(scale)):
        r = torch.rand(m, generator=g, device=device)
        down = r >= (a + b)
        right = ((r >= a) & ~down) | (r >= (a + b + c))
        src |= down.to(torch.int64) << level
        dst |= right.to(torch.int64) << level
        del r, down, right
    perm = torch.randperm(nv, generator=g, device=device)
    src, dst = perm[src], perm[dst]
    s2 = torch.cat([src, dst])
    d2 = torch.cat([dst, src])
    del src, dst
    key = s2 * nv + d2
    del s2, d2
    key, _ = torch.sort(key)
    rows = key // nv
    cols = (key - rows * nv).to(torch.int32)
    counts = torch.bincount(rows, minlength=nv)
    row_offsets = torch.zeros(nv + 1, dtype=torch.int64, device=device)
    torch.cumsum(counts, 0, out=row_offsets[1:])
    return row_offsets, cols
