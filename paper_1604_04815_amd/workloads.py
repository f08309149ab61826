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
