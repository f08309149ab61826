"""Helpers shared by the GPU parity tests: device copies of numpy inputs and
element-by-element comparison of the HIP result with the CPU oracle."""
from __future__ import annotations

import sys

import numpy as np

import oracle

# float add tolerances: |y_j - y64_j| <= tau * sum_{i<=j} |x_i|
TAU_PLAIN = 1e-6
TAU_COMP = 2e-7


def log(msg: str) -> None:
    print(msg, flush=True)
    sys.stdout.flush()


def to_device(x: np.ndarray, dtype: str):
    import torch

    if dtype == "bfloat16":
        t = torch.from_numpy(x.view(np.int16).copy()).view(torch.bfloat16)
    else:
        t = torch.from_numpy(np.ascontiguousarray(x))
    return t.to("cuda")


def to_host(y) -> np.ndarray:
    return y.cpu().numpy()


def compare(got: np.ndarray, x: np.ndarray, dtype: str, op: str, exclusive: bool,
            compensated: bool = False, offsets=None, what: str = "") -> float:
    """Compare a device result with the oracle; returns the float error ratio
    (0 for exact types).  Raises AssertionError with the first mismatches."""
    if op == "add" and dtype in ("float32", "bfloat16"):
        if offsets is None:
            y64, a = oracle.scan(x, dtype, op, exclusive, with_absum=True)
        else:
            y64, a = oracle.segscan(x, offsets, dtype, op, exclusive, with_absum=True)
        tau = TAU_COMP if compensated else TAU_PLAIN
        ratio, j = oracle.float_error_ratio(got, y64, a)
        assert ratio <= tau, (f"{what}: error ratio {ratio:.3e} > {tau:.1e} at j={j} "
                              f"(got {got[j]!r}, want {y64[j]!r}, A={a[j]!r})")
        return ratio
    if offsets is None:
        want = oracle.scan(x, dtype, op, exclusive)
    else:
        want = oracle.segscan(x, offsets, dtype, op, exclusive)
    if got.dtype.kind == "f":
        same = got.view(np.uint32) == want.view(np.uint32)
    else:
        same = got == want
    if not np.all(same):
        bad = np.flatnonzero(~same)
        raise AssertionError(f"{what}: {bad.size} mismatches, first at {bad[:8].tolist()}: "
                             f"got {got[bad[:4]].tolist()} want {want[bad[:4]].tolist()}")
    return 0.0


def make_input(dtype: str, op: str, n: int, seed: int) -> np.ndarray:
    """Inputs for parity cases, following the per-type workload recipes."""
    from paper_1604_04815_amd import workloads as w

    if dtype == "int32":
        return w.uniform_int(n, -1000, 1000, seed) if op == "add" else w.full_range_int32(n, seed)
    if dtype == "int64":
        return w.int64_half_open(n, -(2 ** 31), 2 ** 31, seed) if op == "add" else \
            w.rng(seed).integers(-(2 ** 63), 2 ** 63 - 1, size=n, dtype=np.int64)
    if dtype == "float32":
        return w.signed_lognormal_f32(n, seed)
    if dtype == "bfloat16":
        if op == "add":
            return w.bf16_unit(n, seed)
        # signed values for max/min: random sign bit on unit-interval patterns
        h = w.bf16_unit(n, seed)
        sign = (w.rng(seed + 1).integers(0, 2, size=n, dtype=np.uint16) << 15).astype(np.uint16)
        return h | sign
    raise ValueError(dtype)
