"""Parity of the running argmax / argmin scans (a pair operator carrying the
element index) with the oracle: int64 indices, earliest index among ties."""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import log

pytestmark = pytest.mark.gpu

NP = {"int32": np.int32, "int64": np.int64, "float32": np.float32}
TORCH = {"int32": torch.int32, "int64": torch.int64, "float32": torch.float32}


def keys(dtype, n, seed, spread):
    g = np.random.default_rng(seed)
    if dtype == "float32":
        vals = np.array([-3.5, -0.0, 0.0, 1.25, 2.0, 1e30, -1e30], np.float32)
        return g.choice(vals, n) if spread == "ties" else g.standard_normal(n).astype(np.float32)
    if spread == "ties":
        return g.integers(-3, 4, n).astype(NP[dtype])
    return g.integers(-(2 ** 31), 2 ** 31, n, dtype=np.int64).astype(NP[dtype])


def run(gpu_lib, x, dtype, op, exclusive, params=None, index64=False):
    xd = torch.from_numpy(x).to("cuda")
    fn = gpu_lib.exclusive if exclusive else gpu_lib.inclusive
    y = fn(xd, op, params=params, index64=index64)
    gpu_lib.lscan_check(torch.cuda.current_stream().cuda_stream)
    assert y.dtype == torch.int64
    return y.cpu().numpy()


def check(got, x, dtype, op, exclusive, what):
    want = oracle.argscan(x, dtype, op, exclusive)
    if not np.array_equal(got, want):
        bad = np.flatnonzero(got != want)
        raise AssertionError(f"{what}: {bad.size} mismatches, first at {bad[:8].tolist()}: "
                             f"got {got[bad[:4]].tolist()} want {want[bad[:4]].tolist()}")


# both kernel families: 32-bit index (what arrays below 2^31 elements use)
# and 64-bit index (forced with LSCAN_F_INDEX64; used by itself from 2^31 on)
@pytest.mark.parametrize("index64", [False, True], ids=["idx32", "idx64"])
@pytest.mark.parametrize("dtype", ["int32", "int64", "float32"])
@pytest.mark.parametrize("op", ["argmax", "argmin"])
def test_argscan(gpu_lib, dtype, op, index64):
    xd = torch.zeros(1 << 16, dtype=TORCH[dtype], device="cuda")
    gpu_lib.inclusive(xd, op, index64=index64)
    L = int(gpu_lib.lscan_last_launch().tile_elems)
    for spread in ("ties", "wide"):
        for n in (1, 63, L - 1, L + 1, 3 * L + 5, 1_000_003):
            x = keys(dtype, n, seed=n + len(spread), spread=spread)
            for excl in (False, True):
                check(run(gpu_lib, x, dtype, op, excl, index64=index64), x, dtype, op, excl,
                      f"{dtype} {op} {spread} n={n} excl={excl} index64={index64}")
    log(f"[argscan] {dtype} {op} index64={index64} ok (L={L})")


@pytest.mark.parametrize("index64", [False, True], ids=["idx32", "idx64"])
@pytest.mark.parametrize("shape", range(10))
def test_argscan_every_shape(gpu_lib, shape, index64):
    t, r = gpu_lib.lscan_tile_shapes()[shape]
    for dtype, op in (("int32", "argmax"), ("int64", "argmin"), ("float32", "argmax")):
        x = keys(dtype, 777_777, seed=30 + shape, spread="ties")
        for groups in (1, 2):
            got = run(gpu_lib, x, dtype, op, False, params=gpu_lib.Params(t, r, groups, 0), index64=index64)
            check(got, x, dtype, op, False, f"{dtype} {op} T={t} R={r} g={groups} index64={index64}")


def test_argscan_full_size(gpu_lib):
    from paper_1604_04815_amd import workloads as w
    n = 1 << 28
    x = w.full_range_int32(n, w.seed_for(7))
    log("[argscan] full size 2^28")
    check(run(gpu_lib, x, "int32", "argmax", False), x, "int32", "argmax", False, "2^28")
