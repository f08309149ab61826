"""Parity of stream compaction (lscan_compact) with the oracle: the kept items,
in order and bit for bit, their count, and nothing written past the count."""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import log

pytestmark = pytest.mark.gpu

NP = {"int32": np.int32, "int64": np.int64, "float32": np.float32}
TORCH = {"int32": torch.int32, "int64": torch.int64, "float32": torch.float32}
SENTINEL = {"int32": np.int32(-7), "int64": np.int64(-7), "float32": np.float32(-7.5)}


def items(dtype, n, seed, zero_frac=0.0):
    g = np.random.default_rng(seed)
    if dtype == "float32":
        x = (g.lognormal(0.0, 2.0, n) * g.choice([-1.0, 1.0], n)).astype(np.float32)
        if n:
            x[g.random(n) < 0.01] = -0.0  # bits not all zero: kept when keep is None
    else:
        x = g.integers(-(2 ** 31), 2 ** 31, n, dtype=np.int64).astype(NP[dtype])
    if zero_frac > 0:
        x[g.random(n) < zero_frac] = 0
    return x


def flags(n, density, seed):
    g = np.random.default_rng(seed)
    return (g.random(n) < density).astype(np.uint8) * g.integers(1, 256, n).astype(np.uint8)


def run(gpu_lib, x, keep, dtype, params=None, x_offset=0, keep_offset=0):
    """Compact on the device, with x and keep optionally shifted inside a
    larger allocation (to reach the unaligned path)."""
    n = x.shape[0]
    xbuf = torch.empty(n + x_offset, dtype=TORCH[dtype], device="cuda")
    xd = xbuf[x_offset:]
    xd.copy_(torch.from_numpy(x))
    kd = None
    if keep is not None:
        kbuf = torch.empty(n + keep_offset, dtype=torch.uint8, device="cuda")
        kd = kbuf[keep_offset:]
        kd.copy_(torch.from_numpy(keep))
    out = torch.full((n,), float(SENTINEL[dtype]) if dtype == "float32" else int(SENTINEL[dtype]),
                     dtype=TORCH[dtype], device="cuda")
    out, count = gpu_lib.compact(xd, kd, out=out, params=params)
    gpu_lib.lscan_check(torch.cuda.current_stream().cuda_stream)
    return out.cpu().numpy(), int(count.item())


def check(got, count, x, keep, dtype, what):
    want = oracle.compact(x, keep)
    assert count == want.shape[0], f"{what}: count {count} != {want.shape[0]}"
    g, w = got[:count], want
    if dtype == "float32":
        g, w = g.view(np.uint32), w.view(np.uint32)
    if not np.array_equal(g, w):
        bad = np.flatnonzero(g != w)
        raise AssertionError(f"{what}: {bad.size} mismatches, first at {bad[:8].tolist()}")
    tail = got[count:]
    sentinel = np.full(tail.shape, SENTINEL[dtype], dtype=NP[dtype])
    assert np.array_equal(tail.view(np.uint8), sentinel.view(np.uint8)), f"{what}: written past the count"


def tile_len(gpu_lib, dtype):
    x = torch.ones(1 << 16, dtype=TORCH[dtype], device="cuda")
    gpu_lib.compact(x)
    torch.cuda.synchronize()
    return int(gpu_lib.lscan_last_launch().tile_elems)


@pytest.mark.parametrize("dtype", ["int32", "float32", "int64"])
@pytest.mark.parametrize("density", [0.0, 0.01, 0.5, 0.99, 1.0])
def test_compact_densities(gpu_lib, dtype, density):
    L = tile_len(gpu_lib, dtype)
    for n in (1, 63, L - 1, L, L + 1, 3 * L + 5, 1_000_003):
        x = items(dtype, n, seed=n)
        keep = flags(n, density, seed=n + 1)
        got, count = run(gpu_lib, x, keep, dtype)
        check(got, count, x, keep, dtype, f"{dtype} p={density} n={n}")
    log(f"[compact] {dtype} p={density} ok (L={L})")


@pytest.mark.parametrize("dtype", ["int32", "float32", "int64"])
def test_compact_without_flags(gpu_lib, dtype):
    for n in (5, 100_000, 2_000_017):
        x = items(dtype, n, seed=3 * n, zero_frac=0.4)
        got, count = run(gpu_lib, x, None, dtype)
        check(got, count, x, None, dtype, f"{dtype} no flags n={n}")


def test_compact_unaligned_and_bool_flags(gpu_lib):
    n = 777_777
    for dtype, x_off, k_off in (("int32", 1, 0), ("int32", 0, 3), ("int64", 1, 1), ("float32", 3, 2)):
        x = items(dtype, n, seed=11)
        keep = flags(n, 0.3, seed=12)
        got, count = run(gpu_lib, x, keep, dtype, x_offset=x_off, keep_offset=k_off)
        check(got, count, x, keep, dtype, f"{dtype} x+{x_off} keep+{k_off}")
    # a bool keep tensor is read as bytes
    x = items("int32", n, seed=13)
    kb = torch.from_numpy(flags(n, 0.5, seed=14) != 0).to("cuda")
    out, count = gpu_lib.compact(torch.from_numpy(x).to("cuda"), kb)
    torch.cuda.synchronize()
    want = x[kb.cpu().numpy()]
    assert int(count.item()) == want.shape[0]
    assert np.array_equal(out[:want.shape[0]].cpu().numpy(), want)


def test_compact_empty(gpu_lib):
    x = torch.empty(0, dtype=torch.int32, device="cuda")
    count = torch.full((1,), 99, dtype=torch.int64, device="cuda")
    gpu_lib.compact(x, None, count=count)
    torch.cuda.synchronize()
    assert int(count.item()) == 0


@pytest.mark.parametrize("shape", range(10))
def test_compact_every_shape(gpu_lib, shape):
    t, r = gpu_lib.lscan_tile_shapes()[shape]
    n = 1_234_567
    for dtype in ("int32", "int64"):
        x = items(dtype, n, seed=20 + shape)
        keep = flags(n, 0.37, seed=21 + shape)
        for groups in (1, 2):
            got, count = run(gpu_lib, x, keep, dtype, params=gpu_lib.Params(t, r, groups, 0))
            check(got, count, x, keep, dtype, f"T={t} R={r} g={groups} {dtype}")


def test_compact_full_size(gpu_lib):
    # the measured configuration: int32, 2^28 items, half of them kept
    from paper_1604_04815_amd import workloads as w
    n = 1 << 28
    x = w.uniform_int(n, -1024, 1024, w.seed_for(5))
    keep = flags(n, 0.5, seed=w.seed_for(5, 1))
    log("[compact] full size 2^28")
    got, count = run(gpu_lib, x, keep, "int32")
    check(got, count, x, keep, "int32", "2^28")
