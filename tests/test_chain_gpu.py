"""Parity of the paper's prefix chain (LSCAN_HANDOFF_CHAIN: block i waits for
the inclusive prefix that block i-1 published, Section 4.3, Algorithm 4) with
the oracle, for plain, segmented and batched scans, and its agreement with
the default window hand-off wherever the result is exact."""
import numpy as np
import pytest
import torch

from gpu_util import compare, log, make_input, to_device, to_host

pytestmark = pytest.mark.gpu

CASES = [("int32", "add", False), ("int32", "max", False), ("int64", "add", False), ("int64", "min", False),
         ("float32", "add", False), ("float32", "add", True), ("float32", "max", False),
         ("bfloat16", "add", False), ("bfloat16", "add", True)]


def chain(gpu_lib, t=0, r=0, groups=0):
    return gpu_lib.Params(t, r, groups, gpu_lib.HANDOFF_CHAIN)


def check(gpu_lib):
    gpu_lib.lscan_check(torch.cuda.current_stream().cuda_stream)


@pytest.mark.parametrize("dtype,op,comp", CASES, ids=[f"{d}-{o}{'-comp' if c else ''}" for d, o, c in CASES])
def test_chain_plain(gpu_lib, dtype, op, comp):
    # a ragged tail and several hundred blocks of the default shape
    n = (1 << 22) + 4097
    x = make_input(dtype, op, n, seed=41)
    xd = to_device(x, dtype)
    log(f"[chain] {dtype} {op} comp={comp} n={n}")
    for excl in (False, True):
        fn = gpu_lib.exclusive if excl else gpu_lib.inclusive
        got = fn(xd, op, comp, params=chain(gpu_lib))
        check(gpu_lib)
        assert gpu_lib.lscan_last_launch().num_blocks > 100
        compare(to_host(got), x, dtype, op, excl, comp, what=f"chain {dtype}/{op}/excl={excl}")
        if not (op == "add" and dtype in ("float32", "bfloat16")):
            window = fn(xd, op, comp)
            check(gpu_lib)
            assert torch.equal(got, window)


@pytest.mark.parametrize("shape", [0, 3, 4, 8])
@pytest.mark.parametrize("groups", [1, 2])
def test_chain_shapes(gpu_lib, shape, groups):
    t, r = gpu_lib.lscan_tile_shapes()[shape]
    n = 1_000_003
    x = make_input("int32", "add", n, seed=42)
    xd = to_device(x, "int32")
    got = gpu_lib.inclusive(xd, "add", params=chain(gpu_lib, t, r, groups))
    check(gpu_lib)
    compare(to_host(got), x, "int32", "add", False, what=f"chain T={t} R={r} g={groups}")


def test_chain_segmented(gpu_lib):
    from paper_1604_04815_amd import workloads as w
    off = w.segment_offsets(2000, 1 << 12, seed=w.seed_for(3, 1))
    n = int(off[-1])
    od = torch.from_numpy(off).to("cuda")
    for dtype, op, comp in (("int32", "add", False), ("float32", "add", True), ("int64", "max", False)):
        x = make_input(dtype, op, n, seed=43)
        xd = to_device(x, dtype)
        for excl in (False, True):
            got = gpu_lib.segmented(xd, od, op, exclusive=excl, compensated=comp, params=chain(gpu_lib))
            check(gpu_lib)
            compare(to_host(got), x, dtype, op, excl, comp, offsets=off, what=f"chain seg {dtype}/{op}/excl={excl}")


def test_chain_batched(gpu_lib):
    sizes = [0, 1, 5, 16_384, 16_385, 70_000, 1_234_567, 123, 0, 300_000]
    for dtype, op, comp in (("int32", "min", False), ("bfloat16", "add", True)):
        xs_host = [make_input(dtype, op, n, seed=44 + k) for k, n in enumerate(sizes)]
        xs = [to_device(v, dtype) for v in xs_host]
        ys = gpu_lib.batched(xs, op, compensated=comp, params=chain(gpu_lib))
        check(gpu_lib)
        for k, (xh, y) in enumerate(zip(xs_host, ys)):
            compare(to_host(y), xh, dtype, op, False, comp, what=f"chain batched {dtype}/{op} array {k}")


def test_chain_then_window_on_one_stream(gpu_lib):
    # the two hand-offs share the stream's flag workspace: alternate them and
    # check every result (tags keep advancing across both)
    n = 3_000_017
    x = make_input("int64", "add", n, seed=45)
    xd = to_device(x, "int64")
    want = None
    for k in range(6):
        p = chain(gpu_lib) if k % 2 == 0 else None
        got = gpu_lib.inclusive(xd, "add", params=p)
        check(gpu_lib)
        if want is None:
            compare(to_host(got), x, "int64", "add", False, what="chain/window alternation")
            want = got.clone()
        assert torch.equal(got, want), k
