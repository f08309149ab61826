"""Parity of the segmented scan (one persistent launch over many arrays) with
the oracle's per-segment scans."""
import numpy as np
import pytest
import torch

from gpu_util import compare, log, make_input, to_device, to_host

pytestmark = pytest.mark.gpu


def run(gpu_lib, x, off, dtype, op, excl=False, comp=False, params=None):
    xd = to_device(x, dtype)
    od = torch.from_numpy(off).to("cuda")
    y = gpu_lib.segmented(xd, od, op, exclusive=excl, compensated=comp, params=params)
    gpu_lib.lscan_check(torch.cuda.current_stream().cuda_stream)
    return to_host(y)


CASES = [("int32", "add", False), ("int32", "max", False), ("int64", "add", False), ("int64", "min", False),
         ("float32", "add", False), ("float32", "add", True), ("float32", "max", False),
         ("bfloat16", "add", False), ("bfloat16", "add", True), ("bfloat16", "min", False)]


@pytest.mark.parametrize("dtype,op,comp", CASES, ids=[f"{d}-{o}{'-comp' if c else ''}" for d, o, c in CASES])
def test_log_uniform_segments(gpu_lib, dtype, op, comp):
    from paper_1604_04815_amd import workloads as w
    off = w.segment_offsets(4096, 1 << 13, seed=w.seed_for(3))
    n = int(off[-1])
    x = make_input(dtype, op, n, seed=31)
    log(f"[seg] {dtype} {op} comp={comp} n={n}")
    for excl in (False, True):
        got = run(gpu_lib, x, off, dtype, op, excl, comp)
        compare(got, x, dtype, op, excl, comp, offsets=off, what=f"seg {dtype}/{op}/excl={excl}")


def test_one_segment_equals_plain(gpu_lib):
    n = 3_333_333
    x = make_input("int32", "add", n, seed=2)
    off = np.array([0, n], dtype=np.int64)
    got = run(gpu_lib, x, off, "int32", "add")
    plain = to_host(gpu_lib.inclusive(to_device(x, "int32"), "add"))
    assert np.array_equal(got, plain)
    compare(got, x, "int32", "add", False, what="one segment")


def test_all_length_one(gpu_lib):
    n = 200_003
    x = make_input("int32", "add", n, seed=3)
    off = np.arange(n + 1, dtype=np.int64)
    assert np.array_equal(run(gpu_lib, x, off, "int32", "add"), x)
    assert np.array_equal(run(gpu_lib, x, off, "int32", "add", excl=True), np.zeros(n, np.int32))
    xf = make_input("float32", "max", n, seed=4)
    got = run(gpu_lib, xf, off, "float32", "max", excl=True)
    assert np.all(got == -np.inf)


def test_empty_and_boundary_segments(gpu_lib):
    info_x = torch.zeros(1 << 16, dtype=torch.int32, device="cuda")
    gpu_lib.segmented(info_x, torch.tensor([0, 1 << 16], dtype=torch.int64, device="cuda"))
    L = int(gpu_lib.lscan_last_launch().tile_elems)
    lens = [0, 0, L, L - 1, L + 1, 0, 1, 0, 2 * L, 3, L // 2, 0, 5 * L + 11, 64, 0, 0]
    off = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    n = int(off[-1])
    for dtype, op in (("int32", "add"), ("int64", "max"), ("float32", "add")):
        x = make_input(dtype, op, n, seed=6)
        for excl in (False, True):
            got = run(gpu_lib, x, off, dtype, op, excl)
            compare(got, x, dtype, op, excl, offsets=off, what=f"boundary {dtype}/{op}/excl={excl}")


@pytest.mark.parametrize("shape", range(10))
def test_segmented_every_shape(gpu_lib, shape):
    from paper_1604_04815_amd import workloads as w
    t, r = gpu_lib.lscan_tile_shapes()[shape]
    off = w.segment_offsets(1000, 1 << 12, seed=77 + shape)
    n = int(off[-1])
    for dtype, op, comp in (("int32", "add", False), ("float32", "add", True)):
        x = make_input(dtype, op, n, seed=8)
        for groups in (1, 2):
            p = gpu_lib.Params(t, r, groups, 0)
            got = run(gpu_lib, x, off, dtype, op, False, comp, params=p)
            compare(got, x, dtype, op, False, comp, offsets=off, what=f"seg T={t} R={r} g={groups} {dtype}")


@pytest.mark.parametrize("max_len", [1024, 2048, 96])
def test_heads_per_block_around_matching_limit(gpu_lib, max_len):
    # Segment lengths uniform in [0, max_len] (empty segments included): blocks
    # of 16K elements then hold about 32 heads (max_len 1024), about 16 (2048)
    # or hundreds (96), so both ways of locating heads inside a block are used,
    # often in neighbouring blocks.
    rng = np.random.default_rng(1604 + max_len)
    lens = rng.integers(0, max_len + 1, size=(3 << 21) // max_len)
    off = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    n = int(off[-1])
    log(f"[seg] heads test max_len={max_len} n={n} segments={len(lens)}")
    for dtype, op, comp in (("int32", "add", False), ("float32", "add", True), ("int64", "min", False)):
        x = make_input(dtype, op, n, seed=9)
        for excl in (False, True):
            got = run(gpu_lib, x, off, dtype, op, excl, comp)
            compare(got, x, dtype, op, excl, comp, offsets=off, what=f"heads {max_len} {dtype}/{op}/excl={excl}")


SEG_UNALIGNED = [("int32", "add", False), ("int64", "max", False), ("float32", "add", True),
                 ("bfloat16", "add", False), ("float32", "min", False), ("int64", "add", False)]


@pytest.mark.parametrize("dtype,op,comp", SEG_UNALIGNED,
                         ids=[f"{d}-{o}{'-comp' if c else ''}" for d, o, c in SEG_UNALIGNED])
def test_segmented_unaligned(gpu_lib, dtype, op, comp):
    # x and y a few elements past a vector boundary: with equal phases the
    # block grid and the segment heads shift together and vectors are used,
    # with different phases vector reads and element writes; log-uniform segments with
    # empty ones at the start, inside and at the end; inclusive and exclusive
    from paper_1604_04815_amd import workloads as w
    off = w.segment_offsets(700, 1 << 12, seed=w.seed_for(3, 7))
    off = np.concatenate([[0, 0], off, [off[-1]]]).astype(np.int64)   # empty first and last segments
    off[300] = off[299]                                                # and one inside
    n = int(off[-1])
    x = make_input(dtype, op, n + 4, seed=77)
    od = torch.from_numpy(off).to("cuda")
    t = {"int32": torch.int32, "int64": torch.int64, "float32": torch.float32, "bfloat16": torch.float32}[dtype]
    in_el = {"int32": 4, "int64": 8, "float32": 4, "bfloat16": 2}[dtype]
    out_el = 8 if dtype == "int64" else 4
    vec_in = 8 if dtype == "bfloat16" else 16
    for xo, yo in ((1, 1), (3, 3), (1, 2)):
        base = to_device(x, dtype)
        xd = base[xo:xo + n]
        yb = torch.full((n + 4,), 7, dtype=t, device="cuda")
        yd = yb[yo:yo + n]
        same = ((xo * in_el) % vec_in) // in_el * out_el % 16 == (yo * out_el) % 16
        for excl in (False, True):
            gpu_lib.segmented(xd, od, op, exclusive=excl, compensated=comp, out=yd)
            gpu_lib.lscan_check(torch.cuda.current_stream().cuda_stream)
            assert gpu_lib.lscan_last_launch().vector_path == (1 if same else 2), (xo, yo)
            compare(to_host(yd), x[xo:xo + n], dtype, op, excl, comp, offsets=off,
                    what=f"seg unaligned {dtype}/{op} x+{xo} y+{yo} excl={excl}")
        # nothing written outside y
        assert torch.all(yb[:yo] == 7).item() and torch.all(yb[yo + n:] == 7).item()
