"""Parity of the HIP scan (through the C ABI) with the CPU oracle, element by
element, on seeded inputs at sizes that span several tiles, several rounds of
the persistent grid and ragged tails."""
import numpy as np

import oracle
import pytest
import torch

from gpu_util import TAU_COMP, compare, log, make_input, to_device, to_host

pytestmark = pytest.mark.gpu

CASES = [
    ("int32", "add", False), ("int32", "max", False), ("int32", "min", False),
    ("int64", "add", False), ("int64", "max", False), ("int64", "min", False),
    ("float32", "add", False), ("float32", "add", True), ("float32", "max", False), ("float32", "min", False),
    ("bfloat16", "add", False), ("bfloat16", "add", True), ("bfloat16", "max", False), ("bfloat16", "min", False),
]


def sizes_for(gpu_lib, dtype, op, comp):
    """Edge sizes around the tile length L and the grid span B*L of the
    large-array launch (arrays of at most 32 MiB take smaller tiles, so the
    small sizes below run those)."""
    x = torch.zeros(1 << 26, dtype={"int32": torch.int32, "int64": torch.int64, "float32": torch.float32,
                                    "bfloat16": torch.bfloat16}[dtype], device="cuda")
    fn = gpu_lib.inclusive
    fn(x, op, comp)
    info = gpu_lib.lscan_last_launch()
    L = int(info.tile_elems)
    tdtype = x.dtype
    del x
    # grid of a launch with many blocks
    big = torch.zeros(L * 2048, dtype=tdtype, device="cuda")
    fn(big, op, comp)
    B = int(gpu_lib.lscan_last_launch().grid)
    del big
    return L, B, [1, 2, 3, 63, 64, 65, 255, 256, 257, 1000, L - 1, L, L + 1, 5 * L + 7,
                  B * L - 1, B * L + 1, 2 * B * L + L // 2 + 3]


@pytest.mark.parametrize("dtype,op,comp", CASES, ids=[f"{d}-{o}{'-comp' if c else ''}" for d, o, c in CASES])
def test_inclusive_exclusive(gpu_lib, dtype, op, comp):
    L, B, sizes = sizes_for(gpu_lib, dtype, op, comp)
    log(f"[parity] {dtype} {op} comp={comp} L={L} B={B}")
    for k, n in enumerate(sizes):
        x = make_input(dtype, op, n, seed=1000 + k)
        xd = to_device(x, dtype)
        for excl in (False, True):
            fn = gpu_lib.exclusive if excl else gpu_lib.inclusive
            y = fn(xd, op, comp)
            gpu_lib.lscan_check(torch.cuda.current_stream().cuda_stream)
            compare(to_host(y), x, dtype, op, excl, comp, what=f"{dtype}/{op}/n={n}/excl={excl}")


@pytest.mark.parametrize("shape", range(10))
@pytest.mark.parametrize("groups", [1, 2, 4])
def test_every_tile_shape(gpu_lib, shape, groups):
    t, r = gpu_lib.lscan_tile_shapes()[shape]
    p = gpu_lib.Params(t, r, groups, 0)
    log(f"[shapes] T={t} R={r} groups/CU={groups}")
    for dtype, op, comp in (("int32", "add", False), ("int64", "max", False), ("float32", "add", False),
                            ("float32", "add", True), ("bfloat16", "min", False)):
        for n in (777, 3_000_001):
            x = make_input(dtype, op, n, seed=77 + n + shape)
            xd = to_device(x, dtype)
            for excl in (False, True):
                fn = gpu_lib.exclusive if excl else gpu_lib.inclusive
                y = fn(xd, op, comp, params=p)
                gpu_lib.lscan_check(torch.cuda.current_stream().cuda_stream)
                info = gpu_lib.lscan_last_launch()
                assert info.block_threads == t
                compare(to_host(y), x, dtype, op, excl, comp, what=f"T={t} R={r} g={groups} {dtype}/{op}/n={n}")


def test_float_results_are_deterministic(gpu_lib):
    x = make_input("float32", "add", 20_000_003, seed=5)
    xd = to_device(x, "float32")
    for comp in (False, True):
        a = to_host(gpu_lib.inclusive(xd, "add", comp))
        b = to_host(gpu_lib.inclusive(xd, "add", comp))
        assert np.array_equal(a.view(np.uint32), b.view(np.uint32))


def test_float_exact_cases(gpu_lib):
    # small integers as float32: every association is exact, so the float
    # path must be bit-exact (catches lost or doubled elements)
    from paper_1604_04815_amd import workloads as w
    n = 1 << 14
    for k in range(3):
        x = w.uniform_int(n, -1000, 1000, seed=k).astype(np.float32)
        want = np.cumsum(x.astype(np.int64)).astype(np.float32)
        for comp in (False, True):
            got = to_host(gpu_lib.inclusive(to_device(x, "float32"), "add", comp))
            assert np.array_equal(got, want)
    # all ones: y_j = j + 1 exactly while below 2^24
    n = 3_000_000
    ones = np.ones(n, np.float32)
    got = to_host(gpu_lib.inclusive(to_device(ones, "float32"), "add"))
    assert np.array_equal(got, np.arange(1, n + 1, dtype=np.float32))
    hb = np.full(n, 0x3F80, np.uint16)  # bf16 1.0
    got = to_host(gpu_lib.inclusive(to_device(hb, "bfloat16"), "add"))
    assert np.array_equal(got, np.arange(1, n + 1, dtype=np.float32))


def test_compensated_cancellation(gpu_lib):
    # (2^24, 1, -2^24, 1, ...): the exact prefixes after each cancellation are
    # small integers that float32 represents; the compensated scan returns
    # them exactly, and within 2e-7 * A_j everywhere
    big = float(2 ** 24)
    x = np.array([big, 1.0, -big, 1.0] * 250_000, dtype=np.float32)
    got = to_host(gpu_lib.inclusive(to_device(x, "float32"), "add", True))
    exact = np.cumsum(x.astype(np.float64))
    idx = np.arange(2, x.size, 4)
    assert np.array_equal(got[idx].astype(np.float64), exact[idx])
    compare(got, x, "float32", "add", False, True, what="cancellation")


def test_in_place(gpu_lib):
    for dtype, op in (("int32", "add"), ("int64", "min"), ("float32", "max"), ("float32", "add")):
        n = 4_000_037
        x = make_input(dtype, op, n, seed=3)
        xd = to_device(x, dtype)
        gpu_lib.inclusive(xd, op, out=xd)
        compare(to_host(xd), x, dtype, op, False, what=f"in-place {dtype}/{op}")
        xd = to_device(x, dtype)
        gpu_lib.exclusive(xd, op, out=xd)
        compare(to_host(xd), x, dtype, op, True, what=f"in-place excl {dtype}/{op}")


NP_OF = {"int32": np.int32, "int64": np.int64, "float32": np.float32}


def test_unaligned_pointers(gpu_lib):
    # x and y a few elements past a 16-byte boundary: with the same phase the
    # block grid is shifted and vectors are used; with different phases the
    # grid follows x (vector reads) and y is written element by element; both
    # exact, inclusive and exclusive, a few sizes
    for dtype, op in (("int32", "add"), ("int64", "add"), ("float32", "min"), ("bfloat16", "add"),
                      ("int32", "argmax"), ("float32", "add")):
        out_el = 8 if op == "argmax" else (4 if dtype == "bfloat16" else np.dtype(NP_OF.get(dtype, np.float32)).itemsize)
        in_el = 2 if dtype == "bfloat16" else np.dtype(NP_OF.get(dtype, np.float32)).itemsize
        for n in (2_000_003, 70_001, 5):
            for xo, yo in ((1, 1), (3, 3), (1, 2), (2, 0)):
                x = make_input(dtype, "max" if op == "argmax" else op, n + 4, seed=9 + xo)
                base = to_device(x, dtype)
                xd = base[xo:xo + n]
                y_base = torch.empty(n + 4, dtype=gpu_lib.out_dtype(base, op), device="cuda")
                for excl in (False, True):
                    fn = gpu_lib.exclusive if excl else gpu_lib.inclusive
                    y = fn(xd, op, out=y_base[yo:yo + n])
                    gpu_lib.lscan_check(torch.cuda.current_stream().cuda_stream)
                    info = gpu_lib.lscan_last_launch()
                    vec_in = 8 if dtype == "bfloat16" else 16
                    same_phase = ((xo * in_el) % vec_in) // in_el * out_el % 16 == (yo * out_el) % 16
                    assert info.vector_path == (1 if same_phase else 2), (dtype, op, xo, yo, info.vector_path)
                    what = f"unaligned {dtype}/{op} n={n} x+{xo} y+{yo} excl={excl}"
                    if op == "argmax":
                        want = oracle.argscan(x[xo:xo + n], dtype, "argmax", excl)
                        assert np.array_equal(to_host(y), want), what
                    else:
                        compare(to_host(y), x[xo:xo + n], dtype, op, excl, what=what)


def test_unaligned_compensated(gpu_lib):
    # the compensated sums run lane-major (rows pass through LDS so that each
    # lane scans consecutive elements): full blocks at a shifted grid, output
    # at another phase than the input (staged row stores), partial blocks
    # (lane-major element loads and stores), in place, both forms
    for dtype in ("float32", "bfloat16"):
        in_el, out_el, vec_in = (2, 4, 8) if dtype == "bfloat16" else (4, 4, 16)
        for n in (2_000_003, 70_001, 5):
            for xo, yo in ((0, 0), (1, 1), (3, 3), (1, 2), (2, 0)):
                x = make_input(dtype, "add", n + 4, seed=19 + xo + n % 7)
                base = to_device(x, dtype)
                xd = base[xo:xo + n]
                y_base = torch.empty(n + 4, dtype=torch.float32, device="cuda")
                for excl in (False, True):
                    fn = gpu_lib.exclusive if excl else gpu_lib.inclusive
                    y = fn(xd, "add", True, out=y_base[yo:yo + n])
                    gpu_lib.lscan_check(torch.cuda.current_stream().cuda_stream)
                    info = gpu_lib.lscan_last_launch()
                    same_phase = ((xo * in_el) % vec_in) // in_el * out_el % 16 == (yo * out_el) % 16
                    assert info.vector_path == (1 if same_phase else 2), (dtype, xo, yo, info.vector_path)
                    compare(to_host(y), x[xo:xo + n], dtype, "add", excl, True,
                            what=f"unaligned compensated {dtype} n={n} x+{xo} y+{yo} excl={excl}")
    for n in (3_000_017, 4099):
        x = make_input("float32", "add", n, seed=23)
        xd = to_device(x, "float32")
        gpu_lib.inclusive(xd, "add", True, out=xd)
        gpu_lib.lscan_check(torch.cuda.current_stream().cuda_stream)
        compare(to_host(xd), x, "float32", "add", False, True, what=f"in-place compensated n={n}")


def test_bf16_grid_origin_off_16_bytes(gpu_lib):
    # bf16 lane vectors are 8 bytes, so the shifted block grid may start 8 bytes
    # past a 16-byte boundary: such launches cannot use the 16-byte loads into
    # LDS and read full blocks straight into registers (lane-blocked rows of the
    # compensated sum included); x offsets 4..7 elements put the origin there
    for op, comp in (("add", False), ("add", True), ("max", False)):
        for n in (2_000_003, 70_001):
            for xo, yo in ((4, 4), (5, 5), (7, 3), (4, 1)):
                x = make_input("bfloat16", op, n + 8, seed=31 + xo + n % 5)
                base = to_device(x, "bfloat16")
                xd = base[xo:xo + n]
                y_base = torch.empty(n + 8, dtype=torch.float32, device="cuda")
                for excl in (False, True):
                    fn = gpu_lib.exclusive if excl else gpu_lib.inclusive
                    y = fn(xd, op, comp, out=y_base[yo:yo + n])
                    gpu_lib.lscan_check(torch.cuda.current_stream().cuda_stream)
                    compare(to_host(y), x[xo:xo + n], "bfloat16", op, excl, comp,
                            what=f"bf16 origin 8 bytes off {op} comp={comp} n={n} x+{xo} y+{yo} excl={excl}")


def test_repeated_launches_reuse_flags(gpu_lib):
    # flag slots are never cleared between launches (epoch tags): many
    # launches of varying sizes on one stream must all be right
    rng = np.random.default_rng(2024)
    for k in range(60):
        n = int(rng.integers(1, 3_000_000))
        dtype, op = [("int32", "add"), ("int64", "max"), ("float32", "min")][k % 3]
        x = make_input(dtype, op, n, seed=500 + k)
        y = gpu_lib.inclusive(to_device(x, dtype), op)
        compare(to_host(y), x, dtype, op, False, what=f"repeat {k} n={n}")
    gpu_lib.lscan_check(torch.cuda.current_stream().cuda_stream)


def test_other_stream(gpu_lib):
    s = torch.cuda.Stream()
    x = make_input("int32", "add", 5_000_000, seed=1)
    xd = to_device(x, "int32")
    torch.cuda.synchronize()
    with torch.cuda.stream(s):
        y = gpu_lib.inclusive(xd, "add")
    s.synchronize()
    gpu_lib.lscan_check(s.cuda_stream)
    compare(to_host(y), x, "int32", "add", False, what="side stream")


def test_max_min_special_floats(gpu_lib):
    pool = np.array([-0.0, 0.0, np.inf, -np.inf, 1.0, -1.0, 3.0e38, -3.0e38, 1e-45, -1e-45],
                    dtype=np.float32)
    rng = np.random.default_rng(4)
    x = pool[rng.integers(0, pool.size, 1_000_003)]
    for op in ("max", "min"):
        for excl in (False, True):
            fn = gpu_lib.exclusive if excl else gpu_lib.inclusive
            y = fn(to_device(x, "float32"), op)
            compare(to_host(y), x, "float32", op, excl, what=f"special {op}")


def test_int_wraparound(gpu_lib):
    n = 3_000_000
    x = np.full(n, 2 ** 31 - 1, dtype=np.int32)
    compare(to_host(gpu_lib.inclusive(to_device(x, "int32"), "add")), x, "int32", "add", False, what="wrap32")
    x64 = np.full(n, 2 ** 62 + 12345, dtype=np.int64)
    compare(to_host(gpu_lib.inclusive(to_device(x64, "int64"), "add")), x64, "int64", "add", False,
            what="wrap64")


def test_scans_alternating_on_two_streams_without_sync(gpu_lib):
    # full-device persistent grids enqueued on two streams back to back: the
    # runtime orders them across streams, so none waits for workgroups that
    # cannot become resident, and every result is exact
    n = (1 << 26) + 3
    x = torch.randint(-1000, 1001, (n,), dtype=torch.int32, device="cuda")
    want = torch.cumsum(x.to(torch.int64), 0).to(torch.int32)
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    ys = [torch.empty_like(x) for _ in range(6)]
    torch.cuda.synchronize()
    for k, y in enumerate(ys):
        s = streams[k % 2]
        with torch.cuda.stream(s):
            gpu_lib.inclusive(x, "add", out=y)
    for s in streams:
        s.synchronize()
        gpu_lib.lscan_check(s.cuda_stream)
    for y in ys:
        assert torch.equal(y, want)


def test_small_arrays_take_small_tiles(gpu_lib):
    # plain add / max / min of at most 32 MiB run 512 x 2, 1024 x 2 or 1024 x 4;
    # larger arrays the large-array default; both exact
    for n, want_t in ((1 << 16, 512), (1 << 19, 1024), (1 << 23, 1024), (1 << 24, None)):
        x = make_input("int32", "add", n, seed=n)
        y = gpu_lib.inclusive(to_device(x, "int32"), "add")
        gpu_lib.lscan_check(torch.cuda.current_stream().cuda_stream)
        info = gpu_lib.lscan_last_launch()
        if want_t is not None:
            assert info.block_threads == want_t, (n, info.block_threads)
        else:
            d = gpu_lib.lscan_get_params(gpu_lib.I32, gpu_lib.ADD)
            assert info.block_threads == d.block_threads, (n, info.block_threads)
        compare(to_host(y), x, "int32", "add", False, what=f"small-array shapes n={n}")
