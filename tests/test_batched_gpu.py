"""Parity of the many-array batched scan and of graph-captured launches with
the CPU oracle."""
import numpy as np
import pytest
import torch

from gpu_util import compare, log, make_input, to_device, to_host

pytestmark = pytest.mark.gpu

CASES = [("int32", "add", False), ("int32", "min", False), ("int64", "add", False), ("int64", "max", False),
         ("float32", "add", False), ("float32", "add", True), ("float32", "max", False),
         ("bfloat16", "add", False), ("bfloat16", "add", True), ("bfloat16", "max", False)]


def tile_len(gpu_lib, dtype):
    t = {"int32": torch.int32, "int64": torch.int64, "float32": torch.float32, "bfloat16": torch.bfloat16}[dtype]
    x = torch.zeros(1 << 16, dtype=t, device="cuda")
    gpu_lib.batched([x])
    return int(gpu_lib.lscan_last_launch().tile_elems)


@pytest.mark.parametrize("dtype,op,comp", CASES, ids=[f"{d}-{o}{'-comp' if c else ''}" for d, o, c in CASES])
def test_batched_mixed_sizes(gpu_lib, dtype, op, comp):
    L = tile_len(gpu_lib, dtype)
    rng = np.random.default_rng(11)
    sizes = [0, 1, 2, 63, L - 1, L, L + 1, 3 * L + 5, 0, 1000, 100_000, 1_234_567]
    sizes += [int(v) for v in np.floor(np.exp(rng.uniform(0, np.log(300_000), 40)))]
    xs_host = [make_input(dtype, op, n, seed=100 + k) for k, n in enumerate(sizes)]
    xs = [to_device(x, dtype) for x in xs_host]
    log(f"[batched] {dtype} {op} comp={comp} arrays={len(xs)} L={L}")
    for excl in (False, True):
        ys = gpu_lib.batched(xs, op, exclusive=excl, compensated=comp)
        gpu_lib.lscan_check(torch.cuda.current_stream().cuda_stream)
        for k, (xh, y) in enumerate(zip(xs_host, ys)):
            compare(to_host(y), xh, dtype, op, excl, comp, what=f"batched {dtype}/{op} array {k} n={xh.size}")


def test_batched_equals_alone_for_exact_ops(gpu_lib):
    xs_host = [make_input("int32", "add", n, seed=n) for n in (5, 70_000, 3_000_001, 123)]
    xs = [to_device(x, "int32") for x in xs_host]
    ys = gpu_lib.batched(xs, "add")
    for x, y in zip(xs, ys):
        assert torch.equal(y, gpu_lib.inclusive(x, "add"))


def test_batched_in_place_and_unaligned(gpu_lib):
    xs_host = [make_input("int32", "add", n, seed=n) for n in (10_001, 40_000, 7)]
    xs = [to_device(x, "int32") for x in xs_host]
    base = to_device(make_input("float32", "max", 50_001, seed=3), "float32")
    gpu_lib.lscan_batched([(x.data_ptr(), x.data_ptr(), x.shape[0]) for x in xs], gpu_lib.I32, gpu_lib.ADD)
    for xh, x in zip(xs_host, xs):
        compare(to_host(x), xh, "int32", "add", False, what="batched in place")
    xu = base[1:]
    yu = torch.empty(50_001, dtype=torch.float32, device="cuda")[1:]
    gpu_lib.batched([xu], "max", outs=[yu])
    compare(to_host(yu), to_host(xu), "float32", "max", False, what="batched unaligned")


def test_graph_segmented_replays(gpu_lib):
    from paper_1604_04815_amd import workloads as w
    off = w.segment_offsets(512, 1 << 14, seed=5)
    n = int(off[-1])
    xd = torch.empty(n, dtype=torch.int32, device="cuda")
    yd = torch.empty_like(xd)
    od = torch.from_numpy(off).to("cuda")
    g = gpu_lib.lscan_graph_create_segmented(xd.data_ptr(), yd.data_ptr(), n, od.data_ptr(), off.size - 1,
                                             gpu_lib.I32, gpu_lib.ADD)
    for rep in range(5):
        x = make_input("int32", "add", n, seed=700 + rep)
        xd.copy_(torch.from_numpy(x))
        g.launch()
        g.check()
        compare(to_host(yd), x, "int32", "add", False, offsets=off, what=f"graph replay {rep}")
        # eager work in between replays, on the same stream
        z = gpu_lib.inclusive(xd, "max")
        torch.cuda.synchronize()
        compare(to_host(z), x, "int32", "max", False, what=f"eager between replays {rep}")
    g.destroy()


def test_graph_batched_replays(gpu_lib):
    sizes = [1, 4097, 100_000, 0, 65_536, 3]
    xs = [torch.empty(n, dtype=torch.float32, device="cuda") for n in sizes]
    ys = [torch.empty_like(x) for x in xs]
    g = gpu_lib.lscan_graph_create_batched([(x.data_ptr(), y.data_ptr(), x.shape[0]) for x, y in zip(xs, ys)],
                                           gpu_lib.F32, gpu_lib.ADD, gpu_lib.F_COMPENSATED)
    for rep in range(4):
        hosts = [make_input("float32", "add", n, seed=900 + 7 * rep + k) for k, n in enumerate(sizes)]
        for x, h in zip(xs, hosts):
            x.copy_(torch.from_numpy(h))
        g.launch()
        g.check()
        for k, (h, y) in enumerate(zip(hosts, ys)):
            compare(to_host(y), h, "float32", "add", False, True, what=f"graph batched replay {rep} array {k}")
        torch.cumsum(xs[2], 0)  # unrelated eager work on the stream
    g.destroy()


MISALIGNED = [("int32", "add", False), ("int64", "max", False), ("float32", "add", True),
              ("bfloat16", "add", False), ("float32", "min", False)]


@pytest.mark.parametrize("dtype,op,comp", MISALIGNED, ids=[f"{d}-{o}{'-comp' if c else ''}" for d, o, c in MISALIGNED])
def test_batched_misaligned_arrays(gpu_lib, dtype, op, comp):
    # arrays cut at arbitrary element offsets out of one buffer, outputs cut
    # at the same offsets (equal phases: shifted block grids, vectors) and,
    # for every third array, one element further on (different phases: the
    # element path), sizes across tiles with ragged tails, empty arrays too
    L = tile_len(gpu_lib, dtype)
    rng = np.random.default_rng(23)
    sizes = [1, 2, 5, L - 1, L, L + 3, 0, 2 * L + 7, 3 * L - 2, 17]
    sizes += [int(v) for v in np.floor(np.exp(rng.uniform(0, np.log(200_000), 30)))]
    gaps = rng.integers(1, 5, size=len(sizes))  # outputs one further on must not reach the next array
    starts = np.cumsum(np.concatenate([[1], (np.array(sizes) + gaps)[:-1]]))
    total = int(starts[-1] + sizes[-1] + 2)
    host = make_input(dtype, op, total, seed=71)
    xb = to_device(host, dtype)
    yb = torch.empty(total + 1, dtype=gpu_lib.out_dtype(xb), device="cuda")
    xs, ys = [], []
    for k, (s, n) in enumerate(zip(starts, sizes)):
        s = int(s)
        o = s + (1 if k % 3 == 2 else 0)
        xs.append(xb[s:s + n])
        ys.append(yb[o:o + n])
    log(f"[batched misaligned] {dtype} {op} comp={comp} arrays={len(xs)} L={L}")
    for excl in (False, True):
        yb.fill_(-7)
        gpu_lib.batched(xs, op, exclusive=excl, compensated=comp, outs=ys)
        gpu_lib.lscan_check(torch.cuda.current_stream().cuda_stream)
        for k, (s, n) in enumerate(zip(starts, sizes)):
            s = int(s)
            compare(to_host(ys[k]), host[s:s + n], dtype, op, excl, comp,
                    what=f"batched misaligned {dtype}/{op} array {k} n={n} at {s}")
    if dtype == "int32":  # a captured batch of the same arrays replays the same outputs
        want = [y.clone() for y in ys]
        g = gpu_lib.lscan_graph_create_batched([(x.data_ptr(), y.data_ptr(), x.shape[0]) for x, y in zip(xs, ys)],
                                               gpu_lib.I32, gpu_lib.OPS[op], gpu_lib.F_EXCLUSIVE)
        for rep in range(3):
            yb.fill_(-7)
            g.launch()
            g.check()
            for k in range(len(ys)):
                assert torch.equal(ys[k], want[k]), f"graph replay {rep} array {k}"
        g.destroy()


def test_graph_plain_replays(gpu_lib):
    # one plain scan captured once and replayed with new data each time,
    # eager scans on the same stream in between; int32 add inclusive, float32
    # compensated exclusive, int32 running argmax, and an int32 scan whose x
    # and y sit one element past a vector boundary (shifted block grid)
    import oracle
    n = 3 * 65_536 + 1234
    cases = [("int32", "add", 0, 0), ("float32", "add", gpu_lib.F_EXCLUSIVE | gpu_lib.F_COMPENSATED, 0),
             ("int32", "argmax", 0, 0), ("int32", "add", 0, 1)]
    for dtype, op, flags, off in cases:
        t = {"int32": torch.int32, "float32": torch.float32}[dtype]
        xb = torch.empty(n + off, dtype=t, device="cuda")
        xd = xb[off:]
        yb = torch.empty(n + off, dtype=torch.int64 if op == "argmax" else t, device="cuda")
        yd = yb[off:]
        dt = {"int32": gpu_lib.I32, "float32": gpu_lib.F32}[dtype]
        g = gpu_lib.lscan_graph_create_scan(xd.data_ptr(), yd.data_ptr(), n, dt, gpu_lib.OPS[op], flags)
        assert gpu_lib.lscan_last_launch().vector_path == 1
        excl = bool(flags & gpu_lib.F_EXCLUSIVE)
        for rep in range(4):
            x = make_input(dtype, "max" if op == "argmax" else op, n, seed=1300 + 11 * rep + off)
            xd.copy_(torch.from_numpy(x))
            g.launch()
            g.check()
            what = f"graph plain {dtype}/{op} flags={flags} off={off} replay {rep}"
            if op == "argmax":
                assert np.array_equal(to_host(yd), oracle.argscan(x, dtype, "argmax", excl)), what
            else:
                compare(to_host(yd), x, dtype, op, excl, bool(flags & gpu_lib.F_COMPENSATED), what=what)
            z = gpu_lib.inclusive(xd, "max")  # eager work between replays, on the same stream
            torch.cuda.synchronize()
            compare(to_host(z), x, dtype, "max", False, what=f"eager between replays {rep}")
        g.destroy()
