#!/usr/bin/env python3
"""Benchmark of the single-pass device-wide scan on one MI355X.

One step = one inclusive scan (all stages of the method: tiled loads, wave
and block scans, inter-block prefix hand-off, fix-up and stores) of the
workload "int32 add, N = 2^28, x uniform in [-1024, 1024]", inputs resident
in HBM.  The headline value is scan GB/s = 2 * N * sizeof(int32) / t, with t
the mean device time per step over the whole timed region, measured with HIP
events on the stream the kernel is launched on; roofline.achieved divides the
same bytes by the mean duration of a single launch (an event pair around
each launch).

Prints ONE JSON line on stdout.  Besides the contract keys it carries
  roofline      the scan kernel against the 8 TB/s HBM peak, with the HBM
                traffic measured by rocprofv3 counters (from profiles/) when
                the kernel sources still match the profiled build,
  cpu_baseline  the sequential CPU oracle timed on this host on the same
                array,
  configs       the other workloads (int64 add, int32 max, float32 add plain
                and compensated, bf16 -> float32, a 4096-array segmented scan
                against 4096 plain launches, the 2^20 latency case, and the
                paper's serial prefix chain at 2^20 and 2^28 against the
                default window hand-off, stream compaction of the headline
                array, radix-sort digit offsets, running argmax), plus a
                device copy of the same size.

Before the warmup steps of every measurement the device runs the same call
for about SETTLE_S seconds (untimed), so that clocks have left the idle state
that input generation or a host-side oracle check leaves behind.

Progress lines go to stderr.  ``--gpus N`` with N > 1 is refused: the scan runs on
one GPU and is not sharded across GPUs.
"""
from __future__ import annotations

import argparse
import glob
import hashlib
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
PROFILE_TRAFFIC = os.path.join(ROOT, "profiles", "traffic_int32_add_2p28.txt")


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


DEVICE_SOURCES = ("scan_kernel.hpp", "scan_ops.hpp", "kernel_table.hpp")


def _code_only(text: str) -> str:
    """Source text without comments and blank lines (comments do not change
    the kernels)."""
    import re

    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    lines = [re.sub(r"//.*$", "", l).rstrip() for l in text.splitlines()]
    return "\n".join(l for l in lines if l.strip())


def kernel_source_hash() -> str:
    """Hash of the device code (kernel templates, operators, argument layout
    and instantiation units, comments left out); host-only changes leave it
    unchanged."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1604_04815_amd", "csrc")
    files = [os.path.join(csrc, f) for f in DEVICE_SOURCES] + sorted(glob.glob(os.path.join(csrc, "kernels_*.hip")))
    for f in files:
        h.update(os.path.basename(f).encode())
        h.update(_code_only(open(f).read()).encode())
    return h.hexdigest()[:16]


def read_traffic():
    """HBM bytes per launch from the committed rocprofv3 counter summary, or
    None when it is missing or was taken on different kernel sources."""
    if not os.path.exists(PROFILE_TRAFFIC):
        return None
    kv = {}
    for line in open(PROFILE_TRAFFIC):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernel_source_hash") != kernel_source_hash():
        return None
    try:
        return float(kv["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


# ---------------------------------------------------------------------------
# device timing
# ---------------------------------------------------------------------------

SETTLE_S = 0.15


def settle(fn, seconds: float | None = None):
    """Keep the device busy with fn for about `seconds` before any warmup or
    timing: after an idle stretch (input generation, an oracle check on the
    host) the GPU takes milliseconds to return to its working clocks, which
    a few warmup steps of a sub-millisecond kernel do not cover."""
    import torch

    seconds = SETTLE_S if seconds is None else seconds
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        for _ in range(8):
            fn()
        torch.cuda.synchronize()


def time_steps(fn, steps: int, warmup: int):
    """Settle the device, run fn warmup + steps times on the current stream;
    returns (mean ms per step over the whole timed region, per-step ms list)."""
    import torch

    settle(fn)
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    begin, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    stops = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    torch.cuda.synchronize()
    begin.record()
    for k in range(steps):
        starts[k].record()
        fn()
        stops[k].record()
    end.record()
    torch.cuda.synchronize()
    per = [s.elapsed_time(e) for s, e in zip(starts, stops)]
    return begin.elapsed_time(end) / steps, per


def pct(values, q):
    v = sorted(values)
    if not v:
        return float("nan")
    k = min(len(v) - 1, max(0, int(round(q / 100.0 * (len(v) - 1)))))
    return v[k]


def rate_entry(nbytes: float, n: int, ms: float, per=None):
    d = {"ms": round(ms, 5), "gbs": round(nbytes / (ms * 1e-3) / 1e9, 1),
         "gelem_s": round(n / (ms * 1e-3) / 1e9, 2),
         "frac_hbm_peak": round(nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    if per:
        d["launch_ms_mean"] = round(statistics.mean(per), 5)
        d["ms_p50"] = round(pct(per, 50), 5)
        d["ms_min"] = round(min(per), 5)
        d["ms_p99"] = round(pct(per, 99), 5)
    return d


def float_error(xd, y, offsets=None):
    """max_j |y_j - y64_j| / A_j over the whole array, with y64 the exact
    prefix sums in float64 and A_j = sum_{i<=j} |x_i| (the bound the float
    tolerances are stated in), and the j where it is largest.  The float64
    reference runs on the device (torch.cumsum in float64: its own error,
    about log2(N) * 2^-53 * A_j, is far below the float32 tolerances).
    Segmented scans restart the sums at every segment."""
    import torch

    xf = xd.float().double() if xd.dtype == torch.bfloat16 else xd.double()
    if offsets is None:
        ref = torch.cumsum(xf, 0)
        a = torch.cumsum(xf.abs(), 0)
    else:
        ref = torch.empty_like(xf)
        a = torch.empty_like(xf)
        off = offsets.tolist()
        for s in range(len(off) - 1):
            lo, hi = off[s], off[s + 1]
            if hi > lo:
                torch.cumsum(xf[lo:hi], 0, out=ref[lo:hi])
                torch.cumsum(xf[lo:hi].abs(), 0, out=a[lo:hi])
    err = (y.double() - ref).abs()
    ratio = torch.where(a > 0, err / a.clamp_min(1e-300), torch.where(err > 0, float("inf"), 0.0))
    j = int(torch.argmax(ratio).item())
    out = {"max_error_ratio": float(ratio[j].item()), "argmax": j,
           "reference": "float64 prefix sums on the device", "bound": "|y_j - y64_j| / sum_{i<=j} |x_i|"}
    del xf, ref, a, err, ratio
    torch.cuda.empty_cache()
    return out


# ---------------------------------------------------------------------------
# workloads
# ---------------------------------------------------------------------------

def to_device(x, dtype):
    import numpy as np
    import torch

    if dtype == "bfloat16":
        return torch.from_numpy(x.view(np.int16)).view(torch.bfloat16).to("cuda")
    return torch.from_numpy(x).to("cuda")


def bench_plain(binding, x_host, dtype, op, comp, steps, warmup):
    import torch

    xd = to_device(x_host, dtype)
    n = xd.shape[0]
    y = torch.empty(n, dtype=binding.out_dtype(xd), device="cuda")
    fn = lambda: binding.inclusive(xd, op, comp, out=y)  # noqa: E731
    ms, per = time_steps(fn, steps, warmup)
    binding.lscan_check(torch.cuda.current_stream().cuda_stream)
    info = binding.lscan_last_launch()
    in_b = 2 if dtype == "bfloat16" else xd.element_size()
    nbytes = n * (in_b + y.element_size())
    entry = rate_entry(nbytes, n, ms, per)
    entry.update({"n": n, "dtype": dtype, "op": op, "compensated": comp, "bytes": nbytes,
                  "grid": info.grid, "block_threads": info.block_threads, "tile_elems": info.tile_elems,
                  "num_blocks": info.num_blocks})
    if op == "add" and dtype in ("float32", "bfloat16"):
        entry["error"] = float_error(xd, y)
        entry["error"]["tolerance"] = 2e-7 if comp else 1e-6
    del xd, y
    torch.cuda.empty_cache()
    return entry


CEILING_LIB = os.path.join(ROOT, "paper_1604_04815_amd", "ceiling", "libcopy_ceiling.so")


def bench_copy(n, steps, warmup, scan_shape=(256, 16, 2)):
    """Copies of the headline's bytes (N int32 read, N written): the
    practical ceiling of a kernel that touches every byte once.
      persistent  the scan's structure without the hand-off: the scan's grid
                  (groups per CU), tile (threads x vectors) and one-round
                  load/store pipeline, the same 16-byte non-temporal vectors
      persistent_strips  the same grid and pipeline with each load of the
                  workgroup over one contiguous span (row r of every wave
                  side by side): the best persistent copy measured
      flat        one 4 KiB tile per workgroup, hardware-dispatched grid
      torch       torch's copy_ (the runtime's copy kernel)"""
    import ctypes

    import torch

    a = torch.empty(n, dtype=torch.int32, device="cuda").fill_(1)
    b = torch.empty_like(a)
    out = {}
    lib = ctypes.CDLL(CEILING_LIB)
    lib.ceiling_copy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_int,
                                 ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.POINTER(ctypes.c_int)]
    lib.ceiling_copy.restype = ctypes.c_int
    grid = ctypes.c_int()
    stream = torch.cuda.current_stream().cuda_stream
    t, r, g = scan_shape
    for name, structure, shape in (("persistent", 1, (t, r, g)), ("persistent_strips", 2, (t, r, g)),
                                   ("flat", 0, (256, 1, 0))):
        def fn(structure=structure, shape=shape):
            st = lib.ceiling_copy(a.data_ptr(), b.data_ptr(), 4 * n, structure, shape[0], shape[1], shape[2],
                                  stream, ctypes.byref(grid))
            if st != 0:
                raise RuntimeError(f"ceiling_copy failed: {st}")
        ms, per = time_steps(fn, steps, warmup)
        e = rate_entry(2 * 4 * n, n, ms, per)
        e.update({"structure": name, "block_threads": shape[0], "vectors_per_lane": shape[1], "grid": grid.value})
        if structure != 0:
            e["groups_per_cu"] = shape[2]
        out[name] = e
    assert torch.equal(a, b)
    ms, per = time_steps(lambda: b.copy_(a), steps, warmup)
    out["torch"] = rate_entry(2 * 4 * n, n, ms, per)
    del a, b
    torch.cuda.empty_cache()
    return out


def bench_segmented(binding, workloads, steps, warmup):
    """4096 arrays, log-uniform lengths in [1, 2^20]: one persistent
    segmented launch against 4096 plain launches on one stream."""
    import numpy as np
    import torch

    off = workloads.segment_offsets(4096, 1 << 20, workloads.seed_for(3))
    n = int(off[-1])
    out = {}
    for dtype in ("int32", "float32"):
        if dtype == "int32":
            x = workloads.uniform_int(n, -1000, 1000, workloads.seed_for(3, 1))
        else:
            x = workloads.uniform01_f32(n, workloads.seed_for(3, 2))
        xd = to_device(x, dtype)
        od = torch.from_numpy(off).to("cuda")
        y = torch.empty_like(xd)
        ms_seg, per = time_steps(lambda: binding.segmented(xd, od, "add", out=y), steps, warmup)
        seg_y = y.clone()
        views = [(xd[int(off[s]):int(off[s + 1])], y[int(off[s]):int(off[s + 1])]) for s in range(4096)]

        def plain_all():
            for xs, ys in views:
                if xs.shape[0]:
                    binding.inclusive(xs, "add", out=ys)

        ms_plain, _ = time_steps(plain_all, max(2, steps // 5), 1)
        binding.lscan_check(torch.cuda.current_stream().cuda_stream)
        same = bool(torch.equal(seg_y, y)) if dtype == "int32" else None
        # the same segmented launch captured once in a hipGraph and replayed
        code = binding.I32 if dtype == "int32" else binding.F32
        g = binding.lscan_graph_create_segmented(xd.data_ptr(), y.data_ptr(), n, od.data_ptr(), 4096, code,
                                                 binding.ADD)
        ms_graph, per_graph = time_steps(g.launch, steps, warmup)
        g.check()
        g.destroy()
        graph_same = bool(torch.equal(seg_y, y))
        err = float_error(xd, seg_y, od) if dtype == "float32" else None
        nbytes = n * 8
        e = rate_entry(nbytes, n, ms_seg, per)
        e.update({"n": n, "segments": 4096, "plain_4096_launches_ms": round(ms_plain, 4),
                  "speedup_vs_plain_launches": round(ms_plain / ms_seg, 2),
                  "graph": rate_entry(nbytes, n, ms_graph, per_graph),
                  "graph_speedup_vs_plain_launches": round(ms_plain / ms_graph, 2),
                  "graph_bit_equal_to_eager": graph_same})
        if same is not None:
            e["bit_equal_to_plain_launches"] = same
        if err is not None:
            err["tolerance"] = 1e-6
            e["error"] = err
        if dtype == "int32":
            # the same 4096 arrays as separate arrays of one batched launch
            # (cut at arbitrary element offsets: each array's own alignment
            # phase), eager and as a graph
            table = [(xs.data_ptr(), ys.data_ptr(), xs.shape[0]) for xs, ys in views]
            tab = binding._array_table(table)
            lib = binding.load()
            stream = torch.cuda.current_stream().cuda_stream

            def batched():
                binding._check(lib.lscan_batched(tab, len(table), binding.I32, binding.ADD, 0, stream),
                               "lscan_batched")

            y.zero_()
            ms_b, per_b = time_steps(batched, steps, warmup)
            binding.lscan_check(stream)
            b_same = bool(torch.equal(seg_y, y))
            gb = binding.lscan_graph_create_batched(table, binding.I32, binding.ADD)
            y.zero_()
            ms_bg, per_bg = time_steps(gb.launch, steps, warmup)
            gb.check()
            gb.destroy()
            e.update({"batched": rate_entry(nbytes, n, ms_b, per_b),
                      "batched_graph": rate_entry(nbytes, n, ms_bg, per_bg),
                      "batched_speedup_vs_plain_launches": round(ms_plain / ms_bg, 2),
                      "batched_bit_equal_to_segmented": b_same and bool(torch.equal(seg_y, y))})
        out[f"segmented_4096_{dtype}_add"] = e
        del xd, y, seg_y, views, od
        torch.cuda.empty_cache()
    return out


def bench_compact(binding, x_host, steps, warmup, seed):
    """Stream compaction of the headline array with half of the items kept
    (independent random keep bytes): algorithmic bytes are N items and N
    flags read, the kept items written and the 8-byte count."""
    import numpy as np
    import torch

    n = x_host.shape[0]
    g = np.random.default_rng(seed)
    keep_host = (g.random(n) < 0.5).astype(np.uint8)
    xd = to_device(x_host, "int32")
    kd = torch.from_numpy(keep_host).to("cuda")
    out = torch.empty_like(xd)
    count = torch.empty(1, dtype=torch.int64, device="cuda")
    ms, per = time_steps(lambda: binding.compact(xd, kd, out=out, count=count), steps, warmup)
    binding.lscan_check(torch.cuda.current_stream().cuda_stream)
    info = binding.lscan_last_launch()
    kept = int(count.item())
    nbytes = 4 * n + n + 4 * kept + 8
    e = rate_entry(nbytes, n, ms, per)
    mask = kd.bool()
    ms_torch, _ = time_steps(lambda: torch.masked_select(xd, mask), max(2, steps // 2), 1)
    ref = torch.masked_select(xd, mask)
    e.update({"n": n, "kept": kept, "bytes": nbytes, "grid": info.grid, "block_threads": info.block_threads,
              "tile_elems": info.tile_elems, "equal_to_torch_masked_select": bool(torch.equal(out[:kept], ref)),
              "torch_masked_select_ms": round(ms_torch, 5),
              "speedup_vs_torch_masked_select": round(ms_torch / ms, 2)})
    del xd, kd, out, mask, ref
    torch.cuda.empty_cache()
    return e


def bench_radix(binding, workloads, steps, warmup):
    """Digit offsets of one 8-bit radix-sort pass over 2^28 int32 keys in
    blocks of 16K keys: the digit-count kernel plus the exclusive scan of the
    2^8 x M counts.  Algorithmic bytes: the keys read once, the counts
    written, then read and written by the scan."""
    import torch

    n, block, bits = 1 << 28, 1 << 14, 8
    kd = to_device(workloads.full_range_int32(n, workloads.seed_for(6)), "int32")
    m = (n + block - 1) // block
    out = torch.empty((1 << bits) * m, dtype=torch.int64, device="cuda")
    ms, per = time_steps(lambda: binding.radix_offsets(kd, 0, bits, block, out=out), steps, warmup)
    binding.lscan_check(torch.cuda.current_stream().cuda_stream)
    counts_bytes = 8 * (1 << bits) * m
    nbytes = 4 * n + 3 * counts_bytes
    e = rate_entry(nbytes, n, ms, per)
    e.update({"n": n, "block_items": block, "bits": bits, "blocks": m, "bytes": nbytes,
              "key_gbs": round(4 * n / (ms * 1e-3) / 1e9, 1),
              "last_offset_plus_count_is_n": None})
    # the last digit's offsets end at n
    last = out.view(1 << bits, m)[-1, -1].item()
    hist_last = int(((kd[(m - 1) * block:].to(torch.int64) & 0xFF) == 0xFF).sum().item())
    e["last_offset_plus_count_is_n"] = bool(last + hist_last == n)
    del kd, out
    torch.cuda.empty_cache()
    return e


def bench_bfs(binding, workloads, steps, warmup, num_sources=8):
    """Breadth-first search over an R-MAT graph: 2^22 vertices, edge factor
    16, every edge in both directions (134M column entries), from
    num_sources seeded sources that have at least one edge.  Rate: edges
    scanned per second (the out-degrees of the reached vertices over the
    search time; Graph500 counts each undirected edge once, half of that).
    Algorithmic bytes per search: 16 per vertex (row offsets read once for
    the monotonicity check, level and parent set up), 64 per reached vertex
    (row offsets 16, level and parent 8, frontier entry -- vertex, edge
    offset, first edge, 20 bytes -- written and read), 8 per scanned edge
    (column 4, visited word 4).  Every search is validated on the device: levels of both ends of
    every edge differ by at most one where the tail is reached, every reached
    vertex other than the source has a parent one level up with an edge to
    it."""
    import numpy as np
    import torch

    scale, ef = 22, 16
    row, col = workloads.rmat_csr_torch(scale, ef, workloads.seed_for(9), device="cuda")
    nv = row.shape[0] - 1
    deg = row[1:] - row[:-1]
    cand = torch.nonzero(deg > 0).flatten().cpu().numpy()
    sources = np.random.default_rng(workloads.seed_for(9, 1)).choice(cand, num_sources, replace=False)
    tail = torch.repeat_interleave(torch.arange(nv, device="cuda"), deg)
    keys = tail * nv + col.to(torch.int64)  # sorted: rows in order, columns sorted in each row
    levels = torch.empty(nv, dtype=torch.int32, device="cuda")
    parents = torch.empty(nv, dtype=torch.int32, device="cuda")
    stats = torch.empty(4, dtype=torch.int64, device="cuda")
    runs = []
    valid = True
    for src in sources.tolist():
        fn = lambda: binding.bfs(row, col, src, levels=levels, parents=parents, stats=stats)  # noqa: E731
        ms, per = time_steps(fn, steps, warmup)
        binding.lscan_check(torch.cuda.current_stream().cuda_stream)
        st = stats.cpu().tolist()
        lv = levels.to(torch.int64)
        lt, lh = lv[tail], lv[col.to(torch.int64)]
        ok = bool(((lt < 0) | ((lh >= 0) & (lh <= lt + 1))).all().item())
        ok &= int(lv[src].item()) == 0 and int(parents[src].item()) == src
        reached = lv >= 0
        ok &= int(reached.sum().item()) == st[1] and int(lv.max().item()) + 1 == st[0]
        v = torch.nonzero(reached).flatten()
        v = v[v != src]
        p = parents[v].to(torch.int64)
        ok &= bool(((p >= 0) & (p < nv)).all().item())
        if ok:
            ok &= bool((lv[p] == lv[v] - 1).all().item())
            q = p * nv + v
            i = torch.clamp(torch.searchsorted(keys, q), max=keys.shape[0] - 1)
            ok &= bool((keys[i] == q).all().item())
        ok &= int(deg[reached].sum().item()) == st[2] and st[3] == 0
        valid &= ok
        nbytes = 16 * nv + 64 * st[1] + 8 * st[2]
        runs.append({"source": int(src), "ms": round(ms, 4), "launch_ms_mean": round(statistics.mean(per), 4),
                     "levels": st[0], "reached": st[1], "edges_scanned": st[2],
                     "gteps_scanned": round(st[2] / (ms * 1e-3) / 1e9, 3), "bytes": nbytes,
                     "gbs": round(nbytes / (ms * 1e-3) / 1e9, 1), "valid": ok})
    info = binding.lscan_last_launch()
    teps = [r["gteps_scanned"] for r in runs]
    hmean = len(teps) / sum(1.0 / t for t in teps)
    e = {"workload": f"rmat scale {scale} edge factor {ef}, symmetric", "num_vertices": nv,
         "column_entries": int(col.shape[0]), "sources": num_sources,
         "gteps_scanned_hmean": round(hmean, 3), "gteps_graph500_hmean": round(hmean / 2, 3),
         "ms_median": round(statistics.median(r["ms"] for r in runs), 4),
         "gbs_median": round(statistics.median(r["gbs"] for r in runs), 1),
         "frac_hbm_peak_median": round(statistics.median(r["gbs"] for r in runs) / HBM_PEAK_GBS, 4),
         "grid": info.grid, "block_threads": info.block_threads, "groups_per_cu": info.groups_per_cu,
         "all_valid": valid, "runs": runs}
    del row, col, tail, keys, levels, parents
    torch.cuda.empty_cache()
    return e


def bench_custom_affine(binding, steps, warmup):
    """A scan with a user-defined operator built outside the library
    (include/lscan_custom.hpp): composition of affine maps mod 2^32 over 2^27
    maps, 8 bytes in and 8 bytes out each, for each example tile shape."""
    import numpy as np
    import torch

    n = 1 << 27
    g = np.random.default_rng(1604 + 1100)
    ab = g.integers(0, 1 << 32, (n, 2), dtype=np.uint64).astype(np.uint32)
    x = torch.from_numpy(ab.view(np.int32).reshape(-1)).to("cuda")
    y = torch.empty_like(x)
    del ab
    kernels = binding.affine_example_kernels()
    shapes = {}
    for name in ("default", "small", "wide"):
        k = kernels[name]
        ms, per = time_steps(lambda: binding.scan_custom(k, x, n, out=y), steps, warmup)
        binding.lscan_check(torch.cuda.current_stream().cuda_stream)
        info = binding.lscan_last_launch()
        e = rate_entry(16 * n, n, ms, per)
        e.update({"block_threads": info.block_threads, "tile_elems": info.tile_elems, "grid": info.grid})
        shapes[name] = e
    best = max(shapes, key=lambda k: shapes[k]["gbs"])
    out = dict(shapes[best])
    out.update({"n": n, "bytes": 16 * n, "best_shape": best, "shapes": shapes})
    del x, y
    torch.cuda.empty_cache()
    return out


def cpu_parallel_scan(x, repeats: int = 3):
    """Context, not the oracle: a two-pass chunked scan over all host cores
    (per-chunk totals, a scan of the totals, per-chunk scans with their
    offsets; numpy releases the interpreter lock inside each pass), the
    analogue of a multi-core library scan on the CPU."""
    import numpy as np
    from concurrent.futures import ThreadPoolExecutor

    threads = len(os.sched_getaffinity(0))
    n = x.shape[0]
    y = np.empty_like(x)
    bounds = np.linspace(0, n, threads + 1).astype(np.int64)
    times = []
    with ThreadPoolExecutor(threads) as ex:
        for _ in range(repeats):
            t0 = time.perf_counter()
            totals = list(ex.map(lambda k: x[bounds[k]:bounds[k + 1]].sum(dtype=x.dtype), range(threads)))
            offs = np.concatenate([[0], np.cumsum(np.array(totals, dtype=x.dtype), dtype=x.dtype)[:-1]])

            def chunk(k):
                seg = y[bounds[k]:bounds[k + 1]]
                np.cumsum(x[bounds[k]:bounds[k + 1]], out=seg)
                seg += x.dtype.type(offs[k])

            list(ex.map(chunk, range(threads)))
            times.append(time.perf_counter() - t0)
    t = statistics.median(times)
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), "")
    except OSError:
        pass
    nbytes = 2 * n * x.dtype.itemsize
    ok = bool(y[-1] == x.sum(dtype=x.dtype)) if n else True
    return {"value": round(nbytes / t / 1e9, 3), "unit": "GB/s", "threads": threads, "cpu_model": model,
            "last_equals_total": ok,
            "ms": round(t * 1e3, 2), "kind": "two-pass chunked scan (numpy, threads)",
            "sample": f"the full int32 add N=2^{int(np.log2(n))} array, median of {repeats}"}


def bench_latency(binding, workloads, steps):
    """N = 2^20 int32 add: launch-bound.  Device time of one launch, taken
    with the stream already busy (a spin kernel queued first), so the event
    pair around the launch holds no host time; and the host time of one
    call + synchronize."""
    import torch

    x = workloads.uniform_int(1 << 20, -1000, 1000, workloads.seed_for(0))
    xd = to_device(x, "int32")
    y = torch.empty_like(xd)
    fn = lambda: binding.inclusive(xd, "add", out=y)  # noqa: E731
    ms, per = time_steps(fn, max(steps, 50), 5)
    filler = torch.empty(1 << 26, dtype=torch.int32, device="cuda")

    def busy():  # keeps the stream busy (tens of microseconds) while the launch below is queued
        try:
            torch.cuda._sleep(200_000)
        except Exception:  # noqa: BLE001 - any kernel of that length will do
            filler.fill_(1)

    dev = []
    for _ in range(max(steps, 50)):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        busy()
        a.record()
        fn()
        b.record()
        b.synchronize()
        dev.append(a.elapsed_time(b))
    host = []
    for _ in range(max(steps, 50)):
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        host.append((time.perf_counter() - t0) * 1e3)
    # the same scan captured once into a graph and replayed
    g = binding.lscan_graph_create_scan(xd.data_ptr(), y.data_ptr(), 1 << 20, binding.I32, binding.ADD)
    want = y.clone()
    g.launch()
    g.check()
    if not torch.equal(y, want):
        raise RuntimeError("graph replay differs from the eager scan")
    gms, gper = time_steps(g.launch, max(steps, 50), 5)
    ghost = []
    for _ in range(max(steps, 50)):
        t0 = time.perf_counter()
        g.launch()
        torch.cuda.synchronize()
        ghost.append((time.perf_counter() - t0) * 1e3)
    g.destroy()
    e = rate_entry(8 * (1 << 20), 1 << 20, ms, per)
    e.update({"device_ms_p50": round(pct(dev, 50), 5), "device_ms_min": round(min(dev), 5),
              "device_ms_p99": round(pct(dev, 99), 5),
              "host_call_sync_ms_p50": round(pct(host, 50), 4), "host_call_sync_ms_p99": round(pct(host, 99), 4),
              "graph_replay_ms_per_step": round(gms, 5),
              "graph_host_launch_sync_ms_p50": round(pct(ghost, 50), 4),
              "graph_host_launch_sync_ms_p99": round(pct(ghost, 99), 4)})
    return e


def _serving_pools(workloads):
    """Device-resident value pools (2^26 elements each) that request inputs
    are sliced from; PCIe could not feed fresh inputs at the offered load."""
    n = 1 << 26
    return {
        ("int32", "add"): to_device(workloads.uniform_int(n, -1000, 1000, workloads.seed_for(4, 1)), "int32"),
        ("int32", "max"): to_device(workloads.full_range_int32(n, workloads.seed_for(4, 2)), "int32"),
        ("int64", "add"): to_device(workloads.int64_half_open(n, -(2 ** 31), 2 ** 31, workloads.seed_for(4, 3)),
                                    "int64"),
        ("float32", "add"): to_device(workloads.signed_lognormal_f32(n, workloads.seed_for(4, 4)), "float32"),
    }


def _pool_slice(pools, req, rng):
    key = (req["dtype"], "max" if (req["dtype"] == "int32" and req["op"] == "max") else "add")
    pool = pools[key]
    n = req["n"]
    off = int(rng.integers(0, pool.shape[0] - n + 1)) & ~3  # 16-byte aligned slices
    return pool[off:off + n]


def bench_chain(binding, x_host, steps):
    """The paper's prefix chain (every block waits for its predecessor's
    inclusive prefix) against the default window hand-off, same shape and
    input: time per launch, and the time per hand-off in the chain."""
    import torch

    xd = to_device(x_host, "int32")
    n = xd.shape[0]
    y = torch.empty_like(xd)
    binding.inclusive(xd, "add", out=y)
    window = y.clone()
    p = binding.Params(0, 0, 0, binding.HANDOFF_CHAIN)
    ms, per = time_steps(lambda: binding.inclusive(xd, "add", out=y, params=p), steps, 1)
    binding.lscan_check(torch.cuda.current_stream().cuda_stream)
    info = binding.lscan_last_launch()
    e = rate_entry(8 * n, n, ms, per)
    e.update({"n": n, "num_blocks": info.num_blocks, "grid": info.grid, "block_threads": info.block_threads,
              "us_per_handoff": round(ms * 1e3 / info.num_blocks, 4),
              "bit_equal_to_window": bool(torch.equal(y, window))})
    del xd, y, window
    torch.cuda.empty_cache()
    return e


def bench_serving(binding, workloads, seconds: float, rate: float):
    """Poisson trace through the request server (two streams, continuous
    batching), and the same trace served one request at a time: a server
    with one stream in which every request runs alone as a plain
    full-device scan, launched when the previous one has completed (FIFO,
    no overlap).  Both arms take their timestamps the same way: latency is
    the server's completion time (its completion thread, after the batch's
    event) minus the request's arrival time, both from the host's monotonic
    clock."""
    import numpy as np
    import torch

    trace = workloads.request_trace(rate, seconds, workloads.seed_for(4))
    pools = _serving_pools(workloads)
    torch.cuda.synchronize()
    size_of = {"int32": 4, "int64": 8, "float32": 4}
    total_bytes = sum(2 * size_of[r["dtype"]] * r["n"] for r in trace)
    rng = np.random.default_rng(workloads.seed_for(4, 9))
    xs = [_pool_slice(pools, r, rng) for r in trace]
    out = {"requests": len(trace), "seconds": seconds, "rate_hz": rate, "bytes": total_bytes}
    ops = {"add": binding.ADD, "max": binding.MAX}

    def run_trace(srv, keep_for_check):
        """Submit every request at its arrival time; returns per-request
        latencies (ns), batch sizes, the last completion time, the first
        arrival and the outputs kept for spot checks."""
        torch.cuda.synchronize()
        t0 = time.monotonic_ns() + 20_000_000
        arrivals = [t0 + int(r["t"] * 1e9) for r in trace]
        live = {}
        lat, sizes, t_done_last = [], [], t0
        kept = []
        k = 0
        while k < len(trace) or live:
            now = time.monotonic_ns()
            while k < len(trace) and arrivals[k] <= now:
                r, x = trace[k], xs[k]
                y = torch.empty(r["n"], dtype=x.dtype, device="cuda")
                tk = srv.submit_raw(x.data_ptr(), y.data_ptr(), r["n"], binding.dtype_code(x), ops[r["op"]])
                if tk < 0:
                    raise RuntimeError(f"submit refused: {tk}")
                live[tk] = (k, y)
                k += 1
            for tk in list(live):
                st, res = srv.poll(tk)
                if st == binding.PENDING:
                    continue
                if st != binding.OK:
                    raise RuntimeError(f"request failed: {st}")
                idx, y = live.pop(tk)
                lat.append(res.t_done_ns - arrivals[idx])
                sizes.append(res.batch_size)
                t_done_last = max(t_done_last, res.t_done_ns)
                if keep_for_check(idx):
                    kept.append((idx, y))
        return lat, sizes, t_done_last, arrivals[0], kept

    def summarize(lat_ns, t_first, t_last):
        lat = np.array(lat_ns, dtype=np.float64) / 1e3
        span = (t_last - t_first) / 1e9
        return {"p50_us": round(float(np.percentile(lat, 50)), 1), "p99_us": round(float(np.percentile(lat, 99)), 1),
                "mean_us": round(float(lat.mean()), 1), "gbs": round(total_bytes / span / 1e9, 1),
                "makespan_s": round(span, 3)}

    def size_hist(sizes):
        """Requests by the size of the launch that carried them."""
        buckets = [(1, 1), (2, 2), (3, 4), (5, 8), (9, 16), (17, 64), (65, 1 << 30)]
        hist = {}
        for lo, hi in buckets:
            c = sum(1 for b in sizes if lo <= b <= hi)
            if c:
                hist[str(lo) if lo == hi else (f"{lo}-{hi}" if hi < (1 << 30) else f"{lo}+")] = c
        return hist

    # --- served: two streams, continuous batching
    srv = binding.Server(num_streams=2, hbm_budget_bytes=32 << 30)
    lat, sizes, t_last, t_first, checks = run_trace(srv, lambda idx: idx % 997 == 0)
    stats = srv.stats()
    srv.close()
    served = summarize(lat, t_first, t_last)
    served.update({"batches": int(stats.batches), "peak_bytes_in_flight": int(stats.peak_bytes_in_flight),
                   "requests_by_batch_size": size_hist(sizes),
                   "mean_batch_size_per_request": round(float(np.mean(sizes)), 3)})
    failed = []
    for idx, y in checks:
        alone = binding.inclusive(xs[idx], trace[idx]["op"])
        if trace[idx]["dtype"] == "float32" and trace[idx]["op"] == "add":
            # both within 1e-6 * sum |x_i| of the exact prefix (different tile
            # shapes associate differently), so within twice that of each other
            a = torch.cumsum(xs[idx].abs().to(torch.float64), 0)
            diff = (y.to(torch.float64) - alone.to(torch.float64)).abs()
            ok = bool((diff <= 2e-6 * a).all())
        else:
            ok = bool(torch.equal(y, alone))
        if not ok:
            failed.append({"request": idx, "dtype": trace[idx]["dtype"], "op": trace[idx]["op"], "n": trace[idx]["n"]})
    served["spot_checks_equal_alone"] = not failed
    served["spot_check_failures"] = failed[:8]
    served["spot_checks"] = len(checks)
    out["served"] = served
    del checks

    # --- serial plain launches: one stream, every request alone on the
    # full-device plain kernel, the next launched only after it completes
    srv = binding.Server(num_streams=1, hbm_budget_bytes=32 << 30, max_batch=1, solo_bytes=1)
    lat, sizes, t_last, t_first, _ = run_trace(srv, lambda idx: False)
    stats = srv.stats()
    srv.close()
    serial = summarize(lat, t_first, t_last)
    serial.update({"batches": int(stats.batches), "how": "request server, one stream, every request alone "
                   "(full-device plain kernel), FIFO, no overlap"})
    out["serial_plain"] = serial
    out["p99_speedup_vs_serial"] = round(out["serial_plain"]["p99_us"] / out["served"]["p99_us"], 2)
    out["p50_speedup_vs_serial"] = round(out["serial_plain"]["p50_us"] / out["served"]["p50_us"], 2)
    out["clock"] = "both arms: server completion timestamp minus arrival, host monotonic clock"
    del pools, xs
    torch.cuda.empty_cache()
    return out


def cpu_baseline(x_host, budget_s: float):
    """The sequential oracle (one core) on the same array, repeated for about
    budget_s seconds; median rate."""
    import oracle

    oracle.build(force=False)
    times = []
    t_start = time.perf_counter()
    while True:
        t0 = time.perf_counter_ns()
        oracle.scan(x_host, "int32", "add")
        times.append((time.perf_counter_ns() - t0) * 1e-9)
        if len(times) >= 2 and time.perf_counter() - t_start >= budget_s:
            break
    t = statistics.median(times)
    n = x_host.shape[0]
    return {"value": round(2 * 4 * n / t / 1e9, 3), "unit": "GB/s", "cores": 1, "kind": "oracle",
            "sample": f"the full int32 add N=2^28 array, {len(times)} sequential passes (median "
                      f"{t:.3f} s each, {sum(times):.1f} s total) on one host core",
            "gelem_s": round(n / t / 1e9, 3)}


def cpu_oracle_rows(workloads, configs):
    """The oracle (one core) timed on a bounded sample of each workload line
    present in configs; attaches {"gelem_s", "sample", "cores"} as
    "oracle_cpu" to that line (rates in the line's own element unit)."""
    import numpy as np

    import oracle

    oracle.build(force=False)
    n = 1 << 22

    def timed(fn, elems, sample):
        times = []
        for _ in range(3):
            t0 = time.perf_counter_ns()
            fn()
            times.append((time.perf_counter_ns() - t0) * 1e-9)
        t = statistics.median(times)
        return {"gelem_s": round(elems / t / 1e9, 4), "sample": sample, "cores": 1}

    s = workloads.seed_for(9)
    rows = {}
    if "int64_add_2p27" in configs:
        x = workloads.int64_half_open(n, -(2 ** 31), 2 ** 31, s)
        rows["int64_add_2p27"] = timed(lambda: oracle.scan(x, "int64", "add"), n, "2^22 int64 of the same recipe")
    if "int32_max_2p28" in configs:
        x = workloads.full_range_int32(n, s)
        rows["int32_max_2p28"] = timed(lambda: oracle.scan(x, "int32", "max"), n, "2^22 int32 of the same recipe")
    if "float32_add_2p27" in configs:
        x = workloads.signed_lognormal_f32(n, s)
        r = timed(lambda: oracle.scan(x, "float32", "add"), n, "2^22 float32 of the same recipe (fp64 fold)")
        rows["float32_add_2p27"] = rows["float32_add_2p27_compensated"] = r
    if "bf16_add_2p27" in configs:
        x = workloads.bf16_unit(n, s)
        r = timed(lambda: oracle.scan(x, "bfloat16", "add"), n, "2^22 bf16 of the same recipe (fp64 fold)")
        rows["bf16_add_2p27"] = rows["bf16_add_2p27_compensated"] = r
    if "segmented_4096_int32_add" in configs:
        off = workloads.segment_offsets(64, 1 << 16, s)
        x = workloads.uniform_int(int(off[-1]), -1000, 1000, s)
        rows["segmented_4096_int32_add"] = timed(lambda: oracle.segscan(x, off, "int32", "add"), x.shape[0],
                                                 f"64 log-uniform segments, {x.shape[0]} int32")
    if "compact_int32_2p28_half" in configs:
        x = workloads.uniform_int(n, -1024, 1024, s)
        keep = (np.random.default_rng(s).random(n) < 0.5).astype(np.uint8)
        rows["compact_int32_2p28_half"] = timed(lambda: oracle.compact(x, keep), n, "2^22 int32, half kept")
    if "argmax_int32_2p28" in configs:
        x = workloads.uniform_int(n, -1024, 1024, s)
        rows["argmax_int32_2p28"] = timed(lambda: oracle.argscan(x, "int32", "argmax"), n, "2^22 int32")
    if "radix_offsets_int32_2p28_8bit" in configs:
        x = workloads.full_range_int32(n, s)
        rows["radix_offsets_int32_2p28_8bit"] = timed(lambda: oracle.radix_offsets(x, 0, 8, 1 << 14), n,
                                                      "2^22 int32 keys, 8 bits, 16K-key blocks")
    if "custom_affine_2p27" in configs:
        g = np.random.default_rng(s)
        ab = g.integers(0, 1 << 32, (n, 2), dtype=np.uint64).astype(np.uint32)
        rows["custom_affine_2p27"] = timed(lambda: oracle.affine_scan(ab), n, "2^22 affine maps")
    if "bfs_rmat22" in configs:
        src, dst = workloads.rmat_edges(16, 16, s)
        row, col = workloads.csr_from_edges(src, dst, 1 << 16)
        deg = np.diff(row)
        root = int(np.flatnonzero(deg > 0)[0])
        lev = oracle.bfs_levels(row, col, root)
        scanned = int(deg[lev >= 0].sum())
        r = timed(lambda: oracle.bfs_levels(row, col, root), scanned,
                  "R-MAT 2^16 vertices, edge factor 16, symmetric, one source")
        r["unit"] = "G edges scanned/s"
        rows["bfs_rmat22"] = r
    for k, v in rows.items():
        configs[k]["oracle_cpu"] = v


def main(argv=None) -> int:
    global SETTLE_S
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--only", default="", help="'1a': only the headline scan and the copies of its bytes; a comma "
                    "list of lines (int64_add_2p27, int32_max_2p28, float32_add_2p27[_compensated], "
                    "bf16_add_2p27[_compensated], segmented, serving, latency, compact, argmax, radix, bfs, custom, "
                    "chain, torch_cumsum): the headline plus those; 'serve': only the serving trace; "
                    "'bfs': only the breadth-first search line; 'custom': only the user-operator line")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--serve-seconds", type=float, default=60.0,
                    help="length of the Poisson request trace (the workload's full trace: 60 s)")
    ap.add_argument("--serve-rate", type=float, default=2000.0)
    ap.add_argument("--serve-heavy-rate", type=float, default=20000.0,
                    help="a second, heavier trace where requests queue and batching pays")
    ap.add_argument("--serve-heavy-seconds", type=float, default=1.0)
    ap.add_argument("--settle", type=float, default=SETTLE_S,
                    help="seconds the device runs each measured call, untimed, before its warmup steps")
    args = ap.parse_args(argv)
    SETTLE_S = max(0.0, args.settle)

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the scan is not sharded "
              "across GPUs", file=sys.stderr)
        return 2
    if "WORLD_SIZE" in os.environ and int(os.environ["WORLD_SIZE"]) > 1:
        print("bench.py runs on one GPU only", file=sys.stderr)
        return 2

    import torch

    from paper_1604_04815_amd import binding, workloads

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 2
    binding.load()
    torch.cuda.init()
    dev = torch.cuda.get_device_properties(0)
    log(f"device {dev.name}, {dev.multi_processor_count} CUs")

    if args.only == "custom":
        print(json.dumps({"custom_affine_2p27": bench_custom_affine(binding, args.steps, args.warmup)}), flush=True)
        return 0
    if args.only == "bfs":
        bf = bench_bfs(binding, workloads, max(3, args.steps // 2), 1)
        print(json.dumps({"bfs_rmat22": bf}), flush=True)
        return 0
    if args.only == "serve":
        sv = bench_serving(binding, workloads, args.serve_seconds, args.serve_rate)
        hv = bench_serving(binding, workloads, args.serve_heavy_seconds, args.serve_heavy_rate)
        print(json.dumps({"serving": sv, "serving_heavy": hv}), flush=True)
        return 0

    n = 1 << 28
    x = workloads.uniform_int(n, -1024, 1024, workloads.seed_for(1))
    log("headline: int32 add N=2^28")
    head = bench_plain(binding, x, "int32", "add", False, args.steps, args.warmup)
    log(f"  {head['gbs']} GB/s, {head['ms']} ms/step, grid {head['grid']} x {head['block_threads']}")
    copy = bench_copy(n, args.steps, args.warmup,
                      (head["block_threads"], head["tile_elems"] // head["block_threads"] // 4,
                       head["grid"] // dev.multi_processor_count))
    log(f"  copies of the same bytes: persistent {copy['persistent']['gbs']} GB/s, flat {copy['flat']['gbs']} GB/s, "
        f"torch {copy['torch']['gbs']} GB/s")

    configs = {"copy_int32_2p28": copy}
    only = set(args.only.split(",")) - {""} if args.only not in ("1a",) else set()

    def want(line):
        """Every line unless --only names lines (the headline always runs)."""
        if args.only == "1a":
            return False
        return not only or line in only

    if want("int64_add_2p27"):
        log("int64 add N=2^27")
        configs["int64_add_2p27"] = bench_plain(
            binding, workloads.int64_half_open(1 << 27, -(2 ** 31), 2 ** 31, workloads.seed_for(1, 1)),
            "int64", "add", False, args.steps, args.warmup)
    if want("int32_max_2p28"):
        log("int32 max N=2^28")
        configs["int32_max_2p28"] = bench_plain(
            binding, workloads.full_range_int32(1 << 28, workloads.seed_for(1, 2)),
            "int32", "max", False, args.steps, args.warmup)
    if want("float32_add_2p27") or want("float32_add_2p27_compensated"):
        xf = workloads.signed_lognormal_f32(1 << 27, workloads.seed_for(2))
        for comp in (False, True):
            key = f"float32_add_2p27{'_compensated' if comp else ''}"
            if want(key):
                log(f"float32 add N=2^27 compensated={comp}")
                configs[key] = bench_plain(binding, xf, "float32", "add", comp, args.steps, args.warmup)
        del xf
    if want("bf16_add_2p27") or want("bf16_add_2p27_compensated"):
        xb = workloads.bf16_unit(1 << 27, workloads.seed_for(2, 1))
        for comp in (False, True):
            key = f"bf16_add_2p27{'_compensated' if comp else ''}"
            if want(key):
                log(f"bf16 -> float32 add N=2^27 compensated={comp}")
                configs[key] = bench_plain(binding, xb, "bfloat16", "add", comp, args.steps, args.warmup)
        del xb
    if want("segmented"):
        log("segmented: 4096 arrays")
        configs.update(bench_segmented(binding, workloads, args.steps, args.warmup))
    if args.serve_seconds > 0 and want("serving"):
        log(f"serving: Poisson {args.serve_rate:.0f} req/s for {args.serve_seconds:.0f} s")
        configs["serving"] = bench_serving(binding, workloads, args.serve_seconds, args.serve_rate)
        sv = configs["serving"]
        log(f"  served p50/p99 {sv['served']['p50_us']}/{sv['served']['p99_us']} us, serial "
            f"{sv['serial_plain']['p50_us']}/{sv['serial_plain']['p99_us']} us")
        if args.serve_heavy_seconds > 0:
            log(f"serving: Poisson {args.serve_heavy_rate:.0f} req/s for {args.serve_heavy_seconds:.0f} s")
            configs["serving_heavy"] = bench_serving(binding, workloads, args.serve_heavy_seconds,
                                                     args.serve_heavy_rate)
            hv = configs["serving_heavy"]
            log(f"  served p50/p99 {hv['served']['p50_us']}/{hv['served']['p99_us']} us, serial "
                f"{hv['serial_plain']['p50_us']}/{hv['serial_plain']['p99_us']} us")
    if want("latency"):
        log("latency: int32 add N=2^20")
        configs["int32_add_2p20_latency"] = bench_latency(binding, workloads, args.steps)
    if want("compact"):
        log("stream compaction: int32 N=2^28, half kept")
        configs["compact_int32_2p28_half"] = bench_compact(binding, x, args.steps, args.warmup,
                                                           workloads.seed_for(5, 1))
        log(f"  {configs['compact_int32_2p28_half']['gbs']} GB/s, "
            f"{configs['compact_int32_2p28_half']['speedup_vs_torch_masked_select']}x torch.masked_select")
    if want("argmax"):
        log("running argmax: int32 N=2^28 (int64 indices)")
        xa = to_device(workloads.full_range_int32(1 << 28, workloads.seed_for(7)), "int32")
        ya = torch.empty(1 << 28, dtype=torch.int64, device="cuda")
        ms_a, per_a = time_steps(lambda: binding.inclusive(xa, "argmax", out=ya), args.steps, args.warmup)
        binding.lscan_check(torch.cuda.current_stream().cuda_stream)
        info_a = binding.lscan_last_launch()
        configs["argmax_int32_2p28"] = rate_entry(12 * (1 << 28), 1 << 28, ms_a, per_a)
        configs["argmax_int32_2p28"].update({"bytes": 12 * (1 << 28), "grid": info_a.grid,
                                             "block_threads": info_a.block_threads,
                                             "tile_elems": info_a.tile_elems})
        del xa, ya
        torch.cuda.empty_cache()
        log(f"  {configs['argmax_int32_2p28']['gbs']} GB/s")
    if want("radix"):
        log("radix-sort digit offsets: 2^28 int32 keys, 8 bits, 16K-key blocks")
        configs["radix_offsets_int32_2p28_8bit"] = bench_radix(binding, workloads, args.steps, args.warmup)
        log(f"  {configs['radix_offsets_int32_2p28_8bit']['key_gbs']} GB/s of keys")
    if want("bfs"):
        log("breadth-first search: R-MAT 2^22 vertices, edge factor 16, 8 sources")
        configs["bfs_rmat22"] = bench_bfs(binding, workloads, max(3, args.steps // 2), 1)
        bf = configs["bfs_rmat22"]
        log(f"  {bf['gteps_scanned_hmean']} G edges scanned/s (harmonic mean), median {bf['ms_median']} ms, "
            f"valid={bf['all_valid']}")
    if want("custom"):
        log("user-defined operator: affine maps mod 2^32, 2^27 maps")
        configs["custom_affine_2p27"] = bench_custom_affine(binding, args.steps, args.warmup)
        log(f"  {configs['custom_affine_2p27']['gbs']} GB/s ({configs['custom_affine_2p27']['best_shape']})")
    if want("chain"):
        log("the paper's prefix chain: int32 add N=2^20 and N=2^28")
        configs["int32_add_2p20_chain"] = bench_chain(
            binding, workloads.uniform_int(1 << 20, -1000, 1000, workloads.seed_for(0)), 10)
        configs["int32_add_2p28_chain"] = bench_chain(binding, x, 3)
        log(f"  chain {configs['int32_add_2p28_chain']['gbs']} GB/s, "
            f"{configs['int32_add_2p28_chain']['us_per_handoff']} us per hand-off")
    if want("torch_cumsum"):
        try:
            xd = to_device(x, "int32")
            yd = torch.empty_like(xd)
            ms, _ = time_steps(lambda: torch.cumsum(xd, 0, dtype=torch.int32, out=yd), 5, 1)
            configs["torch_cumsum_int32_2p28_context"] = rate_entry(8 * n, n, ms)
            del xd, yd
        except Exception as exc:  # noqa: BLE001 - context only
            log(f"torch.cumsum context skipped: {exc}")

    cpu = None
    if not args.no_cpu:
        log("CPU parallel scan (context)")
        configs["cpu_parallel_scan_context"] = cpu_parallel_scan(x)
        log(f"CPU oracle baseline (~{args.cpu_seconds:.0f} s)")
        cpu = cpu_baseline(x, args.cpu_seconds)
        cpu["cores_available"] = len(os.sched_getaffinity(0))
        log("CPU oracle on a sample of every other line")
        cpu_oracle_rows(workloads, configs)

    achieved = head["bytes"] / (head["ms"] * 1e-3) / 1e9
    # the kernel alone: algorithmic bytes over the mean of the per-launch
    # event pairs recorded around each launch on its stream (the whole-region
    # mean above also holds the gaps between launches)
    kernel_gbs = head["bytes"] / (head["launch_ms_mean"] * 1e-3) / 1e9
    traffic = read_traffic()
    record = {
        "metric": "scan GB/s (2N*bytes), % HBM peak; batched p50/p99 latency vs plain launches",
        "value": round(achieved, 1),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(head["ms"], 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": "inclusive scan, add, int32, N=2^28, x uniform in [-1024, 1024] (seeded)",
                   "n": n, "bytes_per_step": head["bytes"], "grid": head["grid"],
                   "block_threads": head["block_threads"], "tile_elems": head["tile_elems"],
                   "parallelism": "single GPU"},
        "gelem_per_s": head["gelem_s"],
        "frac_hbm_peak": round(achieved / HBM_PEAK_GBS, 4),
        "roofline": {"bound": "hbm", "achieved": round(kernel_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(kernel_gbs / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "algorithmic_bytes_per_launch": head["bytes"], "launch_ms_mean": head["launch_ms_mean"],
                     "copy_ceiling": {k: copy[k]["gbs"] for k in ("persistent", "persistent_strips", "flat", "torch")},
                     "frac_of_persistent_copy": round(achieved / copy["persistent"]["gbs"], 4),
                     "frac_of_best_persistent_copy": round(
                         achieved / max(copy["persistent"]["gbs"], copy["persistent_strips"]["gbs"]), 4)},
        "cpu_baseline": cpu,
        "settle_s": SETTLE_S,
        "step_ms_p50": head.get("ms_p50"),
        "step_ms_p99": head.get("ms_p99"),
        "configs": configs,
    }
    print(json.dumps(record), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
