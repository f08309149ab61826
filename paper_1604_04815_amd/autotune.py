"""Autotuner for the scan launch parameters.

The paper fixes its launch shape by hand from the register budget of one SM
(T = 1024 threads, K = 44 or 20 items per thread, one block per SM; Section
5.1).  Here the shape is chosen by measurement: for one (dtype, operator,
precision, kernel kind) and a representative size, every compiled tile shape
(threads per workgroup x 16-byte vectors per lane) is timed at every
groups-per-CU count the device admits, and the fastest is installed as the
library default with ``lscan_set_params``.

Results persist in a JSON cache keyed by the device name, the dtype, the
operator, the compensation flag, the kernel kind and the size bucket
(``floor(log2(n))``), so later processes can apply them without re-timing.
"""
from __future__ import annotations

import json
import math
import os
import time
from dataclasses import asdict, dataclass, field

from . import binding

KINDS = {"plain": binding.KIND_PLAIN, "segmented": binding.KIND_SEGMENTED, "batched": binding.KIND_BATCHED,
         "compact": binding.KIND_COMPACT}
DTYPE_CODES = {"int32": binding.I32, "int64": binding.I64, "float32": binding.F32, "bfloat16": binding.BF16}
GROUPS = (1, 2, 3, 4, 5, 6, 8)


@dataclass
class Candidate:
    block_threads: int
    vectors_per_lane: int
    groups_per_cu: int
    grid: int = 0
    ms: float = float("inf")


@dataclass
class Entry:
    device: str
    dtype: str
    op: str
    compensated: bool
    kind: str
    size_bucket: int
    block_threads: int
    vectors_per_lane: int
    groups_per_cu: int
    ms: float
    gbs: float
    tried: int = 0
    when: float = field(default_factory=time.time)

    def key(self) -> str:
        return cache_key(self.device, self.dtype, self.op, self.compensated, self.kind, self.size_bucket)


def cache_key(device, dtype, op, compensated, kind, size_bucket) -> str:
    return f"{device}|{dtype}|{op}|{'comp' if compensated else 'plain'}|{kind}|2^{size_bucket}"


def size_bucket(n: int) -> int:
    return int(math.floor(math.log2(max(1, n))))


def pick_best(candidates):
    """Fastest candidate; ties go to the smaller grid (fewer flag reads per
    block) and then to fewer threads."""
    ok = [c for c in candidates if math.isfinite(c.ms)]
    if not ok:
        raise ValueError("no candidate ran")
    return min(ok, key=lambda c: (round(c.ms, 6), c.grid, c.block_threads))


def distinct_by_grid(candidates):
    """Drop candidates whose (shape, effective grid) repeats an earlier one."""
    seen, out = set(), []
    for c in candidates:
        k = (c.block_threads, c.vectors_per_lane, c.grid)
        if k not in seen:
            seen.add(k)
            out.append(c)
    return out


class Cache:
    """JSON file of tuned entries."""

    def __init__(self, path: str):
        self.path = path
        self.entries: dict[str, Entry] = {}
        if os.path.exists(path):
            with open(path) as f:
                raw = json.load(f)
            for d in raw.get("entries", []):
                e = Entry(**d)
                self.entries[e.key()] = e

    def put(self, e: Entry) -> None:
        self.entries[e.key()] = e

    def get(self, device, dtype, op, compensated, kind, n) -> Entry | None:
        return self.entries.get(cache_key(device, dtype, op, compensated, kind, size_bucket(n)))

    def save(self) -> None:
        tmp = self.path + ".tmp"
        with open(tmp, "w") as f:
            json.dump({"entries": [asdict(e) for e in self.entries.values()]}, f, indent=1, sort_keys=True)
        os.replace(tmp, self.path)


def apply(entry: Entry) -> None:
    """Install a tuned entry as the library default for its key."""
    flags = binding.F_COMPENSATED if entry.compensated else 0
    binding.lscan_set_params(DTYPE_CODES[entry.dtype], binding.OPS[entry.op], flags, KINDS[entry.kind],
                             binding.Params(entry.block_threads, entry.vectors_per_lane, entry.groups_per_cu, 0))


def _time(fn, reps: int, warmup: int) -> float:
    import torch

    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def tune(x, op="add", compensated=False, kind="plain", offsets=None, arrays=None, keep=None, reps=8, warmup=2,
         shapes=None, groups=GROUPS, verbose=False, outs=None) -> Entry:
    """Time every (shape, groups) for scanning device tensor ``x`` (or the
    batch ``arrays`` of device tensors, or ``x`` cut by ``offsets``, or
    compacting ``x`` by the ``keep`` flags) and return the best as an Entry
    (not yet applied).  A batch is timed with the caller's output tensors
    ``outs`` when given: where each output sits relative to its input's
    16-byte alignment decides the kernel's path, so fresh outputs may time
    another path than the caller's."""
    import torch

    binding.load()
    shapes = shapes or binding.lscan_tile_shapes()
    if kind == "batched":
        xs = arrays
        ys = list(outs) if outs is not None else [
            torch.empty(t.shape[0], dtype=binding.out_dtype(t, op), device=t.device) for t in xs]
        n = sum(int(t.shape[0]) for t in xs)
        dtype_t = xs[0]
        # the descriptor table is built once, so a large batch is timed by its
        # launch and not by rebuilding thousands of descriptors in Python
        table = binding.array_table([(t.data_ptr(), u.data_ptr(), t.shape[0]) for t, u in zip(xs, ys)])
        bflags = binding.F_COMPENSATED if compensated else 0
        bdt = binding.dtype_code(dtype_t)
    else:
        y = torch.empty(x.shape[0], dtype=binding.out_dtype(x, op), device=x.device)
        n = int(x.shape[0])
        dtype_t = x
    count = torch.empty(1, dtype=torch.int64, device=x.device) if kind == "compact" else None
    cands = []
    for t, r in shapes:
        for g in groups:
            p = binding.Params(t, r, g, 0)
            if kind == "plain":
                fn = lambda p=p: binding.inclusive(x, op, compensated, out=y, params=p)  # noqa: E731
            elif kind == "segmented":
                fn = lambda p=p: binding.segmented(x, offsets, op, compensated=compensated, out=y,  # noqa: E731
                                                   params=p)
            elif kind == "compact":
                fn = lambda p=p: binding.compact(x, keep, out=y, count=count, params=p)  # noqa: E731
            else:
                fn = lambda p=p: binding.lscan_batched(table, bdt, binding.OPS[op], bflags,  # noqa: E731
                                                       torch.cuda.current_stream().cuda_stream, p)
            fn()
            torch.cuda.synchronize()
            binding.lscan_check(torch.cuda.current_stream().cuda_stream)
            info = binding.lscan_last_launch()
            c = Candidate(t, r, info.groups_per_cu, info.grid)
            if any((d.block_threads, d.vectors_per_lane, d.grid) == (t, r, c.grid) for d in cands):
                continue
            c.ms = _time(fn, reps, warmup)
            binding.lscan_check(torch.cuda.current_stream().cuda_stream)
            cands.append(c)
            if verbose:
                print(f"  T={t} R={r} groups={c.groups_per_cu} grid={c.grid}: {c.ms * 1e3:.1f} us", flush=True)
    best = pick_best(cands)
    in_bytes = 2 if dtype_t.dtype == torch.bfloat16 else dtype_t.element_size()
    out_bytes = torch.empty(0, dtype=binding.out_dtype(dtype_t, op)).element_size()
    if kind == "compact":  # items and flags read, the kept items written
        fn()
        torch.cuda.synchronize()
        kept = int(count.item())
        gbs = (n * (in_bytes + (1 if keep is not None else 0)) + kept * out_bytes) / (best.ms * 1e-3) / 1e9
    else:
        gbs = n * (in_bytes + out_bytes) / (best.ms * 1e-3) / 1e9
    dtype_name = {v: k for k, v in DTYPE_CODES.items()}[binding.dtype_code(dtype_t)]
    return Entry(device=torch.cuda.get_device_name(), dtype=dtype_name, op=op, compensated=bool(compensated),
                 kind=kind, size_bucket=size_bucket(n), block_threads=best.block_threads,
                 vectors_per_lane=best.vectors_per_lane, groups_per_cu=best.groups_per_cu, ms=best.ms, gbs=gbs,
                 tried=len(cands))


def apply_cache(path: str, n_hint: int | None = None) -> int:
    """Apply every cached entry (or those of ``n_hint``'s size bucket) for
    the current device; returns how many were applied."""
    import torch

    cache = Cache(path)
    dev = torch.cuda.get_device_name()
    count = 0
    for e in cache.entries.values():
        if e.device != dev:
            continue
        if n_hint is not None and e.size_bucket != size_bucket(n_hint):
            continue
        apply(e)
        count += 1
    return count
