"""Python binding of the C ABI in ``include/lscan.h`` (argument marshalling only).

Every scan runs in the HIP kernels of ``liblscan.so``; this module converts
torch tensors to device pointers, sizes and the current HIP stream, calls the
C entry point of the same name and turns negative status codes into
exceptions.  There is no CPU fallback: if the library is not built, or there
is no GPU, the calls raise.

torch is imported before the library is loaded so that both share one HIP
runtime (torch ships ``libamdhip64.so.7``, the soname the library links).
"""
from __future__ import annotations

import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "liblscan.so")

I32, I64, F32, BF16 = 0, 1, 2, 3
ADD, MAX, MIN = 0, 1, 2
F_COMPENSATED = 0x1
F_DETERMINISTIC = 0x2
F_EXCLUSIVE = 0x4
F_INDEX64 = 0x8

OK, PENDING = 0, 1
ERR_INVALID_ARG, ERR_UNSUPPORTED, ERR_NO_MEMORY, ERR_DEVICE = -1, -2, -3, -4
ERR_AGAIN, ERR_TIMEOUT, ERR_NOT_FOUND = -5, -6, -7

ARGMAX, ARGMIN = 3, 4
OPS = {"add": ADD, "max": MAX, "min": MIN, "argmax": ARGMAX, "argmin": ARGMIN}


class LscanError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__(f"{what}: {status_string(status)} (status {status})")


class Params(ctypes.Structure):
    _fields_ = [("block_threads", ctypes.c_int32), ("vectors_per_lane", ctypes.c_int32),
                ("groups_per_cu", ctypes.c_int32), ("handoff", ctypes.c_int32)]


class Array(ctypes.Structure):
    _fields_ = [("x", ctypes.c_void_p), ("y", ctypes.c_void_p), ("n", ctypes.c_int64)]


class LaunchInfo(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("num_blocks", ctypes.c_int64), ("tile_elems", ctypes.c_int64),
                ("grid", ctypes.c_int32), ("block_threads", ctypes.c_int32),
                ("slot_words", ctypes.c_int32), ("vector_path", ctypes.c_int32),
                ("groups_per_cu", ctypes.c_int32), ("occupancy", ctypes.c_int32)]


class ServerConfig(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int32), ("num_streams", ctypes.c_int32),
                ("hbm_budget_bytes", ctypes.c_uint64), ("max_queue", ctypes.c_int32),
                ("max_batch", ctypes.c_int32), ("groups_per_cu", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("solo_bytes", ctypes.c_uint64)]


class Request(ctypes.Structure):
    _fields_ = [("dt", ctypes.c_int32), ("op", ctypes.c_int32), ("flags", ctypes.c_uint32),
                ("reserved", ctypes.c_int32), ("n", ctypes.c_int64), ("x", ctypes.c_void_p),
                ("y", ctypes.c_void_p)]


class Result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("batch_size", ctypes.c_int32), ("batch_id", ctypes.c_uint64),
                ("t_submit_ns", ctypes.c_uint64), ("t_admit_ns", ctypes.c_uint64),
                ("t_launch_ns", ctypes.c_uint64), ("t_done_ns", ctypes.c_uint64)]


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64), ("failed", ctypes.c_uint64),
                ("batches", ctypes.c_uint64), ("bytes_in_flight", ctypes.c_uint64),
                ("peak_bytes_in_flight", ctypes.c_uint64), ("pending", ctypes.c_int64)]


_lib = None

# Every symbol declared in include/lscan.h, with its ctypes signature.
_vp, _i64, _i32, _u32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_uint32
SIGNATURES = {
    "lscan_inclusive": ([_vp, _vp, _i64, _i32, _i32, _u32, _vp], _i32),
    "lscan_exclusive": ([_vp, _vp, _i64, _i32, _i32, _u32, _vp], _i32),
    "lscan_inclusive_noalloc": ([_vp, _vp, _i64, _i32, _i32, _u32, _vp], _i32),
    "lscan_segmented": ([_vp, _vp, _i64, _vp, _i64, _i32, _i32, _u32, _vp], _i32),
    "lscan_num_tile_shapes": ([], _i32),
    "lscan_tile_shape": ([_i32, ctypes.POINTER(Params)], _i32),
    "lscan_get_params": ([_i32, _i32, _u32, _i32, ctypes.POINTER(Params)], _i32),
    "lscan_set_params": ([_i32, _i32, _u32, _i32, ctypes.POINTER(Params)], _i32),
    "lscan_scan_with_params": ([_vp, _vp, _i64, _i32, _i32, _u32, _i32, ctypes.POINTER(Params), _vp], _i32),
    "lscan_segmented_with_params": ([_vp, _vp, _i64, _vp, _i64, _i32, _i32, _u32,
                                     ctypes.POINTER(Params), _vp], _i32),
    "lscan_batched": ([ctypes.POINTER(Array), _i64, _i32, _i32, _u32, _vp], _i32),
    "lscan_batched_with_params": ([ctypes.POINTER(Array), _i64, _i32, _i32, _u32, ctypes.POINTER(Params), _vp],
                                  _i32),
    "lscan_compact": ([_vp, _vp, _vp, _vp, _i64, _i32, _vp], _i32),
    "lscan_radix_offsets": ([_vp, _i64, _i32, _i32, _i32, _i64, _vp, _vp], _i32),
    "lscan_compact_with_params": ([_vp, _vp, _vp, _vp, _i64, _i32, ctypes.POINTER(Params), _vp], _i32),
    "lscan_scan_custom": ([_vp, _vp, _vp, _i64, _u32, ctypes.POINTER(Params), _vp], _i32),
    "lscan_bfs": ([_vp, _vp, _i64, _i64, _i32, _vp, _vp, _vp, _vp], _i32),
    "lscan_bfs_with_params": ([_vp, _vp, _i64, _i64, _i32, _vp, _vp, _vp, ctypes.POINTER(Params), _vp], _i32),
    "lscan_graph_create_scan": ([_vp, _vp, _i64, _i32, _i32, _u32, ctypes.POINTER(Params), ctypes.POINTER(_vp)],
                                _i32),
    "lscan_graph_create_segmented": ([_vp, _vp, _i64, _vp, _i64, _i32, _i32, _u32, ctypes.POINTER(Params),
                                      ctypes.POINTER(_vp)], _i32),
    "lscan_graph_create_batched": ([ctypes.POINTER(Array), _i64, _i32, _i32, _u32, ctypes.POINTER(Params),
                                    ctypes.POINTER(_vp)], _i32),
    "lscan_graph_launch": ([_vp, _vp], _i32),
    "lscan_graph_check": ([_vp, _vp], _i32),
    "lscan_graph_destroy": ([_vp], _i32),
    "lscan_server_default_config": ([ctypes.POINTER(ServerConfig)], _i32),
    "lscan_server_create": ([ctypes.POINTER(ServerConfig), ctypes.POINTER(_vp)], _i32),
    "lscan_submit": ([_vp, ctypes.POINTER(Request), ctypes.POINTER(ctypes.c_uint64)], _i32),
    "lscan_poll": ([_vp, ctypes.c_uint64, ctypes.POINTER(Result)], _i32),
    "lscan_wait": ([_vp, ctypes.c_uint64, ctypes.POINTER(Result)], _i32),
    "lscan_server_get_stats": ([_vp, ctypes.POINTER(ServerStats)], _i32),
    "lscan_server_destroy": ([_vp], _i32),
    "lscan_set_watchdog_us": ([_i64], _i32),
    "lscan_get_watchdog_us": ([], _i64),
    "lscan_last_launch": ([ctypes.POINTER(LaunchInfo)], _i32),
    "lscan_check": ([_vp], _i32),
    "lscan_release_workspaces": ([], _i32),
    "lscan_status_string": ([_i32], ctypes.c_char_p),
    "lscan_last_device_error": ([], _i32),
    # include/lscan_testing.h
    "lscan_test_epoch_limit": ([], ctypes.c_uint64),
    "lscan_test_seed_epoch": ([_vp, ctypes.c_uint64, _u32, _u32], _i32),
    "lscan_test_graph_seed_epoch": ([_vp, ctypes.c_uint64, _u32, _u32], _i32),
    "lscan_test_epoch_state": ([_vp, ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(_u32)], _i32),
    "lscan_test_graph_epoch_state": ([_vp, ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(_u32)], _i32),
}


def load(path: str | None = None):
    """Load ``liblscan.so`` (raises if it has not been built)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    import torch  # noqa: F401  -- share torch's HIP runtime

    p = path or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(f"{p} is not built: run __graft_entry__.build() "
                           "(python -m paper_1604_04815_amd.build)")
    lib = ctypes.CDLL(p)
    for name, (args, res) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    if path is None:
        _lib = lib
    return lib


def status_string(status: int) -> str:
    try:
        return load().lscan_status_string(int(status)).decode()
    except Exception:  # noqa: BLE001 - used while formatting errors
        return "status"


def _check(status: int, what: str) -> int:
    if status < 0:
        if status == ERR_DEVICE:
            raise LscanError(status, f"{what} (hip error {load().lscan_last_device_error()})")
        raise LscanError(status, what)
    return status


# ---------------------------------------------------------------------------
# C entry points under their own names (raw pointers and sizes).
# ---------------------------------------------------------------------------

def lscan_inclusive(x: int, y: int, n: int, dt: int, op: int, flags: int = 0, stream: int = 0) -> int:
    return _check(load().lscan_inclusive(x, y, n, dt, op, flags, stream), "lscan_inclusive")


def lscan_exclusive(x: int, y: int, n: int, dt: int, op: int, flags: int = 0, stream: int = 0) -> int:
    return _check(load().lscan_exclusive(x, y, n, dt, op, flags, stream), "lscan_exclusive")


def lscan_inclusive_noalloc(x: int, y: int, n: int, dt: int, op: int, flags: int = 0, stream: int = 0) -> int:
    return _check(load().lscan_inclusive_noalloc(x, y, n, dt, op, flags, stream), "lscan_inclusive_noalloc")


def lscan_segmented(x: int, y: int, n_total: int, offsets: int, num_segments: int, dt: int, op: int,
                    flags: int = 0, stream: int = 0) -> int:
    return _check(load().lscan_segmented(x, y, n_total, offsets, num_segments, dt, op, flags, stream),
                  "lscan_segmented")


def lscan_scan_with_params(x, y, n, dt, op, flags, exclusive, params: Params | None, stream=0) -> int:
    p = ctypes.byref(params) if params is not None else None
    return _check(load().lscan_scan_with_params(x, y, n, dt, op, flags, int(exclusive), p, stream),
                  "lscan_scan_with_params")


def lscan_segmented_with_params(x, y, n_total, offsets, num_segments, dt, op, flags,
                                params: Params | None, stream=0) -> int:
    p = ctypes.byref(params) if params is not None else None
    return _check(load().lscan_segmented_with_params(x, y, n_total, offsets, num_segments, dt, op, flags,
                                                     p, stream), "lscan_segmented_with_params")


def _array_table(arrays):
    tab = (Array * max(1, len(arrays)))()
    for i, (x, y, n) in enumerate(arrays):
        tab[i].x, tab[i].y, tab[i].n = x, y, n
    return tab


class ArrayTable:
    """A batch's lscan_array table, built once: len() is the array count and
    the object passes to the C call as the table itself."""

    def __init__(self, arrays):
        self._tab = _array_table(arrays)
        self._count = len(arrays)
        self._as_parameter_ = ctypes.cast(self._tab, ctypes.POINTER(Array))

    def __len__(self):
        return self._count


def array_table(arrays) -> ArrayTable:
    """arrays: list of (x_ptr, y_ptr, n)."""
    return ArrayTable(arrays)


def lscan_batched(arrays, dt: int, op: int, flags: int = 0, stream: int = 0,
                  params: Params | None = None) -> int:
    """arrays: list of (x_ptr, y_ptr, n), or a table built once with
    array_table (what a caller that launches the same batch many times
    passes, so the per-call cost is the C call alone)."""
    tab = arrays if isinstance(arrays, ArrayTable) else _array_table(arrays)
    if params is None:
        st = load().lscan_batched(tab, len(arrays), dt, op, flags, stream)
    else:
        st = load().lscan_batched_with_params(tab, len(arrays), dt, op, flags, ctypes.byref(params), stream)
    return _check(st, "lscan_batched")


class Graph:
    """A captured segmented or batched launch (lscan_graph_*)."""

    def __init__(self, handle):
        self.handle = handle

    def launch(self, stream=None):
        _check(load().lscan_graph_launch(self.handle, _stream(stream)), "lscan_graph_launch")

    def check(self, stream=None):
        _check(load().lscan_graph_check(self.handle, _stream(stream)), "lscan_graph_check")

    def destroy(self):
        if self.handle:
            _check(load().lscan_graph_destroy(self.handle), "lscan_graph_destroy")
            self.handle = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:  # noqa: BLE001 - interpreter shutdown
            pass


def lscan_graph_create_scan(x, y, n, dt, op, flags=0, params: Params | None = None) -> Graph:
    """Capture one plain scan of the device pointers x -> y (n elements;
    F_EXCLUSIVE in flags for the exclusive scan) into a graph."""
    h = ctypes.c_void_p()
    p = ctypes.byref(params) if params is not None else None
    _check(load().lscan_graph_create_scan(x, y, n, dt, op, flags, p, ctypes.byref(h)), "lscan_graph_create_scan")
    return Graph(h.value)


def lscan_graph_create_segmented(x, y, n_total, offsets, num_segments, dt, op, flags=0,
                                 params: Params | None = None) -> Graph:
    h = ctypes.c_void_p()
    p = ctypes.byref(params) if params is not None else None
    _check(load().lscan_graph_create_segmented(x, y, n_total, offsets, num_segments, dt, op, flags, p,
                                               ctypes.byref(h)), "lscan_graph_create_segmented")
    return Graph(h.value)


def lscan_graph_create_batched(arrays, dt, op, flags=0, params: Params | None = None) -> Graph:
    h = ctypes.c_void_p()
    tab = _array_table(arrays)
    p = ctypes.byref(params) if params is not None else None
    _check(load().lscan_graph_create_batched(tab, len(arrays), dt, op, flags, p, ctypes.byref(h)),
           "lscan_graph_create_batched")
    return Graph(h.value)


def lscan_tile_shapes() -> list[tuple[int, int]]:
    lib = load()
    out = []
    for i in range(lib.lscan_num_tile_shapes()):
        p = Params()
        _check(lib.lscan_tile_shape(i, ctypes.byref(p)), "lscan_tile_shape")
        out.append((p.block_threads, p.vectors_per_lane))
    return out


KIND_PLAIN, KIND_SEGMENTED, KIND_BATCHED, KIND_COMPACT = 0, 1, 2, 3
HANDOFF_WINDOW, HANDOFF_CHAIN = 0, 1


def lscan_get_params(dt, op, flags=0, kind=KIND_PLAIN) -> Params:
    p = Params()
    _check(load().lscan_get_params(dt, op, flags, int(kind), ctypes.byref(p)), "lscan_get_params")
    return p


def lscan_set_params(dt, op, flags, kind, params: Params) -> None:
    _check(load().lscan_set_params(dt, op, flags, int(kind), ctypes.byref(params)), "lscan_set_params")


def lscan_last_launch() -> LaunchInfo:
    info = LaunchInfo()
    _check(load().lscan_last_launch(ctypes.byref(info)), "lscan_last_launch")
    return info


def lscan_check(stream: int = 0) -> None:
    _check(load().lscan_check(stream), "lscan_check")


def lscan_release_workspaces() -> None:
    _check(load().lscan_release_workspaces(), "lscan_release_workspaces")


def lscan_test_epoch_limit() -> int:
    return int(load().lscan_test_epoch_limit())


def lscan_test_seed_epoch(launches: int, tag: int, abort_tag: int = 0, stream=None,
                          graph: Graph | None = None) -> None:
    """Seed the flag workspace of a stream (or of a graph) near the epoch
    reset (include/lscan_testing.h)."""
    if graph is not None:
        _check(load().lscan_test_graph_seed_epoch(graph.handle, launches, tag, abort_tag),
               "lscan_test_graph_seed_epoch")
    else:
        _check(load().lscan_test_seed_epoch(_stream(stream), launches, tag, abort_tag), "lscan_test_seed_epoch")


def lscan_test_epoch_state(stream=None, graph: Graph | None = None):
    """(launch count, [ctrl0, ctrl1, ctrl2, ctrl3]) of a stream's or a
    graph's flag workspace."""
    n = ctypes.c_uint64()
    ctrl = (ctypes.c_uint32 * 4)()
    if graph is not None:
        _check(load().lscan_test_graph_epoch_state(graph.handle, ctypes.byref(n), ctrl),
               "lscan_test_graph_epoch_state")
    else:
        _check(load().lscan_test_epoch_state(_stream(stream), ctypes.byref(n), ctrl), "lscan_test_epoch_state")
    return int(n.value), [int(c) for c in ctrl]


# ---------------------------------------------------------------------------
# torch tensor marshalling
# ---------------------------------------------------------------------------

def dtype_code(t) -> int:
    import torch

    table = {torch.int32: I32, torch.int64: I64, torch.float32: F32, torch.bfloat16: BF16}
    if t.dtype not in table:
        raise TypeError(f"unsupported dtype {t.dtype}")
    return table[t.dtype]


def out_dtype(t, op="add"):
    import torch

    if op in ("argmax", "argmin"):
        return torch.int64  # indices
    return torch.float32 if t.dtype == torch.bfloat16 else t.dtype


def _stream(stream) -> int:
    import torch

    if stream is None:
        raw = getattr(torch._C, "_cuda_getCurrentRawStream", None)
        if raw is not None:  # the raw handle without building a Stream object (a few microseconds less)
            return raw(torch.cuda.current_device())
        return torch.cuda.current_stream().cuda_stream
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)


def _flat(t, name):
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dim() != 1 or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous 1-D tensor")
    return t


def _out_for(x, out, op="add"):
    import torch

    if out is None:
        return torch.empty(x.shape[0], dtype=out_dtype(x, op), device=x.device)
    _flat(out, "out")
    if out.dtype != out_dtype(x, op) or out.shape[0] != x.shape[0]:
        raise ValueError("out has the wrong dtype or length")
    return out


def inclusive(x, op="add", compensated=False, out=None, stream=None, params: Params | None = None,
              index64=False):
    """y_j = x_0 (+) ... (+) x_j on the device; returns y (for argmax /
    argmin the int64 index of the best element of each prefix)."""
    _flat(x, "x")
    y = _out_for(x, out, op)
    flags = (F_COMPENSATED if compensated else 0) | (F_INDEX64 if index64 else 0)
    if params is None:
        lscan_inclusive(x.data_ptr(), y.data_ptr(), x.shape[0], dtype_code(x), OPS[op], flags, _stream(stream))
    else:
        lscan_scan_with_params(x.data_ptr(), y.data_ptr(), x.shape[0], dtype_code(x), OPS[op], flags, 0,
                               params, _stream(stream))
    return y


def exclusive(x, op="add", compensated=False, out=None, stream=None, params: Params | None = None,
              index64=False):
    """y_0 = e, y_j = x_0 (+) ... (+) x_{j-1} on the device; returns y."""
    _flat(x, "x")
    y = _out_for(x, out, op)
    flags = (F_COMPENSATED if compensated else 0) | (F_INDEX64 if index64 else 0)
    if params is None:
        lscan_exclusive(x.data_ptr(), y.data_ptr(), x.shape[0], dtype_code(x), OPS[op], flags, _stream(stream))
    else:
        lscan_scan_with_params(x.data_ptr(), y.data_ptr(), x.shape[0], dtype_code(x), OPS[op], flags, 1,
                               params, _stream(stream))
    return y


def segmented(x, offsets, op="add", exclusive=False, compensated=False, out=None, stream=None,
              params: Params | None = None):
    """Scan of every segment x[off[s]:off[s+1]] in one launch; returns y."""
    import torch

    _flat(x, "x")
    _flat(offsets, "offsets")
    if offsets.dtype != torch.int64:
        raise TypeError("offsets must be int64")
    y = _out_for(x, out)
    flags = (F_COMPENSATED if compensated else 0) | (F_EXCLUSIVE if exclusive else 0)
    nseg = offsets.shape[0] - 1
    if params is None:
        lscan_segmented(x.data_ptr(), y.data_ptr(), x.shape[0], offsets.data_ptr(), nseg, dtype_code(x),
                        OPS[op], flags, _stream(stream))
    else:
        lscan_segmented_with_params(x.data_ptr(), y.data_ptr(), x.shape[0], offsets.data_ptr(), nseg,
                                    dtype_code(x), OPS[op], flags, params, _stream(stream))
    return y


def batched(xs, op="add", exclusive=False, compensated=False, outs=None, stream=None,
            params: Params | None = None):
    """Scan each tensor of ``xs`` (1-D device tensors of one dtype) in one
    launch; returns the list of outputs."""
    if not xs:
        return []
    dt = dtype_code(xs[0])
    ys = []
    table = []
    for k, x in enumerate(xs):
        _flat(x, "x")
        if dtype_code(x) != dt:
            raise TypeError("all arrays of a batch share one dtype")
        y = _out_for(x, outs[k] if outs is not None else None)
        ys.append(y)
        table.append((x.data_ptr(), y.data_ptr(), x.shape[0]))
    flags = (F_COMPENSATED if compensated else 0) | (F_EXCLUSIVE if exclusive else 0)
    lscan_batched(table, dt, OPS[op], flags, _stream(stream), params)
    return ys


def compact(x, keep=None, out=None, count=None, stream=None, params: Params | None = None):
    """Stream compaction on the device: the items of ``x`` whose ``keep``
    byte (a uint8 or bool device tensor) is non-zero, or with ``keep`` None
    whose bits are not all zero, in order.  Returns ``(out, count)``: ``out``
    has room for every item and holds the kept ones in ``out[:count]``;
    ``count`` is a one-element int64 device tensor (read it after the stream
    has synchronized)."""
    import torch

    _flat(x, "x")
    n = x.shape[0]
    if keep is not None:
        _flat(keep, "keep")
        if keep.dtype not in (torch.uint8, torch.bool) or keep.shape[0] != n:
            raise ValueError("keep must be uint8 or bool with one flag per item")
    if out is None:
        out = torch.empty_like(x)
    else:
        _flat(out, "out")
        if out.dtype != x.dtype or out.shape[0] < n:
            raise ValueError("out must have x's dtype and room for every item")
    if count is None:
        count = torch.empty(1, dtype=torch.int64, device=x.device)
    keep_ptr = keep.data_ptr() if keep is not None else None
    p = ctypes.byref(params) if params is not None else None
    _check(load().lscan_compact_with_params(x.data_ptr(), keep_ptr, out.data_ptr(), count.data_ptr(), n,
                                            dtype_code(x), p, _stream(stream)), "lscan_compact")
    return out, count


def radix_offsets(keys, shift, bits, block_items, out=None, stream=None):
    """Digit offsets of one radix-sort pass over the device tensor ``keys``
    (int32 / float32 / int64, read as unsigned bit patterns): an int64 device
    tensor of shape (2**bits, M), M = ceil(n / block_items)."""
    import torch

    _flat(keys, "keys")
    n = keys.shape[0]
    m = (n + block_items - 1) // block_items if n else 0
    if out is None:
        out = torch.empty((1 << bits) * m, dtype=torch.int64, device=keys.device)
    else:
        _flat(out, "out")
        if out.dtype != torch.int64 or out.shape[0] != (1 << bits) * m:
            raise ValueError("out must be int64 with 2**bits * M entries")
    _check(load().lscan_radix_offsets(keys.data_ptr(), n, dtype_code(keys), shift, bits, block_items,
                                      out.data_ptr(), _stream(stream)), "lscan_radix_offsets")
    return out.view(1 << bits, m)


def scan_custom(kernel, x, n, out=None, exclusive=False, stream=None, params: Params | None = None):
    """Scan n elements of a user operator's In type held in the device
    tensor ``x`` with the kernel handle ``kernel`` (made in the user's own
    library with include/lscan_custom.hpp); ``out`` (default: a tensor like
    ``x``) receives n elements of its Out type.  Returns ``out``."""
    import torch

    _flat(x, "x")
    if out is None:
        out = torch.empty_like(x)
    else:
        _flat(out, "out")
    flags = F_EXCLUSIVE if exclusive else 0
    p = ctypes.byref(params) if params is not None else None
    _check(load().lscan_scan_custom(ctypes.c_void_p(kernel), x.data_ptr(), out.data_ptr(), int(n), flags, p,
                                    _stream(stream)), "lscan_scan_custom")
    return out


# The example library of a user operator (composition of affine maps mod
# 2^32), built beside the package by the build step.
AFFINE_EXAMPLE_LIB = os.path.join(os.path.dirname(os.path.abspath(__file__)), "custom", "libaffine_scan.so")


def affine_example_kernels(path: str | None = None) -> dict:
    """Handles of the example affine-map scan kernels: 'default' (256 x 8),
    'small' (64 x 1) and 'wide' (1024 x 2)."""
    p = path or AFFINE_EXAMPLE_LIB
    if not os.path.exists(p):
        raise RuntimeError(f"{p} is not built: run __graft_entry__.build()")
    lib = ctypes.CDLL(p)
    out = {}
    for name, sym in (("default", "lscan_affine_kernel"), ("small", "lscan_affine_kernel_small"),
                      ("wide", "lscan_affine_kernel_wide")):
        f = getattr(lib, sym)
        f.argtypes = []
        f.restype = ctypes.c_void_p
        out[name] = f()
    out["_lib"] = lib  # keeps the code object loaded
    return out

def bfs(row_offsets, cols, source, levels=None, parents=True, stats=None, stream=None,
        params: Params | None = None):
    """Breadth-first search on the device over a directed graph in compressed
    rows (``row_offsets``: int64, V + 1 entries; ``cols``: int32, E
    entries; both device tensors).  Returns ``(levels, parents, stats)``:
    int32 levels (-1 unreached); int32 parents of a breadth-first tree, or
    None when ``parents`` is False; an int64 device tensor of 4 (levels,
    vertices reached, edges scanned, malformed entries)."""
    import torch

    _flat(row_offsets, "row_offsets")
    _flat(cols, "cols")
    if row_offsets.dtype != torch.int64 or cols.dtype != torch.int32:
        raise TypeError("row_offsets must be int64 and cols int32")
    nv = row_offsets.shape[0] - 1
    if nv < 0:
        raise ValueError("row_offsets needs V + 1 >= 1 entries")
    dev = row_offsets.device

    def out_vec(t, name):
        if t is None:
            return torch.empty(nv, dtype=torch.int32, device=dev)
        _flat(t, name)
        if t.dtype != torch.int32 or t.shape[0] != nv:
            raise ValueError(f"{name} must be int32 with one entry per vertex")
        return t

    levels = out_vec(levels, "levels")
    par = None
    if parents is not False and parents is not None:
        par = out_vec(None if parents is True else parents, "parents")
    if stats is None:
        stats = torch.empty(4, dtype=torch.int64, device=dev)
    else:
        _flat(stats, "stats")
        if stats.dtype != torch.int64 or stats.shape[0] != 4:
            raise ValueError("stats must be int64 with 4 entries")
    ne = cols.shape[0]
    p = ctypes.byref(params) if params is not None else None
    _check(load().lscan_bfs_with_params(row_offsets.data_ptr(), cols.data_ptr() if ne else None, nv, ne,
                                        int(source), levels.data_ptr(), par.data_ptr() if par is not None else None,
                                        stats.data_ptr(), p, _stream(stream)), "lscan_bfs")
    return levels, par, stats

class Server:
    """Request server (lscan_server_*): submit device arrays, poll tickets."""

    def __init__(self, device=0, num_streams=2, hbm_budget_bytes=32 << 30, max_queue=1 << 16, max_batch=4096,
                 groups_per_cu=0, solo_bytes=0):
        lib = load()
        cfg = ServerConfig()
        _check(lib.lscan_server_default_config(ctypes.byref(cfg)), "lscan_server_default_config")
        cfg.device, cfg.num_streams, cfg.hbm_budget_bytes = device, num_streams, hbm_budget_bytes
        cfg.max_queue, cfg.max_batch, cfg.groups_per_cu = max_queue, max_batch, groups_per_cu
        cfg.solo_bytes = solo_bytes
        h = ctypes.c_void_p()
        _check(lib.lscan_server_create(ctypes.byref(cfg), ctypes.byref(h)), "lscan_server_create")
        self.handle = h.value
        self._req = Request()
        self._ticket = ctypes.c_uint64()
        self._res = Result()

    def submit_raw(self, x_ptr, y_ptr, n, dt, op, flags=0) -> int:
        """Returns a ticket (> 0) or a negative status (no exception)."""
        r = self._req
        r.dt, r.op, r.flags, r.n, r.x, r.y = dt, op, flags, n, x_ptr, y_ptr
        st = load().lscan_submit(self.handle, ctypes.byref(r), ctypes.byref(self._ticket))
        return int(self._ticket.value) if st == OK else st

    def submit(self, x, y, op="add", exclusive=False, compensated=False) -> int:
        _flat(x, "x")
        _flat(y, "y")
        flags = (F_COMPENSATED if compensated else 0) | (F_EXCLUSIVE if exclusive else 0)
        t = self.submit_raw(x.data_ptr(), y.data_ptr(), x.shape[0], dtype_code(x), OPS[op], flags)
        if t < 0:
            raise LscanError(t, "lscan_submit")
        return t

    def poll(self, ticket: int):
        """(status, Result copy); status is PENDING, OK or an error code."""
        st = load().lscan_poll(self.handle, ticket, ctypes.byref(self._res))
        res = Result()
        ctypes.pointer(res)[0] = self._res
        return st, res

    def wait(self, ticket: int):
        res = Result()
        st = load().lscan_wait(self.handle, ticket, ctypes.byref(res))
        return st, res

    def stats(self) -> ServerStats:
        s = ServerStats()
        _check(load().lscan_server_get_stats(self.handle, ctypes.byref(s)), "lscan_server_get_stats")
        return s

    def close(self):
        if self.handle:
            _check(load().lscan_server_destroy(self.handle), "lscan_server_destroy")
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
