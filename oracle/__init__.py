"""Sequential CPU oracle for the device-wide scan -- TEST INFRASTRUCTURE.

Only the test suite, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg
of ``bench.py`` may import this package.  The product path (the HIP library
and its Python binding) never imports, links or runs it, and this package
imports nothing from the product.

The arithmetic lives in ``lscan_oracle.c`` (plain C, one left fold per scan,
written from the problem statement in Section 1 of the paper).  This module
only builds that file with gcc, loads it with ctypes and marshals numpy
arrays.  Results:

* int32 / int64, any operator: exact, wrap-around add (two's complement).
* float32 / bf16 with max / min: exact, IEEE 754 totalOrder (-0 < +0).
* float32 / bf16 with add: the exact prefix sums rounded to FP64 (Neumaier
  compensated fold) together with ``A_j = sum_{i<=j} |x_i|``; a GPU result
  is accepted when ``|y_j - y64_j| <= tau * A_j``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lscan_oracle.c")
_LIB = os.path.join(_HERE, "liblscan_oracle.so")

I32, I64, F32, BF16 = 0, 1, 2, 3
ADD, MAX, MIN = 0, 1, 2

_DTYPES = {"int32": I32, "int64": I64, "float32": F32, "bfloat16": BF16}
_OPS = {"add": ADD, "max": MAX, "min": MIN}
_IN_NP = {I32: np.int32, I64: np.int64, F32: np.float32, BF16: np.uint16}

def compile_library(src: str, out: str) -> str:
    """Compile a C oracle source file into a shared library (gcc)."""
    tmp = out + ".tmp"
    subprocess.run(
        ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
         "-fPIC", "-shared", "-o", tmp, src, "-lm"],
        check=True,
    )
    os.replace(tmp, out)
    return out


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc into ``liblscan_oracle.so``."""
    if force or not os.path.exists(_LIB) or (
        os.path.getmtime(_LIB) < os.path.getmtime(_SRC)
    ):
        compile_library(_SRC, _LIB)
    return _LIB


def _codes(dtype, op):
    dt = _DTYPES[dtype] if isinstance(dtype, str) else int(dtype)
    o = _OPS[op] if isinstance(op, str) else int(op)
    return dt, o


def _out_np(dt, o):
    if dt == I32:
        return np.int32
    if dt == I64:
        return np.int64
    return np.float64 if o == ADD else np.float32


def _as_input(x, dt):
    x = np.ascontiguousarray(x)
    want = _IN_NP[dt]
    if x.dtype != want:
        if dt == BF16 and x.dtype == np.int16:
            x = x.view(np.uint16)
        else:
            raise TypeError(f"oracle expects {np.dtype(want)} input, got {x.dtype}")
    return x


class Oracle:
    """ctypes view of one compiled oracle library."""

    def __init__(self, path: str):
        lib = ctypes.CDLL(path)
        vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
        lib.oracle_scan.argtypes = [vp, vp, vp, i64, i32, i32, i32]
        lib.oracle_scan.restype = i32
        lib.oracle_segscan.argtypes = [vp, vp, vp, vp, i64, i32, i32, i32]
        lib.oracle_segscan.restype = i32
        lib.oracle_compact.argtypes = [vp, vp, i64, i32, vp]
        lib.oracle_compact.restype = i64
        lib.oracle_radix_offsets.argtypes = [vp, i64, i32, i32, i32, i64, vp]
        lib.oracle_radix_offsets.restype = i64
        lib.oracle_argscan.argtypes = [vp, vp, i64, i32, i32, i32]
        lib.oracle_argscan.restype = i32
        lib.oracle_affine_scan.argtypes = [vp, vp, i64, i32]
        lib.oracle_affine_scan.restype = i32
        lib.oracle_bfs_levels.argtypes = [vp, vp, i64, i64, vp, vp]
        lib.oracle_bfs_levels.restype = i64
        self.lib = lib
        self.path = path

    def scan(self, x, dtype="int32", op="add", exclusive=False, with_absum=False, out=None):
        """Sequential scan of ``x`` (1-D numpy array; bf16 given as uint16 bits).

        Returns ``y`` or, for float add with ``with_absum``, ``(y64, absum)``.
        ``out`` may be ``x`` itself (in-place) when the output type equals
        the input type.
        """
        dt, o = _codes(dtype, op)
        x = _as_input(x, dt)
        n = x.shape[0]
        y = out if out is not None else np.empty(n, dtype=_out_np(dt, o))
        want_abs = with_absum and o == ADD and dt in (F32, BF16)
        absum = np.empty(n, dtype=np.float64) if want_abs else None
        rc = self.lib.oracle_scan(
            x.ctypes.data, y.ctypes.data,
            absum.ctypes.data if absum is not None else None,
            n, dt, o, int(bool(exclusive)))
        if rc != 0:
            raise ValueError(f"oracle_scan rejected its arguments (rc={rc})")
        return (y, absum) if absum is not None else y

    def segscan(self, x, offsets, dtype="int32", op="add", exclusive=False, with_absum=False):
        """The plain scan applied to each segment ``x[off[s]:off[s+1]]``."""
        dt, o = _codes(dtype, op)
        x = _as_input(x, dt)
        off = np.ascontiguousarray(offsets, dtype=np.int64)
        n = x.shape[0]
        y = np.zeros(n, dtype=_out_np(dt, o))
        want_abs = with_absum and o == ADD and dt in (F32, BF16)
        absum = np.zeros(n, dtype=np.float64) if want_abs else None
        rc = self.lib.oracle_segscan(
            x.ctypes.data, y.ctypes.data,
            absum.ctypes.data if absum is not None else None,
            off.ctypes.data, off.shape[0] - 1, dt, o, int(bool(exclusive)))
        if rc != 0:
            raise ValueError(f"oracle_segscan rejected its arguments (rc={rc})")
        return (y, absum) if absum is not None else y


    def compact(self, x, keep=None):
        """Stream compaction: the elements of ``x`` (1-D numpy array of 2-, 4-
        or 8-byte items) whose ``keep`` flag (uint8) is non-zero, or with
        ``keep`` None whose bytes are not all zero, in order."""
        x = np.ascontiguousarray(x)
        n = x.shape[0]
        if keep is not None:
            keep = np.ascontiguousarray(keep, dtype=np.uint8)
            if keep.shape[0] != n:
                raise ValueError("keep must have one flag per element")
        out = np.zeros(n, dtype=x.dtype)
        count = self.lib.oracle_compact(x.ctypes.data, keep.ctypes.data if keep is not None else None,
                                        n, x.dtype.itemsize, out.ctypes.data)
        if count < 0:
            raise ValueError(f"oracle_compact rejected its arguments (rc={count})")
        return out[:count]


    def radix_offsets(self, keys, shift, bits, block_items):
        """Digit offsets of one radix-sort pass over ``keys`` (uint32 or
        uint64 numpy array): an int64 array of shape (2**bits, M), entry
        [d, b] = keys with a smaller digit + keys of digit d in earlier blocks."""
        keys = np.ascontiguousarray(keys)
        if keys.dtype.itemsize not in (4, 8):
            raise TypeError("keys must have 4- or 8-byte items")
        n = keys.shape[0]
        m = (n + block_items - 1) // block_items
        out = np.zeros((1 << bits) * max(m, 0), dtype=np.int64)
        rc = self.lib.oracle_radix_offsets(keys.ctypes.data, n, keys.dtype.itemsize, shift, bits, block_items,
                                           out.ctypes.data)
        if rc < 0:
            raise ValueError(f"oracle_radix_offsets rejected its arguments (rc={rc})")
        return out.reshape(1 << bits, m)


    def argscan(self, x, dtype="int32", op="argmax", exclusive=False):
        """Running argmax / argmin: int64 indices of the best element of each
        prefix (earliest among ties; -1 for the empty prefix)."""
        dt, _ = _codes(dtype, "max")
        x = _as_input(x, dt)
        y = np.empty(x.shape[0], dtype=np.int64)
        rc = self.lib.oracle_argscan(x.ctypes.data, y.ctypes.data, x.shape[0], dt, int(op == "argmax"),
                                     int(bool(exclusive)))
        if rc != 0:
            raise ValueError(f"oracle_argscan rejected its arguments (rc={rc})")
        return y


    def affine_scan(self, ab, exclusive=False):
        """Scan of affine maps x -> a*x + b mod 2^32 under composition (the
        earlier map first); ``ab`` is a uint32 array of shape (n, 2) holding
        (a, b) per map; returns the composed prefixes in the same shape."""
        ab = np.ascontiguousarray(ab, dtype=np.uint32).reshape(-1, 2)
        out = np.empty_like(ab)
        rc = self.lib.oracle_affine_scan(ab.ctypes.data, out.ctypes.data, ab.shape[0], int(bool(exclusive)))
        if rc != 0:
            raise ValueError(f"oracle_affine_scan rejected its arguments (rc={rc})")
        return out


    def bfs_levels(self, row_ptr, col, src):
        """BFS levels from ``src`` over a CSR graph (int64 row_ptr, int32
        col): int32 array, -1 for unreachable vertices."""
        row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int64)
        col = np.ascontiguousarray(col, dtype=np.int32)
        nv = row_ptr.shape[0] - 1
        level = np.empty(nv, dtype=np.int32)
        queue = np.empty(max(nv, 1), dtype=np.int32)
        rc = self.lib.oracle_bfs_levels(row_ptr.ctypes.data, col.ctypes.data, nv, int(src), level.ctypes.data,
                                        queue.ctypes.data)
        if rc < 0:
            raise ValueError(f"oracle_bfs_levels rejected its arguments (rc={rc})")
        return level


_default = None


def default() -> Oracle:
    """The oracle built from ``lscan_oracle.c`` (compiled on first use)."""
    global _default
    if _default is None:
        if not os.path.exists(_LIB) or (
            os.path.getmtime(_LIB) < os.path.getmtime(_SRC)
        ):
            build(force=True)
        _default = Oracle(_LIB)
    return _default


def scan(x, dtype="int32", op="add", exclusive=False, with_absum=False, out=None):
    return default().scan(x, dtype, op, exclusive, with_absum, out)


def segscan(x, offsets, dtype="int32", op="add", exclusive=False, with_absum=False):
    return default().segscan(x, offsets, dtype, op, exclusive, with_absum)


def compact(x, keep=None):
    return default().compact(x, keep)


def radix_offsets(keys, shift, bits, block_items):
    return default().radix_offsets(keys, shift, bits, block_items)


def argscan(x, dtype="int32", op="argmax", exclusive=False):
    return default().argscan(x, dtype, op, exclusive)


def affine_scan(ab, exclusive=False):
    return default().affine_scan(ab, exclusive)


def bfs_levels(row_ptr, col, src):
    return default().bfs_levels(row_ptr, col, src)


def float_error_ratio(y, y64, absum):
    """max_j |y_j - y64_j| / A_j (A_j = 0 demands an exact match).

    Returns ``(ratio, argmax)``; ``ratio`` is ``inf`` when some ``A_j = 0``
    entry is not matched exactly.
    """
    y = np.asarray(y, dtype=np.float64)
    err = np.abs(y - y64)
    zero = absum == 0
    if np.any(err[zero] != 0):
        j = int(np.flatnonzero(zero & (err != 0))[0])
        return float("inf"), j
    ratio = np.zeros_like(err)
    nz = ~zero
    ratio[nz] = err[nz] / absum[nz]
    if ratio.size == 0:
        return 0.0, -1
    j = int(np.argmax(ratio))
    return float(ratio[j]), j
