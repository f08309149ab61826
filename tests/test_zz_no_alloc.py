"""lscan_inclusive_noalloc (the entry point for callers that cannot
allocate) against lscan_inclusive through the C ABI: the same kernels on
the same shapes, so the outputs must be equal bit for bit, and both match
the oracle (exact for integer / max / min, float sums within the tolerance
of the plain or compensated form).  Two calls in a row on each case, the
second with a smaller input, since every call on a GPU reuses the same
static flag words."""
import numpy as np
import pytest
import torch

from gpu_util import compare, log, make_input, to_host

pytestmark = pytest.mark.gpu

CASES = [
    # dtype, op, compensated, first n (several tiles, ragged tail), second n (smaller)
    ("int32", "add", False, (1 << 22) + 3, (1 << 18) + 1),
    ("int32", "add", False, (1 << 27) + 1001, 3 * 16384 + 17),
    ("int64", "max", False, (1 << 24) + 9, 5000),
    ("float32", "add", False, (1 << 25) + 7, (1 << 20) + 3),
    ("float32", "add", True, (1 << 23) + 5, 3 * 4096 + 7),
    ("bfloat16", "add", False, (1 << 22) + 11, 777),
    ("int32", "argmax", False, (1 << 22) + 1, 4099),
]

DT = {"int32": 0, "int64": 1, "float32": 2, "bfloat16": 3}
OPS = {"add": 0, "max": 1, "min": 2, "argmax": 3, "argmin": 4}
TORCH = {"int32": torch.int32, "int64": torch.int64, "float32": torch.float32, "bfloat16": torch.bfloat16}


@pytest.mark.parametrize("dtype,op,comp,n1,n2", CASES)
def test_noalloc_equals_inclusive(gpu_lib, dtype, op, comp, n1, n2):
    import oracle

    lib = gpu_lib.load()
    out_t = torch.int64 if op == "argmax" else (torch.float32 if dtype == "bfloat16" else TORCH[dtype])
    flags = gpu_lib.F_COMPENSATED if comp else 0
    for call, n in enumerate((n1, n2)):
        log(f"[noalloc] {dtype} {op} comp={comp} call {call} n={n}")
        x = make_input(dtype, "max" if op == "argmax" else op, n, seed=4242 + 17 * call + n % 97)
        if dtype == "bfloat16":
            xd = torch.from_numpy(x.view(np.int16).copy()).view(torch.bfloat16).to("cuda")
        else:
            xd = torch.from_numpy(x).to("cuda")
        y = torch.full((n,), -3, dtype=out_t, device="cuda") if out_t != torch.float32 else \
            torch.full((n,), float("nan"), dtype=out_t, device="cuda")
        yr = torch.empty_like(y)
        s = torch.cuda.current_stream().cuda_stream
        st = lib.lscan_inclusive_noalloc(xd.data_ptr(), y.data_ptr(), n, DT[dtype], OPS[op], flags, s)
        assert st == 0, gpu_lib.status_string(st)
        gpu_lib.lscan_check(s)
        st = lib.lscan_inclusive(xd.data_ptr(), yr.data_ptr(), n, DT[dtype], OPS[op], flags, s)
        assert st == 0, gpu_lib.status_string(st)
        gpu_lib.lscan_check(s)
        got, ref = to_host(y), to_host(yr)
        if got.dtype.kind == "f":
            same = got.view(np.uint32) == ref.view(np.uint32)
        else:
            same = got == ref
        bad = np.flatnonzero(~same)
        assert bad.size == 0, f"call {call}: {bad.size} differences from lscan_inclusive, first at {bad[:8]}"
        if op == "argmax":
            assert np.array_equal(got, oracle.argscan(x, dtype, "argmax", False))
        else:
            compare(got, x, dtype, op, False, comp, what=f"noalloc {dtype}/{op} call {call} n={n}")
