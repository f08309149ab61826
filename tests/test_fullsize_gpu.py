"""Parity at the full workload sizes, in the launch configuration the
benchmark times (the library defaults): every output element is compared
with the oracle, which finishes these sizes in about a second each."""
import numpy as np
import pytest
import torch

from gpu_util import compare, log, to_device, to_host

pytestmark = pytest.mark.gpu


def _run(gpu_lib, x, dtype, op, comp=False):
    xd = to_device(x, dtype)
    y = gpu_lib.inclusive(xd, op, comp)
    gpu_lib.lscan_check(torch.cuda.current_stream().cuda_stream)
    out = to_host(y)
    del xd, y
    return out


def test_int32_add_2p28(gpu_lib):
    from paper_1604_04815_amd import workloads as w
    x = w.uniform_int(1 << 28, -1024, 1024, w.seed_for(1))
    log("[full] int32 add N=2^28")
    compare(_run(gpu_lib, x, "int32", "add"), x, "int32", "add", False, what="1a")


def test_int64_add_2p27(gpu_lib):
    from paper_1604_04815_amd import workloads as w
    x = w.int64_half_open(1 << 27, -(2 ** 31), 2 ** 31, w.seed_for(1, 1))
    log("[full] int64 add N=2^27")
    compare(_run(gpu_lib, x, "int64", "add"), x, "int64", "add", False, what="1b")


def test_int32_max_2p28(gpu_lib):
    from paper_1604_04815_amd import workloads as w
    x = w.full_range_int32(1 << 28, w.seed_for(1, 2))
    log("[full] int32 max N=2^28")
    compare(_run(gpu_lib, x, "int32", "max"), x, "int32", "max", False, what="1c")


@pytest.mark.parametrize("comp", [False, True])
def test_f32_lognormal_2p27(gpu_lib, comp):
    from paper_1604_04815_amd import workloads as w
    x = w.signed_lognormal_f32(1 << 27, w.seed_for(2))
    log(f"[full] float32 add N=2^27 comp={comp}")
    r = compare(_run(gpu_lib, x, "float32", "add", comp), x, "float32", "add", False, comp, what="2")
    log(f"[full] float32 comp={comp} max error ratio {r:.3e}")


@pytest.mark.parametrize("comp", [False, True])
def test_bf16_unit_2p27(gpu_lib, comp):
    from paper_1604_04815_amd import workloads as w
    x = w.bf16_unit(1 << 27, w.seed_for(2, 1))
    log(f"[full] bf16 add N=2^27 comp={comp}")
    r = compare(_run(gpu_lib, x, "bfloat16", "add", comp), x, "bfloat16", "add", False, comp, what="2-bf16")
    log(f"[full] bf16 comp={comp} max error ratio {r:.3e}")


def test_segmented_4096_log_uniform(gpu_lib):
    from paper_1604_04815_amd import workloads as w
    off = w.segment_offsets(4096, 1 << 20, w.seed_for(3))
    n = int(off[-1])
    log(f"[full] segmented 4096 arrays n={n}")
    for dtype, op in (("int32", "add"), ("float32", "add")):
        x = w.uniform_int(n, -1000, 1000, w.seed_for(3, 1)) if dtype == "int32" else w.uniform01_f32(n, w.seed_for(3, 2))
        xd = to_device(x, dtype)
        od = torch.from_numpy(off).to("cuda")
        y = gpu_lib.segmented(xd, od, op)
        gpu_lib.lscan_check(torch.cuda.current_stream().cuda_stream)
        compare(to_host(y), x, dtype, op, False, offsets=off, what=f"3 {dtype}")
        del xd, y
