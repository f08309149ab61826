"""The autotuner on the device: it times candidates, installs the winner as
the default, and scans with the winner stay exact."""
import torch
import pytest

from gpu_util import compare, make_input, to_device, to_host

pytestmark = pytest.mark.gpu


def test_tune_apply_and_scan(gpu_lib, tmp_path):
    from paper_1604_04815_amd import autotune
    x_host = make_input("int32", "add", 6_000_001, seed=12)
    x = to_device(x_host, "int32")
    before = gpu_lib.lscan_get_params(gpu_lib.I32, gpu_lib.ADD)
    e = autotune.tune(x, "add", shapes=[(256, 8), (512, 4), (1024, 2)], groups=(1, 2, 4), reps=3, warmup=1)
    assert e.tried >= 3 and e.gbs > 0
    cache = autotune.Cache(str(tmp_path / "t.json"))
    cache.put(e)
    cache.save()
    assert autotune.apply_cache(str(tmp_path / "t.json")) == 1
    now = gpu_lib.lscan_get_params(gpu_lib.I32, gpu_lib.ADD)
    assert (now.block_threads, now.vectors_per_lane) == (e.block_threads, e.vectors_per_lane)
    y = gpu_lib.inclusive(x, "add")
    compare(to_host(y), x_host, "int32", "add", False, what="tuned default")
    gpu_lib.lscan_set_params(gpu_lib.I32, gpu_lib.ADD, 0, gpu_lib.KIND_PLAIN, before)


def test_tune_batched_and_segmented(gpu_lib):
    from paper_1604_04815_amd import autotune, workloads as w
    xs = [to_device(make_input("float32", "add", n, seed=n), "float32") for n in (1000, 200_000, 3_000_000)]
    e = autotune.tune(None, "add", compensated=True, kind="batched", arrays=xs, shapes=[(256, 8), (1024, 4)],
                      groups=(1, 2), reps=2, warmup=1)
    assert e.kind == "batched" and e.compensated
    off = w.segment_offsets(64, 1 << 14, seed=2)
    xh = make_input("int32", "add", int(off[-1]), seed=3)
    od = torch.from_numpy(off).to("cuda")
    e = autotune.tune(to_device(xh, "int32"), "add", kind="segmented", offsets=od, shapes=[(256, 8), (512, 4)],
                      groups=(1, 2), reps=2, warmup=1)
    assert e.kind == "segmented"


def test_tune_compact(gpu_lib):
    import numpy as np
    from paper_1604_04815_amd import autotune
    n = 2_000_003
    x = to_device(make_input("int32", "add", n, seed=14), "int32")
    keep = torch.from_numpy((np.random.default_rng(15).random(n) < 0.4).astype(np.uint8)).to("cuda")
    before = gpu_lib.lscan_get_params(gpu_lib.I32, gpu_lib.ADD, 0, gpu_lib.KIND_COMPACT)
    e = autotune.tune(x, "add", kind="compact", keep=keep, shapes=[(256, 8), (1024, 4)], groups=(1, 2), reps=2,
                      warmup=1)
    assert e.kind == "compact" and e.gbs > 0
    autotune.apply(e)
    out, count = gpu_lib.compact(x, keep)
    torch.cuda.synchronize()
    want = torch.masked_select(x, keep.bool())
    assert int(count.item()) == want.shape[0] and torch.equal(out[:want.shape[0]], want)
    gpu_lib.lscan_set_params(gpu_lib.I32, gpu_lib.ADD, 0, gpu_lib.KIND_COMPACT, before)


def test_tune_argmax(gpu_lib):
    """The tuner sizes the running argmax's output as int64 indices; the
    installed winner still matches the oracle element by element."""
    import numpy as np
    import oracle
    from paper_1604_04815_amd import autotune
    n = 3_000_017
    x_host = np.random.default_rng(16).integers(-50, 50, n).astype(np.int32)  # many ties
    x = to_device(x_host, "int32")
    before = gpu_lib.lscan_get_params(gpu_lib.I32, gpu_lib.OPS["argmax"])
    e = autotune.tune(x, "argmax", shapes=[(256, 8), (1024, 4)], groups=(1, 2), reps=2, warmup=1)
    assert e.op == "argmax" and e.gbs > 0
    autotune.apply(e)
    y = gpu_lib.inclusive(x, "argmax")
    torch.cuda.synchronize()
    assert y.dtype == torch.int64
    assert np.array_equal(to_host(y), oracle.argscan(x_host, "int32", "argmax", False))
    gpu_lib.lscan_set_params(gpu_lib.I32, gpu_lib.OPS["argmax"], 0, gpu_lib.KIND_PLAIN, before)
