"""The timeout path, forced from the host: with the watchdog at 0 every wait
between workgroups that is not already satisfied gives up at once, the whole
grid stops through the abort word, and lscan_check reports the timeout.  The
kernels still exit normally (every wait is bounded).  After the watchdog is
restored, the same workspaces give exact results again: the epoch tags of
the stopped launches do not leak into later ones."""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import log
from paper_1604_04815_amd import workloads as w

pytestmark = pytest.mark.gpu


def statuses(gpu_lib, fn, times):
    out = []
    for _ in range(times):
        fn()
        try:
            gpu_lib.lscan_check(torch.cuda.current_stream().cuda_stream)
            out.append("ok")
        except gpu_lib.LscanError as exc:
            assert exc.status == gpu_lib.ERR_TIMEOUT, exc
            out.append("timeout")
    return out


@pytest.fixture
def watchdog(gpu_lib):
    lib = gpu_lib.load()
    default = lib.lscan_get_watchdog_us()
    assert default == 2_000_000
    yield lib
    assert lib.lscan_set_watchdog_us(default) == 0
    assert lib.lscan_get_watchdog_us() == default


def test_scan_timeout_then_exact(gpu_lib, watchdog):
    n = 1 << 24
    x = w.uniform_int(n, -1000, 1000, w.seed_for(12))
    xd = torch.from_numpy(x).to("cuda")
    y = torch.empty_like(xd)
    assert watchdog.lscan_set_watchdog_us(0) == 0
    log("[watchdog] int32 scans with the watchdog at 0")
    got = statuses(gpu_lib, lambda: gpu_lib.inclusive(xd, "add", out=y), 6)
    assert watchdog.lscan_set_watchdog_us(2_000_000) == 0
    assert "timeout" in got, got
    for _ in range(3):
        gpu_lib.inclusive(xd, "add", out=y)
        gpu_lib.lscan_check(torch.cuda.current_stream().cuda_stream)
        assert np.array_equal(y.cpu().numpy(), oracle.scan(x, "int32", "add"))


def test_compaction_and_chain_timeout_then_exact(gpu_lib, watchdog):
    n = 1 << 23
    x = w.uniform_int(n, -5, 5, w.seed_for(12, 1))
    xd = torch.from_numpy(x).to("cuda")
    chain = gpu_lib.Params(0, 0, 0, gpu_lib.HANDOFF_CHAIN)
    assert watchdog.lscan_set_watchdog_us(0) == 0
    got_c = statuses(gpu_lib, lambda: gpu_lib.compact(xd), 4)
    got_h = statuses(gpu_lib, lambda: gpu_lib.inclusive(xd, "add", params=chain), 4)
    assert watchdog.lscan_set_watchdog_us(2_000_000) == 0
    assert "timeout" in got_c + got_h, (got_c, got_h)
    out, count = gpu_lib.compact(xd)
    gpu_lib.lscan_check(torch.cuda.current_stream().cuda_stream)
    want = oracle.compact(x, None)
    assert int(count.item()) == want.shape[0]
    assert np.array_equal(out[:want.shape[0]].cpu().numpy(), want)
    y = gpu_lib.inclusive(xd, "add", params=chain)
    gpu_lib.lscan_check(torch.cuda.current_stream().cuda_stream)
    assert np.array_equal(y.cpu().numpy(), oracle.scan(x, "int32", "add"))


def test_bfs_timeout_then_exact(gpu_lib, watchdog):
    s, d = w.rmat_edges(16, 16, w.seed_for(12, 2))
    row, col = w.csr_from_edges(s, d, 1 << 16, symmetric=True)
    src = int(np.argmax(np.diff(row)))
    rd, cd = torch.from_numpy(row).to("cuda"), torch.from_numpy(col).to("cuda")
    assert watchdog.lscan_set_watchdog_us(0) == 0
    log("[watchdog] searches with the watchdog at 0")
    got = statuses(gpu_lib, lambda: gpu_lib.bfs(rd, cd, src), 4)
    assert watchdog.lscan_set_watchdog_us(2_000_000) == 0
    assert "timeout" in got, got
    levels, _, stats = gpu_lib.bfs(rd, cd, src)
    gpu_lib.lscan_check(torch.cuda.current_stream().cuda_stream)
    assert np.array_equal(levels.cpu().numpy(), oracle.bfs_levels(row, col, src))


def test_watchdog_validation(gpu_lib, watchdog):
    assert watchdog.lscan_set_watchdog_us(-1) == gpu_lib.ERR_INVALID_ARG
    assert watchdog.lscan_set_watchdog_us(3_600_000_001) == gpu_lib.ERR_INVALID_ARG
    assert watchdog.lscan_get_watchdog_us() == 2_000_000
