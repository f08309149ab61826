"""The flag workspace across its epoch reset.

Every launch tags the flag words it writes with a 32-bit epoch taken from a
device control word (the paper leaves the reset of its flag array between
scans unstated, Section 4.3, Algorithm 4; here tags advance per launch and
the words are cleared only before the tag could wrap).  The reset clears the
flag words, restarts the tag and clears the word holding the tag of the last
launch that gave up.  A real workspace reaches it after ~4e9 launches, so
the test hooks of include/lscan_testing.h seed a workspace a few launches
before it; every launch across the reset is then checked element by element
against the oracle, and the control words are read back.

Kinds covered: plain inclusive / exclusive, segmented and batched scans on
one stream's workspace (they share it), and graph replays (a graph owns its
workspace).  A stale last-abort word equal to a tag that a post-reset launch
uses would stop that launch at its first wait: the tests plant such a word
before the reset, once through the watchdog (a launch really stopped with the
watchdog at 0) and once directly through the seed hook, and check that the
launches after the reset are exact."""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import compare, log, to_host
from paper_1604_04815_amd import workloads as w

pytestmark = pytest.mark.gpu


def _stream():
    return torch.cuda.current_stream().cuda_stream


class Kinds:
    """Plain, segmented and batched int32 add scans over one input, each
    checked exactly against the oracle."""

    def __init__(self, gpu_lib, n, seed):
        self.lib = gpu_lib
        self.x = w.uniform_int(n, -1000, 1000, seed)
        self.xd = torch.from_numpy(self.x).to("cuda")
        self.y = torch.empty_like(self.xd)
        cuts = np.sort(w.rng(seed + 1).integers(0, n, size=7))
        self.off = np.concatenate([[0], cuts, [n]]).astype(np.int64)
        self.offd = torch.from_numpy(self.off).to("cuda")
        # batched: three arrays cut from the input, outputs at the same offsets
        self.parts = [(0, n // 3), (n // 3, n // 3 + 1000), (n // 3 + 1000, n)]

    def run(self, k):
        lib, xd, y = self.lib, self.xd, self.y
        kind = ("plain", "exclusive", "segmented", "batched")[k % 4]
        y.fill_(-7)
        if kind == "plain":
            lib.inclusive(xd, "add", out=y)
        elif kind == "exclusive":
            lib.exclusive(xd, "add", out=y)
        elif kind == "segmented":
            lib.segmented(xd, self.offd, "add", out=y)
        else:
            lib.batched([xd[a:b] for a, b in self.parts], "add", outs=[y[a:b] for a, b in self.parts])
        return kind

    def check(self, kind, what):
        got = to_host(self.y)
        if kind == "plain":
            compare(got, self.x, "int32", "add", False, what=what)
        elif kind == "exclusive":
            compare(got, self.x, "int32", "add", True, what=what)
        elif kind == "segmented":
            compare(got, self.x, "int32", "add", False, offsets=self.off, what=what)
        else:
            for a, b in self.parts:
                compare(got[a:b], self.x[a:b], "int32", "add", False, what=f"{what} array [{a}, {b})")


def test_eager_scans_cross_the_epoch_reset(gpu_lib):
    limit = gpu_lib.lscan_test_epoch_limit()
    assert limit == 0xFFFFFFF0
    ks = Kinds(gpu_lib, (1 << 21) + 77, w.seed_for(20))
    for k in range(4):  # every kind once: workspace, segment table, residency tests
        ks.check(ks.run(k), f"warm-up {k}")
    gpu_lib.lscan_check(_stream())
    # the realistic state: tags near 2^32, a few launches before the reset
    gpu_lib.lscan_test_seed_epoch(limit - 3, limit - 3, 0)
    launches, ctrl = gpu_lib.lscan_test_epoch_state()
    assert launches == limit - 3 and ctrl[0] == limit - 3 and ctrl[1] == 0 and ctrl[3] == 0
    want = [(limit - 2, limit - 2), (limit - 1, limit - 1), (limit, limit), (1, 1), (2, 2), (3, 3), (4, 4), (5, 5)]
    for k, (n_want, tag_want) in enumerate(want):
        kind = ks.run(k)
        log(f"[epoch] eager launch {k} ({kind}), expecting tag {tag_want:#x}")
        gpu_lib.lscan_check(_stream())
        ks.check(kind, f"eager {kind} launch {k} (tag {tag_want:#x})")
        launches, ctrl = gpu_lib.lscan_test_epoch_state()
        assert (launches, ctrl[0], ctrl[1], ctrl[3]) == (n_want, tag_want, 0, 0), (k, launches, ctrl)


def test_planted_abort_tag_is_cleared_by_the_reset(gpu_lib):
    # the last-abort word names tag 3; the run is seeded so that tag 3 is
    # used only after the reset, where a stale word would stop that launch
    limit = gpu_lib.lscan_test_epoch_limit()
    ks = Kinds(gpu_lib, (1 << 22) + 5, w.seed_for(20, 1))
    for k in range(4):
        ks.check(ks.run(k), f"warm-up {k}")
    gpu_lib.lscan_test_seed_epoch(limit - 1, 10, 3)
    launches, ctrl = gpu_lib.lscan_test_epoch_state()
    assert ctrl[3] == 3
    for k in range(6):  # tags 11, then 1 .. 5 after the reset
        kind = ks.run(k)
        gpu_lib.lscan_check(_stream())
        ks.check(kind, f"planted abort tag, {kind} launch {k}")
        launches, ctrl = gpu_lib.lscan_test_epoch_state()
        if k == 0:
            assert (launches, ctrl[0], ctrl[3]) == (limit, 11, 3), ctrl
        else:
            assert (launches, ctrl[0], ctrl[3]) == (k, k, 0), (k, launches, ctrl)


@pytest.fixture
def watchdog(gpu_lib):
    lib = gpu_lib.load()
    default = lib.lscan_get_watchdog_us()
    yield lib
    assert lib.lscan_set_watchdog_us(default) == 0


def test_watchdog_stop_just_before_the_reset(gpu_lib, watchdog):
    # launches with the watchdog at 0 until one gives up (its tag lands in the
    # last-abort word), then normal launches through the reset and past that
    # tag's next use, every one exact
    limit = gpu_lib.lscan_test_epoch_limit()
    n = 1 << 24
    x = w.uniform_int(n, -1000, 1000, w.seed_for(20, 2))
    xd = torch.from_numpy(x).to("cuda")
    y = torch.empty_like(xd)
    gpu_lib.inclusive(xd, "add", out=y)
    gpu_lib.lscan_check(_stream())
    gpu_lib.lscan_test_seed_epoch(limit - 8, 1, 0)
    assert watchdog.lscan_set_watchdog_us(0) == 0
    stopped = None
    for k in range(6):  # tags 2 .. 7
        gpu_lib.inclusive(xd, "add", out=y)
        try:
            gpu_lib.lscan_check(_stream())
        except gpu_lib.LscanError as exc:
            assert exc.status == gpu_lib.ERR_TIMEOUT, exc
            stopped = 2 + k
            break
    assert watchdog.lscan_set_watchdog_us(2_000_000) == 0
    if stopped is None:
        pytest.skip("no launch gave up with the watchdog at 0 (every wait was already satisfied)")
    launches, ctrl = gpu_lib.lscan_test_epoch_state()
    log(f"[epoch] launch with tag {stopped} gave up; last-abort word {ctrl[3]}")
    assert ctrl[3] == stopped and ctrl[0] == stopped
    want = oracle.scan(x, "int32", "add")
    tag = stopped
    while True:  # the rest of the run, then the reset, then past the stopped tag
        y.fill_(-7)
        gpu_lib.inclusive(xd, "add", out=y)
        gpu_lib.lscan_check(_stream())
        assert np.array_equal(to_host(y), want)
        launches, ctrl = gpu_lib.lscan_test_epoch_state()
        if launches == limit:
            tag += 1
            assert ctrl[0] == tag and ctrl[3] == stopped
            continue
        if launches < 100:  # after the reset
            assert ctrl[0] == launches and ctrl[3] == 0, (launches, ctrl)
            if launches >= stopped + 2:
                break
        else:
            tag += 1
            assert ctrl[0] == tag and ctrl[3] == stopped, (launches, ctrl)


def test_graph_replays_cross_the_epoch_reset(gpu_lib):
    limit = gpu_lib.lscan_test_epoch_limit()
    n = (1 << 21) + 13
    xd = torch.empty(n, dtype=torch.int32, device="cuda")
    yd = torch.empty_like(xd)
    g = gpu_lib.lscan_graph_create_scan(xd.data_ptr(), yd.data_ptr(), n, gpu_lib.I32, gpu_lib.ADD, 0)
    try:
        xd.copy_(torch.from_numpy(w.uniform_int(n, -1000, 1000, w.seed_for(20, 3))))
        g.launch()
        g.check()
        # tags near 2^32, and a planted last-abort word (tag 2) that the
        # second replay after the reset would meet
        gpu_lib.lscan_test_seed_epoch(limit - 2, limit - 2, 2, graph=g)
        want = [(limit - 1, limit - 1, 2), (limit, limit, 2), (1, 1, 0), (2, 2, 0), (3, 3, 0)]
        for rep, (n_want, tag_want, abort_want) in enumerate(want):
            x = w.uniform_int(n, -1000, 1000, w.seed_for(20, 10 + rep))
            xd.copy_(torch.from_numpy(x))
            g.launch()
            g.check()
            compare(to_host(yd), x, "int32", "add", False, what=f"graph replay {rep} (tag {tag_want:#x})")
            launches, ctrl = gpu_lib.lscan_test_epoch_state(graph=g)
            assert (launches, ctrl[0], ctrl[1], ctrl[3]) == (n_want, tag_want, 0, abort_want), (rep, launches, ctrl)
            z = gpu_lib.inclusive(xd, "max")  # eager work between replays, on the same stream
            torch.cuda.synchronize()
            compare(to_host(z), x, "int32", "max", False, what=f"eager between replays {rep}")
    finally:
        g.destroy()


def test_eager_calls_refused_under_capture(gpu_lib):
    # a kernel node captured from an eager call would hold the per-stream
    # workspace's pointers, which later calls may free; such calls are
    # refused (graphs come from lscan_graph_create_*), and so are the
    # zero-size calls that would otherwise record a memset
    lib = gpu_lib.load()
    n = 1 << 16
    x = w.uniform_int(n, -1000, 1000, w.seed_for(20, 4))
    xd = torch.from_numpy(x).to("cuda")
    y = torch.empty_like(xd)
    off = torch.tensor([0, n // 2, n], dtype=torch.int64, device="cuda")
    out = torch.empty_like(xd)
    count = torch.zeros(1, dtype=torch.int64, device="cuda")
    row = torch.zeros(1, dtype=torch.int64, device="cuda")
    stats = torch.zeros(4, dtype=torch.int64, device="cuda")
    keys_off = torch.empty(256, dtype=torch.int64, device="cuda")
    gpu_lib.inclusive(xd, "add", out=y)  # the workspace exists: only the capture refuses
    gpu_lib.segmented(xd, off, "add", out=y)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    got = {}
    with torch.cuda.graph(graph, stream=side):
        s = torch.cuda.current_stream().cuda_stream
        z = xd + 1  # something for the graph to hold
        got["inclusive"] = lib.lscan_inclusive(xd.data_ptr(), y.data_ptr(), n, gpu_lib.I32, gpu_lib.ADD, 0, s)
        got["exclusive"] = lib.lscan_exclusive(xd.data_ptr(), y.data_ptr(), n, gpu_lib.I32, gpu_lib.MAX, 0, s)
        got["segmented"] = lib.lscan_segmented(xd.data_ptr(), y.data_ptr(), n, off.data_ptr(), 2, gpu_lib.I32,
                                               gpu_lib.ADD, 0, s)
        got["compact"] = lib.lscan_compact(xd.data_ptr(), None, out.data_ptr(), count.data_ptr(), n, gpu_lib.I32, s)
        got["compact n=0"] = lib.lscan_compact(xd.data_ptr(), None, out.data_ptr(), count.data_ptr(), 0,
                                               gpu_lib.I32, s)
        got["radix"] = lib.lscan_radix_offsets(xd.data_ptr(), n, gpu_lib.I32, 0, 8, n, keys_off.data_ptr(), s)
        got["bfs V=0"] = lib.lscan_bfs(row.data_ptr(), None, 0, 0, 0, None, None, stats.data_ptr(), s)
    torch.cuda.synchronize()
    assert all(v == gpu_lib.ERR_UNSUPPORTED for v in got.values()), got
    graph.replay()
    torch.cuda.synchronize()
    assert torch.equal(z, xd + 1)
    gpu_lib.inclusive(xd, "add", out=y)  # eager again, unaffected
    gpu_lib.lscan_check(_stream())
    assert np.array_equal(to_host(y), oracle.scan(x, "int32", "add"))
