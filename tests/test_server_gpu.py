"""The request server on the device: each result in a mixed stream equals the
same request run alone (bit-exact for integer, max and min; float within the
stated bound of the oracle), admission keeps the bytes in flight within the
budget, and destroy finishes every submitted request."""
import numpy as np
import pytest
import torch

from gpu_util import TAU_COMP, TAU_PLAIN, compare, log, make_input, to_device, to_host

pytestmark = pytest.mark.gpu

KINDS = [("int32", "add", False, False), ("int32", "max", False, True), ("int64", "add", False, False),
         ("int64", "max", False, False), ("float32", "add", False, False), ("float32", "add", True, False),
         ("float32", "max", False, True), ("bfloat16", "add", True, False), ("int32", "min", False, False)]


def _alone(gpu_lib, x, op, comp, excl):
    fn = gpu_lib.exclusive if excl else gpu_lib.inclusive
    return fn(x, op, comp)


@pytest.mark.parametrize("solo_bytes", [0, 4 << 20], ids=["solo64MiB", "solo4MiB"])
def test_mix_equals_alone(gpu_lib, solo_bytes):
    rng = np.random.default_rng(42)
    reqs = []
    for k in range(240):
        dtype, op, comp, excl = KINDS[int(rng.integers(0, len(KINDS)))]
        n = int(np.floor(2.0 ** rng.uniform(0, 21)))
        xh = make_input(dtype, op, n, seed=3000 + k)
        x = to_device(xh, dtype)
        y = torch.empty(n, dtype=gpu_lib.out_dtype(x), device="cuda")
        reqs.append((dtype, op, comp, excl, xh, x, y))
    torch.cuda.synchronize()
    with gpu_lib.Server(num_streams=2, solo_bytes=solo_bytes) as srv:
        tickets = [srv.submit(x, y, op, excl, comp) for dtype, op, comp, excl, xh, x, y in reqs]
        results = [srv.wait(t) for t in tickets]
        st = srv.stats()
    assert all(s == gpu_lib.OK for s, _ in results), [s for s, _ in results if s != gpu_lib.OK][:5]
    sizes = [r.batch_size for _, r in results]
    log(f"[server] {len(reqs)} requests in {st.batches} batches, largest batch {max(sizes)}")
    assert st.completed == len(reqs) and st.failed == 0
    for (dtype, op, comp, excl, xh, x, y), (s, r) in zip(reqs, results):
        assert r.t_submit_ns <= r.t_admit_ns <= r.t_launch_ns <= r.t_done_ns
        got = to_host(y)
        compare(got, xh, dtype, op, excl, comp, what=f"served {dtype}/{op} n={xh.size}")
        alone = to_host(_alone(gpu_lib, x, op, comp, excl))
        if dtype in ("int32", "int64") or op != "add":
            assert np.array_equal(got.view(np.uint8), alone.view(np.uint8)), f"{dtype}/{op} mix != alone"
        else:
            # both are within tau * A_j of the exact prefix, so within 2 tau * A_j of each other
            import oracle
            _, a = oracle.scan(xh, dtype, "add", excl, with_absum=True)
            tau = TAU_COMP if comp else TAU_PLAIN
            assert np.all(np.abs(got.astype(np.float64) - alone.astype(np.float64)) <= 2 * tau * a)


def test_budget_and_refusal(gpu_lib):
    budget = 48 << 20
    with gpu_lib.Server(num_streams=2, hbm_budget_bytes=budget) as srv:
        big = torch.zeros((budget // 8) + 1, dtype=torch.int32, device="cuda")
        with pytest.raises(gpu_lib.LscanError) as ei:
            srv.submit(big, torch.empty_like(big))
        assert ei.value.status == gpu_lib.ERR_NO_MEMORY
        xs = [to_device(make_input("int32", "add", 1_500_000, seed=k), "int32") for k in range(24)]
        hosts = [to_host(x) for x in xs]
        ys = [torch.empty_like(x) for x in xs]
        tickets = [srv.submit(x, y) for x, y in zip(xs, ys)]
        for t in tickets:
            s, _ = srv.wait(t)
            assert s == gpu_lib.OK
        st = srv.stats()
        assert 0 < st.peak_bytes_in_flight <= budget
        assert st.bytes_in_flight == 0 and st.pending == 0
    for h, y in zip(hosts, ys):
        compare(to_host(y), h, "int32", "add", False, what="budgeted")


def test_destroy_finishes_work_and_poll(gpu_lib):
    xs = [to_device(make_input("float32", "max", n, seed=n), "float32") for n in (10, 100_000, 2_000_000, 0)]
    hosts = [to_host(x) for x in xs]
    ys = [torch.empty_like(x) for x in xs]
    srv = gpu_lib.Server(num_streams=1)
    tickets = [srv.submit(x, y, "max") for x, y in zip(xs, ys)]
    s, r = srv.poll(tickets[-1])   # n == 0 completes at submit
    assert s == gpu_lib.OK
    s, r = srv.poll(tickets[-1])   # and is forgotten after reporting
    assert s == gpu_lib.ERR_NOT_FOUND
    srv.close()
    for h, y in zip(hosts, ys):
        compare(to_host(y), h, "float32", "max", False, what="after destroy")
