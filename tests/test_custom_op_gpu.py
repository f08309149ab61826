"""Parity of a scan with a user-defined operator (lscan_scan_custom): the
library's persistent kernel instantiated outside the library, in
paper_1604_04815_amd/custom/affine_scan.hip, from the public header
include/lscan_custom.hpp, for composition of affine maps x -> a*x + b mod 2^32
(associative, not commutative).  Compared bit for bit with the oracle's
affine_scan."""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def kernels(gpu_lib):
    return gpu_lib.affine_example_kernels()


def maps(n, seed):
    g = np.random.default_rng(seed)
    ab = g.integers(0, 1 << 32, (n, 2), dtype=np.uint64).astype(np.uint32)
    if n:
        ab[g.random(n) < 0.05, 0] = 0          # maps that forget their argument
        ab[g.random(n) < 0.05, 0] = 0xFFFFFFFF
    return ab


def to_dev(ab):
    return torch.from_numpy(ab.view(np.int32).reshape(-1).copy()).to("cuda")


def run(gpu_lib, k, ab, exclusive=False, params=None, inplace=False):
    x = to_dev(ab)
    out = x if inplace else None
    y = gpu_lib.scan_custom(k, x, ab.shape[0], out=out, exclusive=exclusive, params=params)
    gpu_lib.lscan_check(torch.cuda.current_stream().cuda_stream)
    return y.cpu().numpy().view(np.uint32).reshape(-1, 2)


def check(got, ab, exclusive, what):
    want = oracle.affine_scan(ab, exclusive)
    if not np.array_equal(got, want):
        bad = np.flatnonzero(np.any(got != want, axis=1))
        raise AssertionError(f"{what}: {bad.size} mismatches, first at {bad[:6].tolist()}")


@pytest.mark.parametrize("shape", ["default", "small", "wide"])
def test_affine_sizes(gpu_lib, kernels, shape):
    k = kernels[shape]
    x = to_dev(maps(4096, 1))
    gpu_lib.scan_custom(k, x, 4096)
    torch.cuda.synchronize()
    L = int(gpu_lib.lscan_last_launch().tile_elems)
    for n in (1, 2, 3, 63, L - 1, L, L + 1, 5 * L + 7, 1_000_003):
        ab = maps(n, n)
        for excl in (False, True):
            check(run(gpu_lib, k, ab, excl), ab, excl, f"{shape} n={n} excl={excl}")
    log(f"[custom] affine {shape} (L={L}) ok")


def test_affine_in_place_and_params(gpu_lib, kernels):
    n = 777_777
    ab = maps(n, 5)
    check(run(gpu_lib, kernels["default"], ab, inplace=True), ab, False, "in place")
    for groups in (1, 2, 4):
        for handoff in (gpu_lib.HANDOFF_WINDOW, gpu_lib.HANDOFF_CHAIN):
            p = gpu_lib.Params(0, 0, groups, handoff)
            check(run(gpu_lib, kernels["default"], ab, params=p), ab, False, f"groups {groups} handoff {handoff}")
            assert gpu_lib.lscan_last_launch().groups_per_cu <= groups


def test_affine_recurrence_closed_form(gpu_lib, kernels):
    # a = 2, b = 1: h_j = 2 h_{j-1} + 1 = 2^(j+1) - 1 (mod 2^32)
    n = 100_000
    ab = np.tile(np.array([[2, 1]], np.uint32), (n, 1))
    got = run(gpu_lib, kernels["wide"], ab)
    j = np.arange(n, dtype=np.uint64)
    want_b = ((np.uint64(1) << np.minimum(j + 1, 32)) - 1).astype(np.uint64) & 0xFFFFFFFF
    assert np.array_equal(got[:, 1].astype(np.uint64), want_b)
    want_a = np.where(j + 1 < 32, np.uint64(1) << np.minimum(j + 1, 31), 0)
    assert np.array_equal(got[:, 0].astype(np.uint64), want_a)


def test_affine_two_streams(gpu_lib, kernels):
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    jobs = []
    for k in range(4):
        ab = maps(300_000 + k, 40 + k)
        st = s1 if k % 2 == 0 else s2
        with torch.cuda.stream(st):
            x = to_dev(ab)
            y = gpu_lib.scan_custom(kernels["default"], x, ab.shape[0], stream=st)
        jobs.append((ab, x, y))
    torch.cuda.synchronize()
    for ab, _, y in jobs:
        check(y.cpu().numpy().view(np.uint32).reshape(-1, 2), ab, False, "two streams")


def test_affine_full_size(gpu_lib, kernels):
    # the measured configuration: 2^27 maps (1 GiB in, 1 GiB out)
    n = 1 << 27
    ab = maps(n, 9)
    log("[custom] affine 2^27")
    check(run(gpu_lib, kernels["default"], ab), ab, False, "2^27")


def test_affine_misaligned(gpu_lib, kernels):
    # maps (8 bytes each; two per 16-byte vector) starting one map past a
    # vector boundary: with the output at the same phase the block grid is
    # shifted and vectors are used, with the output aligned the maps are read
    # as vectors and written one by one; both bit-exact, inclusive and exclusive
    k = kernels["default"]
    for n in (5, 4097, 300_001):
        ab = maps(n, 40 + n)
        base = to_dev(np.concatenate([maps(1, 1), ab, maps(2, 2)]))   # one map before the data
        x = base[2:2 + 2 * n]
        for y_words, vec in ((2, 1), (4, 2)):
            ybase = torch.zeros(2 * n + 8, dtype=torch.int32, device="cuda")
            y = ybase[y_words:y_words + 2 * n]
            for excl in (False, True):
                gpu_lib.scan_custom(k, x, n, out=y, exclusive=excl)
                gpu_lib.lscan_check(torch.cuda.current_stream().cuda_stream)
                assert gpu_lib.lscan_last_launch().vector_path == vec, (n, y_words)
                got = y.cpu().numpy().view(np.uint32).reshape(-1, 2)
                check(got, ab, excl, f"misaligned n={n} y+{y_words} words excl={excl}")
            # nothing written outside y
            assert not torch.any(ybase[:y_words]).item() and not torch.any(ybase[y_words + 2 * n:]).item()
