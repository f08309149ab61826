"""Sizes beyond 2^31 elements: every index, block number and count in the
kernels is 64-bit.  Checked on the device through properties that hold at
any size (the difference of neighbouring outputs is the input; closed forms),
over every element, in chunks so that the checks need little extra memory."""
import pytest
import torch

from gpu_util import log

pytestmark = pytest.mark.gpu

N_BIG = (1 << 31) + 12_345
CHUNK = 1 << 28


def test_int64_ones_closed_form_in_place(gpu_lib):
    # y_j = j + 1, scanned in place (16 GiB)
    x = torch.ones(N_BIG, dtype=torch.int64, device="cuda")
    log(f"[big] int64 add of ones, n={N_BIG}, in place")
    gpu_lib.inclusive(x, "add", out=x)
    gpu_lib.lscan_check(torch.cuda.current_stream().cuda_stream)
    assert gpu_lib.lscan_last_launch().n == N_BIG
    for lo in range(0, N_BIG, CHUNK):
        hi = min(lo + CHUNK, N_BIG)
        want = torch.arange(lo + 1, hi + 1, dtype=torch.int64, device="cuda")
        assert torch.equal(x[lo:hi], want), lo
    del x
    torch.cuda.empty_cache()


def test_int32_random_neighbour_differences(gpu_lib):
    # y_0 = x_0 and y_j - y_{j-1} = x_j (mod 2^32) for every j: the scan, exactly
    g = torch.Generator(device="cuda").manual_seed(1604)
    x = torch.randint(-1000, 1001, (N_BIG,), dtype=torch.int32, device="cuda", generator=g)
    log(f"[big] int32 add, n={N_BIG}")
    y = gpu_lib.inclusive(x, "add")
    gpu_lib.lscan_check(torch.cuda.current_stream().cuda_stream)
    assert y[0].item() == x[0].item()
    for lo in range(1, N_BIG, CHUNK):
        hi = min(lo + CHUNK, N_BIG)
        d = y[lo:hi].to(torch.int64) - y[lo - 1:hi - 1].to(torch.int64)
        d = torch.remainder(d + (1 << 31), 1 << 32) - (1 << 31)  # back to the wrapped int32 step
        assert torch.equal(d, x[lo:hi].to(torch.int64)), lo
    # the last element is the full sum modulo 2^32
    total = int(x.to(torch.int64).sum().item())
    assert y[-1].item() == ((total + (1 << 31)) % (1 << 32)) - (1 << 31)
    del x, y
    torch.cuda.empty_cache()


def test_compact_count_beyond_2p31(gpu_lib):
    # all ones but a zero every 1000 items: count and contents by closed form
    x = torch.ones(N_BIG, dtype=torch.int32, device="cuda")
    x[::1000] = 0
    log(f"[big] compaction, n={N_BIG}")
    out, count = gpu_lib.compact(x)
    torch.cuda.synchronize()
    zeros = (N_BIG + 999) // 1000
    assert int(count.item()) == N_BIG - zeros
    kept = N_BIG - zeros
    for lo in range(0, kept, CHUNK):
        hi = min(lo + CHUNK, kept)
        assert bool((out[lo:hi] == 1).all()), lo
    del x, out
    torch.cuda.empty_cache()


def test_argmax_index_beyond_2p31(gpu_lib):
    # zeros with one larger value past index 2^31: the running argmax is 0
    # before it and its index from it on
    p = (1 << 31) + 5
    x = torch.zeros(N_BIG, dtype=torch.int32, device="cuda")
    x[p] = 7
    log(f"[big] argmax, n={N_BIG}")
    y = gpu_lib.inclusive(x, "argmax")
    gpu_lib.lscan_check(torch.cuda.current_stream().cuda_stream)
    for lo in range(0, N_BIG, CHUNK):
        hi = min(lo + CHUNK, N_BIG)
        idx = torch.arange(lo, hi, dtype=torch.int64, device="cuda")
        want = torch.where(idx < p, torch.zeros_like(idx), torch.full_like(idx, p))
        assert torch.equal(y[lo:hi], want), lo
    del x, y
    torch.cuda.empty_cache()
