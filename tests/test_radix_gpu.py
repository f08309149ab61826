"""Parity of the radix-sort digit offsets (lscan_radix_offsets: a digit-count
kernel, then the single-pass exclusive scan of the counts) with the oracle,
and a stable partition by digit built from them."""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import log

pytestmark = pytest.mark.gpu

TORCH = {"int32": torch.int32, "float32": torch.float32, "int64": torch.int64}
BITS_OF = {"int32": np.uint32, "float32": np.uint32, "int64": np.uint64}


def keys_for(dtype, n, seed, equal=False):
    g = np.random.default_rng(seed)
    raw = g.integers(0, 1 << 63, n, dtype=np.uint64)
    if equal:
        raw[:] = raw[0] if n else 0
    bits = raw.astype(BITS_OF[dtype])
    host = bits.view({"int32": np.int32, "float32": np.float32, "int64": np.int64}[dtype])
    return bits, host


def device_offsets(gpu_lib, host, dtype, shift, bits, block, offset_items=0):
    buf = torch.empty(host.shape[0] + offset_items, dtype=TORCH[dtype], device="cuda")
    kd = buf[offset_items:]
    kd.copy_(torch.from_numpy(host))
    off = gpu_lib.radix_offsets(kd, shift, bits, block)
    gpu_lib.lscan_check(torch.cuda.current_stream().cuda_stream)
    return off.cpu().numpy()


CASES = [("int32", 0, 8), ("int32", 24, 8), ("int32", 3, 1), ("float32", 23, 8), ("float32", 5, 5),
         ("int64", 0, 8), ("int64", 56, 8), ("int64", 30, 3)]


@pytest.mark.parametrize("dtype,shift,bits", CASES, ids=[f"{d}-s{s}-b{b}" for d, s, b in CASES])
def test_radix_offsets(gpu_lib, dtype, shift, bits):
    for n, block in ((1, 1), (100, 7), (100_003, 64), (3_000_000, 1000), (3_000_000, 16_384), (2_000_001, 4096)):
        kbits, host = keys_for(dtype, n, seed=n + bits)
        got = device_offsets(gpu_lib, host, dtype, shift, bits, block)
        want = oracle.radix_offsets(kbits, shift, bits, block)
        assert got.shape == want.shape and np.array_equal(got, want), (n, block)
    log(f"[radix] {dtype} shift={shift} bits={bits} ok")


def test_radix_offsets_equal_keys_and_unaligned(gpu_lib):
    # every key in one digit: one LDS counter takes every atomic
    kbits, host = keys_for("int32", 1_000_000, seed=5, equal=True)
    got = device_offsets(gpu_lib, host, "int32", 8, 8, 16_384)
    assert np.array_equal(got, oracle.radix_offsets(kbits, 8, 8, 16_384))
    # keys not 16-byte aligned, and a block size that is not a multiple of the vector
    for dtype, off_items, block in (("int32", 1, 4096), ("int64", 1, 1000), ("int32", 0, 1001)):
        kbits, host = keys_for(dtype, 777_777, seed=6)
        got = device_offsets(gpu_lib, host, dtype, 4, 6, block, offset_items=off_items)
        assert np.array_equal(got, oracle.radix_offsets(kbits, 4, 6, block)), (dtype, off_items, block)


def test_radix_offsets_give_a_stable_partition(gpu_lib):
    n, block, shift, bits = 200_000, 2048, 7, 4
    kbits, host = keys_for("int32", n, seed=7)
    off = device_offsets(gpu_lib, host, "int32", shift, bits, block)
    dig = ((kbits >> np.uint32(shift)) & np.uint32((1 << bits) - 1)).astype(np.int64)
    # within a block, the r-th key of digit d goes to off[d, b] + r
    pos = np.empty(n, np.int64)
    for b in range((n + block - 1) // block):
        d = dig[b * block:(b + 1) * block]
        order = np.argsort(d, kind="stable")
        rank = np.empty_like(order)
        first = np.searchsorted(d[order], np.arange(1 << bits))
        rank[order] = np.arange(order.shape[0]) - first[d[order]]
        pos[b * block:(b + 1) * block] = off[d, b] + rank
    placed = np.empty_like(kbits)
    placed[pos] = kbits
    assert np.array_equal(placed, kbits[np.argsort(dig, kind="stable")])


def test_radix_offsets_full_size(gpu_lib):
    # the measured configuration: 2^28 int32 keys, 8-bit digits, 16K-key blocks
    from paper_1604_04815_amd import workloads as w
    n = 1 << 28
    kbits = w.full_range_int32(n, w.seed_for(6)).view(np.uint32)
    log("[radix] full size 2^28")
    got = device_offsets(gpu_lib, kbits.view(np.int32), "int32", 0, 8, 16_384)
    assert np.array_equal(got, oracle.radix_offsets(kbits, 0, 8, 16_384))
