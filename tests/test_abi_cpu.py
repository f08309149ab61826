"""The C ABI library on the CPU host: it loads, exports every symbol that
include/lscan.h declares, and rejects bad arguments before any device work
(no GPU call is made by these tests)."""
import ctypes
import glob
import os
import re

import pytest

from paper_1604_04815_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lscan.h")
HEADERS = sorted(glob.glob(os.path.join(ROOT, "include", "*.h")))


def declared_symbols(headers=None):
    syms = set()
    for h in headers or HEADERS:
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        syms.update(re.findall(r"\b(lscan_[a-z_0-9]+)\s*\(", text))
    return sorted(syms)


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(binding.LIB_PATH):
        pytest.fail("liblscan.so is not built (run __graft_entry__.build())")
    return binding.load()


def test_header_declares_the_abi():
    syms = declared_symbols([HEADER])
    for name in ("lscan_inclusive", "lscan_exclusive", "lscan_segmented", "lscan_check",
                 "lscan_status_string"):
        assert name in syms
    assert os.path.join(ROOT, "include", "lscan_testing.h") in HEADERS
    assert "lscan_test_seed_epoch" in declared_symbols()


def test_every_declared_symbol_is_exported(lib):
    for name in declared_symbols():
        assert hasattr(lib, name), name
        assert name in binding.SIGNATURES, f"binding lacks {name}"


def test_status_strings(lib):
    for code in (0, -1, -2, -3, -4, -5, -6, -7):
        assert lib.lscan_status_string(code)
    assert binding.status_string(-1) == "invalid argument"


def test_tile_shapes(lib):
    shapes = binding.lscan_tile_shapes()
    assert len(shapes) >= 1
    for t, r in shapes:
        assert t % 64 == 0 and 64 <= t <= 1024 and r >= 1


def test_default_params_roundtrip(lib):
    p = binding.lscan_get_params(binding.I32, binding.ADD)
    assert (p.block_threads, p.vectors_per_lane) in binding.lscan_tile_shapes()
    assert p.groups_per_cu >= 1
    q = binding.Params(p.block_threads, p.vectors_per_lane, p.groups_per_cu + 1, 0)
    binding.lscan_set_params(binding.I32, binding.ADD, 0, False, q)
    r = binding.lscan_get_params(binding.I32, binding.ADD)
    assert r.groups_per_cu == p.groups_per_cu + 1
    binding.lscan_set_params(binding.I32, binding.ADD, 0, False, p)
    with pytest.raises(binding.LscanError):
        binding.lscan_set_params(binding.I32, binding.ADD, 0, False, binding.Params(100, 3, 1, 0))


FAKE_X = 1 << 20     # never dereferenced: every call below is rejected or a no-op
FAKE_Y = 1 << 30


@pytest.mark.parametrize("call,status", [
    # n < 0
    (lambda l: l.lscan_inclusive(FAKE_X, FAKE_Y, -1, 0, 0, 0, None), binding.ERR_INVALID_ARG),
    # bad dtype / op / flags
    (lambda l: l.lscan_inclusive(FAKE_X, FAKE_Y, 8, 9, 0, 0, None), binding.ERR_INVALID_ARG),
    (lambda l: l.lscan_inclusive(FAKE_X, FAKE_Y, 8, 0, 5, 0, None), binding.ERR_INVALID_ARG),
    (lambda l: l.lscan_inclusive(FAKE_X, FAKE_Y, 8, 0, 0, 0x100, None), binding.ERR_INVALID_ARG),
    # the exclusive flag belongs to lscan_segmented only
    (lambda l: l.lscan_inclusive(FAKE_X, FAKE_Y, 8, 0, 0, binding.F_EXCLUSIVE, None), binding.ERR_INVALID_ARG),
    # null pointers with n > 0
    (lambda l: l.lscan_inclusive(None, FAKE_Y, 8, 0, 0, 0, None), binding.ERR_INVALID_ARG),
    (lambda l: l.lscan_exclusive(FAKE_X, None, 8, 0, 0, 0, None), binding.ERR_INVALID_ARG),
    # compensation only for float add
    (lambda l: l.lscan_inclusive(FAKE_X, FAKE_Y, 8, binding.I32, binding.ADD, binding.F_COMPENSATED, None),
     binding.ERR_UNSUPPORTED),
    (lambda l: l.lscan_inclusive(FAKE_X, FAKE_Y, 8, binding.F32, binding.MAX, binding.F_COMPENSATED, None),
     binding.ERR_UNSUPPORTED),
    # misaligned element pointers
    (lambda l: l.lscan_inclusive(FAKE_X + 2, FAKE_Y, 8, binding.I32, 0, 0, None), binding.ERR_INVALID_ARG),
    (lambda l: l.lscan_inclusive(FAKE_X, FAKE_Y + 4, 8, binding.I64, 0, 0, None), binding.ERR_INVALID_ARG),
    # partial overlap (in place is allowed, a shifted alias is not)
    (lambda l: l.lscan_inclusive(FAKE_X, FAKE_X + 4, 8, binding.I32, 0, 0, None), binding.ERR_INVALID_ARG),
    # bf16 in place is impossible (2-byte input, 4-byte output)
    (lambda l: l.lscan_inclusive(FAKE_X, FAKE_X, 8, binding.BF16, 0, 0, None), binding.ERR_INVALID_ARG),
    # n == 0 is a no-op, even with null pointers
    (lambda l: l.lscan_inclusive(None, None, 0, 0, 0, 0, None), binding.OK),
    (lambda l: l.lscan_exclusive(None, None, 0, binding.F32, binding.MIN, 0, None), binding.OK),
    # segmented: negative count, zero segments with elements, null offsets, bad flag
    (lambda l: l.lscan_segmented(FAKE_X, FAKE_Y, 8, FAKE_X, -1, 0, 0, 0, None), binding.ERR_INVALID_ARG),
    (lambda l: l.lscan_segmented(FAKE_X, FAKE_Y, 8, FAKE_X, 0, 0, 0, 0, None), binding.ERR_INVALID_ARG),
    (lambda l: l.lscan_segmented(FAKE_X, FAKE_Y, 8, None, 2, 0, 0, 0, None), binding.ERR_INVALID_ARG),
    (lambda l: l.lscan_segmented(FAKE_X, FAKE_Y, 8, FAKE_X + 4, 2, 0, 0, 0, None), binding.ERR_INVALID_ARG),
    (lambda l: l.lscan_segmented(FAKE_X, FAKE_Y, 8, FAKE_X, 2, 0, 0, 0x80, None), binding.ERR_INVALID_ARG),
    (lambda l: l.lscan_segmented(None, None, 0, None, 0, 0, 0, binding.F_EXCLUSIVE, None), binding.OK),
])
def test_argument_validation(lib, call, status):
    assert call(lib) == status


def test_params_validation(lib):
    bad_shape = binding.Params(192, 3, 1, 0)
    st = lib.lscan_scan_with_params(FAKE_X, FAKE_Y, 8, 0, 0, 0, 0, ctypes.byref(bad_shape), None)
    assert st == binding.ERR_UNSUPPORTED
    neg = binding.Params(0, 0, -1, 0)
    st = lib.lscan_scan_with_params(FAKE_X, FAKE_Y, 8, 0, 0, 0, 0, ctypes.byref(neg), None)
    assert st == binding.ERR_INVALID_ARG
    for handoff in (-1, 2, 7):
        bad = binding.Params(0, 0, 0, handoff)
        st = lib.lscan_scan_with_params(FAKE_X, FAKE_Y, 8, 0, 0, 0, 0, ctypes.byref(bad), None)
        assert st == binding.ERR_INVALID_ARG, handoff
        st = lib.lscan_set_params(binding.I32, binding.ADD, 0, binding.KIND_PLAIN,
                                  ctypes.byref(binding.Params(256, 8, 1, handoff)))
        assert st == binding.ERR_INVALID_ARG, handoff


def test_handoff_default_roundtrip(lib):
    p = binding.lscan_get_params(binding.I64, binding.MAX)
    assert p.handoff == binding.HANDOFF_WINDOW
    q = binding.Params(p.block_threads, p.vectors_per_lane, p.groups_per_cu, binding.HANDOFF_CHAIN)
    binding.lscan_set_params(binding.I64, binding.MAX, 0, False, q)
    assert binding.lscan_get_params(binding.I64, binding.MAX).handoff == binding.HANDOFF_CHAIN
    binding.lscan_set_params(binding.I64, binding.MAX, 0, False, p)
    assert binding.lscan_get_params(binding.I64, binding.MAX).handoff == binding.HANDOFF_WINDOW


def test_raising_wrappers(lib):
    with pytest.raises(binding.LscanError) as ei:
        binding.lscan_inclusive(FAKE_X, FAKE_Y, -5, binding.I32, binding.ADD)
    assert ei.value.status == binding.ERR_INVALID_ARG


def _table(entries):
    tab = (binding.Array * max(1, len(entries)))()
    for i, (x, y, n) in enumerate(entries):
        tab[i].x, tab[i].y, tab[i].n = x, y, n
    return tab


@pytest.mark.parametrize("entries,count,status", [
    ([], 0, binding.OK),                                         # nothing to do
    ([(None, None, 0), (None, None, 0)], 2, binding.OK),         # all empty
    ([(FAKE_X, FAKE_Y, 8)], -1, binding.ERR_INVALID_ARG),        # negative count
    ([(FAKE_X, FAKE_Y, -3)], 1, binding.ERR_INVALID_ARG),        # negative length
    ([(FAKE_X, None, 8)], 1, binding.ERR_INVALID_ARG),           # null y
    ([(FAKE_X + 2, FAKE_Y, 8)], 1, binding.ERR_INVALID_ARG),     # misaligned x
    ([(FAKE_X, FAKE_X + 8, 8)], 1, binding.ERR_INVALID_ARG),     # partial overlap
    ([(FAKE_X, FAKE_Y, 8), (FAKE_X, FAKE_Y + 4, -1)], 2, binding.ERR_INVALID_ARG),
])
def test_batched_validation(lib, entries, count, status):
    tab = _table(entries)
    assert lib.lscan_batched(tab, count, binding.I32, binding.ADD, 0, None) == status


def test_batched_null_table(lib):
    assert lib.lscan_batched(None, 3, binding.I32, binding.ADD, 0, None) == binding.ERR_INVALID_ARG
    assert lib.lscan_batched(None, 0, binding.I32, binding.ADD, 0, None) == binding.OK


def test_graph_validation(lib):
    h = ctypes.c_void_p()
    # nothing to capture
    st = lib.lscan_graph_create_segmented(None, None, 0, None, 0, binding.I32, binding.ADD, 0, None,
                                          ctypes.byref(h))
    assert st == binding.ERR_INVALID_ARG
    st = lib.lscan_graph_create_batched(_table([]), 0, binding.I32, binding.ADD, 0, None, ctypes.byref(h))
    assert st == binding.ERR_INVALID_ARG
    # bad arguments are rejected before any device work
    st = lib.lscan_graph_create_segmented(FAKE_X, FAKE_Y, 8, FAKE_X, -1, binding.I32, binding.ADD, 0, None,
                                          ctypes.byref(h))
    assert st == binding.ERR_INVALID_ARG
    assert lib.lscan_graph_launch(None, None) == binding.ERR_INVALID_ARG
    assert lib.lscan_graph_destroy(None) == binding.ERR_INVALID_ARG
    # plain scans: nothing to capture, bad flags, types, pointers
    g = lib.lscan_graph_create_scan
    assert g(None, None, 0, binding.I32, binding.ADD, 0, None, ctypes.byref(h)) == binding.ERR_INVALID_ARG
    assert g(FAKE_X, FAKE_Y, 8, binding.I32, binding.ADD, 0x100, None, ctypes.byref(h)) == binding.ERR_INVALID_ARG
    assert g(FAKE_X, FAKE_Y, 8, binding.I32, binding.ADD, binding.F_COMPENSATED, None,
             ctypes.byref(h)) == binding.ERR_UNSUPPORTED
    assert g(FAKE_X, FAKE_Y, 8, binding.I32, binding.ADD, binding.F_INDEX64, None,
             ctypes.byref(h)) == binding.ERR_INVALID_ARG
    assert g(FAKE_X, FAKE_Y, 8, 9, binding.ADD, 0, None, ctypes.byref(h)) == binding.ERR_INVALID_ARG
    assert g(None, FAKE_Y, 8, binding.I32, binding.ADD, 0, None, ctypes.byref(h)) == binding.ERR_INVALID_ARG
    assert g(FAKE_X + 2, FAKE_Y, 8, binding.I32, binding.ADD, 0, None, ctypes.byref(h)) == binding.ERR_INVALID_ARG
    assert g(FAKE_X, FAKE_X + 4, 8, binding.I32, binding.ADD, 0, None, ctypes.byref(h)) == binding.ERR_INVALID_ARG
    assert g(FAKE_X, FAKE_Y, 8, binding.I32, binding.ADD, binding.F_EXCLUSIVE, None, None) == binding.ERR_INVALID_ARG


def test_params_kinds(lib):
    p = binding.Params()
    for kind in (binding.KIND_PLAIN, binding.KIND_SEGMENTED, binding.KIND_BATCHED, binding.KIND_COMPACT):
        assert lib.lscan_get_params(binding.F32, binding.ADD, binding.F_COMPENSATED, kind, ctypes.byref(p)) == 0
    assert lib.lscan_get_params(binding.F32, binding.ADD, 0, 4, ctypes.byref(p)) == binding.ERR_INVALID_ARG
    assert lib.lscan_get_params(binding.F32, binding.ADD, 0, -1, ctypes.byref(p)) == binding.ERR_INVALID_ARG
    assert lib.lscan_get_params(binding.I32, binding.MAX, binding.F_COMPENSATED, 0,
                                ctypes.byref(p)) == binding.ERR_UNSUPPORTED


def test_deterministic_flag_is_accepted(lib):
    # n == 0 is a no-op after validation, so these reach the flag check only
    for flags in (binding.F_DETERMINISTIC, binding.F_DETERMINISTIC | binding.F_COMPENSATED):
        assert lib.lscan_inclusive(FAKE_X, FAKE_Y, 0, binding.F32, binding.ADD, flags, None) == binding.OK
    assert lib.lscan_inclusive(FAKE_X, FAKE_Y, 0, binding.I32, binding.ADD, 0x8, None) == binding.ERR_INVALID_ARG
    assert lib.lscan_segmented(None, None, 0, None, 0, binding.I32, binding.MAX,
                               binding.F_DETERMINISTIC | binding.F_EXCLUSIVE, None) == binding.OK


def test_compact_validation(lib):
    cnt = FAKE_Y + (1 << 24)  # aligned, never dereferenced
    # bf16 items are not supported; bad enum is invalid
    assert lib.lscan_compact(FAKE_X, None, FAKE_Y, cnt, 8, binding.BF16, None) == binding.ERR_UNSUPPORTED
    assert lib.lscan_compact(FAKE_X, None, FAKE_Y, cnt, 8, 9, None) == binding.ERR_INVALID_ARG
    # count missing or misaligned, negative n
    assert lib.lscan_compact(FAKE_X, None, FAKE_Y, None, 8, binding.I32, None) == binding.ERR_INVALID_ARG
    assert lib.lscan_compact(FAKE_X, None, FAKE_Y, cnt + 4, 8, binding.I32, None) == binding.ERR_INVALID_ARG
    assert lib.lscan_compact(FAKE_X, None, FAKE_Y, cnt, -1, binding.I32, None) == binding.ERR_INVALID_ARG
    # out may not overlap x (not even exactly), the flags or the count
    assert lib.lscan_compact(FAKE_X, None, FAKE_X, cnt, 8, binding.I32, None) == binding.ERR_INVALID_ARG
    assert lib.lscan_compact(FAKE_X, None, FAKE_X + 16, cnt, 8, binding.I64, None) == binding.ERR_INVALID_ARG
    assert lib.lscan_compact(FAKE_X, FAKE_Y + 4, FAKE_Y, cnt, 64, binding.I32, None) == binding.ERR_INVALID_ARG
    assert lib.lscan_compact(FAKE_X, None, FAKE_Y, FAKE_Y + 8, 8, binding.I32, None) == binding.ERR_INVALID_ARG
    # the chain hand-off is not offered for compaction; bad shapes as for scans
    chain = binding.Params(0, 0, 0, binding.HANDOFF_CHAIN)
    assert lib.lscan_compact_with_params(FAKE_X, None, FAKE_Y, cnt, 8, binding.I32, ctypes.byref(chain),
                                         None) == binding.ERR_UNSUPPORTED
    bad = binding.Params(192, 3, 1, 0)
    assert lib.lscan_compact_with_params(FAKE_X, None, FAKE_Y, cnt, 8, binding.I32, ctypes.byref(bad),
                                         None) == binding.ERR_UNSUPPORTED


def test_compact_params_kind(lib):
    p = binding.lscan_get_params(binding.F32, binding.MAX, 0, binding.KIND_COMPACT)
    q = binding.lscan_get_params(binding.I32, binding.ADD, 0, binding.KIND_COMPACT)
    assert (p.block_threads, p.vectors_per_lane, p.groups_per_cu) == (q.block_threads, q.vectors_per_lane,
                                                                      q.groups_per_cu)
    with pytest.raises(binding.LscanError):
        binding.lscan_get_params(binding.BF16, binding.ADD, 0, binding.KIND_COMPACT)
    with pytest.raises(binding.LscanError):
        binding.lscan_set_params(binding.I64, binding.ADD, 0, binding.KIND_COMPACT,
                                 binding.Params(q.block_threads, q.vectors_per_lane, 1, binding.HANDOFF_CHAIN))


def test_radix_offsets_validation(lib):
    off = FAKE_Y
    f = lib.lscan_radix_offsets
    assert f(FAKE_X, 8, binding.BF16, 0, 8, 4, off, None) == binding.ERR_UNSUPPORTED
    assert f(FAKE_X, 8, 7, 0, 8, 4, off, None) == binding.ERR_INVALID_ARG
    for shift, bits in ((0, 0), (0, 9), (-1, 4), (25, 8), (28, 5)):
        assert f(FAKE_X, 8, binding.I32, shift, bits, 4, off, None) == binding.ERR_INVALID_ARG, (shift, bits)
    assert f(FAKE_X, 8, binding.I32, 0, 8, 0, off, None) == binding.ERR_INVALID_ARG
    assert f(FAKE_X, -1, binding.I32, 0, 8, 4, off, None) == binding.ERR_INVALID_ARG
    assert f(FAKE_X + 2, 8, binding.I32, 0, 8, 4, off, None) == binding.ERR_INVALID_ARG
    assert f(FAKE_X, 8, binding.I32, 0, 8, 4, off + 4, None) == binding.ERR_INVALID_ARG
    assert f(FAKE_X, 8, binding.I32, 0, 8, 4, None, None) == binding.ERR_INVALID_ARG
    # offsets over the keys
    assert f(FAKE_X, 1024, binding.I32, 0, 8, 64, FAKE_X + 64, None) == binding.ERR_INVALID_ARG
    # nothing to do
    assert f(None, 0, binding.I32, 0, 8, 4, None, None) == binding.OK


def test_argscan_validation(lib):
    f = lib.lscan_inclusive
    assert f(FAKE_X, FAKE_Y, 8, binding.BF16, binding.ARGMAX, 0, None) == binding.ERR_UNSUPPORTED
    assert f(FAKE_X, FAKE_Y, 8, binding.F32, binding.ARGMIN, binding.F_COMPENSATED, None) == binding.ERR_UNSUPPORTED
    assert f(FAKE_X, FAKE_Y, 8, binding.I32, 5, 0, None) == binding.ERR_INVALID_ARG
    # int64 indices may not share memory with the int32 keys, not even exactly
    assert f(FAKE_X, FAKE_X, 8, binding.I32, binding.ARGMAX, 0, None) == binding.ERR_INVALID_ARG
    # y must be 8-byte aligned for the indices
    assert f(FAKE_X, FAKE_Y + 4, 8, binding.I32, binding.ARGMAX, 0, None) == binding.ERR_INVALID_ARG
    # plain scans only
    assert lib.lscan_segmented(FAKE_X, FAKE_Y, 8, FAKE_X, 1, binding.I32, binding.ARGMAX, 0,
                               None) == binding.ERR_UNSUPPORTED
    tab = (binding.Array * 1)(binding.Array(FAKE_X, FAKE_Y, 8))
    assert lib.lscan_batched(tab, 1, binding.I32, binding.ARGMIN, 0, None) == binding.ERR_UNSUPPORTED



def test_bfs_validation(lib):
    f = lib.lscan_bfs
    row, col, lev, par, st = FAKE_X, FAKE_X + (1 << 16), FAKE_Y, FAKE_Y + (1 << 16), FAKE_Y + (1 << 17)
    ok_args = dict(row=row, col=col, nv=100, ne=400, src=0, lev=lev, par=par, st=st)

    def call(**kw):
        a = dict(ok_args, **kw)
        return f(a["row"], a["col"], a["nv"], a["ne"], a["src"], a["lev"], a["par"], a["st"], None)

    assert call(nv=-1) == binding.ERR_INVALID_ARG
    assert call(nv=1 << 31) == binding.ERR_INVALID_ARG        # vertex ids are int32
    assert call(ne=-1) == binding.ERR_INVALID_ARG
    assert call(src=-1) == binding.ERR_INVALID_ARG
    assert call(src=100) == binding.ERR_INVALID_ARG
    assert call(row=None) == binding.ERR_INVALID_ARG
    assert call(col=None) == binding.ERR_INVALID_ARG            # edges but no columns
    assert call(lev=None) == binding.ERR_INVALID_ARG
    assert call(row=row + 4) == binding.ERR_INVALID_ARG          # int64 offsets: 8-byte aligned
    assert call(col=col + 2) == binding.ERR_INVALID_ARG
    assert call(lev=lev + 2) == binding.ERR_INVALID_ARG
    assert call(par=par + 1) == binding.ERR_INVALID_ARG
    assert call(st=st + 4) == binding.ERR_INVALID_ARG
    # outputs over inputs or over each other
    assert call(lev=row + 64) == binding.ERR_INVALID_ARG
    assert call(lev=col + 64) == binding.ERR_INVALID_ARG
    assert call(par=lev + 200) == binding.ERR_INVALID_ARG
    assert call(st=lev + 8) == binding.ERR_INVALID_ARG
    # nothing to do: no vertices and no stats
    assert call(nv=0, ne=0, src=0, st=None) == binding.OK
    # parameters: only groups_per_cu applies
    g = lib.lscan_bfs_with_params
    for p, status in ((binding.Params(256, 8, 0, 0), binding.ERR_UNSUPPORTED),
                      (binding.Params(0, 0, 0, binding.HANDOFF_CHAIN), binding.ERR_UNSUPPORTED),
                      (binding.Params(0, 0, -1, 0), binding.ERR_INVALID_ARG),
                      (binding.Params(0, 0, 0, 7), binding.ERR_INVALID_ARG)):
        assert g(row, col, 100, 400, 0, lev, par, st, ctypes.byref(p), None) == status, p


def test_custom_scan_validation(lib):
    kernels = binding.affine_example_kernels()
    k = kernels["default"]
    f = lib.lscan_scan_custom
    assert f(None, FAKE_X, FAKE_Y, 8, 0, None, None) == binding.ERR_INVALID_ARG
    bogus = (ctypes.c_char * 256)()       # not an entry made by lscan_custom.hpp
    assert f(ctypes.addressof(bogus), FAKE_X, FAKE_Y, 8, 0, None, None) == binding.ERR_INVALID_ARG
    assert f(k, FAKE_X, FAKE_Y, -1, 0, None, None) == binding.ERR_INVALID_ARG
    assert f(k, FAKE_X, FAKE_Y, 8, binding.F_COMPENSATED, None, None) == binding.ERR_INVALID_ARG
    assert f(k, None, FAKE_Y, 8, 0, None, None) == binding.ERR_INVALID_ARG
    assert f(k, FAKE_X + 4, FAKE_Y, 8, 0, None, None) == binding.ERR_INVALID_ARG   # 8-byte elements
    assert f(k, FAKE_X, FAKE_Y + 4, 8, 0, None, None) == binding.ERR_INVALID_ARG
    assert f(k, FAKE_X, FAKE_X + 8, 8, 0, None, None) == binding.ERR_INVALID_ARG   # partial overlap
    p = binding.Params(256, 8, 0, 0)
    assert f(k, FAKE_X, FAKE_Y, 8, 0, ctypes.byref(p), None) == binding.ERR_UNSUPPORTED
    p = binding.Params(0, 0, -1, 0)
    assert f(k, FAKE_X, FAKE_Y, 8, 0, ctypes.byref(p), None) == binding.ERR_INVALID_ARG
    assert f(k, None, None, 0, 0, None, None) == binding.OK                        # nothing to do
    # the three example shapes are distinct kernels
    assert len({kernels["default"], kernels["small"], kernels["wide"]}) == 3
    # a handle built against another layout of the headers: its layout tag
    # (the first 32-bit word) keeps the mark but not the revision
    copy = (ctypes.c_char * 56)()
    ctypes.memmove(copy, k, 56)
    tag = ctypes.c_uint32.from_buffer(copy)
    assert tag.value >> 16 == 0x4C53
    tag.value ^= 0x1
    assert f(ctypes.addressof(copy), FAKE_X, FAKE_Y, 8, 0, None, None) == binding.ERR_UNSUPPORTED
    tag.value = 0
    assert f(ctypes.addressof(copy), FAKE_X, FAKE_Y, 8, 0, None, None) == binding.ERR_INVALID_ARG


def test_watchdog_setter(lib):
    default = lib.lscan_get_watchdog_us()
    assert default == 2_000_000
    assert lib.lscan_set_watchdog_us(-5) == binding.ERR_INVALID_ARG
    assert lib.lscan_set_watchdog_us(3_600_000_001) == binding.ERR_INVALID_ARG
    assert lib.lscan_set_watchdog_us(1234) == binding.OK
    assert lib.lscan_get_watchdog_us() == 1234
    assert lib.lscan_set_watchdog_us(default) == binding.OK
    assert lib.lscan_get_watchdog_us() == default


def test_index64_flag_validation(lib):
    f = lib.lscan_inclusive
    # only the running argmax / argmin take it
    assert f(FAKE_X, FAKE_Y, 8, binding.I32, binding.ADD, binding.F_INDEX64, None) == binding.ERR_INVALID_ARG
    assert f(FAKE_X, FAKE_Y, 8, binding.F32, binding.MAX, binding.F_INDEX64, None) == binding.ERR_INVALID_ARG
    # not for segmented scans
    assert lib.lscan_segmented(FAKE_X, FAKE_Y, 8, FAKE_X, 1, binding.I32, binding.ARGMAX, binding.F_INDEX64,
                               None) == binding.ERR_INVALID_ARG
    # an argmax with the flag and nothing to do is accepted
    assert f(None, None, 0, binding.I32, binding.ARGMAX, binding.F_INDEX64, None) == binding.OK


def test_epoch_test_hooks_validation(lib):
    # include/lscan_testing.h: the limit, and the null-graph checks made
    # before any device call
    assert lib.lscan_test_epoch_limit() == 0xFFFFFFF0
    assert lib.lscan_test_graph_seed_epoch(None, 0, 0, 0) == binding.ERR_INVALID_ARG
    n = ctypes.c_uint64()
    ctrl = (ctypes.c_uint32 * 4)()
    assert lib.lscan_test_graph_epoch_state(None, ctypes.byref(n), ctrl) == binding.ERR_INVALID_ARG


def test_noalloc_size_limit_before_device_work(lib):
    # lscan_inclusive_noalloc refuses scans whose flag words would not fit
    # its static array, from host data alone (these pointers are never read)
    x, y = 0x1000_0000_0000, 0x3000_0000_0000
    assert lib.lscan_inclusive_noalloc(x, y, 1 << 34, binding.I32, binding.ADD, 0, None) == binding.ERR_NO_MEMORY
    assert lib.lscan_inclusive_noalloc(x, y, 1 << 31, binding.I32, binding.ARGMAX, 0, None) == binding.ERR_NO_MEMORY
    # argument checks come first, as for lscan_inclusive
    assert lib.lscan_inclusive_noalloc(x, y, -1, binding.I32, binding.ADD, 0, None) == binding.ERR_INVALID_ARG
    assert lib.lscan_inclusive_noalloc(x, y, 4, binding.I32, binding.MAX, binding.F_COMPENSATED, None) == \
        binding.ERR_UNSUPPORTED
    assert lib.lscan_inclusive_noalloc(None, None, 0, binding.I32, binding.ADD, 0, None) == binding.OK


def test_array_table_built_once():
    """A batch's descriptor table built once (what repeated launches of one
    batch pass) holds every array's pointers and length in order."""
    from paper_1604_04815_amd import binding
    rows = [(0x1000, 0x2000, 5), (0x3010, 0x4020, 0), (0x5000, 0x6000, 1 << 33)]
    t = binding.array_table(rows)
    assert len(t) == 3
    p = t._as_parameter_
    assert [(p[i].x, p[i].y, p[i].n) for i in range(3)] == rows
