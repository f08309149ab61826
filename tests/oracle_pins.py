"""Pins of the CPU oracle: checks against what the paper and mathematics fix.

Each check takes an ``Oracle`` (a compiled oracle library) and raises
``AssertionError`` on a mismatch.  ``tests/test_oracle.py`` runs them on the
real oracle; ``tests/test_oracle_mutants.py`` runs them on copies of the
oracle with planted mistakes and requires every mutant to fail one.

The expected values never come from the oracle itself: they are hand-worked
fixtures (``tests/golden``), closed forms, brute force over Python integers
and ``math.fsum``, and numpy library routines.
"""
from __future__ import annotations

import functools
import math
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "scan_small.txt")

NP_OF = {"int32": np.int32, "int64": np.int64, "float32": np.float32}


def wrap(v: int, bits: int) -> int:
    """Two's complement wrap of a Python integer to ``bits`` bits."""
    m = 1 << bits
    v %= m
    return v - m if v >= m // 2 else v


# --------------------------------------------------------------------------
# golden fixtures
# --------------------------------------------------------------------------

def load_golden():
    cases = []
    with open(GOLDEN) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            parts = [p.strip() for p in line.split("|")]
            name, dtype, op, kind = parts[:4]
            if kind.startswith("seg"):
                off = [int(v) for v in parts[4].split()]
                xs, ys = parts[5].split(), parts[6].split()
            else:
                off = None
                xs, ys = parts[4].split(), parts[5].split()
            conv = float if dtype == "float32" else int
            cases.append(dict(name=name, dtype=dtype, op=op, kind=kind, off=off,
                              x=[conv(v) for v in xs], y=[conv(v) for v in ys]))
    return cases


def check_golden(orc):
    for c in load_golden():
        x = np.array(c["x"], dtype=NP_OF[c["dtype"]])
        excl = c["kind"].endswith("excl")
        if c["off"] is not None:
            y = orc.segscan(x, np.array(c["off"], dtype=np.int64), c["dtype"], c["op"], excl)
        else:
            y = orc.scan(x, c["dtype"], c["op"], excl)
        want = c["y"]
        if c["dtype"] == "float32":
            got = [float(v) for v in y]
            assert all(g == w and math.copysign(1, g) == math.copysign(1, w)
                       for g, w in zip(got, want)), (c["name"], got, want)
        else:
            assert [int(v) for v in y] == want, (c["name"], list(y), want)


# --------------------------------------------------------------------------
# closed forms
# --------------------------------------------------------------------------

def check_closed_forms(orc):
    n = 1 << 17                                   # crosses the int32 wrap of j(j+1)/2
    j = np.arange(n, dtype=np.int64)
    ones32 = np.ones(n, dtype=np.int32)
    assert np.array_equal(orc.scan(ones32, "int32", "add"), (j + 1).astype(np.int32))
    assert np.array_equal(orc.scan(ones32, "int32", "add", exclusive=True), j.astype(np.int32))
    assert np.array_equal(orc.scan(np.ones(n, np.int64), "int64", "add"), j + 1)

    # x_i = i  ->  y_j = j (j + 1) / 2, modulo 2^32 for int32
    tri = [wrap(k * (k + 1) // 2, 32) for k in range(0, n, 997)]
    got = orc.scan(j.astype(np.int32), "int32", "add")[::997]
    assert [int(v) for v in got] == tri
    got64 = orc.scan(j, "int64", "add")
    assert np.array_equal(got64, j * (j + 1) // 2)

    # monotone inputs: max of increasing is the identity map, of decreasing is x_0
    inc = np.arange(-500, 500, dtype=np.int32)
    dec = inc[::-1].copy()
    assert np.array_equal(orc.scan(inc, "int32", "max"), inc)
    assert np.array_equal(orc.scan(dec, "int32", "max"), np.full_like(dec, dec[0]))
    assert np.array_equal(orc.scan(inc, "int32", "min"), np.full_like(inc, inc[0]))
    assert np.array_equal(orc.scan(dec, "int32", "min"), dec)
    inc64 = np.arange(-(1 << 40), -(1 << 40) + 300, dtype=np.int64)
    assert np.array_equal(orc.scan(inc64, "int64", "max"), inc64)
    assert np.array_equal(orc.scan(inc64[::-1].copy(), "int64", "min"), inc64[::-1])
    incf = np.linspace(-3.0, 7.0, 257, dtype=np.float32)
    assert np.array_equal(orc.scan(incf, "float32", "max"), incf)
    assert np.array_equal(orc.scan(incf, "float32", "min"), np.full_like(incf, incf[0]))

    # float all-ones: exact prefix j + 1, A_j = j + 1
    y64, a = orc.scan(np.ones(n, np.float32), "float32", "add", with_absum=True)
    assert np.array_equal(y64, (j + 1).astype(np.float64))
    assert np.array_equal(a, (j + 1).astype(np.float64))
    # bf16 1.0 = 0x3f80: widened exactly, prefix j + 1
    yb = orc.scan(np.full(n, 0x3F80, np.uint16), "bfloat16", "add")
    assert np.array_equal(yb, (j + 1).astype(np.float64))
    # bf16 max of increasing bit patterns of positive numbers is the identity map
    hb = np.arange(0x3F80, 0x4000, dtype=np.uint16)
    wide = (hb.astype(np.uint32) << 16).view(np.float32)
    assert np.array_equal(orc.scan(hb, "bfloat16", "max"), wide)
    assert np.array_equal(orc.scan(hb, "bfloat16", "min"), np.full_like(wide, wide[0]))


# --------------------------------------------------------------------------
# brute force on tiny inputs
# --------------------------------------------------------------------------

def _total_order_key(v: float):
    """Sort key for IEEE totalOrder on non-NaN floats (-0 before +0)."""
    return (v, math.copysign(1.0, v))


def check_brute_force(orc, seed=7):
    g = np.random.default_rng(seed)
    for n in (0, 1, 2, 3, 17, 63, 64):
        for dtype, bits in (("int32", 32), ("int64", 64)):
            lo, hi = (-(2 ** 31), 2 ** 31) if bits == 32 else (-(2 ** 63), 2 ** 63)
            x = g.integers(lo, hi, size=n, dtype=np.int64 if bits == 64 else np.int64)
            x = x.astype(NP_OF[dtype])
            xs = [int(v) for v in x]
            for op, f, e in (("add", lambda a, b: a + b, 0),
                             ("max", max, -(2 ** (bits - 1))),
                             ("min", min, 2 ** (bits - 1) - 1)):
                want_in = [wrap(functools.reduce(f, xs[: k + 1]), bits) for k in range(n)]
                want_ex = [wrap(functools.reduce(f, xs[:k], e), bits) for k in range(n)]
                assert [int(v) for v in orc.scan(x, dtype, op)] == want_in, (dtype, op, n)
                assert [int(v) for v in orc.scan(x, dtype, op, exclusive=True)] == want_ex, (dtype, op, n)

        # float32 add: exact sum by math.fsum, A_j by fsum of magnitudes
        xf = (g.standard_normal(n) * np.exp(g.uniform(-8, 8, n))).astype(np.float32)
        y64, a = orc.scan(xf, "float32", "add", with_absum=True)
        for k in range(n):
            exact = math.fsum(float(v) for v in xf[: k + 1])
            mag = math.fsum(abs(float(v)) for v in xf[: k + 1])
            assert abs(y64[k] - exact) <= 1e-15 * mag, (k, y64[k], exact)
            assert abs(a[k] - mag) <= 1e-15 * mag
        y64e, ae = orc.scan(xf, "float32", "add", exclusive=True, with_absum=True)
        for k in range(n):
            exact = math.fsum(float(v) for v in xf[:k])
            mag = math.fsum(abs(float(v)) for v in xf[:k])
            assert abs(y64e[k] - exact) <= 1e-15 * mag and abs(ae[k] - mag) <= 1e-15 * mag

        # float32 max / min under totalOrder, with signed zeros and infinities mixed in
        pool = np.array([-0.0, 0.0, 1.5, -1.5, np.inf, -np.inf, 3.0, -7.25], dtype=np.float32)
        xo = pool[g.integers(0, pool.size, n)]
        for op, pick in (("max", max), ("min", min)):
            y = orc.scan(xo, "float32", op)
            for k in range(n):
                want = pick((float(v) for v in xo[: k + 1]), key=_total_order_key)
                assert float(y[k]) == want and math.copysign(1, y[k]) == math.copysign(1, want), (op, k)


# --------------------------------------------------------------------------
# invariants and library special cases on larger random inputs
# --------------------------------------------------------------------------

def check_invariants(orc, seed=11):
    g = np.random.default_rng(seed)
    n = 100_003
    x32 = g.integers(-(2 ** 31), 2 ** 31, size=n, dtype=np.int64).astype(np.int32)
    x64 = g.integers(-(2 ** 63), 2 ** 63, size=n, dtype=np.int64)
    for x, dtype, bits in ((x32, "int32", 32), (x64, "int64", 64)):
        inc = orc.scan(x, dtype, "add")
        exc = orc.scan(x, dtype, "add", exclusive=True)
        # y_{N-1} equals the full reduction (Python integers, wrapped)
        assert int(inc[-1]) == wrap(sum(int(v) for v in x), bits)
        # exclusive is inclusive shifted by one, identity first
        assert exc[0] == 0 and np.array_equal(exc[1:], inc[:-1])
        # numpy's sequential accumulate wraps the same way
        assert np.array_equal(inc, np.add.accumulate(x, dtype=x.dtype))
        assert np.array_equal(orc.scan(x, dtype, "max"), np.maximum.accumulate(x))
        assert np.array_equal(orc.scan(x, dtype, "min"), np.minimum.accumulate(x))
        info = np.iinfo(x.dtype)
        excm = orc.scan(x, dtype, "max", exclusive=True)
        assert excm[0] == info.min and np.array_equal(excm[1:], np.maximum.accumulate(x)[:-1])
        excn = orc.scan(x, dtype, "min", exclusive=True)
        assert excn[0] == info.max and np.array_equal(excn[1:], np.minimum.accumulate(x)[:-1])
        # in-place gives the same bits
        xi = x.copy()
        orc.scan(xi, dtype, "add", out=xi)
        assert np.array_equal(xi, inc)
        xi = x.copy()
        orc.scan(xi, dtype, "add", exclusive=True, out=xi)
        assert np.array_equal(xi, exc)

    # float exactness: small integers as float32 sum exactly in any order
    xi = g.integers(-1000, 1000, size=1 << 14, endpoint=True).astype(np.float32)
    y64 = orc.scan(xi, "float32", "add")
    assert np.array_equal(y64, np.cumsum(xi.astype(np.int64)).astype(np.float64))
    # f32 max/min equals numpy's accumulate for data without zeros
    xf = (g.standard_normal(n) * 100).astype(np.float32)
    xf[xf == 0] = 1.0
    assert np.array_equal(orc.scan(xf, "float32", "max"), np.maximum.accumulate(xf))
    assert np.array_equal(orc.scan(xf, "float32", "min"), np.minimum.accumulate(xf))
    exf = orc.scan(xf, "float32", "max", exclusive=True)
    assert exf[0] == -np.inf and np.array_equal(exf[1:], np.maximum.accumulate(xf)[:-1])
    # float add on random data: within FP64 rounding of math.fsum at sampled points
    y64, a = orc.scan(xf, "float32", "add", with_absum=True)
    for k in (0, 1, 999, 50_000, n - 1):
        exact = math.fsum(float(v) for v in xf[: k + 1])
        assert abs(y64[k] - exact) <= 1e-14 * a[k]
    y64e = orc.scan(xf, "float32", "add", exclusive=True)
    assert y64e[0] == 0.0 and np.array_equal(y64e[1:], y64[:-1])
    # bf16 add equals the float32 add of the widened values, bit for bit
    hb = g.integers(0, 1 << 16, size=4096, dtype=np.uint16)
    hb = hb[((hb >> 7) & 0xFF) != 0xFF]            # drop inf / nan patterns
    wide = (hb.astype(np.uint32) << 16).view(np.float32)
    yb, ab = orc.scan(hb, "bfloat16", "add", with_absum=True)
    yf, af = orc.scan(wide, "float32", "add", with_absum=True)
    assert np.array_equal(yb, yf) and np.array_equal(ab, af)


# --------------------------------------------------------------------------
# compensated-sum pin: cancellation pattern with an exact answer
# --------------------------------------------------------------------------

def check_cancellation(orc):
    big = float(2 ** 24)
    x = np.array([big, 1.0, -big, 1.0] * 256, dtype=np.float32)
    y64, a = orc.scan(x, "float32", "add", with_absum=True)
    want = []
    s = 0
    for v in x:
        s += int(v)
        want.append(float(s))
    assert np.array_equal(y64, np.array(want))
    assert a[-1] == 256 * (2 * big + 2)
    # The same pattern at 2^60 defeats a plain FP64 fold (2^60 + 1 rounds to
    # 2^60, so 2^60 + 1 - 2^60 would give 0): only a compensated fold returns
    # the exact small prefixes.  Expected: the exact integer prefix, rounded
    # once to FP64 by Python's correctly rounded int -> float conversion.
    huge = float(2 ** 60)
    x = np.array([huge, 1.0, -huge, 1.0] * 64, dtype=np.float32)
    y64 = orc.scan(x, "float32", "add")
    s = 0
    for k, v in enumerate(x):
        s += int(v)
        assert y64[k] == float(s), (k, y64[k], s)


# --------------------------------------------------------------------------
# segmented scan
# --------------------------------------------------------------------------

def check_segmented(orc, seed=13):
    g = np.random.default_rng(seed)
    n = 5000
    x = g.integers(-1000, 1000, size=n, endpoint=True).astype(np.int32)
    # one segment == plain scan
    off1 = np.array([0, n], dtype=np.int64)
    for op in ("add", "max", "min"):
        assert np.array_equal(orc.segscan(x, off1, "int32", op), orc.scan(x, "int32", op))
    # all segments of length one: inclusive gives x, exclusive gives the identity
    offs = np.arange(n + 1, dtype=np.int64)
    assert np.array_equal(orc.segscan(x, offs, "int32", "add"), x)
    assert np.array_equal(orc.segscan(x, offs, "int32", "add", exclusive=True), np.zeros(n, np.int32))
    assert np.array_equal(orc.segscan(x, offs, "int32", "max", exclusive=True),
                          np.full(n, np.iinfo(np.int32).min, np.int32))
    # random segments with empty ones, against a per-segment Python fold
    cuts = np.sort(g.integers(0, n + 1, size=60))
    off = np.concatenate([[0], cuts, cuts[:5], [n]]).astype(np.int64)
    off.sort()
    for op, f in (("add", lambda a, b: a + b), ("max", max), ("min", min)):
        got = orc.segscan(x, off, "int32", op)
        gote = orc.segscan(x, off, "int32", op, exclusive=True)
        e = {"add": 0, "max": -(2 ** 31), "min": 2 ** 31 - 1}[op]
        want, wante = [], []
        for s in range(off.size - 1):
            acc = e
            for v in x[off[s]:off[s + 1]]:
                wante.append(acc)
                acc = f(acc, int(v))
                want.append(acc)
        assert [int(v) for v in got] == want, op
        assert [int(v) for v in gote] == wante, op
    # float add per segment: restarts the sum and the magnitude sum
    xf = g.random(n).astype(np.float32)
    y64, a = orc.segscan(xf, off, "float32", "add", with_absum=True)
    for s in range(off.size - 1):
        lo, hi = off[s], off[s + 1]
        if hi > lo:
            assert abs(y64[hi - 1] - math.fsum(float(v) for v in xf[lo:hi])) <= 1e-14 * a[hi - 1]
            assert a[lo] == abs(float(xf[lo]))


def check_compact(orc, seed=17):
    """Stream compaction against closed forms and numpy's boolean indexing."""
    g = np.random.default_rng(seed)
    n = 1000
    for dt in (np.int32, np.int64, np.float32, np.uint16):
        x = g.integers(1, 1 << 15, n).astype(dt)
        # closed forms: keep everything / nothing / every other element
        assert np.array_equal(orc.compact(x, np.ones(n, np.uint8)), x), dt
        assert orc.compact(x, np.zeros(n, np.uint8)).shape[0] == 0, dt
        alt = (np.arange(n) % 2 == 0).astype(np.uint8)
        assert np.array_equal(orc.compact(x, alt), x[0::2]), dt
        # random flags (any non-zero byte keeps): numpy boolean indexing
        keep = g.integers(0, 4, n).astype(np.uint8)
        assert np.array_equal(orc.compact(x, keep), x[keep != 0]), dt
    # distinct values 0..n-1: the kept values are the kept indices, in order
    idx = np.arange(n, dtype=np.int64)
    keep = (g.random(n) < 0.3).astype(np.uint8)
    assert np.array_equal(orc.compact(idx, keep), np.flatnonzero(keep))
    # no flags: keep the elements whose bits are not all zero (-0.0 is kept)
    xf = np.array([0.0, -0.0, 1.5, 0.0, -2.0, 0.0], dtype=np.float32)
    assert np.array_equal(orc.compact(xf).view(np.uint32), np.array([-0.0, 1.5, -2.0], np.float32).view(np.uint32))
    xi = g.integers(-3, 4, n).astype(np.int64)
    assert np.array_equal(orc.compact(xi), xi[xi != 0])
    # empty input
    assert orc.compact(np.zeros(0, np.int32), np.zeros(0, np.uint8)).shape[0] == 0


def check_radix_offsets(orc, seed=19):
    """Digit offsets against numpy (bincount per block, cumulative sums) and
    against a stable sort by digit that uses them."""
    g = np.random.default_rng(seed)
    for dt, kb in ((np.uint32, 32), (np.uint64, 64)):
        n, blk = 5000, 384
        keys = g.integers(0, 1 << 62, n, dtype=np.uint64).astype(dt)
        for shift, bits in ((0, 8), (kb - 8, 8), (3, 1), (kb - 5, 5)):
            off = orc.radix_offsets(keys, shift, bits, blk)
            nd, m = 1 << bits, (n + blk - 1) // blk
            assert off.shape == (nd, m)
            dig = ((keys.astype(np.uint64) >> np.uint64(shift)) & np.uint64(nd - 1)).astype(np.int64)
            counts = np.zeros((nd, m), np.int64)
            for b in range(m):
                counts[:, b] = np.bincount(dig[b * blk:(b + 1) * blk], minlength=nd)
            flat = counts.reshape(-1)
            want = np.concatenate([[0], np.cumsum(flat)[:-1]]).reshape(nd, m)
            assert np.array_equal(off, want), (dt, shift, bits)
            # placing every key at its block's offset for its digit, then one
            # past the previous key of the same digit and block, is a stable
            # sort by digit
            pos = np.empty(n, np.int64)
            nxt = off.copy()
            for i in range(n):
                d, b = dig[i], i // blk
                pos[i] = nxt[d, b]
                nxt[d, b] += 1
            placed = np.empty_like(keys)
            placed[pos] = keys
            assert np.array_equal(placed, keys[np.argsort(dig, kind="stable")]), (dt, shift, bits)
    # closed forms: all keys equal -> one digit takes block offsets b * blk
    keys = np.full(1000, 0xAB, np.uint32)
    off = orc.radix_offsets(keys, 0, 8, 100)
    assert np.array_equal(off[0xAB], np.arange(10) * 100)
    assert np.all(off[:0xAB] == 0) and np.all(off[0xAB + 1:] == 1000)
    # empty input
    assert orc.radix_offsets(np.zeros(0, np.uint32), 0, 4, 64).shape == (16, 0)


def check_argscan(orc, seed=23):
    """Running argmax / argmin against closed forms, brute force over the
    prefixes (Python max / min with the earliest index) and numpy."""
    g = np.random.default_rng(seed)
    n = 40
    # closed forms: increasing -> j (argmax) / 0 (argmin); constant -> 0
    inc = np.arange(n, dtype=np.int32)
    assert np.array_equal(orc.argscan(inc, "int32", "argmax"), np.arange(n))
    assert np.array_equal(orc.argscan(inc, "int32", "argmin"), np.zeros(n, np.int64))
    assert np.array_equal(orc.argscan(np.full(n, 5, np.int64), "int64", "argmax"), np.zeros(n, np.int64))
    excl = orc.argscan(inc, "int32", "argmax", exclusive=True)
    assert excl[0] == -1 and np.array_equal(excl[1:], np.arange(n - 1))
    for dtype in ("int32", "int64", "float32"):
        if dtype == "float32":
            x = g.choice(np.array([-1.5, -0.0, 0.0, 2.0, 2.0, 7.25], np.float32), n)
            key = lambda v: (float(v), math.copysign(1.0, float(v)))  # totalOrder on non-NaN: -0 < +0
        else:
            x = g.integers(-4, 5, n).astype(NP_OF[dtype])
            key = lambda v: int(v)
        for op in ("argmax", "argmin"):
            got = orc.argscan(x, dtype, op)
            gote = orc.argscan(x, dtype, op, exclusive=True)
            pick = max if op == "argmax" else min
            for j in range(n):
                best = pick(range(j + 1), key=lambda i: (key(x[i]), -i if op == "argmax" else i))
                assert got[j] == best, (dtype, op, j)
                assert gote[j] == (got[j - 1] if j else -1), (dtype, op, j)
    # numpy: the value at the running argmax is the running maximum
    x = g.integers(-1000, 1000, 5000).astype(np.int32)
    idx = orc.argscan(x, "int32", "argmax")
    assert np.array_equal(x[idx], np.maximum.accumulate(x))
    first = np.array([np.flatnonzero(x[:j + 1] == m)[0] for j, m in enumerate(np.maximum.accumulate(x[:300]))])
    assert np.array_equal(idx[:300], first)


def check_affine(orc, seed=29):
    """Composition of affine maps mod 2^32: the special cases that reduce to
    numpy's running sum and product, the linear recurrence evaluated by brute
    force with Python integers (which pins the order of composition: the
    operator is not commutative), and the exclusive shift."""
    g = np.random.default_rng(seed)
    M = 1 << 32
    n = 3000
    # a = 1: x -> x + b, the prefixes are running sums of b
    ab = np.stack([np.ones(n, np.uint32), g.integers(0, M, n, dtype=np.uint64).astype(np.uint32)], 1)
    out = orc.affine_scan(ab)
    assert np.all(out[:, 0] == 1)
    assert np.array_equal(out[:, 1], np.cumsum(ab[:, 1].astype(np.uint64)).astype(np.uint32))
    # b = 0: x -> a * x, the prefixes are running products of a
    ab = np.stack([g.integers(0, M, n, dtype=np.uint64).astype(np.uint32), np.zeros(n, np.uint32)], 1)
    out = orc.affine_scan(ab)
    assert np.all(out[:, 1] == 0)
    prod, want = 1, []
    for a in ab[:, 0].tolist():
        prod = (prod * a) % M
        want.append(prod)
    assert out[:, 0].tolist() == want
    # general maps: prefix j applied to x equals the recurrence run from x
    n = 60
    ab = g.integers(0, M, (n, 2), dtype=np.uint64).astype(np.uint32)
    ab[::7, 0] = 0              # maps that forget their argument
    ab[3::11, 0] = 0xFFFFFFFF   # -1 mod 2^32
    out = orc.affine_scan(ab)
    excl = orc.affine_scan(ab, exclusive=True)
    for x0 in (0, 1, 12345, M - 1):
        h = x0
        for j in range(n):
            h = (int(ab[j, 0]) * h + int(ab[j, 1])) % M
            assert (int(out[j, 0]) * x0 + int(out[j, 1])) % M == h, (x0, j)
    assert excl[0].tolist() == [1, 0]
    assert np.array_equal(excl[1:], out[:-1])
    assert orc.affine_scan(np.zeros((0, 2), np.uint32)).shape == (0, 2)


def _csr(n, edges):
    edges = sorted(edges)
    row_ptr = np.zeros(n + 1, np.int64)
    for u, _ in edges:
        row_ptr[u + 1] += 1
    return np.cumsum(row_ptr), np.array([v for _, v in edges], np.int32)


def check_bfs(orc, seed=29):
    """BFS levels against closed forms (path, star, cycle, two components)
    and a Floyd-Warshall all-pairs shortest-path table on small random graphs."""
    # path 0 -> 1 -> ... -> 9: level = index; reversed source: only itself
    rp, c = _csr(10, [(i, i + 1) for i in range(9)])
    assert np.array_equal(orc.bfs_levels(rp, c, 0), np.arange(10))
    lv = orc.bfs_levels(rp, c, 9)
    assert lv[9] == 0 and np.all(lv[:9] == -1)
    # star from 0: everything at level 1
    rp, c = _csr(50, [(0, v) for v in range(1, 50)])
    assert np.array_equal(orc.bfs_levels(rp, c, 0), np.array([0] + [1] * 49))
    # undirected cycle of 12: level = min(i, 12 - i)
    ed = [(i, (i + 1) % 12) for i in range(12)] + [((i + 1) % 12, i) for i in range(12)]
    rp, c = _csr(12, ed)
    assert np.array_equal(orc.bfs_levels(rp, c, 0), np.array([min(i, 12 - i) for i in range(12)]))
    # random directed graphs against Floyd-Warshall on hop counts
    g = np.random.default_rng(seed)
    for n, m in ((30, 60), (40, 200), (25, 20)):
        ed = set()
        while len(ed) < m:
            u, v = (int(t) for t in g.integers(0, n, 2))
            if u != v:
                ed.add((u, v))
        rp, c = _csr(n, list(ed))
        inf = 10 ** 9
        d = np.full((n, n), inf, np.int64)
        np.fill_diagonal(d, 0)
        for u, v in ed:
            d[u, v] = 1
        for k in range(n):
            d = np.minimum(d, d[:, k:k + 1] + d[k:k + 1, :])
        for s in (0, n // 2):
            want = np.where(d[s] >= inf, -1, d[s])
            assert np.array_equal(orc.bfs_levels(rp, c, s), want), (n, m, s)


ALL_CHECKS = (check_golden, check_closed_forms, check_brute_force, check_invariants,
              check_cancellation, check_segmented, check_compact, check_radix_offsets, check_argscan,
              check_affine, check_bfs)


def failing_checks(orc):
    """Names of the pin checks that fail (or crash) on ``orc``."""
    bad = []
    for chk in ALL_CHECKS:
        try:
            chk(orc)
        except Exception as exc:  # noqa: BLE001 - a crash counts as a failure
            bad.append(f"{chk.__name__}: {type(exc).__name__}")
    return bad
