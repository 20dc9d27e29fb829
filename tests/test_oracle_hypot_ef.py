"""Pins of the oracle's primitives (Sect. 2) against exact integer references.

* correctly rounded hypot: exact integer square roots (tests/exact_ref.py),
  random pairs at every exponent gap, subnormals, exact Pythagorean midpoints
  (ties), Lemma nu and its corollaries;
* (e,f) operations (eqs. plus, minus, unary, binary, prec) against exact rational
  arithmetic with one rounding and an unbounded exponent range; Lemma minus by an
  exhaustive sweep over exponent pairs.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

from exact_ref import F32, F64, exact_hypot, fmt_of, frac, rn_unbounded, ef_value

DTYPES = [np.float64, np.float32]


def _rand_pairs(rng, n, dtype, gap_max=64):
    p, emin, emax = fmt_of(dtype)
    e1 = rng.integers(emin - p + 1, emax + 1, n)
    gap = rng.integers(0, gap_max, n)
    e2 = np.maximum(e1 - gap, emin - p + 1)
    m1 = 1 + rng.random(n)
    m2 = 1 + rng.random(n)
    x = np.ldexp(m1, e1).astype(dtype)
    y = np.ldexp(m2, e2).astype(dtype)
    return x, y


@pytest.mark.parametrize("dtype", DTYPES)
def test_hypot_random_exponent_gaps(orc, dtype):
    rng = np.random.default_rng(123)
    x, y = _rand_pairs(rng, 4000, dtype)
    sx = np.where(rng.random(x.size) < 0.5, -1, 1).astype(dtype)
    got = orc.hypot(x * sx, y)
    for i in range(x.size):
        want = exact_hypot(x[i], y[i], dtype)
        assert got[i] == want, (x[i], y[i], got[i], want)


@pytest.mark.parametrize("dtype", DTYPES)
def test_hypot_subnormal_and_overflow(orc, dtype):
    f = np.finfo(dtype)
    tiny = f.smallest_subnormal
    rng = np.random.default_rng(5)
    ks = rng.integers(1, 1 << (f.nmant), 500)
    x = (ks * np.float64(tiny)).astype(dtype)
    y = (rng.integers(1, 1 << (f.nmant), 500) * np.float64(tiny)).astype(dtype)
    got = orc.hypot(x, y)
    for i in range(x.size):
        assert got[i] == exact_hypot(x[i], y[i], dtype)
    # overflow boundary: hypot(nu, nu) overflows, hypot(nu/2, nu/2) does not
    big = np.array([f.max, f.max / 2, f.max / 4 * 3], dtype)
    got = orc.hypot(big, big)
    for i in range(3):
        assert got[i] == exact_hypot(big[i], big[i], dtype)
    assert np.isinf(got[0]) and np.isfinite(got[1])


def _pythagorean_midpoints(p, count, rng):
    """Triples (a, b, m) with a^2 + b^2 = m^2, a, b < 2^p and m an odd (p+1)-bit integer:
    sqrt is exactly halfway between two p-bit neighbours (a tie)."""
    out = []
    lo = int(math.isqrt(1 << (p - 1)))
    hi = int(math.isqrt(1 << p))
    while len(out) < count:
        u = int(rng.integers(lo, hi))
        v = int(rng.integers(1, u))
        if (u - v) % 2 == 0 or math.gcd(u, v) != 1:
            continue
        a, b, m = u * u - v * v, 2 * u * v, u * u + v * v
        if m.bit_length() == p + 1 and m % 2 == 1 and a < (1 << p) and b < (1 << p):
            out.append((a, b, m))
    return out


@pytest.mark.parametrize("dtype", DTYPES)
def test_hypot_exact_ties(orc, dtype):
    p = fmt_of(dtype)[0]
    rng = np.random.default_rng(7)
    trip = _pythagorean_midpoints(p, 200, rng)
    for sc in (0, -40, 60):
        a = np.array([np.ldexp(t[0], sc) for t in trip], dtype)
        b = np.array([np.ldexp(t[1], sc) for t in trip], dtype)
        got = orc.hypot(a, b)
        for i, (_, _, m) in enumerate(trip):
            # tie between m-1 and m+1 (both even): the even significand wins
            lo, hi = m - 1, m + 1
            want = lo if (lo // 2) % 2 == 0 else hi
            assert got[i] == np.ldexp(float(want), sc), (trip[i], got[i])
            assert got[i] == exact_hypot(a[i], b[i], dtype)


@pytest.mark.parametrize("dtype", DTYPES)
def test_lemma_nu_and_corollaries(orc, dtype):
    f = np.finfo(dtype)
    nu = f.max
    one = dtype(1)
    # Lemma nu: fl(nu + 1) = nu = hypot(nu, 1)
    assert dtype(nu + one) == nu
    assert orc.hypot(np.array([nu], dtype), np.array([1], dtype))[0] == nu
    # Cor. tf: |tan phi| <= 1 for finite tan(2 phi), including tan(2 phi) = nu
    t2 = np.array([nu, -nu, 1e30, 1.0, 1e-30, f.smallest_subnormal], dtype)
    h = orc.hypot(t2, np.ones_like(t2))
    tphi = t2 / (one + h)
    assert np.all(np.abs(tphi) <= 1)
    # Cor. sec: sec = hypot(tan, 1) is finite for finite tan, exact sec for exact tan
    assert np.all(np.isfinite(h))
    tt = np.array([0.75], dtype)  # tan = 3/4 -> sec = 5/4 exactly
    assert orc.hypot(tt, np.ones_like(tt))[0] == dtype(1.25)


@pytest.mark.parametrize("dtype", DTYPES)
def test_hypot_symmetry_monotone_zero(orc, dtype):
    rng = np.random.default_rng(9)
    x, y = _rand_pairs(rng, 2000, dtype, gap_max=8)
    a = orc.hypot(x, y)
    assert np.array_equal(a, orc.hypot(y, x))
    assert np.array_equal(a, orc.hypot(-x, -y))
    bigger = np.nextafter(x, np.array(np.inf, dtype))
    assert np.all(orc.hypot(bigger, y) >= a)
    z = np.zeros(3, dtype)
    assert np.all(orc.hypot(z, z) == 0)
    assert np.all(orc.hypot(np.array([0, 1e-30, 0], dtype), np.array([1e-30, 0, -2], dtype)) > 0)


# ---------------------------------------------------------------- (e,f) ops

def _ef_check(e, f, want: Fraction, p):
    if want == 0:
        assert (e, float(f)) == (0, 0.0)
        return
    assert 1 <= abs(float(f)) < 2, f
    assert ef_value(e, f) == want


@pytest.mark.parametrize("dtype", DTYPES)
def test_ef_mul_div_exact(orc, dtype):
    p = fmt_of(dtype)[0]
    rng = np.random.default_rng(11)
    x, y = _rand_pairs(rng, 1500, dtype, gap_max=400)
    for i in range(x.size):
        xi, yi = x[i], y[i]
        e, f = orc.ef_op("mul", xi, yi, dtype)
        _ef_check(e, f, rn_unbounded(frac(xi) * frac(yi), p), p)
        e, f = orc.ef_op("div", xi, yi, dtype)
        _ef_check(e, f, rn_unbounded(frac(xi) / frac(yi), p), p)


@pytest.mark.parametrize("dtype", DTYPES)
def test_ef_plus_never_overflows(orc, dtype):
    p = fmt_of(dtype)[0]
    f = np.finfo(dtype)
    rng = np.random.default_rng(12)
    xs = np.concatenate([(f.max * (0.5 + 0.5 * rng.random(300))).astype(dtype),
                         _rand_pairs(rng, 300, dtype)[0]])
    ys = np.concatenate([(f.max * (0.5 + 0.5 * rng.random(300))).astype(dtype),
                         _rand_pairs(rng, 300, dtype)[1]])
    for xi, yi in zip(np.abs(xs), np.abs(ys)):
        e, fv = orc.ef_op("plus", xi, yi, dtype)
        _ef_check(e, fv, rn_unbounded(frac(xi) + frac(yi), p), p)
        assert np.isfinite(fv)


@pytest.mark.parametrize("dtype", DTYPES)
def test_lemma_minus_exhaustive_exponents(orc, dtype):
    """Lemma minus: x (-) y never underflows; its value is the exact x - y rounded once."""
    p, emin, emax = fmt_of(dtype)
    rng = np.random.default_rng(13)
    # every exponent of x in a band over the subnormal/normal boundary, paired with every
    # y within p+2 binades below (where the difference can be small)
    for ex in range(emin - p + 1, emin + 3 * p, 3 if dtype == np.float64 else 1):
        for gap in range(0, p + 3):
            ey = ex - gap
            if ey < emin - p + 1:
                continue
            x = np.ldexp(1 + rng.random(), ex).astype(dtype)
            y = np.ldexp(1 + rng.random(), ey).astype(dtype)
            for a, b in ((x, y), (y, x)):
                if a == b:
                    continue
                e, f = orc.ef_op("minus", a, b, dtype)
                want = rn_unbounded(frac(a) - frac(b), p)
                _ef_check(e, f, want, p)
    # x == y gives (0, 0)
    assert orc.ef_op("minus", 3.0, 3.0, dtype) == (0, 0.0)


def test_ef_prec_orders_sigma(orc):
    """eq. prec orders (e,f) pairs like the represented values: for diagonal inputs the
    outputs satisfy sigma1 >= sigma2 as exact rationals and sigma1 = max |g_ii|."""
    g11 = np.array([1.0, 2.0, 1e-300, 5e-324, 3.0, -7.0])
    g22 = np.array([2.0, 1.0, 1e300, 1e-320, -3.0, 7.0])
    z = np.zeros(g11.size)
    o = orc.ksvd2(g11, z, z, g22)
    s1 = [ef_value(e, f) for e, f in zip(o["e1"], o["f1"])]
    s2 = [ef_value(e, f) for e, f in zip(o["e2"], o["f2"])]
    for a, b, x, y in zip(s1, s2, g11, g22):
        assert a >= b
        assert a == max(abs(frac(x)), abs(frac(y))) and b == min(abs(frac(x)), abs(frac(y)))
