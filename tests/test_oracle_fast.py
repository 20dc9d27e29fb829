"""Pins of the oracle's variant for a hypot that is not correctly rounded (Algorithm tf,
its branch for that case; the hypot itself read as hi sqrt(1 + (lo/hi)^2)).

* the fast hypot: within its error bound of the exact value (3 units of eps for a normal
  result: half a unit from the rounded quotient, half from the fma, one each from the
  square root and the product; within one unit in the last place for a subnormal one),
  exact where every step is (a zero argument, the 3-4-5 triangle, equal powers of two);
* the SVD: both sub-branches of the tan(2 phi) branch (r11 > r12 and r11 <= r12) and the
  general families give singular values within the bound the correctly rounded method
  meets (Sect. 4), orthogonal U, V and a small residual; class 9 involves no hypot and is
  bitwise the method's; the class and prescaling bits of the info word are the method's.
"""
from fractions import Fraction

import mpmath
import numpy as np
import pytest

from exact_ref import exact_hypot, fmt_of, frac
from paper_2407_13116_amd import inputs
from sigma_ref import exact_sigmas, rel_err_eps

DTYPES = [np.float64, np.float32]
SIGMA_BOUND = 8.0


def _eps(dtype):
    return 2.0 ** (-fmt_of(dtype)[0])


def _pairs(rng, n, dtype, gap_max=40):
    p, emin, emax = fmt_of(dtype)
    e1 = rng.integers(emin + 2, emax - 1, n)
    e2 = e1 - rng.integers(0, gap_max, n)
    x = np.ldexp(1 + rng.random(n), e1).astype(dtype)
    y = np.ldexp(1 + rng.random(n), np.maximum(e2, emin + 1)).astype(dtype)
    return x, y


@pytest.mark.parametrize("dtype", DTYPES)
def test_fast_hypot_error_bound(orc, dtype):
    rng = np.random.default_rng(77)
    x, y = _pairs(rng, 3000, dtype)
    sx = np.where(rng.random(x.size) < 0.5, -1, 1).astype(dtype)
    got = orc.hypot(x * sx, y, fast=True)
    got_sw = orc.hypot(y, x * sx, fast=True)
    assert np.array_equal(got, got_sw)
    bound = 3 * _eps(dtype) * (1 + 4 * _eps(dtype))
    worst = 0.0
    with mpmath.workprec(200):
        for i in range(x.size):
            v = frac(x[i]) ** 2 + frac(y[i]) ** 2
            ex = mpmath.sqrt(mpmath.mpf(v.numerator) / v.denominator)
            rel = float(abs(mpmath.mpf(float(got[i])) - ex) / ex)
            worst = max(worst, rel)
    assert worst <= bound, worst / _eps(dtype)
    # not the correctly rounded function (else the variant would not be one)
    cr = orc.hypot(x, y)
    assert np.any(cr != got)


@pytest.mark.parametrize("dtype", DTYPES)
def test_fast_hypot_subnormal(orc, dtype):
    f = np.finfo(dtype)
    tiny = np.float64(f.smallest_subnormal)
    rng = np.random.default_rng(9)
    x = (rng.integers(1, 1 << (f.nmant - 1), 400) * tiny).astype(dtype)
    y = (rng.integers(1, 1 << (f.nmant - 1), 400) * tiny).astype(dtype)
    got = orc.hypot(x, y, fast=True)
    for i in range(x.size):
        want = exact_hypot(x[i], y[i], dtype)
        assert abs(frac(got[i]) - frac(want)) <= frac(f.smallest_subnormal)


@pytest.mark.parametrize("dtype", DTYPES)
def test_fast_hypot_exact_cases(orc, dtype):
    f = np.finfo(dtype)
    ks = np.arange(f.minexp + 2, f.maxexp - 3)
    p2 = np.ldexp(1.0, ks).astype(dtype)
    # a zero argument: |x| exactly
    assert np.array_equal(orc.hypot(-p2 * 3, np.zeros_like(p2), fast=True), p2 * 3)
    # 3-4-5: r = 3/4, 1 + r^2 = 25/16 and its root 5/4 are exact
    assert np.array_equal(orc.hypot(p2 * 3, p2 * 4, fast=True), p2 * 5)
    # equal powers of two: 2^k fl(sqrt 2), the correctly rounded value
    got = orc.hypot(p2, p2, fast=True)
    for i in range(0, ks.size, 7):
        assert got[i] == exact_hypot(p2[i], p2[i], dtype)
    z = np.zeros(1, dtype)
    inf = np.array([np.inf], dtype)
    assert orc.hypot(z, z, fast=True)[0] == 0
    assert np.isinf(orc.hypot(inf, np.ones(1, dtype), fast=True)[0])
    assert np.isinf(orc.hypot(np.ones(1, dtype), -inf, fast=True)[0])


def _tri(rng, n, dtype, emax, big_first):
    """Upper triangular [a b; 0 d] with a > b (big_first) or a <= b, a > d > 0."""
    a = np.ldexp(1 + rng.random(n), rng.integers(-emax, emax, n))
    if big_first:
        b = a * np.ldexp(1 + rng.random(n), -rng.integers(1, 30, n)) / 2
    else:
        b = a * np.ldexp(1 + rng.random(n), rng.integers(0, 30, n))
    d = a * np.ldexp(1 + rng.random(n), -rng.integers(1, 30, n)) / 2
    G = np.stack([a, np.zeros(n), b, d], 1).astype(dtype)
    return G


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("big_first", [True, False], ids=["r11>r12", "r11<=r12"])
def test_fast_tan2phi_branches_sigma(orc, dtype, big_first):
    eps = _eps(dtype)
    rng = np.random.default_rng(3 + big_first)
    emax = 400 if dtype == np.float64 else 40
    G = _tri(rng, 1000, dtype, emax, big_first)
    o = orc.ksvd2(G[:, 0], G[:, 1], G[:, 2], G[:, 3], fast=True)
    w1 = w2 = 0.0
    for i in range(len(G)):
        s1, s2 = exact_sigmas(*G[i])
        w1 = max(w1, rel_err_eps(o["e1"][i], o["f1"][i], s1, eps))
        w2 = max(w2, rel_err_eps(o["e2"][i], o["f2"][i], s2, eps))
    assert w1 <= SIGMA_BOUND and w2 <= SIGMA_BOUND, (w1, w2)


FAMILIES = [
    ("narrow", 20, 20, False, True),
    ("half-range", 480, 60, False, True),
    ("triangular-wide", 1000, 120, True, True),
    ("general-wide", 1000, 120, False, False),
]


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("fam", FAMILIES, ids=[f[0] for f in FAMILIES])
def test_fast_sigma_accuracy(orc, dtype, fam):
    name, e64, e32, tri, s2ok = fam
    eps = _eps(dtype)
    emax = e64 if dtype == np.float64 else e32
    rng = np.random.default_rng(52)
    n = 1000
    G = inputs.signed_pow2_entries(rng, (n, 4), -emax, emax, dtype)
    if tri:
        G[:, 1] = 0
    o = orc.ksvd2(G[:, 0], G[:, 1], G[:, 2], G[:, 3], fast=True)
    w1 = w2 = 0.0
    for i in range(n):
        s1, s2 = exact_sigmas(*G[i])
        w1 = max(w1, rel_err_eps(o["e1"][i], o["f1"][i], s1, eps))
        w2 = max(w2, rel_err_eps(o["e2"][i], o["f2"][i], s2, eps))
    assert w1 <= SIGMA_BOUND, w1
    if s2ok:
        assert w2 <= SIGMA_BOUND, w2


@pytest.mark.parametrize("dtype", DTYPES)
def test_fast_orthogonality_residual_and_plumbing(orc, dtype):
    eps = _eps(dtype)
    g = inputs.special_set(dtype, per_type=1024)
    o = orc.ksvd2(*g, fast=True)
    c = orc.ksvd2(*g)
    for k in ("cu", "su", "cv", "sv", "f1", "f2"):
        assert np.all(np.isfinite(o[k]))
    U, V = orc.full_uv(o)
    ou = np.linalg.norm(np.transpose(U, (0, 2, 1)) @ U - np.eye(2), axis=(1, 2))
    ov = np.linalg.norm(np.transpose(V, (0, 2, 1)) @ V - np.eye(2), axis=(1, 2))
    assert ou.max() <= 8 * eps and ov.max() <= 8 * eps
    # classification (bits 0-7) and the prescaling exponent (bits 16-31) precede any hypot
    mask = np.int64(0xFFFF00FF)
    assert np.array_equal(o["info"].astype(np.int64) & mask, c["info"].astype(np.int64) & mask)
    # class 9 (at most one non-zero per row and column) uses no hypot: bitwise equal
    t1 = (c["info"] >> 4) & 15
    z9 = np.isin(t1, [0, 1, 2, 4, 8, 6, 9])
    assert z9.sum() > 0
    for k in ("cu", "su", "cv", "sv", "f1", "f2", "e1", "e2", "info"):
        assert np.array_equal(o[k][z9].view(np.uint8), c[k][z9].view(np.uint8)), k
    # residual in exact rationals on a subset
    worst = Fraction(0)
    info = o["info"].astype(np.int64)
    for i in range(0, g[0].size, 41):
        du = -1 if (info[i] >> 8) & 1 else 1
        dv = -1 if (info[i] >> 9) & 1 else 1
        cu, su, cv, sv = (frac(o[k][i]) for k in ("cu", "su", "cv", "sv"))
        Uf = ((cu, -du * su), (su, du * cu))
        Vf = ((cv, -dv * sv), (sv, dv * cv))
        s = (frac(o["f1"][i]) * Fraction(2) ** int(o["e1"][i]),
             frac(o["f2"][i]) * Fraction(2) ** int(o["e2"][i]))
        assert s[0] >= s[1] >= 0
        G = ((frac(g[0][i]), frac(g[2][i])), (frac(g[1][i]), frac(g[3][i])))
        num = sum((sum(Uf[r][k] * s[k] * Vf[cc][k] for k in range(2)) - G[r][cc]) ** 2
                  for r in range(2) for cc in range(2))
        den = sum(G[r][cc] ** 2 for r in range(2) for cc in range(2))
        if den:
            worst = max(worst, num / den)
    assert float(worst) ** 0.5 <= 8 * eps
