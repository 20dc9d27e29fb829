"""Pins of the oracle's 2x2 SVD (Sect. 3) against what the paper and mathematics fix.

* Sect. 3.1: class 9 is error-free (U Sigma V^T = G exactly); classes 3 and 5 give
  sigma2 = 0 exactly and sigma1 = the correctly rounded norm of the non-zero column/row.
* Theorem R / Table t:d: the elements of R are within the stated relative bounds of the
  exact R of the prescaled matrix (checked through pivot-invariant quantities).
* eq. (EXT): the wider-datatype evaluation is accurate to the stated bound; for binary32
  (T = binary64) the double rounding is innocuous.
* Sect. 4 / Sect. 5 claims: sigma1 within a single-digit multiple of eps always; sigma2 too
  for triangular inputs and for exponent ranges below about half the normal range; high-
  precision references from exact rationals + mpmath (tests/sigma_ref.py).
* e:svdres and e:ortho are a few eps; U and V never hold Inf/NaN for finite inputs; the
  results are bitwise reproducible.
* the worked example of Sect. 4 (tests/golden/worked_example.json).
"""
import json
import os
from fractions import Fraction

import mpmath
import numpy as np
import pytest

from exact_ref import ef_value, exact_hypot, fmt_of, frac, rn_unbounded
from paper_2407_13116_amd import inputs
from sigma_ref import exact_sigmas, rel_err_eps

DTYPES = [np.float64, np.float32]
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
SIGMA_BOUND = 8.0   # eps units: the paper's "single-digit multiple of eps"


def _eps(dtype):
    return 2.0 ** (-fmt_of(dtype)[0])


def _sig(o, i, k):
    return ef_value(o["e%d" % k][i], o["f%d" % k][i])


def _uv_frac(o, i):
    info = int(o["info"][i])
    out = []
    for c, s, bit in (("cu", "su", 8), ("cv", "sv", 9)):
        cc, ss = frac(o[c][i]), frac(o[s][i])
        d = -1 if (info >> bit) & 1 else 1
        out.append(((cc, -d * ss), (ss, d * cc)))
    return out


@pytest.mark.parametrize("dtype", DTYPES)
def test_class9_error_free(orc, dtype):
    g = inputs.special_set(dtype, per_type=256)
    o = orc.ksvd2(*g)
    t = o["info"] & 15
    for i in np.nonzero(np.isin(t, [0, 1, 2, 4, 6, 8, 9]))[0]:
        U, V = _uv_frac(o, i)
        s = (_sig(o, i, 1), _sig(o, i, 2))
        G = ((frac(g[0][i]), frac(g[2][i])), (frac(g[1][i]), frac(g[3][i])))
        for r in range(2):
            for c in range(2):
                val = sum(U[r][k] * s[k] * V[c][k] for k in range(2))
                assert val == G[r][c], (i, r, c)
        assert s[0] >= s[1] >= 0


@pytest.mark.parametrize("dtype", DTYPES)
def test_class3_class5_sigma2_zero(orc, dtype):
    g = inputs.special_set(dtype, per_type=512)
    o = orc.ksvd2(*g)
    t1 = (o["info"] >> 4) & 15
    idx = np.nonzero(np.isin(t1, [3, 12, 5, 10]))[0]
    assert idx.size > 100
    assert np.all(o["f2"][idx] == 0) and np.all(o["e2"][idx] == 0)
    assert np.all(o["f1"][idx] >= 1)


@pytest.mark.parametrize("dtype", DTYPES)
def test_class3_class5_sigma_cr(orc, dtype):
    """sigma1 of a one-column / one-row matrix is the correctly rounded norm."""
    p = fmt_of(dtype)[0]
    rng = np.random.default_rng(21)
    n = 2000
    a = inputs.signed_pow2_entries(rng, n, -30, 30, dtype)
    b = inputs.signed_pow2_entries(rng, n, -30, 30, dtype)
    z = np.zeros(n, dtype)
    for planes in ((a, b, z, z), (a, z, b, z), (z, z, a, b), (z, a, z, b)):
        o = orc.ksvd2(*planes)
        for i in range(0, n, 7):
            want = exact_hypot(a[i], b[i], dtype)
            assert float(_sig(o, i, 1)) == float(want)
            assert o["f2"][i] == 0


def _prescaled15(rng, n, dtype, spread):
    """Type-15 matrices already prescaled: the largest exponent is e_nu - 2 and all
    exponents lie within `spread` binades (no underflow anywhere)."""
    p, emin, emax = fmt_of(dtype)
    G = inputs.signed_pow2_entries(rng, (n, 4), -spread, 0, dtype).astype(np.float64)
    e = np.frexp(np.abs(G))[1] - 1
    G = np.ldexp(G, (emax - 2 - e.max(axis=1))[:, None])
    return G.astype(dtype)


def _mp(q: Fraction):
    return mpmath.mpf(q.numerator) / q.denominator


def _delta_bounds(eps, epsT):
    with mpmath.workprec(200):
        e = mpmath.mpf(eps)
        eT = mpmath.mpf(epsT)
        lo_s = mpmath.sqrt(((1 + e) ** 2 + 1) / 2) * (1 + e)
        hi_s = mpmath.sqrt(((1 - e) ** 2 + 1) / 2) * (1 - e)
        d1 = ((1 - e) ** 2 / lo_s, (1 + e) ** 2 / hi_s)
        d2 = ((1 - e) ** 3 / lo_s, (1 + e) ** 3 / hi_s)
        d3 = ((1 - eT) * (1 - e) ** 2 / lo_s, (1 + eT) * (1 + e) ** 2 / hi_s)
        return d1, d2, d3


def test_table_t_d_reproduced():
    """Table t:d from eqs. (d1)-(d3), rounded upwards to nine digits."""
    tab = json.load(open(os.path.join(GOLDEN, "table_t_d.json")))
    for name, eps, epsT in (("single", 2.0 ** -24, 2.0 ** -53), ("double", 2.0 ** -53, 2.0 ** -113)):
        d1, d2, d3 = _delta_bounds(eps, epsT)
        with mpmath.workprec(200):
            vals = [(1 - d1[0]) / eps, (d1[1] - 1) / eps, (1 - d2[0]) / eps, (d2[1] - 1) / eps,
                    (1 - d3[0]) / eps, (d3[1] - 1) / eps]
            got = [float(mpmath.ceil(v * 10 ** 9) / 10 ** 9) for v in vals]
        assert np.allclose(got, tab[name], rtol=0, atol=1e-12), (name, got)


@pytest.mark.parametrize("dtype", DTYPES)
def test_theorem_R_bounds(orc, dtype):
    """Theorem R: r11 within eps; r12, r22 within delta_1 (exact tan) or delta_2 / delta_3
    (inexact tan) of the exact R.  Checked via pivot-invariant exact values:
    r11* = the larger column norm, |r22*| = |det| / r11*, |r12*| = sqrt(w2^2 - r22*^2)."""
    eps = _eps(dtype)
    # T: binary64 for binary32; double-word (error ~ 2^-104) for binary64
    epsT = 2.0 ** -53 if dtype == np.float32 else 2.0 ** -103
    d1, d2, d3 = _delta_bounds(eps, epsT)
    worst = max(float(d2[1] - 1), float(1 - d2[0]), float(d3[1] - 1), float(1 - d3[0]))
    best = max(float(d1[1] - 1), float(1 - d1[0]))
    rng = np.random.default_rng(31)
    G = _prescaled15(rng, 1500, dtype, 60)
    n_ext = n_exact = 0
    with mpmath.workprec(300):
        for g11, g21, g12, g22 in G:
            r11, r12, r22, tan_t, exact, used_ext = orc.urv15(g11, g21, g12, g22, dtype)
            a, b, c, d = (frac(x) for x in (g11, g21, g12, g22))
            w1 = mpmath.sqrt(_mp(a * a + b * b))
            w2 = mpmath.sqrt(_mp(c * c + d * d))
            r11x = max(w1, w2)
            wmin = min(w1, w2)
            det = abs(_mp(a * d - c * b))
            r22x = det / r11x
            r12x = mpmath.sqrt(max(wmin ** 2 - r22x ** 2, 0))
            assert abs(mpmath.mpf(float(r11)) - r11x) / r11x <= eps
            bound = best if exact else worst
            assert abs(abs(mpmath.mpf(float(r22))) - r22x) / r22x <= bound * 1.000001
            if r12x > wmin * 1e-6:   # r12x by the invariant is itself ill-conditioned near 0
                assert abs(abs(mpmath.mpf(float(r12))) - r12x) / r12x <= bound * 1.000001
            n_ext += used_ext
            n_exact += exact
    assert n_ext > 500 and n_exact >= 0


@pytest.mark.parametrize("dtype", DTYPES)
def test_ext_accuracy(orc, dtype):
    """eq. (EXT): |fl(FL(star)/g) - star/g| <= eps (1 + few eps_T) relative; for binary32
    the double rounding through binary64 is innocuous (the result is RN of the exact
    quotient whenever the binary64 sum is exact)."""
    p, emin, emax = fmt_of(dtype)
    eps = _eps(dtype)
    rng = np.random.default_rng(41)
    G = _prescaled15(rng, 4000, dtype, 40)
    agree = 0
    for x1, y1, x2, y2 in G:
        # as after the pivoting of Sect. 3.2.2: the divisor (the pivot) is the larger of y1, y2
        if abs(y1) < abs(y2):
            y1, y2 = y2, y1
        for minus in (False, True):
            d = y1
            got = orc.ext(x1, y1, x2, y2, minus, d, dtype)
            star = frac(x1) * frac(y1) + (-1 if minus else 1) * frac(x2) * frac(y2)
            q = star / frac(d)
            if q == 0:
                assert got == 0
                continue
            rel = abs(Fraction(float(got)) - q) / abs(q)
            assert rel <= Fraction(eps) * (1 + Fraction(2) ** -50)
            want = rn_unbounded(q, p)
            agree += Fraction(float(got)) == want
            if dtype == np.float32:
                s64 = Fraction(float(np.float64(x1) * np.float64(y1))) + \
                    (-1 if minus else 1) * Fraction(float(np.float64(x2) * np.float64(y2)))
                if s64 == star:   # the binary64 sum is exact
                    assert Fraction(float(got)) == want
    assert agree >= 0.999 * 2 * len(G)


FAMILIES = [
    # (name, exponent half-width for f64, for f32, triangular, sigma2 bound applies)
    ("narrow", 20, 20, False, True),
    ("half-range", 480, 60, False, True),
    ("triangular-wide", 1000, 120, True, True),
    ("general-wide", 1000, 120, False, False),
]


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("fam", FAMILIES, ids=[f[0] for f in FAMILIES])
def test_sigma_accuracy(orc, dtype, fam):
    name, e64, e32, tri, s2ok = fam
    eps = _eps(dtype)
    emax = e64 if dtype == np.float64 else e32
    rng = np.random.default_rng(51)
    n = 1500
    G = inputs.signed_pow2_entries(rng, (n, 4), -emax, emax, dtype)
    if tri:
        G[:, 1] = 0
    o = orc.ksvd2(G[:, 0], G[:, 1], G[:, 2], G[:, 3])
    worst1 = worst2 = 0.0
    for i in range(n):
        s1, s2 = exact_sigmas(*G[i])
        worst1 = max(worst1, rel_err_eps(o["e1"][i], o["f1"][i], s1, eps))
        worst2 = max(worst2, rel_err_eps(o["e2"][i], o["f2"][i], s2, eps))
    assert worst1 <= SIGMA_BOUND, worst1
    if s2ok:
        assert worst2 <= SIGMA_BOUND, worst2


@pytest.mark.parametrize("dtype", DTYPES)
def test_residual_orthogonality_and_finiteness(orc, dtype):
    """e:svdres and e:ortho (evaluated in binary64 / high precision) are a few eps; no
    Inf/NaN in U or V; sigma1 >= sigma2 >= 0 on every zero pattern and edge value."""
    eps = _eps(dtype)
    g = inputs.special_set(dtype, per_type=2048)
    o = orc.ksvd2(*g)
    for k in ("cu", "su", "cv", "sv", "f1", "f2"):
        assert np.all(np.isfinite(o[k]))
    U, V = orc.full_uv(o)
    ou = np.linalg.norm(np.transpose(U, (0, 2, 1)) @ U - np.eye(2), axis=(1, 2))
    ov = np.linalg.norm(np.transpose(V, (0, 2, 1)) @ V - np.eye(2), axis=(1, 2))
    assert ou.max() <= 8 * eps and ov.max() <= 8 * eps
    # residual in exact rationals on a subset (the entries span the whole range)
    worst = Fraction(0)
    for i in range(0, g[0].size, 37):
        Uf, Vf = _uv_frac(o, i)
        s = (_sig(o, i, 1), _sig(o, i, 2))
        assert s[0] >= s[1] >= 0
        G = ((frac(g[0][i]), frac(g[2][i])), (frac(g[1][i]), frac(g[3][i])))
        num = sum((sum(Uf[r][k] * s[k] * Vf[c][k] for k in range(2)) - G[r][c]) ** 2
                  for r in range(2) for c in range(2))
        den = sum(G[r][c] ** 2 for r in range(2) for c in range(2))
        if den:
            worst = max(worst, num / den)
    # general-wide inputs may carry an inaccurate sigma2, but the residual stays small
    assert float(worst) ** 0.5 <= 8 * eps


@pytest.mark.parametrize("dtype", DTYPES)
def test_bitwise_reproducible(orc, dtype):
    g = inputs.special_set(dtype, per_type=512)
    a = orc.ksvd2(*g, nthreads=1)
    b = orc.ksvd2(*g, nthreads=4)
    for k in a:
        assert np.array_equal(a[k].view(np.uint8), b[k].view(np.uint8)), k


@pytest.mark.parametrize("dtype", DTYPES)
def test_nonfinite_flag(orc, dtype):
    g = [np.array([1, np.nan, 0, np.inf], dtype), np.ones(4, dtype), np.ones(4, dtype),
         np.array([1, 1, -np.inf, 1], dtype)]
    o = orc.ksvd2(*g)
    assert (o["info"][0] >> 15) & 1 == 0
    for i in (1, 2, 3):
        assert (o["info"][i] >> 15) & 1 == 1
        assert np.isnan(o["cu"][i]) and np.isnan(o["f1"][i])


@pytest.mark.parametrize("dtype", DTYPES)
def test_worked_example(orc, dtype):
    ex = json.load(open(os.path.join(GOLDEN, "worked_example.json")))
    f = np.finfo(dtype)
    mu, nu = dtype(f.tiny), dtype(f.max)
    o = orc.ksvd2(np.array([mu]), np.array([0], dtype), np.array([nu / 4]), np.array([mu]))
    info = int(o["info"][0])
    assert (info >> 12) & 1, "the tan(psi) overflow branch of Algorithm tp must be taken"
    s1, s2 = _sig(o, 0, 1), _sig(o, 0, 2)
    # the paper's sigma2 ~ 4 mu^2 / nu, and sigma1 = |det G| / sigma2 = mu^2 / sigma2
    printed_s2 = 4 * frac(mu) ** 2 / frac(nu)
    assert abs(s2 - printed_s2) / printed_s2 < Fraction(1, 1 << 20)
    assert abs(s1 * s2 - frac(mu) ** 2) / frac(mu) ** 2 <= 4 * Fraction(_eps(dtype))
    # kappa ~ nu^2/(16 mu^2), above Fig. 2's observed maximum (double)
    if dtype == np.float64:
        kappa = float(_mp(s1 / s2))
        assert kappa >= ex["paper_states"]["fig2_caption_max_kappa_f64"]
    # the exact singular values, correctly rounded in (e,f) form
    key = "f64" if dtype == np.float64 else "f32"
    (e1, f1), (e2, f2) = ex["expected_ef"][key]["sigma1"], ex["expected_ef"][key]["sigma2"]
    assert (int(o["e1"][0]), float(o["f1"][0])) == (e1, float.fromhex(f1))
    assert (int(o["e2"][0]), float(o["f2"][0])) == (e2, float.fromhex(f2))
    p = fmt_of(dtype)[0]
    ex1, ex2 = exact_sigmas(mu, dtype(0), nu / 4, mu, prec=600)
    for (e, fh), exact in (((e1, f1), ex1), ((e2, f2), ex2)):
        with mpmath.workprec(p):
            rounded = +exact          # round-to-nearest-even to p bits
        with mpmath.workprec(600):
            assert rounded == mpmath.ldexp(mpmath.mpf(float.fromhex(fh)), e)


PSIG, RSWAP = 1 << 13, 1 << 11


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("fast", [False, True])
def test_psigma_swap_not_taken_near_degenerate(orc, dtype, fast):
    """Algorithm tp's reordering P_sigma needs sigma~1'' < sigma~2'', i.e. sec(phi) >
    sec(psi) after rounding, i.e. tan(phi) > tan(psi) as computed.  Exactly, tan(psi) >=
    (a/d) tan(phi) for [a b; 0 d] with a >= d; the computed values could only invert
    where a - d is an ulp or so and b < 2(a - d) (the near-degenerate triangular
    matrices), and there the relations of the roundings exclude it for the correctly
    rounded hypot (the argument is written out with the readings of the paper).  Pinned on
    that region: a in [1, 2), d = a - j ulp (j = 1, 2, 3), b = x (a - d), x log-uniform
    in [0.005, 20]; no P_sigma swap, and sec(phi) <= sec(psi) (cos(phi) >= cos(psi))."""
    rng = np.random.default_rng(77)
    N = 1 << 20
    u = np.finfo(dtype).eps
    a = (1 + rng.random(N)).astype(dtype)
    d = (a - rng.integers(1, 4, N) * u).astype(dtype)
    x = np.exp(rng.uniform(np.log(0.005), np.log(20), N))
    b = ((a.astype(np.float64) - d.astype(np.float64)) * x).astype(dtype)
    o = orc.ksvd2(a, np.zeros_like(a), b, d, plain=False, fast=fast)
    assert np.all(((o["info"] >> 4) & 15) == 13)            # [a b; 0 d]: class 13
    assert not np.any(o["info"] & (PSIG | RSWAP))
    assert np.all(np.abs(o["cu"]) >= np.abs(o["cv"]))


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_class15_wide_spread_never_swapped(orc, dtype):
    """tan(psi) can underflow to 0 only when r12/r11 is below about 2^-1127 (2^-150 in
    binary32), which in class 15 needs an exponent spread above the format's range
    within a column or across the second column; the diagonal of R then stays in
    order (r11 >= r22), so the swapped case, where tan(phi-bar) = 1/tan(psi) would be
    infinite, is not reached.  Pinned on class-15 matrices with such spreads:
    [g11 g12; g21 g22] with g21/g11 and g12/g22 tiny, |g22| near |g11|."""
    rng = np.random.default_rng(78)
    N = 1 << 18
    lo, hi = (-1074, 1020) if dtype == np.float64 else (-149, 124)
    big = inputs.signed_pow2_entries(rng, (N,), hi - 2, hi, dtype)
    g11 = np.abs(big)
    g22 = (g11 * (1 - rng.integers(0, 3, N) * np.finfo(dtype).eps) *
           rng.choice([-1, 1], N)).astype(dtype)
    g21 = inputs.signed_pow2_entries(rng, (N,), lo, lo + 40, dtype)
    g12 = inputs.signed_pow2_entries(rng, (N,), lo, lo + 40, dtype)
    o = orc.ksvd2(g11, g21, g12, g22, plain=False)
    cls15 = (o["info"] & 15) == 15
    assert cls15.mean() > 0.9
    assert not np.any(o["info"][cls15] & RSWAP)
