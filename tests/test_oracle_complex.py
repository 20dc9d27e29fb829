"""Pins of the oracle's complex 2x2 SVD (Sect. 3.4): G = U diag(sigma) V^H.

* singular values against high-precision references formed from exact rationals
  (||G||_F^2 and |det G|^2 are exact rationals of the inputs; sigma_1 and sigma_2 then
  follow without cancellation in mpmath), on narrow, half-range and triangular families:
  sigma_1 within 8 eps relatively; sigma_2 within 8 eps sigma_1 (no wider datatype, so
  no relative guarantee for general matrices), and within 8 eps relatively for
  triangular ones;
* U and V unitary and the residual U Sigma V^H - G small, in exact rational arithmetic on
  a sample spanning every zero pattern and edge value, with no Inf/NaN in U or V;
* special cases that reduce to textbook values: a diagonal (or single-element) matrix has
  the correctly rounded moduli |g_ii| as singular values; a real matrix is the real method
  (its sigma within the real method's bound of the exact value); a purely imaginary one
  gives the same sigma and V, and i U;
* invariances: multiplying G by i or conjugating it leaves the singular values within the
  bound.
"""
from fractions import Fraction

import mpmath
import numpy as np
import pytest

from exact_ref import exact_hypot, frac
from paper_2407_13116_amd import inputs

CDT = [np.complex128, np.complex64]
BOUND = 8.0


def _rt(cdt):
    return np.float64 if cdt == np.complex128 else np.float32


def _eps(cdt):
    return 2.0 ** (-53 if cdt == np.complex128 else -24)


def _exact(G2, prec=320):
    a, b, c, d = (complex(G2[0, 0]), complex(G2[0, 1]), complex(G2[1, 0]), complex(G2[1, 1]))
    fr = [(Fraction(z.real), Fraction(z.imag)) for z in (a, b, c, d)]
    F = sum(x * x + y * y for x, y in fr)
    (ar, ai), (br, bi), (cr, ci), (dr, di) = fr
    # det = a d - b c
    Dr = ar * dr - ai * di - (br * cr - bi * ci)
    Di = ar * di + ai * dr - (br * ci + bi * cr)
    D2 = Dr * Dr + Di * Di
    with mpmath.workprec(prec):
        if F == 0:
            return mpmath.mpf(0), mpmath.mpf(0)
        Fm = mpmath.mpf(F.numerator) / F.denominator
        disc = F * F - 4 * D2
        s1 = mpmath.sqrt((Fm + mpmath.sqrt(mpmath.mpf(disc.numerator) / disc.denominator)) / 2)
        s2 = mpmath.sqrt(mpmath.mpf(D2.numerator) / D2.denominator) / s1
        return s1, s2


def _rel(o, b, k, ex, eps, prec=320):
    with mpmath.workprec(prec):
        got = mpmath.ldexp(mpmath.mpf(float(o["f"][b, k])), int(o["e"][b, k]))
        if ex == 0:
            return 0.0 if got == 0 else float("inf")
        return float(abs(got - ex) / ex / eps)


@pytest.mark.parametrize("cdt", CDT)
@pytest.mark.parametrize("emax,tri", [(20, False), (480, False), (1000, True)],
                         ids=["narrow", "half-range", "triangular-wide"])
def test_complex_sigma_accuracy(orc, cdt, emax, tri):
    if cdt == np.complex64:
        emax = min(emax // 8, 60)
    eps = _eps(cdt)
    G = inputs.complex_batch(cdt, seed=31, B=1500, emax=emax)
    if tri:
        G[:, 1, 0] = 0
    o = orc.ksvd2c(G)
    w1 = w2 = wn = 0.0
    for b in range(len(G)):
        s1, s2 = _exact(G[b])
        w1 = max(w1, _rel(o, b, 0, s1, eps))
        w2 = max(w2, _rel(o, b, 1, s2, eps))
        with mpmath.workprec(320):
            got = mpmath.ldexp(mpmath.mpf(float(o["f"][b, 1])), int(o["e"][b, 1]))
            if s1 > 0:
                wn = max(wn, float(abs(got - s2) / s1 / eps))
    assert w1 <= BOUND, w1
    # without eq. EXT (Sect. 3.4 drops the wider datatype) sigma_2 of a general complex
    # matrix is accurate relative to sigma_1; triangular inputs need no rotation and
    # keep sigma_2 relatively accurate
    assert wn <= BOUND, wn
    if tri:
        assert w2 <= BOUND, w2


@pytest.mark.parametrize("cdt", CDT)
def test_complex_unitary_residual_special_set(orc, cdt):
    eps = _eps(cdt)
    G = inputs.complex_special_set(cdt, per_type=512)
    o = orc.ksvd2c(G)
    assert np.all(np.isfinite(o["U"])) and np.all(np.isfinite(o["V"]))
    U = o["U"].astype(np.complex128)
    V = o["V"].astype(np.complex128)
    I = np.eye(2)
    eu = np.abs(np.conj(np.transpose(U, (0, 2, 1))) @ U - I).max()
    ev = np.abs(np.conj(np.transpose(V, (0, 2, 1))) @ V - I).max()
    assert eu <= 8 * eps and ev <= 8 * eps, (eu / eps, ev / eps)
    worst = Fraction(0)
    for b in range(0, len(G), 29):
        s = [frac(o["f"][b, k]) * Fraction(2) ** int(o["e"][b, k]) for k in range(2)]
        assert s[0] >= s[1] >= 0
        num = Fraction(0)
        den = Fraction(0)
        for i in range(2):
            for j in range(2):
                re = im = Fraction(0)
                for k in range(2):
                    ur, ui = frac(U[b, i, k].real), frac(U[b, i, k].imag)
                    vr, vi = frac(V[b, j, k].real), -frac(V[b, j, k].imag)  # conj(v_jk)
                    re += s[k] * (ur * vr - ui * vi)
                    im += s[k] * (ur * vi + ui * vr)
                gr, gi = frac(G[b, i, j].real), frac(G[b, i, j].imag)
                num += (re - gr) ** 2 + (im - gi) ** 2
                den += gr * gr + gi * gi
        if den:
            worst = max(worst, num / den)
    assert float(worst) ** 0.5 <= 8 * eps


@pytest.mark.parametrize("cdt", CDT)
def test_complex_diagonal_moduli_correctly_rounded(orc, cdt):
    rt = _rt(cdt)
    rng = np.random.default_rng(5)
    n = 600
    G = np.zeros((n, 2, 2), cdt)
    for i in range(2):
        G[:, i, i].real = inputs.signed_pow2_entries(rng, n, -40, 40, rt)
        G[:, i, i].imag = inputs.signed_pow2_entries(rng, n, -40, 40, rt)
    G[: n // 3, 1, 1] = 0          # a single element
    o = orc.ksvd2c(G)
    for b in range(n):
        m = sorted((exact_hypot(G[b, i, i].real, G[b, i, i].imag, rt) for i in range(2)),
                   reverse=True)
        assert o["S"][b, 0] == m[0] and o["S"][b, 1] == m[1], b


@pytest.mark.parametrize("cdt", CDT)
def test_complex_real_and_imaginary_reduce_to_real(orc, cdt):
    rt = _rt(cdt)
    eps = _eps(cdt)
    rng = np.random.default_rng(6)
    n = 500
    Gr = inputs.signed_pow2_entries(rng, (n, 2, 2), -30, 30, rt)
    G = Gr.astype(cdt)
    o = orc.ksvd2c(G)
    oi = orc.ksvd2c((1j * Gr).astype(cdt))
    assert np.array_equal(o["S"], oi["S"]) and np.array_equal(o["V"], oi["V"])
    assert np.array_equal(oi["U"].imag, o["U"].real) and np.all(oi["U"].real == 0)
    assert np.all(o["U"].imag == 0) and np.all(o["V"].imag == 0)
    for b in range(0, n, 5):
        s1, s2 = _exact(G[b])
        assert _rel(o, b, 0, s1, eps) <= BOUND and _rel(o, b, 1, s2, eps) <= BOUND


@pytest.mark.parametrize("cdt", CDT)
def test_complex_phase_and_conjugate_invariance(orc, cdt):
    eps = _eps(cdt)
    G = inputs.complex_batch(cdt, seed=33, B=800)
    o = orc.ksvd2c(G)
    oi = orc.ksvd2c((1j * G).astype(cdt))   # exact: (re, im) -> (-im, re)
    oc = orc.ksvd2c(np.conj(G))
    for other in (oi, oc):
        for k in range(2):
            a = o["S"][:, k].astype(np.float64)
            b = other["S"][:, k].astype(np.float64)
            nz = a > 0
            assert np.all(np.abs(a[nz] - b[nz]) <= 2 * BOUND * eps * a[nz])
