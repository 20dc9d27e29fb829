"""High-precision singular values of 2x2 matrices (test reference, independent of the oracle).

F = ||G||_F^2 and D = det G are formed exactly as rationals; then, with mpmath at
`prec` bits, sigma1 = sqrt((F + sqrt(F^2 - 4 D^2)) / 2) and sigma2 = |D| / sigma1
(no cancellation in either formula)."""
from fractions import Fraction

import mpmath
import numpy as np


def exact_sigmas(g11, g21, g12, g22, prec=320):
    a, b, c, d = (Fraction(float(v)) for v in (g11, g21, g12, g22))
    F = a * a + b * b + c * c + d * d
    D = a * d - c * b
    with mpmath.workprec(prec):
        if F == 0:
            return mpmath.mpf(0), mpmath.mpf(0)
        Fm = mpmath.mpf(F.numerator) / F.denominator
        disc = F * F - 4 * D * D
        Dm = mpmath.mpf(disc.numerator) / disc.denominator
        s1 = mpmath.sqrt((Fm + mpmath.sqrt(Dm)) / 2)
        s2 = abs(mpmath.mpf(D.numerator) / D.denominator) / s1
        return s1, s2


def rel_err_eps(e, f, exact, eps, prec=320):
    """Relative error of sigma = f 2^e against `exact`, in units of eps (eq. relerr:
    0/0 counts as 0)."""
    with mpmath.workprec(prec):
        got = mpmath.ldexp(mpmath.mpf(float(f)), int(e))
        if exact == 0:
            return 0.0 if got == 0 else float("inf")
        return float(abs(got - exact) / exact / eps)
