"""Exact references for pinning the oracle (pure Python integers / Fraction).

Nothing here calls the oracle or the GPU library: each function is the plain
mathematical definition (exact rational arithmetic, then one round-to-nearest-
even), so agreement with it is evidence about the oracle, not a restatement of
its code.
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np

# (p, e_min, e_max) of Sect. 2: p significand bits, e_mu, e_nu
F64 = (53, -1022, 1023)
F32 = (24, -126, 127)


def fmt_of(dtype):
    return F64 if np.dtype(dtype) == np.float64 else F32


def floor_log2(a: Fraction) -> int:
    """floor(lg a) for a > 0."""
    n, d = a.numerator, a.denominator
    e = n.bit_length() - d.bit_length()
    # now 2^(e-1) < n/d < 2^(e+1)
    if e >= 0:
        if n < d << e:
            e -= 1
    else:
        if n << (-e) < d:
            e -= 1
    return e


def _pow2(k: int) -> Fraction:
    return Fraction(1 << k) if k >= 0 else Fraction(1, 1 << (-k))


def round_rn(v: Fraction, p: int, emin=None, emax=None):
    """Round v to p significant bits, ties to even.  With emin: gradual underflow
    (quantum 2^(emin-p+1)).  With emax: overflow to +-inf.  Returns Fraction or float inf."""
    if v == 0:
        return Fraction(0)
    sign = -1 if v < 0 else 1
    a = abs(v)
    e = floor_log2(a)
    q = e - p + 1
    if emin is not None:
        q = max(q, emin - p + 1)
    num, den = a.numerator, a.denominator
    if q >= 0:
        den <<= q
    else:
        num <<= -q
    n, r = divmod(num, den)
    if 2 * r > den or (2 * r == den and (n & 1)):
        n += 1
    res = Fraction(n) * _pow2(q)
    if emax is not None and res >= _pow2(emax + 1):
        return sign * math.inf
    return sign * res


def to_float(v, dtype=np.float64):
    if isinstance(v, float) and math.isinf(v):
        return np.array(v, dtype)[()]
    return np.array(float(v), dtype)[()] if np.dtype(dtype) == np.float64 else np.float32(float(v))


def rn(v: Fraction, dtype=np.float64):
    """IEEE round-to-nearest-even of an exact rational into dtype (with subnormals/overflow)."""
    p, emin, emax = fmt_of(dtype)
    r = round_rn(v, p, emin, emax)
    if isinstance(r, float):
        return np.array(r, dtype)[()]
    # r is exactly representable in dtype; float() of a Fraction is correctly rounded,
    # and for float32 the value is representable in binary64 too.
    return np.array(float(r), dtype)[()]


def rn_unbounded(v: Fraction, p: int) -> Fraction:
    """Round to p bits with an unbounded exponent range (the (e,f) pairs' semantics)."""
    return round_rn(v, p)


def exact_hypot(x, y, dtype=np.float64):
    """Correctly rounded sqrt(x^2 + y^2) by integer square roots."""
    p, emin, emax = fmt_of(dtype)
    fx, fy = Fraction(float(x)), Fraction(float(y))
    v = fx * fx + fy * fy
    if v == 0:
        return np.array(0.0, dtype)[()]
    e = floor_log2(v) // 2               # floor(lg sqrt v)
    q = max(e - p + 1, emin - p + 1)     # quantum of the result's grid
    W = v / (_pow2(q) * _pow2(q))        # sqrt(W) = sqrt(v) / 2^q
    W4 = 4 * W
    fl = W4.numerator // W4.denominator  # floor(4W)
    t = math.isqrt(fl)                   # floor(2 sqrt(W))
    exact_mid = (W4.denominator == 1) and (t * t == W4.numerator)
    if t % 2 == 0:
        n = t // 2
    elif exact_mid:
        lo, hi = (t - 1) // 2, (t + 1) // 2
        n = lo if lo % 2 == 0 else hi
    else:
        n = (t + 1) // 2
    res = Fraction(n) * _pow2(q)
    if res >= _pow2(emax + 1):
        return np.array(np.inf, dtype)[()]
    return np.array(float(res), dtype)[()]


def ef_value(e: int, f) -> Fraction:
    return Fraction(float(f)) * _pow2(int(e))


def frac(x) -> Fraction:
    return Fraction(float(x))
