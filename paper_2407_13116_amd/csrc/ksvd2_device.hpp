// Device side of the enhanced Kogbetliantz SVD of order two (gfx950).
//
// One matrix per lane.  Everything here is straight-line scalar code in the
// working precision W (double or float), with explicit fma and no contraction
// (the library is built with -ffp-contract=off), IEEE division and square
// root, and gradual underflow.  The paper's steps, in order (Sect. 3):
//   phase 1  type/class of the zero pattern (eq. ts), prescaling by a power of
//            two (eqs. eG, s), re-examination of the pattern, simple classes
//            (Sect. 3.1);
//   phase 2  error-free triangularisation of class 13 (Sect. 3.2.1) or the
//            fully pivoted URV of class 15 with the wider-precision element
//            (Sect. 3.2.2, eqs. QR15, EXT, Theorem R);
//   phase 3  SVD of the triangular factor (Sect. 3.3.1, Algorithms tf, tp),
//            assembly with the left-vector heuristic (Sect. 3.3.2, eqs. p+t,
//            p-t, tan+-, UV) and backscaling in (e,f) form.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ksvd2 {

// ---------------------------------------------------------------------------
// Format constants (Sect. 2): p, eps = 2^-p, e_mu, e_nu.
// ---------------------------------------------------------------------------
template <class R> struct Lim;
template <> struct Lim<double> {
  static constexpr int p = 53, e_mu = -1022, e_nu = 1023;
  __device__ static double mu() { return 0x1p-1022; }
  __device__ static double nu() { return 0x1.fffffffffffffp+1023; }
  __device__ static double eps() { return 0x1p-53; }
  __device__ static double eps_normal_from() { return 0x1p-960; }  // b eps normal above
};
template <> struct Lim<float> {
  static constexpr int p = 24, e_mu = -126, e_nu = 127;
  __device__ static float mu() { return 0x1p-126f; }
  __device__ static float nu() { return 0x1.fffffep+127f; }
  __device__ static float eps() { return 0x1p-24f; }
  __device__ static float eps_normal_from() { return 0x1p-100f; }
};

// floor(lg|x|) for finite x != 0 (also for subnormal x).
__device__ inline int ilog2(double x) {
  int e;
  (void)frexp(x, &e);
  return e - 1;
}
__device__ inline int ilog2(float x) {
  int e;
  (void)frexpf(x, &e);
  return e - 1;
}

// x 2^n rounded once to nearest-even, as IEEE scaleB: exact while the result
// is normal, gradual underflow below that, +-inf on overflow.  v_ldexp_f64 and
// v_ldexp_f32 are IEEE scaleB (with denormals enabled, as this library is
// built), so this is one instruction.
__device__ inline double scale2(double x, int n) { return ldexp(x, n); }
__device__ inline float scale2(float x, int n) { return ldexpf(x, n); }

__device__ inline double ldexp_w(double x, int n) { return ldexp(x, n); }
__device__ inline double frexp_w(double x, int *e) { return frexp(x, e); }
__device__ inline float frexp_w(float x, int *e) { return frexpf(x, e); }
__device__ inline float ldexp_w(float x, int n) { return ldexpf(x, n); }

// ---------------------------------------------------------------------------
// Error-free transformations (Dekker/Knuth; Joldes-Muller-Popescu 2017).
// ---------------------------------------------------------------------------
__device__ inline void two_sum(double a, double b, double &s, double &t) {
  s = a + b;
  double bb = s - a;
  double aa = s - bb;
  t = (a - aa) + (b - bb);
}
__device__ inline void fast_two_sum(double a, double b, double &s, double &t) {
  s = a + b;
  t = b - (s - a);
}
__device__ inline void two_prod(double a, double b, double &p, double &e) {
  p = a * b;
  e = fma(a, b, -p);
}

// Exact sign of the sum of n doubles (Shewchuk's grow-expansion: the
// components stay non-overlapping, so the sign of the sum is the sign of the
// most significant non-zero component).  Used only on rare rounding-boundary
// paths.
__device__ __attribute__((noinline)) int exact_sign(double t0, double t1, double t2, double t3,
                                                    double t4, double t5, double t6, double t7) {
  const double t[8] = {t0, t1, t2, t3, t4, t5, t6, t7};
  double e[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    double q = t[i];
#pragma unroll
    for (int j = 0; j < i; ++j) {
      double s, r;
      two_sum(q, e[j], s, r);
      e[j] = r;
      q = s;
    }
    e[i] = q;
  }
  int sg = 0;
#pragma unroll
  for (int j = 0; j < 8; ++j)
    if (e[j] != 0.0) sg = e[j] > 0.0 ? 1 : -1;
  return sg;
}

__device__ inline bool even_sig(double y) { return (__double_as_longlong(y) & 1) == 0; }
__device__ inline bool even_sig(float y) { return (__float_as_uint(y) & 1u) == 0; }

// ---------------------------------------------------------------------------
// Correctly rounded hypot, binary64.
//   hi >= lo > 0.  Both subnormal: the result lies on the 2^-1074 grid;
//   integer rounding of sqrt(H^2 + L^2) with an exact sign test (no ties are
//   possible there).  Otherwise scale hi into [1,2) (exact), form S = A^2 + B^2
//   as a double-word, take a candidate root y and prove it correctly rounded
//   from its residual S - y^2 (sqrt_dw_cr below); only next to a rounding
//   midpoint does an exact expansion sign test decide (this includes exact
//   ties, e.g. Pythagorean midpoints).
// ---------------------------------------------------------------------------
__device__ __attribute__((noinline)) double hypot_tiny(double hi, double lo) {
  double H = ldexp(hi, 1074), L = ldexp(lo, 1074);  // integers < 2^52, exact
  double p, pe, q, qe;
  two_prod(H, H, p, pe);
  two_prod(L, L, q, qe);
  double k = rint(sqrt(p + q));
  double kk, kke;
  two_prod(k, k, kk, kke);
  // S - k^2 - k > 0  <=>  sqrt(S) > k + 1/2 (S integer, so never a tie)
  if (exact_sign(p, pe, q, qe, -kk, -kke, -k, 0.0) > 0) {
    k += 1.0;
  } else if (exact_sign(p, pe, q, qe, -kk, -kke, k, 0.0) <= 0) {
    k -= 1.0;  // S <= k^2 - k  <=>  sqrt(S) < k - 1/2
  }
  return k * 0x1p-1074;
}

__device__ __attribute__((noinline)) double hypot_resolve(double p, double pe, double q,
                                                          double qe, double y, double up_gap,
                                                          double dn_gap) {
  // sign(S - m^2) at the upper midpoint m = y + up_gap/2, then at the lower one
  double yy, yye;
  two_prod(y, y, yy, yye);
  double h = 0.5 * up_gap;
  int cu = exact_sign(p, pe, q, qe, -yy, -yye, -2.0 * y * h, -h * h);
  if (cu > 0) return y + up_gap;
  if (cu == 0) return even_sig(y) ? y : y + up_gap;
  h = 0.5 * dn_gap;
  int cd = exact_sign(p, pe, q, qe, -yy, -yye, 2.0 * y * h, -h * h);
  if (cd < 0) return y - dn_gap;
  if (cd == 0) return even_sig(y) ? y : y - dn_gap;
  return y;
}

// sqrt(S), S = sh + sl a double-word in [1, 8), correctly rounded to binary64.
// A reciprocal square root estimate and one Goldschmidt step give g ~ sqrt(S)
// and h ~ 1/(2 sqrt S); one Newton step on the double-word S gives the
// candidate y, within far less than an ulp of sqrt(S) except next to a
// rounding midpoint.  Its residual rho = S - y^2 (sh - y^2 by one fma, then
// + sl) is within 2^-100 y^2 of the exact one, and sqrt(S) - y = rho /
// (sqrt(S) + y).  So |rho| < y ulp(y) (1 - 2^-40) proves |sqrt(S) - y| <
// ulp(y)/2, i.e. y is the correctly rounded root (below y = 2 the gap is half
// as wide, so that side is left to the fallback).  Otherwise the exact
// expansion sign test settles it (p, pe, q, qe are the exact parts of S).
__device__ __attribute__((always_inline)) inline double sqrt_dw_cr(double sh, double sl,
                                                                    double p, double pe,
                                                                    double q, double qe) {
  double s = sh + sl;
  double r0 = __builtin_amdgcn_rsq(s);
  double g = s * r0, h = 0.5 * r0;
  double e = fma(-h, g, 0.5);
  g = fma(g, e, g);
  h = fma(h, e, h);
  double d = fma(-g, g, sh) + sl;
  double y = fma(d, h, g);
  double rho = fma(-y, y, sh) + sl;
  constexpr double c1 = 0x1p-52 * (1.0 - 0x1p-40), c2 = 0x1p-51 * (1.0 - 0x1p-40);
  bool big = y >= 2.0;
  double thr = y * (big ? c2 : c1);
  bool ok = fabs(rho) < thr && !(y == 2.0 && rho < 0.0);
  if (ok) return y;
  double hg = big ? 0x1p-52 : 0x1p-53;          // half an ulp of y (y in [1, 4))
  bool pow2 = (y == 1.0) || (y == 2.0);         // the gap below y is half as wide
  return hypot_resolve(p, pe, q, qe, y, 2.0 * hg, pow2 ? hg : 2.0 * hg);
}

__device__ __attribute__((always_inline)) inline double hypot_cr(double x, double y) {
  double a = fabs(x), b = fabs(y);
  double hi = fmax(a, b), lo = fmin(a, b);
  if (lo == 0.0 || isinf(hi)) return hi;
  int eh = ilog2(hi), el = ilog2(lo);
  // beyond an exponent gap of 30, lo^2 < 2^-60 hi^2 cannot move the rounding
  // of hi (the general path would return hi as well; on wide-range data whole
  // waves skip it here)
  if (eh - el > 30) return hi;
  if (eh < -1022) return hypot_tiny(hi, lo);
  double A = ldexp(hi, -eh), B = ldexp(lo, -eh);  // A in [1,2), B >= 2^-31: exact
  double p, pe, q, qe;
  two_prod(A, A, p, pe);
  two_prod(B, B, q, qe);
  double sh = p + q;                               // p >= q: Fast2Sum
  double sl = (q - (sh - p)) + (pe + qe);
  return ldexp(sqrt_dw_cr(sh, sl, p, pe, q, qe), eh);
}

// hypot(t, 1) for 0 <= t <= 1 (the secants of angles up to pi/4): the larger
// argument is exactly 1, so no scaling is needed; below 2^-30 the result is 1.
// S = 1 + t^2 lies in [1, 2], so the root lies in [1, sqrt 2]: sqrt_dw_cr's
// tests for roots of 2 and above are dropped (the same candidate, acceptance
// test and fallback for this range).
__device__ __attribute__((always_inline)) inline double hypot1_le1(double t) {
  if (t < 0x1p-30) return 1.0;
  double q, qe;
  two_prod(t, t, q, qe);
  double sh = 1.0 + q;
  double sl = (q - (sh - 1.0)) + qe;
  double s = sh + sl;
  double r0 = __builtin_amdgcn_rsq(s);
  double g = s * r0, h = 0.5 * r0;
  double e = fma(-h, g, 0.5);
  g = fma(g, e, g);
  h = fma(h, e, h);
  double d = fma(-g, g, sh) + sl;
  double y = fma(d, h, g);
  double rho = fma(-y, y, sh) + sl;
  constexpr double c1 = 0x1p-52 * (1.0 - 0x1p-40);
  if (fabs(rho) < y * c1) return y;
  return hypot_resolve(1.0, 0.0, q, qe, y, 0x1p-52, y == 1.0 ? 0x1p-53 : 0x1p-52);
}

// ---------------------------------------------------------------------------
// Correctly rounded hypot, binary32, the general route: evaluate in binary64
// (squares exact), round to binary32, and settle the one float midpoint that can separate the binary64
// value from the exact one by an exact sign test of S - m^2 (hi^2 - m^2 is
// exact in binary64, so only the addition of lo^2 rounds, which keeps the sign).
// ---------------------------------------------------------------------------
__device__ __attribute__((noinline)) float hypot_cr32_slow(float x, float y) {
  double a = fabs((double)x), b = fabs((double)y);
  double hi = fmax(a, b), lo = fmin(a, b);
  if (isinf(hi)) return (float)hi;
  double S = fma(hi, hi, lo * lo);
  if (S == 0.0) return 0.0f;
  // sqrt(S) to about 2^-40 relative: a reciprocal square root estimate and one
  // Goldschmidt step (S is far inside binary64's normal range).  The exact
  // midpoint test below needs r only within a small fraction of a binary32 ulp.
  double r0 = __builtin_amdgcn_rsq(S);
  double r = S * r0, h = 0.5 * r0;
  double e = fma(-h, r, 0.5);
  r = fma(r, e, r);
  float f = (float)r;
  double fd = isinf(f) ? 0x1p128 : (double)f;  // +inf stands for 2^128 here
  if (fd == r) return f;
  // f is the correctly rounded root unless sqrt(x^2 + y^2) lies beyond one of
  // the two rounding boundaries around f.  With d = sqrt(S) - r, S - r^2 =
  // d (2 r + d) and 2 r + d > r, so |d| < |S - r^2| / r; the residual comes from
  // one fma, and the rounding of S itself moves the root by at most r 2^-54.  So
  // f is certified when |r - f| + r 2^-52 + |S - r^2| / r stays below the
  // smaller distance from f to a rounding boundary (half the spacing of binary32
  // numbers at f; the spacing below a power of two is half as wide), tested
  // without a division; only the rare uncertified lanes take the exact test.
  if (f != 0.0f && !isinf(f)) {
    int ef = max(ilog2(fd), -126);
    double side = ldexp(1.0, ef - 24);
    if ((__float_as_uint(f) & 0x7fffffu) == 0u && ef > -126) side *= 0.5;
    double slack = side - fabs(r - fd) - r * 0x1p-52;
    double rho = fma(-r, r, S);
    if (slack > 0.0 && fabs(rho) < r * slack * 0.5) return f;
  }
  bool above = r > fd;
  float g;
  double gd;
  if (above) {
    if (f == 0x1.fffffep+127f) {
      g = __int_as_float(0x7f800000);
      gd = 0x1p128;
    } else {
      g = __uint_as_float(__float_as_uint(f) + 1u);
      gd = (double)g;
    }
  } else {
    g = __uint_as_float(__float_as_uint(f) - 1u);  // f > 0 here
    gd = (double)g;
  }
  double m = (fd + gd) * 0.5;
  double sgn = fma(-m, m, hi * hi) + lo * lo;  // sign of S - m^2, exactly
  if (above) {
    if (sgn > 0.0) return g;
    if (sgn == 0.0) return even_sig(f) ? f : g;
    return f;
  }
  if (sgn < 0.0) return g;
  if (sgn == 0.0) return even_sig(f) ? f : g;
  return f;
}


// ---------------------------------------------------------------------------
// Correctly rounded hypot, binary32, in binary32 arithmetic.  With hi >= lo > 0
// and hi = A 2^e (A in [1, 2)), an exponent gap above 13 leaves hi (lo^2 <
// 2^-26 hi^2 moves the root by less than a quarter ulp); otherwise S = A^2 + B^2
// (B = lo 2^-e, exact) is formed as a double-float sh + sl from exact squares
// (error below 2^-46 S), a reciprocal square root estimate (about 2^-23) and one
// Newton step on sh + sl give the candidate y, and y is the correctly rounded root when
// its residual rho = S - y^2 (one fma, exact by Sterbenz, plus sl) satisfies
// |rho| < y ulp(y) (1 - 2^-16): then |sqrt(S) - y| = |rho| / (sqrt(S) + y) stays
// below ulp(y)/2 with a margin of 2^-40 y^2 over every rounding error above.
// Below y = 2 the gap to the next smaller float is half as wide, so a negative
// residual there is left to the general route, as are uncertified lanes (about
// 2^-16 of them), results that could be subnormal (hi below 2^-126) and the
// overflow edge (handled by the final scaling, see below).
// ---------------------------------------------------------------------------
__device__ __attribute__((always_inline)) inline float hypot_cr(float x, float y) {
  const float a = fabsf(x), b = fabsf(y);
  const float hi = fmaxf(a, b), lo = fminf(a, b);
  if (lo == 0.0f || isinf(hi)) return hi;
  const int eh = ilog2(hi), el = ilog2(lo);
  if (eh - el > 13) return hi;
  if (eh < -126) return hypot_cr32_slow(x, y);
  const float A = ldexpf(hi, -eh), B = ldexpf(lo, -eh);  // exact
  const float p = A * A, pe = fmaf(A, A, -p), q = B * B, qe = fmaf(B, B, -q);
  const float sh = p + q;                                  // p >= q: Fast2Sum
  const float sl = (q - (sh - p)) + (pe + qe);
  const float r0 = __builtin_amdgcn_rsqf(sh);
  const float g = sh * r0, h = 0.5f * r0;
  const float d = fmaf(-g, g, sh) + sl;
  const float yv = fmaf(d, h, g);
  const float rho = fmaf(-yv, yv, sh) + sl;
  constexpr float c1 = 0x1p-23f * (1.0f - 0x1p-16f), c2 = 0x1p-22f * (1.0f - 0x1p-16f);
  const float thr = yv * (yv >= 2.0f ? c2 : c1);
  if (fabsf(rho) < thr && !(yv == 2.0f && rho < 0.0f))
    return ldexpf(yv, eh);  // y 2^e: exact, or +inf when the root rounds to 2^128
  return hypot_cr32_slow(x, y);
}

// hypot(t, 1) for 0 <= t <= 1: A = 1, no scaling; below 2^-13 the result is 1
__device__ __attribute__((always_inline)) inline float hypot1_le1(float t) {
  if (t < 0x1p-13f) return 1.0f;
  const float q = t * t, qe = fmaf(t, t, -q);
  const float sh = 1.0f + q;
  const float sl = (q - (sh - 1.0f)) + qe;
  const float r0 = __builtin_amdgcn_rsqf(sh);
  const float g = sh * r0, h = 0.5f * r0;
  const float d = fmaf(-g, g, sh) + sl;
  const float yv = fmaf(d, h, g);
  const float rho = fmaf(-yv, yv, sh) + sl;
  constexpr float c1 = 0x1p-23f * (1.0f - 0x1p-16f);
  if (fabsf(rho) < yv * c1) return yv;  // y in [1, sqrt 2]
  return hypot_cr32_slow(t, 1.0f);
}

// ---------------------------------------------------------------------------
// Divisions.  hipcc lowers a binary64 a / b to a reciprocal estimate, two
// Newton steps, a product, its residual and one correction (Markstein's
// scheme), bracketed by two range-scaling instructions and a fix-up for
// special operands.  Where the operands are known to need no scaling (normal
// operands and quotient, numerator above 2^-960, divisor below 2^1020) the
// bracket does nothing and is left out; one reciprocal then also serves two
// numerators.  The results are the IEEE quotients, bit for bit.  The binary32
// sequence (reciprocal estimate, one Newton step, a product, two residual
// corrections) is bracketed the same way and needs no scaling for normal
// operands and quotient, a numerator above 2^-100 and a divisor below 2^124;
// it is used unguarded for the (e,f) mantissa quotients, which always qualify.
// ---------------------------------------------------------------------------
__device__ inline double rcp_refined(double b) {
  double y = __builtin_amdgcn_rcp(b);
  double e = fma(-b, y, 1.0);
  y = fma(y, e, y);
  e = fma(-b, y, 1.0);
  return fma(y, e, y);
}
__device__ inline double div_with(double a, double b, double y) {
  double q = a * y;
  double r = fma(-b, q, a);
  return fma(r, y, q);
}

// a / b for a, b in [1/2, 1) (mantissas in frexp form)
__device__ inline double div_unit(double a, double b) { return div_with(a, b, rcp_refined(b)); }
__device__ inline float rcp_refined(float b) {
  float y = __builtin_amdgcn_rcpf(b);
  float e = fmaf(-b, y, 1.0f);
  return fmaf(e, y, y);
}
__device__ inline float div_with(float a, float b, float y) {
  float q = a * y;
  float r = fmaf(-b, q, a);
  q = fmaf(r, y, q);
  r = fmaf(-b, q, a);
  return fmaf(r, y, q);
}
__device__ inline float div_unit(float a, float b) { return div_with(a, b, rcp_refined(b)); }

// c = 1 / sec and s = t / sec, where sec = sqrt(1 + t^2) rounded (the secant of
// the angle with tangent t): the quotients are normal whenever t is 0 or
// |t| >= 2^-960, so only a huge secant (above 2^1020) or a tiny tangent takes
// the plain route.  In binary32 the guards cost more than the division steps
// they save (measured), so binary32 divides plainly here.
__device__ inline void cos_sin(double t, double sec, double &c, double &s) {
  if (sec <= 0x1p1020 && (t == 0.0 || fabs(t) >= 0x1p-960)) {
    double y = rcp_refined(sec);
    c = div_with(1.0, sec, y);
    s = (t == 0.0) ? t : div_with(t, sec, y);
  } else {
    c = 1.0 / sec;
    s = t / sec;
  }
}
__device__ inline void cos_sin(float t, float sec, float &c, float &s) {
  c = 1.0f / sec;
  s = t / sec;
}

// a1 / sec and a2 / sec for sec in [1, 2): one reciprocal serves both wherever
// 2^-960 <= |a_i| <= 2^1020 (normal quotients, exact residuals); zero and
// extreme numerators take the plain division (binary32: always, as above).
__device__ inline void div_by_sec(double a1, double a2, double sec, double &q1, double &q2) {
  bool f1 = fabs(a1) >= 0x1p-960 && fabs(a1) <= 0x1p1020;
  bool f2 = fabs(a2) >= 0x1p-960 && fabs(a2) <= 0x1p1020;
  if (f1 && f2) {
    double y = rcp_refined(sec);
    q1 = div_with(a1, sec, y);
    q2 = div_with(a2, sec, y);
  } else {
    q1 = a1 / sec;
    q2 = a2 / sec;
  }
}
__device__ inline void div_by_sec(float a1, float a2, float sec, float &q1, float &q2) {
  q1 = a1 / sec;
  q2 = a2 / sec;
}

// ---------------------------------------------------------------------------
// A hypot that is not correctly rounded, for the fast variant of the method
// (Algorithm tf has a branch of its own for it): with hi = max(|x|, |y|) and
// lo = min(|x|, |y|), hi sqrt(fma(r, r, 1)) for r = lo / hi, each operation
// rounded once (a few ulps from the exact value).  Computed here so that the
// result is that value bit for bit, with less work:
//  - r < 2^-27 (2^-12 in binary32) leaves fma(r, r, 1) = 1, so an exponent gap
//    that guarantees it returns hi at once, as does lo = 0;
//  - r is the quotient of lo and hi both scaled by 2^-e(hi) (exact: hi lands
//    in [1, 2) and lo, at least 2^-28 of it, stays normal), where the
//    reciprocal-based IEEE division needs no range scaling;
//  - 1 + r^2 lies in [1, 2], where sqrt_1p gives the correctly rounded root.
// hypot1_fast is the same function for (t, 1) with 0 <= t <= 1, where hi = 1
// and no division is needed.
// ---------------------------------------------------------------------------

// Correctly rounded sqrt(s) for s in [1, 2].  Just above 1, s = 1 + k 2^-52
// with a small k puts sqrt(s) = 1 + k 2^-53 - (k 2^-52)^2 / 8 + ... within far
// less than an ulp below 1 + k 2^-53: the nearest double for even k, a rounding
// midpoint for odd k, which then rounds down.  Such near-midpoints would send
// sqrt_dw_cr to its exact fallback for a large share of small tangents, so for
// s - 1 < 2^-26 (where the second-order term stays below 2^-55) the root is
// formed directly: 1 + ((s - 1)/2 - 2^-54) rounds to exactly that value (the
// inner terms are exact; the offset breaks the midpoint downwards and moves an
// even k's result by a quarter ulp only).
__device__ __attribute__((always_inline)) inline double sqrt_1p(double s) {
  if (s < 1.0 + 0x1p-26) return 1.0 + fma(s - 1.0, 0.5, -0x1p-54);
  return sqrt_dw_cr(s, 0.0, s, 0.0, 0.0, 0.0);
}
__device__ __attribute__((always_inline)) inline double hypot_fast(double x, double y) {
  double a = fabs(x), b = fabs(y);
  double hi = fmax(a, b), lo = fmin(a, b);
  if (lo == 0.0 || isinf(hi)) return hi;
  int eh = ilog2(hi);
  if (eh - ilog2(lo) >= 28) return hi;
  double hs = scale2(hi, -eh), ls = scale2(lo, -eh);
  double r = div_with(ls, hs, rcp_refined(hs));
  return hi * sqrt_1p(fma(r, r, 1.0));
}
__device__ __attribute__((always_inline)) inline double hypot1_fast(double t) {
  if (t < 0x1p-27) return 1.0;
  return sqrt_1p(fma(t, t, 1.0));
}
__device__ __attribute__((always_inline)) inline float hypot_fast(float x, float y) {
  float a = fabsf(x), b = fabsf(y);
  float hi = fmaxf(a, b), lo = fminf(a, b);
  if (lo == 0.0f || isinf(hi)) return hi;
  if (ilog2(hi) - ilog2(lo) >= 13) return hi;
  float r = lo / hi;
  float s = fmaf(r, r, 1.0f);
  return hi * sqrtf(s);  // correctly rounded: the library is built for it
}
__device__ __attribute__((always_inline)) inline float hypot1_fast(float t) {
  if (t < 0x1p-12f) return 1.0f;
  return sqrtf(fmaf(t, t, 1.0f));
}

// the hypot of the variant: correctly rounded (CR) or fast
template <bool CR, class R> __device__ __attribute__((always_inline)) inline R hyp(R x, R y) {
  if constexpr (CR)
    return hypot_cr(x, y);
  else
    return hypot_fast(x, y);
}
// the same for (t, 1) with 0 <= t <= 1
template <bool CR, class R> __device__ __attribute__((always_inline)) inline R hyp1(R t) {
  if constexpr (CR)
    return hypot1_le1(t);
  else
    return hypot1_fast(t);
}

// ---------------------------------------------------------------------------
// (e,f) pairs (Sect. 2, eqs. unary, binary, plus, minus, prec).  Kept as frexp
// returns them: x = f 2^e with f in [1/2, 1), and (0, 0) for zero; the pair of
// the paper is (e - 1, 2 f), formed on output.  The two forms differ by exact
// power-of-two scalings, so every product, quotient and comparison rounds and
// orders as in the paper's form.
// ---------------------------------------------------------------------------
template <class R> struct EF {
  int e;
  R f;
};

template <class R> __device__ inline EF<R> nrm(R x) {  // N(x)
  EF<R> r;
  r.f = frexp_w(x, &r.e);  // frexp(0) = (0, 0)
  return r;
}

template <class R> __device__ inline R flo(EF<R> x) { return scale2(x.f, x.e); }  // fl(w)

template <class R> __device__ inline EF<R> ef_twice(EF<R> x) {  // 2 (.) x
  if (x.f != (R)0) x.e += 1;
  return x;
}

// products and quotients of non-zero pairs: the mantissa product lies in
// [1/4, 1) and the quotient in (1/2, 2), both normal and non-zero
template <class R> __device__ inline EF<R> ef_mul(EF<R> x, EF<R> y) {
  EF<R> z = nrm(x.f * y.f);
  z.e += x.e + y.e;
  return z;
}

template <class R> __device__ inline EF<R> ef_div(EF<R> x, EF<R> y) {
  EF<R> z = nrm(div_unit(x.f, y.f));
  z.e += x.e - y.e;
  return z;
}

template <class R> __device__ inline EF<R> ef_plus(R x, R y) {  // x, y > 0
  R z = x + y;
  if (z <= Lim<R>::nu()) return nrm(z);
  EF<R> w = nrm(x * (R)0.5 + y * (R)0.5);
  w.e += 1;
  return w;
}

template <class R> __device__ inline EF<R> ef_minus(R x, R y) {  // x, y > 0
  EF<R> w;
  if (x == y) {
    w.e = 0;
    w.f = (R)0;
    return w;
  }
  R z = x - y;
  if (fabs(z) >= Lim<R>::mu()) return nrm(z);
  int lx = ilog2(x), ly = ilog2(y);
  int c = Lim<R>::e_mu + Lim<R>::p - 1 - (lx < ly ? lx : ly);
  w = nrm(ldexp_w(x, c) - ldexp_w(y, c));  // upscaling: exact
  w.e -= c;
  return w;
}

template <class R> __device__ inline int sign3(R f) { return (f > (R)0) - (f < (R)0); }

template <class R> __device__ inline bool ef_prec(EF<R> x, EF<R> y) {
  int sx = sign3(x.f), sy = sign3(y.f);
  if (sx != sy) return sx < sy;
  return (x.e < y.e) || (x.e == y.e && x.f < y.f);
}

// ---------------------------------------------------------------------------
// The wider-precision element of eq. (EXT):
//   fl(FL(FL(x1 y1 + x2 y2) / d))    (subtraction: the caller negates x2).
// binary32: T = binary64 (products exact, sum and quotient rounded in binary64,
// then one rounding to binary32).
// binary64: T = double-word.  Both products are formed exactly from the
// factors' mantissas; both are scaled by the larger product's exponent;
// AccurateDWPlusDW, then DWDivFP3 by d's mantissa (Joldes-Muller-Popescu 2017,
// Algorithms 6 and 15); the leading word is scaled back with one rounding.
// ---------------------------------------------------------------------------
__device__ inline float ext_w(float x1, float y1, float x2, float y2, float d) {
  double s = (double)x1 * (double)y1 + (double)x2 * (double)y2;
  return (float)(s / (double)d);
}

__device__ __attribute__((always_inline)) inline double ext_w(double x1, double y1, double x2, double y2,
                                                             double d) {
  // factors as frexp mantissas in [1/2, 1): each product of two is 4 times
  // smaller than the product of the [1, 2) mantissas, and the scalings below
  // carry the factor 4 back before anything can round
  int a1, b1, a2, b2;
  double m1 = frexp(x1, &a1), n1 = frexp(y1, &b1), m2 = frexp(x2, &a2), n2 = frexp(y2, &b2);
  int k1 = a1 + b1, k2 = a2 + b2;
  int K = k1 > k2 ? k1 : k2;
  double p1h, p1l, p2h, p2l;
  two_prod(m1, n1, p1h, p1l);
  two_prod(m2, n2, p2h, p2l);
  p1h = scale2(p1h, k1 - K + 2);
  p1l = scale2(p1l, k1 - K + 2);
  p2h = scale2(p2h, k2 - K + 2);
  p2l = scale2(p2l, k2 - K + 2);
  // AccurateDWPlusDW
  double sh, sl, th, tl, vh, vl, xh, xl;
  two_sum(p1h, p2h, sh, sl);
  two_sum(p1l, p2l, th, tl);
  fast_two_sum(sh, sl + th, vh, vl);
  fast_two_sum(vh, tl + vl, xh, xl);
  if (xh == 0.0) return 0.0;
  // DWDivFP3 by the mantissa of d
  int ed = ilog2(d);
  double dm = ldexp(d, -ed);
  // both quotients by dm in [1, 2) share one refined reciprocal while their
  // numerators are zero or at least 2^-960 (see the division section)
  double yd = rcp_refined(dm);
  double qh;
  if (fabs(xh) >= 0x1p-960)
    qh = div_with(xh, dm, yd);
  else
    qh = xh / dm;
  double ph, pl;
  two_prod(qh, dm, ph, pl);
  double r2 = (xh - ph) + (xl - pl);
  double dl;
  if (r2 == 0.0 || fabs(r2) >= 0x1p-960)
    dl = div_with(r2, dm, yd);
  else
    dl = r2 / dm;
  double zh, zl;
  fast_two_sum(qh, dl, zh, zl);
  return scale2(zh, K - 2 - ed);  // K counts the two factors of 2 of the frexp form
}

// ---------------------------------------------------------------------------
// Factored orthogonal matrices.  Every U and V the method builds is a signed
// permutation times a plane rotation times a signed permutation (the P and S
// factors around U_theta, U_phi, V_psi in Sect. 3), so they are kept as
// L rot(c, s) R with L, R coded in three bits and multiplied symbolically; the
// entries are formed once, at the end (each is +-c or +-s, exactly).
// ---------------------------------------------------------------------------

// Signed permutation Q: column j of Q is (-1)^{n_j} e_{pi(j)}, pi swaps iff x.
struct SP {
  uint32_t x, n0, n1;
};
__device__ inline SP sp_id() { return SP{0u, 0u, 0u}; }
__device__ inline SP sp_x(bool on) { return SP{on ? 1u : 0u, 0u, 0u}; }
__device__ inline SP sp_diag(bool neg0, bool neg1) {
  return SP{0u, neg0 ? 1u : 0u, neg1 ? 1u : 0u};
}
// (A B) e_j = (-1)^{nB_j} A e_{piB(j)} = (-1)^{nB_j + nA_{piB(j)}} e_{piA(piB(j))}
__device__ inline SP sp_mul(SP a, SP b) {
  SP r;
  r.x = a.x ^ b.x;
  r.n0 = b.n0 ^ (b.x ? a.n1 : a.n0);
  r.n1 = b.n1 ^ (b.x ? a.n0 : a.n1);
  return r;
}

// L rot(c, s) Rt with rot(c, s) = [c -s; s c]
template <class R> struct Fac {
  SP L;
  R c, s;
  SP Rt;
};

template <class R> __device__ inline Fac<R> fac(SP L, R c, R s, SP Rt) {
  Fac<R> f;
  f.L = L;
  f.c = c;
  f.s = s;
  f.Rt = Rt;
  return f;
}

template <class R> __device__ inline R neg_if(R v, uint32_t n) { return n ? -v : v; }

// The first column (c, s) of L rot(c, s) Rt, and whether its determinant is -1.
template <class R> __device__ inline void fac_out(const Fac<R> &f, R &c1, R &s1, bool &detneg) {
  // rot Rt e_0 = (-1)^{n0} rot e_{pi(0)}
  R v0 = f.Rt.x ? -f.s : f.c, v1 = f.Rt.x ? f.c : f.s;
  v0 = neg_if(v0, f.Rt.n0);
  v1 = neg_if(v1, f.Rt.n0);
  // L v: component k lands in row pi_L(k) with the sign (-1)^{nL_k}
  R w0 = neg_if(v0, f.L.n0), w1 = neg_if(v1, f.L.n1);
  R u0 = f.L.x ? w1 : w0, u1 = f.L.x ? w0 : w1;
  c1 = u0 + (R)0;  // canonical zero: -0 -> +0
  s1 = u1 + (R)0;
  detneg = ((f.L.x ^ f.L.n0 ^ f.L.n1 ^ f.Rt.x ^ f.Rt.n0 ^ f.Rt.n1) & 1u) != 0;
}

template <class R> __device__ inline bool negative(R x) { return x < (R)0; }

// Result of one 2x2 SVD: U = [cu, -dU su; su, dU cu], V likewise, sigma_i =
// f_i 2^e_i (sigma1 >= sigma2 >= 0), info bits as in the public header.
template <class R> struct Svd2 {
  R cu, su, cv, sv, f1, f2;
  int e1, e2;
  uint32_t info;
};

enum : uint32_t {
  I_DETU = 1u << 8, I_DETV = 1u << 9, I_EXT = 1u << 10, I_RSWAP = 1u << 11,
  I_TPSI_OVF = 1u << 12, I_PSIG = 1u << 13, I_DEGEN = 1u << 14, I_NONFINITE = 1u << 15,
};

// class masks over the 16 types of eq. (ts)
constexpr uint32_t CL9 = (1u << 0) | (1u << 1) | (1u << 2) | (1u << 4) | (1u << 6) | (1u << 8) |
                         (1u << 9);
constexpr uint32_t CL3 = (1u << 3) | (1u << 12);
constexpr uint32_t CL5 = (1u << 5) | (1u << 10);
constexpr uint32_t CL13 = (1u << 7) | (1u << 11) | (1u << 13) | (1u << 14);

template <class R> __device__ inline int ztype(R g11, R g21, R g12, R g22) {
  return (g11 != (R)0) | ((g21 != (R)0) << 1) | ((g12 != (R)0) << 2) | ((g22 != (R)0) << 3);
}

// A (prescaled) 2x2 matrix [a b; c d], row-major.
template <class R> struct M2 {
  R a, b, c, d;
};

// A partial SVD of a (prescaled) matrix: G' = U diag(s1, s2) V^T.
template <class R> struct Part {
  Fac<R> U, V;
  EF<R> s1, s2;
};

// Sect. 3.1, class 9: at most one permutation per side into the 0/1/9 form
// with |d11| >= |d22|; the row signs go into U (U = P_U S, V = P_V).
template <class R> __device__ __attribute__((always_inline)) Part<R> part9(M2<R> G, int t) {
  bool pu = false, pv = false;
  if (t == 2) pu = true;
  else if (t == 4) pv = true;
  else if (t == 8) pu = pv = true;
  else if (t == 6) {
    if (fabs(G.c) >= fabs(G.b)) pu = true; else pv = true;
  } else if (t == 9) {
    if (fabs(G.a) < fabs(G.d)) pu = pv = true;
  }
  // the diagonal of D = P_U^T G P_V
  R d11 = pu ? (pv ? G.d : G.c) : (pv ? G.b : G.a);
  R d22 = pu ? (pv ? G.a : G.b) : (pv ? G.c : G.d);
  Part<R> r;
  r.U = fac(sp_mul(sp_x(pu), sp_diag(negative(d11), negative(d22))), (R)1, (R)0, sp_id());
  r.V = fac(sp_x(pv), (R)1, (R)0, sp_id());
  r.s1 = nrm(fabs(d11));
  r.s2 = nrm(fabs(d22));
  return r;
}

// Sect. 3.1, classes 3 (one non-zero column) and 5 (one non-zero row): the
// non-zero pair made non-negative by signs, the larger one first, and one Givens
// rotation with tangent smaller/larger (eq. Givens, Lemma sincostheta).
template <class R, bool CR> __device__ __attribute__((always_inline)) Part<R> part35(M2<R> G, int t) {
  bool col = (t == 3 || t == 12);
  bool pfirst = (t == 12 || t == 10);  // P_V for t = 12, P_U for t = 10
  R a, b;
  if (col) { a = pfirst ? G.b : G.a; b = pfirst ? G.d : G.c; }
  else { a = pfirst ? G.c : G.a; b = pfirst ? G.d : G.b; }
  bool na = negative(a), nb = negative(b);
  a = fabs(a);
  b = fabs(b);
  bool sw = a < b;
  if (sw) { R t2 = a; a = b; b = t2; }
  R tn = b / a;
  R sec = hyp1<CR>(tn);  // 0 <= tan <= 1
  R gc, gs;
  cos_sin(tn, sec, gc, gs);
  Fac<R> W = fac(sp_mul(sp_diag(na, nb), sp_x(sw)), gc, gs, sp_id());
  Fac<R> P = fac(sp_x(pfirst), (R)1, (R)0, sp_id());
  Part<R> r;
  r.U = col ? W : P;
  r.V = col ? P : W;
  r.s1 = nrm(hyp<CR>(a, b));
  r.s2 = nrm((R)0);
  return r;
}

// fl(a / b) < eps for a >= 0, b > 0, without the division.  eps is a power of
// two, so the quotient rounds below eps iff it lies below the midpoint
// eps (1 - 2^-(p+1)) (a tie rounds up to the even eps), and since the float
// next below b eps is at least b eps 2^-p away, that holds iff a < b eps
// exactly.  fma(-b, eps, a) rounds a - b eps once, keeping its sign whenever
// b eps is normal (a non-zero difference is then at least 2^-1074 in size).
template <class R> __device__ inline bool ratio_below_eps(R a, R b) {
  if (b >= Lim<R>::eps_normal_from()) return fma(-b, Lim<R>::eps(), a) < (R)0;
  return a / b < Lim<R>::eps();
}

// The SVD of R~ = [a b; 0 d], a >= d > 0, b > 0 (Sect. 3.3.1).
template <class R> struct Tri {
  R cphi, sphi, tphi, cpsi, spsi, tpsi;
  EF<R> s1, s2;
  bool psig, ovf;
};

template <class R, bool CR> __device__ __attribute__((always_inline)) Tri<R> tri_svd(R a, R b, R d) {
  const R inf = (R)INFINITY;
  Tri<R> o;
  // Algorithm tf: tan(2 phi), cases in their listed order.  The two cases that
  // end in the (e,f) quotient 2bd / (x y) share one copy of it (x = y = a for
  // eq. t2f''', x, y = h -+ d in the general case), and so do the two cases of
  // eq. t2f'', so lanes of a wave that take different cases do not execute
  // them twice.
  R t2 = (R)0;
  bool simple = (a == d);  // eq. t2f''
  bool ef_case = false;
  EF<R> x = nrm(a), y = x;
  if (!simple) {
    if (b == d) {  // eq. t2f'''
      ef_case = true;
    } else if (ratio_below_eps(a, b)) {
      simple = true;  // eq. t2f''
    } else if (!CR) {
      // the branch for a hypot that is not correctly rounded: x and y are the
      // smaller of a, b and d divided by the larger of a, b, and tan(2 phi) =
      // 2xy / (1 + (x-y)(x+y)) for a > b, 2y / (1 + (x-y)(x+y)) otherwise (no
      // squares of the inputs; a negative denominator counts as 0).  Written
      // without a branch so that lanes of both kinds share the divisions.
      R m = fmax(a, b);
      R xq = fmin(a, b) / m, yq = d / m;
      R num = (a > b) ? ((R)2 * xq) * yq : (R)2 * yq;
      t2 = num / fmax(fma(xq - yq, xq + yq, (R)1), (R)0);
    } else {
      R h = hypot_cr(a, b);
      if (h == d) {
        t2 = inf;
      } else {
        y = ef_plus(h, d);
        x = ef_minus(h, d);
        ef_case = true;
      }
    }
  }
  if (simple) t2 = ((R)2 * d) / b;
  if (ef_case) t2 = flo(ef_div(ef_mul(ef_twice(nrm(b)), nrm(d)), ef_mul(x, y)));
  R tphi = (t2 == inf) ? (R)1 : t2 / ((R)1 + hyp<CR>(t2, (R)1));  // eq. tf
  R sphi_sec = hyp1<CR>(tphi);  // 0 <= tan(phi) <= 1
  o.tphi = tphi;
  cos_sin(tphi, sphi_sec, o.cphi, o.sphi);
  // Algorithm tp
  R tt = fma(d, tphi, b);
  R tpsi = tt / a;
  o.tpsi = tpsi;
  EF<R> s1, s2;
  if (tpsi == inf) {  // eq. tp' and the sigma assignment of Algorithm tp
    o.ovf = true;
    EF<R> et = nrm(tt);
    EF<R> bcos = ef_div(nrm(a), et);
    o.cpsi = flo(bcos);
    o.spsi = (R)1;
    s1 = et;
    s2 = ef_mul(nrm(d), bcos);
  } else {  // eq. s'
    o.ovf = false;
    R spsi_sec = hyp<CR>(tpsi, (R)1);
    cos_sin(tpsi, spsi_sec, o.cpsi, o.spsi);
    EF<R> sp = ef_div(nrm(sphi_sec), nrm(spsi_sec));
    s1 = ef_div(nrm(a), sp);
    s2 = ef_mul(nrm(d), sp);
  }
  o.psig = ef_prec(s1, s2);
  o.s1 = o.psig ? s2 : s1;
  o.s2 = o.psig ? s1 : s2;
  return o;
}

// The whole method for one matrix; CR selects the correctly rounded hypot (the
// method as analysed) or the fast variant.
template <class R, bool CR = true>
__device__ __attribute__((always_inline)) Svd2<R> svd2(R g11, R g21, R g12, R g22) {
  Svd2<R> out;
  int t = ztype(g11, g21, g12, g22);
  if (!(isfinite(g11) && isfinite(g21) && isfinite(g12) && isfinite(g22))) {
    R nan = (R)NAN;
    out.cu = out.su = out.cv = out.sv = out.f1 = out.f2 = nan;
    out.e1 = out.e2 = 0;
    out.info = (uint32_t)t | I_NONFINITE;
    return out;
  }
  // phase 1: prescaling (class 9 is not scaled)
  int s = 0;
  uint32_t tb = 1u << t;
  if (!(tb & CL9)) {
    int eg = -0x7fffffff;
    if (g11 != (R)0) eg = max(eg, ilog2(g11));
    if (g21 != (R)0) eg = max(eg, ilog2(g21));
    if (g12 != (R)0) eg = max(eg, ilog2(g12));
    if (g22 != (R)0) eg = max(eg, ilog2(g22));
    int stype = (t == 15) ? 2 : 1;
    s = Lim<R>::e_nu - eg - stype;
  }
  M2<R> G;
  if (s >= 0) {
    G = M2<R>{ldexp_w(g11, s), ldexp_w(g12, s), ldexp_w(g21, s), ldexp_w(g22, s)};
  } else {  // s in {-1, -2}: one IEEE rounding each
    R f = (s == -1) ? (R)0.5 : (R)0.25;
    G = M2<R>{g11 * f, g12 * f, g21 * f, g22 * f};
  }
  int t1 = ztype(G.a, G.c, G.b, G.d);
  uint32_t tb1 = 1u << t1;
  uint32_t info = (uint32_t)t | ((uint32_t)t1 << 4);

  Part<R> part;
  bool tri = false;
  R r11 = 0, r12 = 0, r22 = 0;
  // left factors of U and V in front of the triangular SVD (U_+, V_+)
  SP UL = sp_id(), VL = sp_id();
  // class 15 pieces kept for the heuristic
  R tan_t = 0, sec_t = 1;
  bool is15 = false, s22neg = false;

  // the simple classes of Sect. 3.1, entered directly or from the degenerate
  // exit of class 15 (one inlined copy serves both)
  bool simple = (tb1 & (CL9 | CL3 | CL5)) != 0, degen = false;
  M2<R> Gs = G;
  int ts = t1;
  if (simple) {
  } else if (tb1 & CL13) {
    // Sect. 3.2.1: permute into [x y; 0 z], then three sign changes:
    // U_+ = P_U S11 S22 = P_U diag(sgn x, sgn z'), V_+ = P_V S12 = P_V diag(1, sgn y')
    bool pu = (t1 == 14 || t1 == 11), pv = (t1 == 7 || t1 == 11);
    R x = pu ? (pv ? G.d : G.c) : (pv ? G.b : G.a);
    R y = pu ? (pv ? G.c : G.d) : (pv ? G.a : G.b);
    R z = pu ? (pv ? G.a : G.b) : (pv ? G.c : G.d);
    bool nx = negative(x);
    y = nx ? -y : y;
    bool ny = negative(y);
    z = ny ? -z : z;
    bool nz = negative(z);
    r11 = fabs(x);
    r12 = fabs(y);
    r22 = fabs(z);
    UL = sp_mul(sp_x(pu), sp_diag(nx, nz));
    VL = sp_mul(sp_x(pv), sp_diag(false, ny));
    tri = true;
  } else {
    // Sect. 3.2.2: class 15, the fully pivoted URV
    is15 = true;
    R w1 = hyp<CR>(G.a, G.c), w2 = hyp<CR>(G.b, G.d);
    bool pv = w1 < w2;
    if (pv) {
      R tw = w1; w1 = w2; w2 = tw;
      tw = G.a; G.a = G.b; G.b = tw;
      tw = G.c; G.c = G.d; G.d = tw;
    }
    bool s1n0 = negative(G.a), s1n1 = negative(G.c);
    if (s1n0) { G.a = -G.a; G.b = -G.b; }
    if (s1n1) { G.c = -G.c; G.d = -G.d; }
    bool pu15 = G.a < G.c;
    if (pu15) {
      R tw = G.a; G.a = G.c; G.c = tw;
      tw = G.b; G.b = G.d; G.d = tw;
    }
    // G''' = [G.a G.b; G.c G.d], G.a >= G.c > 0
    tan_t = G.c / G.a;
    sec_t = hyp1<CR>(tan_t);  // 0 < tan(theta) <= 1
    r11 = w1;
    bool exact = fma(-tan_t, G.a, G.c) == (R)0;
    bool same = negative(G.b) == negative(G.d);
    // the element without cancellation: r12 (same signs) or r22 (opposite)
    R P = same ? G.d : -G.b, Q = same ? G.b : G.d;
    R ngood = fma(P, tan_t, Q), nother;
    if (exact) {
      R P2 = same ? -G.b : G.d, Q2 = same ? G.d : G.b;
      nother = fma(P2, tan_t, Q2);
    } else {
      // eq. EXT: r22 = (g22 g11 - g12 g21)/g11/sec or r12 = (g12 g11 + g22 g21)/g11/sec
      R x1 = same ? G.d : G.b, x2 = same ? -G.b : G.d;
      nother = ext_w(x1, G.a, x2, G.c, G.a);
      info |= I_EXT;
    }
    R rgood, rother;
    div_by_sec(ngood, nother, sec_t, rgood, rother);
    r12 = same ? rgood : rother;
    r22 = same ? rother : rgood;
    UL = sp_mul(sp_diag(s1n0, s1n1), sp_x(pu15));  // S_1 P_U
    VL = sp_x(pv);                                  // P_V
    if (r12 == (R)0 || r22 == (R)0) {
      // a zero appeared: R'' = [r11 r12; 0 r22] is of type 9/1 or 5 and is
      // finished as in Sect. 3.1; U = S_1 P_U U_theta U_R, V = P_V V_R, where
      // U_R is a signed permutation in both cases
      info |= I_DEGEN;
      Gs = M2<R>{r11, r12, (R)0, r22};
      ts = ztype(Gs.a, Gs.c, Gs.b, Gs.d);
      simple = degen = true;
    } else {
      bool n12 = negative(r12);
      if (n12) r22 = -r22;
      VL = sp_mul(VL, sp_diag(false, n12));  // V_+ = P_V S12
      r12 = fabs(r12);
      s22neg = negative(r22);
      r22 = fabs(r22);
      tri = true;
    }
  }

  if (simple) {
    part = ((1u << ts) & CL9) ? part9(Gs, ts) : part35<R, CR>(Gs, ts);
    if (degen) {
      R ct, st;
      cos_sin(tan_t, sec_t, ct, st);
      part.U = fac(UL, ct, st, part.U.L);
      part.V = fac(sp_mul(VL, part.V.L), part.V.c, part.V.s, part.V.Rt);
    }
  }

  if (tri) {
    // phase 3: swap the diagonal through R^T (eq. RT) if r11 < r22
    bool swp = r11 < r22;
    if (swp) info |= I_RSWAP;
    R ta_ = swp ? r22 : r11, td_ = swp ? r11 : r22;  // one inlined copy for both cases
    Tri<R> tr = tri_svd<R, CR>(ta_, r12, td_);
    if (tr.ovf) info |= I_TPSI_OVF;
    if (tr.psig) info |= I_PSIG;
    // common right factor S2 P_sigma (S2 = diag(1,-1) when swapped); the
    // rotations of eq. RT are rot(sin psi, cos psi), rot(sin phi, cos phi) then
    SP RT = sp_mul(sp_diag(false, swp), sp_x(tr.psig));
    R cu_ = swp ? tr.spsi : tr.cphi, su_ = swp ? tr.cpsi : tr.sphi;
    R cv_ = swp ? tr.sphi : tr.cpsi, sv_ = swp ? tr.cphi : tr.spsi;
    part.V = fac(VL, cv_, sv_, RT);  // V = V_+ V_bpsi P_sigma
    if (!is15) {
      part.U = fac(UL, cu_, su_, RT);  // U = U_+ U_bphi P_sigma
    } else {
      // class 15: merge U_theta and U_bphi into one rotation by tan(bphi +- theta)
      // (eqs. p+t, p-t, tan+-); S22 = diag(1, sgn r22) joins the left factor
      R tbp = swp ? (R)1 / tr.tpsi : tr.tphi;
      R ca, sa;
      if (isinf(tbp)) {
        R ct, st;
        cos_sin(tan_t, sec_t, ct, st);
        ca = s22neg ? st : -st;
        sa = ct;
      } else {
        R num = s22neg ? tbp - tan_t : tbp + tan_t;
        R den = fma(s22neg ? tbp : -tbp, tan_t, (R)1);
        if (den == (R)0) {
          ca = (R)0;
          sa = negative(num) ? (R)-1 : (R)1;
        } else {
          R ta = num / den;
          R sa_sec = hyp<CR>(ta, (R)1);
          R sd = negative(den) ? (R)-1 : (R)1;
          R c0, s0;
          cos_sin(ta, sa_sec, c0, s0);
          ca = sd * c0;
          sa = sd * s0;
        }
      }
      part.U = fac(sp_mul(UL, sp_diag(false, s22neg)), ca, sa, RT);
    }
    part.s1 = tr.s1;
    part.s2 = tr.s2;
  }

  // backscale: sigma_i = 2^-s (.) sigma~_i' (Sect. 3.3.2)
  bool nu_, nv_;
  fac_out(part.U, out.cu, out.su, nu_);
  fac_out(part.V, out.cv, out.sv, nv_);
  if (nu_) info |= I_DETU;
  if (nv_) info |= I_DETV;
  out.f1 = part.s1.f * (R)2;  // frexp form -> the paper's (e, f), f in [1, 2)
  out.f2 = part.s2.f * (R)2;
  out.e1 = (part.s1.f != (R)0) ? part.s1.e - 1 - s : 0;
  out.e2 = (part.s2.f != (R)0) ? part.s2.e - 1 - s : 0;
  out.info = info | ((uint32_t)(uint16_t)(int16_t)s << 16);
  return out;
}

}  // namespace ksvd2
