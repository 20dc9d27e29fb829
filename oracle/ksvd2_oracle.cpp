/*
 * CPU oracle for the enhanced Kogbetliantz SVD of order two
 * (V. Novakovic, "Arithmetical enhancements of the Kogbetliantz method for
 * the SVD of order two", arXiv 2407.13116), and for the batched two-sided
 * Kogbetliantz sweep that calls it.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * reference that the GPU path is checked against.  Only the test-suite, the
 * smoke check and the CPU-baseline leg of the benchmark may load it.  It
 * shares no code, header or table with the GPU library, and the GPU library
 * never loads it.
 *
 * Build: g++ -O2 -std=c++17 -ffp-contract=off -fno-fast-math -fopenmp -fPIC
 *        -shared (no contraction: every fused multiply-add below is an
 *        explicit std::fma call, every other operation is one IEEE rounding).
 *
 * Organisation (each part cites the passage of the paper it follows):
 *   1. exact, integer-based, correctly rounded hypot            (Sect. 2)
 *   2. (e,f) exponent-"mantissa" pairs and their operations      (Sect. 2)
 *   3. double-word arithmetic for the wider datatype T of eq. (EXT), f64 only
 *   4. the 2x2 SVD: classification + prescaling (Sect. 3.1), the simple
 *      classes (Sect. 3.1), the URV factorisation (Sect. 3.2), the SVD of
 *      the triangular factor (Sect. 3.3.1, Algorithms tf/tp) and the
 *      assembly with the left-vector heuristic (Sect. 3.3.2)
 *   4b. the complex 2x2 SVD (Sect. 3.4)
 *   5. the Kogbetliantz sweep over an n x n matrix (Sect. 1, eq. (SVD))
 *   5b. rectangular inputs: QR with column pivoting before, Q after the sweep
 *   6. extern "C" batch drivers (OpenMP) for the test-suite
 */
#include <algorithm>
#include <cfloat>
#include <climits>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

/* ------------------------------------------------------------------------ */
/* Floating-point format constants (Sect. 2: p, eps = 2^-p, e_mu, e_nu).      */
/* ------------------------------------------------------------------------ */
template <class R> struct Fmt;
template <> struct Fmt<double> {
  static constexpr int p = 53;
  static constexpr int e_mu = -1022;
  static constexpr int e_nu = 1023;
  static double mu() { return DBL_MIN; }
  static double nu() { return DBL_MAX; }
  static double eps() { return 0x1p-53; }
};
template <> struct Fmt<float> {
  static constexpr int p = 24;
  static constexpr int e_mu = -126;
  static constexpr int e_nu = 127;
  static float mu() { return FLT_MIN; }
  static float nu() { return FLT_MAX; }
  static float eps() { return 0x1p-24f; }
};

/* ------------------------------------------------------------------------ */
/* 1. Correctly rounded hypot (Sect. 2: hypot(a,b) = fl(sqrt(a^2+b^2)),      */
/*    assumed correctly rounded).  Construction: a candidate from long       */
/*    double, then exact integer comparisons of a^2+b^2 against the squares  */
/*    of the rounding midpoints around the candidate, moving the candidate   */
/*    until it is the round-to-nearest-even value.  Obviously correct; slow.  */
/* ------------------------------------------------------------------------ */
struct U256 {
  uint64_t w[4];
};

static U256 u_from128(unsigned __int128 v) {
  U256 r;
  r.w[0] = (uint64_t)v;
  r.w[1] = (uint64_t)(v >> 64);
  r.w[2] = 0;
  r.w[3] = 0;
  return r;
}

static U256 u_shl(U256 a, int s) {
  U256 r = {{0, 0, 0, 0}};
  int limbs = s / 64, bits = s % 64;
  for (int i = 3; i >= 0; --i) {
    int src = i - limbs;
    if (src < 0) continue;
    uint64_t v = a.w[src] << bits;
    if (bits && src - 1 >= 0) v |= a.w[src - 1] >> (64 - bits);
    r.w[i] = v;
  }
  return r;
}

static U256 u_add(U256 a, U256 b) {
  U256 r;
  unsigned __int128 c = 0;
  for (int i = 0; i < 4; ++i) {
    c += (unsigned __int128)a.w[i] + b.w[i];
    r.w[i] = (uint64_t)c;
    c >>= 64;
  }
  return r;
}

static int u_cmp(U256 a, U256 b) {
  for (int i = 3; i >= 0; --i) {
    if (a.w[i] != b.w[i]) return a.w[i] < b.w[i] ? -1 : 1;
  }
  return 0;
}

/* Exact dyadic m * 2^k of a non-negative double (floats convert exactly). */
struct Dy {
  uint64_t m;
  int k;
};

static Dy dy_of(double x) {
  Dy d;
  if (x == 0) {
    d.m = 0;
    d.k = 0;
    return d;
  }
  int e;
  double f = std::frexp(x, &e); /* x = f 2^e, f in [1/2, 1) */
  d.m = (uint64_t)std::ldexp(f, 53);
  d.k = e - 53;
  return d;
}

/* sign(a^2 + b^2 - ((lo + hi)/2)^2), exactly.  `hi` may stand for 2^(e_nu+1)
   (the value "just above the largest finite", used for the overflow
   midpoint), passed as hi_pow2 >= 0 with hi ignored. */
static int cmp_sumsq_mid(double a, double b, double lo, double hi, int hi_pow2) {
  Dy A = dy_of(a), B = dy_of(b), L = dy_of(lo), H;
  if (hi_pow2 >= 0) {
    H.m = 1;
    H.k = hi_pow2;
  } else {
    H = dy_of(hi);
  }
  /* midpoint = (L + H)/2 = M 2^(kq-1) */
  int kq = std::min(L.m ? L.k : H.k, H.k);
  unsigned __int128 M = 0;
  if (L.m) M += (unsigned __int128)L.m << (L.k - kq);
  M += (unsigned __int128)H.m << (H.k - kq);
  /* exponents of the three squares */
  int ea = 2 * A.k, eb = 2 * B.k, em = 2 * (kq - 1);
  int E = em;
  if (A.m) E = std::min(E, ea);
  if (B.m) E = std::min(E, eb);
  U256 lhs = {{0, 0, 0, 0}};
  if (A.m) lhs = u_add(lhs, u_shl(u_from128((unsigned __int128)A.m * A.m), ea - E));
  if (B.m) lhs = u_add(lhs, u_shl(u_from128((unsigned __int128)B.m * B.m), eb - E));
  /* M < 2^56, M^2 < 2^112: square in two 128-bit halves */
  uint64_t Mlo = (uint64_t)M, Mhi = (uint64_t)(M >> 64);
  U256 m2 = u_from128((unsigned __int128)Mlo * Mlo);
  if (Mhi) {
    U256 cross = u_shl(u_from128((unsigned __int128)Mlo * Mhi), 65);
    U256 top = u_shl(u_from128((unsigned __int128)Mhi * Mhi), 128);
    m2 = u_add(u_add(m2, cross), top);
  }
  U256 rhs = u_shl(m2, em - E);
  return u_cmp(lhs, rhs);
}

template <class R> static bool is_even(R x);
template <> bool is_even<double>(double x) {
  uint64_t u;
  std::memcpy(&u, &x, 8);
  return (u & 1) == 0;
}
template <> bool is_even<float>(float x) {
  uint32_t u;
  std::memcpy(&u, &x, 4);
  return (u & 1) == 0;
}

template <class R>
static R cr_hypot(R x, R y) {
  R a = std::fabs(x), b = std::fabs(y);
  if (a < b) std::swap(a, b);
  if (std::isinf(a)) return a;
  if (std::isnan(a) || std::isnan(b)) return a + b;
  if (b == 0) return a;
  int ea, eb;
  std::frexp((double)a, &ea);
  std::frexp((double)b, &eb);
  /* b/a < 2^(eb-ea+1), so sqrt(a^2+b^2) - a < a 2^(2(eb-ea)+1) < half an
     ulp of a once ea - eb > 30: the result is a. */
  if (ea - eb > 30) return a;
  long double la = a, lb = b;
  R r = (R)std::sqrt(la * la + lb * lb);
  const R inf = (R)INFINITY;
  const int top = Fmt<R>::e_nu + 1; /* 2^top is the overflow "neighbour" */
  for (;;) {
    if (std::isinf(r)) r = Fmt<R>::nu();
    R up = std::nextafter(r, inf);
    int c = std::isinf(up) ? cmp_sumsq_mid(a, b, r, 0, top) : cmp_sumsq_mid(a, b, r, up, -1);
    if (c > 0) {
      if (std::isinf(up)) return up;
      r = up;
      continue;
    }
    if (c == 0) {
      if (std::isinf(up)) return up; /* the largest finite is odd */
      return is_even(r) ? r : up;
    }
    R dn = std::nextafter(r, (R)0);
    c = cmp_sumsq_mid(a, b, dn, r, -1);
    if (c < 0) {
      r = dn;
      continue;
    }
    if (c == 0) return is_even(dn) ? dn : r;
    return r;
  }
}

/* 1b. The hypot of the variant for a hypot that is not correctly rounded
   (Algorithm tf names that case without fixing the function; read here as the
   textbook scaled form): with hi = max(|x|,|y|), lo = min(|x|,|y|),
   hypot(x, y) = hi sqrt(1 + (lo/hi)^2), every operation rounded once and the
   sum of 1 and the square taken by one fma; hi itself if hi is 0 or inf. */
template <class R> static R fast_hypot(R x, R y) {
  R hi = std::max(std::fabs(x), std::fabs(y));
  R lo = std::min(std::fabs(x), std::fabs(y));
  if (hi == 0 || std::isinf(hi)) return hi;
  R r = lo / hi;
  return hi * std::sqrt(std::fma(r, r, (R)1));
}

/* the hypot of the method: CR = true is the correctly rounded one the
   analysis of Sect. 3 assumes, false the variant above */
template <bool CR, class R> static R hyp(R x, R y) {
  return CR ? cr_hypot(x, y) : fast_hypot(x, y);
}

/* ------------------------------------------------------------------------ */
/* 2. (e,f) pairs (Sect. 2): w = 2^e f with 1 <= |f| < 2, zero is (0,0).     */
/* ------------------------------------------------------------------------ */
template <class R> struct EF {
  int e;
  R f;
};

/* N(x) = (e_x, f_x), e_x = floor(lg|x|) (also for subnormal x). */
template <class R> static EF<R> ef_of(R x) {
  EF<R> r;
  if (x == 0) {
    r.e = 0;
    r.f = 0;
    return r;
  }
  r.e = std::ilogb(x);
  r.f = std::scalbn(x, -r.e);
  return r;
}

/* fl(w) = scalbn(f_w, e_w): a single rounding, may under- or overflow. */
template <class R> static R ef_fl(EF<R> x) { return std::scalbn(x.f, x.e); }

/* 2^s (.) x   (eq. unary) */
template <class R> static EF<R> ef_pow2(int s, EF<R> x) {
  if (x.f != 0) x.e += s;
  return x;
}

/* x (.) y = (e_x + e_y + e_z, f_z), z = fl(f_x f_y)   (eq. binary) */
template <class R> static EF<R> ef_mul(EF<R> x, EF<R> y) {
  R z = x.f * y.f;
  EF<R> n = ef_of(z);
  if (n.f != 0) n.e += x.e + y.e;
  return n;
}

/* x (/) y = (e_x - e_y + e_z, f_z), z = fl(f_x / f_y)   (eq. binary) */
template <class R> static EF<R> ef_div(EF<R> x, EF<R> y) {
  R z = x.f / y.f;
  EF<R> n = ef_of(z);
  if (n.f != 0) n.e += x.e - y.e;
  return n;
}

/* x (+) y for positive finite x, y (eq. plus): overflow-avoiding addition. */
template <class R> static EF<R> ef_plus(R x, R y) {
  R z = x + y;
  if (z <= Fmt<R>::nu()) return ef_of(z);
  z = (x * (R)0.5) + (y * (R)0.5);
  EF<R> n = ef_of(z);
  n.e += 1;
  return n;
}

/* x (-) y for positive finite x, y (eq. minus, Lemma minus):
   underflow-avoiding subtraction; x = y gives (0,0). */
template <class R> static EF<R> ef_minus(R x, R y) {
  EF<R> zero = {0, (R)0};
  if (x == y) return zero;
  R z = x - y;
  if (std::fabs(z) >= Fmt<R>::mu()) return ef_of(z);
  int c = Fmt<R>::e_mu + Fmt<R>::p - 1 - std::min(std::ilogb(x), std::ilogb(y));
  z = std::scalbn(x, c) - std::scalbn(y, c);
  EF<R> n = ef_of(z);
  n.e -= c;
  return n;
}

template <class R> static int sgn3(R f) { return (f > 0) - (f < 0); }

/* x < y in the sense of the represented values (eq. prec). */
template <class R> static bool ef_prec(EF<R> x, EF<R> y) {
  int sx = sgn3(x.f), sy = sgn3(y.f);
  if (sx < sy) return true;
  if (sx != sy) return false;
  return (x.e < y.e) || ((x.e == y.e) && (x.f < y.f));
}

/* ------------------------------------------------------------------------ */
/* 3. Double-word arithmetic (Joldes, Muller, Popescu, "Tight and rigorous   */
/*    error bounds for basic building blocks of double-word arithmetic",     */
/*    ACM TOMS 44(2), 2017): the wider datatype T of eq. (EXT) for binary64.  */
/* ------------------------------------------------------------------------ */
static void two_sum(double a, double b, double &s, double &t) {
  s = a + b;
  double ap = s - b;
  double bp = s - ap;
  double da = a - ap;
  double db = b - bp;
  t = da + db;
}

static void fast_two_sum(double a, double b, double &s, double &t) {
  s = a + b;
  double z = s - a;
  t = b - z;
}

static void two_prod(double a, double b, double &p, double &e) {
  p = a * b;
  e = std::fma(a, b, -p);
}

/* AccurateDWPlusDW (Algorithm 6 of the cited paper). */
static void dw_plus_dw(double xh, double xl, double yh, double yl, double &zh, double &zl) {
  double sh, sl, th, tl, vh, vl;
  two_sum(xh, yh, sh, sl);
  two_sum(xl, yl, th, tl);
  double c = sl + th;
  fast_two_sum(sh, c, vh, vl);
  double w = tl + vl;
  fast_two_sum(vh, w, zh, zl);
}

/* DWDivFP3 (Algorithm 15 of the cited paper). */
static void dw_div_fp(double xh, double xl, double y, double &zh, double &zl) {
  double th = xh / y;
  double ph, pl;
  two_prod(th, y, ph, pl);
  double dh = xh - ph; /* exact */
  double dl = xl - pl;
  double d = dh + dl;
  double tl = d / y;
  fast_two_sum(th, tl, zh, zl);
}

/* fl(FL(FL(x1 y1 +- x2 y2) / d)) of eq. (EXT), with T = double-word for
   binary64.  Each product is formed exactly from the factors' normalised
   mantissas, both are scaled by the larger product's exponent (so the sum
   cannot overflow and the smaller addend only loses bits far below 2^-106
   of the larger), summed, divided by d's mantissa, and the leading word
   scaled back by one rounding. */
static double ext_f64(double x1, double y1, double x2, double y2, bool minus, double d) {
  int a1 = std::ilogb(x1), b1 = std::ilogb(y1), a2 = std::ilogb(x2), b2 = std::ilogb(y2);
  int k1 = a1 + b1, k2 = a2 + b2, K = std::max(k1, k2);
  double p1h, p1l, p2h, p2l;
  two_prod(std::scalbn(x1, -a1), std::scalbn(y1, -b1), p1h, p1l);
  two_prod(std::scalbn(x2, -a2), std::scalbn(y2, -b2), p2h, p2l);
  p1h = std::scalbn(p1h, k1 - K);
  p1l = std::scalbn(p1l, k1 - K);
  p2h = std::scalbn(p2h, k2 - K);
  p2l = std::scalbn(p2l, k2 - K);
  if (minus) {
    p2h = -p2h;
    p2l = -p2l;
  }
  double xh, xl;
  dw_plus_dw(p1h, p1l, p2h, p2l, xh, xl);
  if (xh == 0) return 0.0;
  int ed = std::ilogb(d);
  double qh, ql;
  dw_div_fp(xh, xl, std::scalbn(d, -ed), qh, ql);
  return std::scalbn(qh, K - ed);
}

/* Same for binary32, with T = binary64 exactly as in the paper: both
   products are exact in binary64, the sum and the quotient are rounded in
   binary64 (FL), and the quotient is rounded to binary32 (fl). */
static float ext_f32(float x1, float y1, float x2, float y2, bool minus, float d) {
  double p1 = (double)x1 * (double)y1;
  double p2 = (double)x2 * (double)y2;
  double s = minus ? (p1 - p2) : (p1 + p2);
  double q = s / (double)d;
  return (float)q;
}

template <class R> static R ext(R x1, R y1, R x2, R y2, bool minus, R d);
template <> double ext<double>(double x1, double y1, double x2, double y2, bool minus, double d) {
  return ext_f64(x1, y1, x2, y2, minus, d);
}
template <> float ext<float>(float x1, float y1, float x2, float y2, bool minus, float d) {
  return ext_f32(x1, y1, x2, y2, minus, d);
}

/* ------------------------------------------------------------------------ */
/* 4. The SVD of order two.                                                 */
/* ------------------------------------------------------------------------ */
template <class R> struct M2 {
  R a[2][2]; /* a[row][col] */
};

template <class R> static M2<R> m_id() { return M2<R>{{{1, 0}, {0, 1}}}; }
template <class R> static M2<R> m_x() { return M2<R>{{{0, 1}, {1, 0}}}; }
template <class R> static M2<R> m_diag(R d1, R d2) { return M2<R>{{{d1, 0}, {0, d2}}}; }
/* plane rotation [c -s; s c] (eq. tfp) */
template <class R> static M2<R> m_rot(R c, R s) { return M2<R>{{{c, -s}, {s, c}}}; }
template <class R> static M2<R> m_t(const M2<R> &A) {
  return M2<R>{{{A.a[0][0], A.a[1][0]}, {A.a[0][1], A.a[1][1]}}};
}
/* Plain matrix product.  Every product formed below has a signed
   permutation as one factor, so every entry is a single non-zero term and
   the product is exact. */
template <class R> static M2<R> m_mul(const M2<R> &A, const M2<R> &B) {
  M2<R> C;
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) C.a[i][j] = A.a[i][0] * B.a[0][j] + A.a[i][1] * B.a[1][j];
  return C;
}

/* sign as used for the sign matrices: sgn(x) = -1 if x < 0, else +1 (zeros
   of either sign give +1). */
template <class R> static R sgn(R x) { return x < 0 ? (R)-1 : (R)1; }

/* type t = [g11!=0] + 2[g21!=0] + 4[g12!=0] + 8[g22!=0], read off the
   pictures of eq. (ts). */
template <class R> static int type_of(const M2<R> &G) {
  return (G.a[0][0] != 0) | ((G.a[1][0] != 0) << 1) | ((G.a[0][1] != 0) << 2) |
         ((G.a[1][1] != 0) << 3);
}

enum Cls { Z9 = 0, Z3 = 1, Z5 = 2, Z13 = 3, Z15 = 4 };

/* permutational classes of eq. (ts) */
static Cls cls_of(int t) {
  switch (t) {
    case 3:
    case 12:
      return Z3;
    case 5:
    case 10:
      return Z5;
    case 7:
    case 11:
    case 13:
    case 14:
      return Z13;
    case 15:
      return Z15;
    default:
      return Z9; /* 0, 1, 2, 4, 6, 8, 9 */
  }
}

/* scale type of eq. (ts) */
static int scale_type(Cls c) {
  switch (c) {
    case Z9:
      return 0;
    case Z15:
      return 2;
    default:
      return 1;
  }
}

/* Result of the SVD of a (prescaled) matrix: G' = U diag(s1, s2) V^T. */
template <class R> struct Part {
  M2<R> U, V;
  EF<R> s1, s2;
};

/* Class t ~ 9 (Sect. 3.1): permute into the 0 / 1 / 9 form with
   |d11| >= |d22| using at most one permutation per side, then take the
   signs of the diagonal out of the rows: U = P_U S, V = P_V. */
template <class R> static Part<R> svd_z9(const M2<R> &G, int t) {
  M2<R> PU = m_id<R>(), PV = m_id<R>();
  switch (t) {
    case 2:
      PU = m_x<R>();
      break;
    case 4:
      PV = m_x<R>();
      break;
    case 8:
      PU = m_x<R>();
      PV = m_x<R>();
      break;
    case 6:
      if (std::fabs(G.a[1][0]) >= std::fabs(G.a[0][1]))
        PU = m_x<R>();
      else
        PV = m_x<R>();
      break;
    case 9:
      if (std::fabs(G.a[0][0]) < std::fabs(G.a[1][1])) {
        PU = m_x<R>();
        PV = m_x<R>();
      }
      break;
    default:
      break; /* 0, 1 */
  }
  M2<R> D = m_mul(m_t(PU), m_mul(G, PV));
  M2<R> S = m_diag(sgn(D.a[0][0]), sgn(D.a[1][1]));
  Part<R> r;
  r.U = m_mul(PU, S);
  r.V = PV;
  r.s1 = ef_of(std::fabs(D.a[0][0]));
  r.s2 = ef_of(std::fabs(D.a[1][1]));
  return r;
}

/* Givens rotation by theta from tan(theta) (eq. Givens, Lemma sincostheta):
   sec = hypot(tan, 1), cos = fl(1/sec), sin = fl(tan/sec). */
template <bool CR, class R> static M2<R> givens(R tan_t) {
  R sec = hyp<CR>(tan_t, (R)1);
  return m_rot((R)1 / sec, tan_t / sec);
}

/* Class t ~ 3 (Sect. 3.1): one non-zero column.  Swap the columns of a
   t = 12 matrix (P_V), make the column positive by row signs (S_U), put the
   larger element on top (P_U), one QR rotation with tan = g21''/g11''
   (eq. theta); sigma1 = hypot, sigma2 = 0; U = S_U P_U U_theta, V = P_V. */
template <bool CR, class R> static Part<R> svd_z3(const M2<R> &G, int t) {
  M2<R> PV = (t == 12) ? m_x<R>() : m_id<R>();
  M2<R> H = m_mul(G, PV);
  R a = H.a[0][0], b = H.a[1][0];
  M2<R> SU = m_diag(sgn(a), sgn(b));
  a = std::fabs(a);
  b = std::fabs(b);
  M2<R> PU = m_id<R>();
  if (a < b) {
    PU = m_x<R>();
    std::swap(a, b);
  }
  Part<R> r;
  r.U = m_mul(m_mul(SU, PU), givens<CR>(b / a));
  r.V = PV;
  r.s1 = ef_of(hyp<CR>(a, b));
  r.s2 = ef_of((R)0);
  return r;
}

/* Class t ~ 5 (Sect. 3.1): one non-zero row; the transposed analogue:
   P_U for t = 10, column signs S_V, column order P_V, one RQ rotation with
   tan = g12''/g11''; U = P_U, V = S_V P_V V_theta. */
template <bool CR, class R> static Part<R> svd_z5(const M2<R> &G, int t) {
  M2<R> PU = (t == 10) ? m_x<R>() : m_id<R>();
  M2<R> H = m_mul(m_t(PU), G);
  R a = H.a[0][0], b = H.a[0][1];
  M2<R> SV = m_diag(sgn(a), sgn(b));
  a = std::fabs(a);
  b = std::fabs(b);
  M2<R> PV = m_id<R>();
  if (a < b) {
    PV = m_x<R>();
    std::swap(a, b);
  }
  Part<R> r;
  r.U = PU;
  r.V = m_mul(m_mul(SV, PV), givens<CR>(b / a));
  r.s1 = ef_of(hyp<CR>(a, b));
  r.s2 = ef_of((R)0);
  return r;
}

/* The SVD of R~ = [a b; 0 d] with a >= d > 0, b > 0 (Sect. 3.3.1). */
template <class R> struct Tri {
  R cphi, sphi, tphi, sec_phi; /* functions of phi */
  R cpsi, spsi, tpsi;          /* functions of psi */
  EF<R> s1, s2;                /* sigma~' after the ordering */
  bool psig;                   /* P_sigma = X */
  bool ovf;                    /* tan(psi) overflowed */
};

/* The expressions Sect. 3.3.1 gives for tan(2 phi) of [a b; 0 d], and the
   conditions under which each one is the one to use.  When several conditions
   hold, the one named first below decides (the precedence of Algorithm tf). */
enum class T2phi {
  diag_equal,   /* a = d: the squares cancel exactly; eq. t2f'', 2d/b         */
  offd_equal,   /* b = d: eq. t2f''', 2bd / a^2 in (e,f) arithmetic           */
  a_negligible, /* fl(a/b) < eps: a^2 vanishes beside b^2; eq. t2f'' again    */
  no_cr_hypot,  /* the variant for a hypot that is not correctly rounded      */
  right_angle,  /* hypot(a, b) = d: the denominator is zero, 2 phi = pi/2    */
  general       /* eq. t2f': 2bd / ((h - d)(h + d)) with h = hypot(a, b)      */
};

template <bool CR, class R> static T2phi t2phi_case(R a, R b, R d, R &h) {
  h = (R)0;
  if (a == d) return T2phi::diag_equal;
  if (b == d) return T2phi::offd_equal;
  if (a / b < Fmt<R>::eps()) return T2phi::a_negligible;
  if (!CR) return T2phi::no_cr_hypot;
  h = cr_hypot(a, b);
  return (h == d) ? T2phi::right_angle : T2phi::general;
}

/* tan(2 phi) = 2bd / (a^2 + b^2 - d^2) of R~, evaluated by the expression
   t2phi_case selects; (e,f) expressions are evaluated left to right. */
template <bool CR, class R> static R tan_2phi(R a, R b, R d) {
  R h;
  const EF<R> two_bd = ef_mul(ef_pow2(1, ef_of(b)), ef_of(d)); /* 2 (.) b (.) d */
  switch (t2phi_case<CR>(a, b, d, h)) {
    case T2phi::diag_equal:
    case T2phi::a_negligible:
      return ((R)2 * d) / b;
    case T2phi::offd_equal:
      return ef_fl(ef_div(two_bd, ef_mul(ef_of(a), ef_of(a))));
    case T2phi::right_angle:
      return (R)INFINITY;
    case T2phi::general:
      return ef_fl(ef_div(two_bd, ef_mul(ef_minus(h, d), ef_plus(h, d))));
    case T2phi::no_cr_hypot:
      break;
  }
  /* No squares of the inputs: divide the numerator and the denominator by the
     square of m = max(a, b).  With x = min(a, b)/m and y = d/m, the denominator
     becomes 1 + (x - y)(x + y) (one fma); the numerator is 2xy when a is the
     larger and 2y when b is.  A negative denominator counts as zero. */
  const bool a_big = a > b;
  const R x = a_big ? b / a : a / b;
  const R y = a_big ? d / a : d / b;
  const R num = a_big ? ((R)2 * x) * y : (R)2 * y;
  return num / std::max(std::fma(x - y, x + y, (R)1), (R)0);
}

template <bool CR, class R> static Tri<R> tri_svd(R a, R b, R d) {
  Tri<R> o;
  /* phi: tan(phi) from tan(2 phi) by eq. tf (2 phi = pi/2 gives tan(phi) = 1),
     then sec, cos, sin */
  const R t2 = tan_2phi<CR>(a, b, d);
  o.tphi = std::isinf(t2) ? (R)1 : t2 / ((R)1 + hyp<CR>(t2, (R)1));
  o.sec_phi = hyp<CR>(o.tphi, (R)1);
  o.cphi = (R)1 / o.sec_phi;
  o.sphi = o.tphi / o.sec_phi;
  /* psi: tan(psi) = (b + d tan(phi)) / a by eq. tp, the numerator by one fma */
  const R num = std::fma(d, o.tphi, b);
  o.tpsi = num / a;
  o.ovf = std::isinf(o.tpsi);
  EF<R> big, small;
  if (o.ovf) {
    /* eq. tp': cos(psi) = a / num in (e,f) form, sin(psi) = 1; the singular
       values then follow Algorithm tp: num and d cos(psi) */
    const EF<R> cos_psi = ef_div(ef_of(a), ef_of(num));
    o.cpsi = ef_fl(cos_psi);
    o.spsi = (R)1;
    big = ef_of(num);
    small = ef_mul(ef_of(d), cos_psi);
  } else {
    /* eq. s': with the ratio sec(phi) / sec(psi), sigma_1 = a / ratio and
       sigma_2 = d * ratio */
    const R sec_psi = hyp<CR>(o.tpsi, (R)1);
    o.cpsi = (R)1 / sec_psi;
    o.spsi = o.tpsi / sec_psi;
    const EF<R> ratio = ef_div(ef_of(o.sec_phi), ef_of(sec_psi));
    big = ef_div(ef_of(a), ratio);
    small = ef_mul(ef_of(d), ratio);
  }
  /* order by eq. prec: P_sigma = X when the first is strictly the smaller */
  o.psig = ef_prec(big, small);
  o.s1 = o.psig ? small : big;
  o.s2 = o.psig ? big : small;
  return o;
}

/* Sect. 3.2.2: the fully pivoted URV of a prescaled type-15 matrix.
   Column pivoting by the column norms w1, w2 (P_V), row signs from the new
   first column (S_1), row pivoting (P_U), then the QR rotation of eq. QR15
   with tan(theta) = g21/g11 of the pivoted matrix and r11 = w1.  r12 and r22
   are returned with their signs (before S_12 and S_22). */
template <class R> struct Urv15 {
  M2<R> S1, PU, PV;
  R tan_t, sec_t, r11, r12, r22;
  bool ext, exact;
};

template <bool CR, class R> static Urv15<R> urv15(const M2<R> &Gp) {
  Urv15<R> q;
  R w1 = hyp<CR>(Gp.a[0][0], Gp.a[1][0]);
  R w2 = hyp<CR>(Gp.a[0][1], Gp.a[1][1]);
  q.PV = m_id<R>();
  if (w1 < w2) {
    q.PV = m_x<R>();
    std::swap(w1, w2);
  }
  M2<R> Gt = m_mul(Gp, q.PV);
  q.S1 = m_diag(sgn(Gt.a[0][0]), sgn(Gt.a[1][0]));
  M2<R> G2 = m_mul(q.S1, Gt);
  q.PU = (G2.a[0][0] < G2.a[1][0]) ? m_x<R>() : m_id<R>();
  M2<R> G3 = m_mul(m_t(q.PU), G2);
  R g11 = G3.a[0][0], g21 = G3.a[1][0], g12 = G3.a[0][1], g22 = G3.a[1][1];
  q.tan_t = g21 / g11;
  q.sec_t = hyp<CR>(q.tan_t, (R)1);
  q.r11 = w1;
  /* Theorem R: tan(theta) is exact iff g21 - tan g11 = 0; that residual of
     a correctly rounded quotient is representable, so fma yields it exactly */
  q.exact = std::fma(-q.tan_t, g11, g21) == 0;
  R r12f = std::fma(g22, q.tan_t, g12) / q.sec_t;
  R r22f = std::fma(-g12, q.tan_t, g22) / q.sec_t;
  q.ext = false;
  if (q.exact) {
    q.r12 = r12f;
    q.r22 = r22f;
  } else if (sgn(g12) == sgn(g22)) {
    /* same signs: r12 is accurate, r22 suffers cancellation: eq. EXT */
    q.r12 = r12f;
    q.r22 = ext(g22, g11, g12, g21, true, g11) / q.sec_t;
    q.ext = true;
  } else {
    /* opposite signs: r22 is accurate, r12 by eq. EXT */
    q.r22 = r22f;
    q.r12 = ext(g12, g11, g22, g21, false, g11) / q.sec_t;
    q.ext = true;
  }
  return q;
}

/* info word layout (also documented in the GPU library's header) */
enum : uint32_t {
  INFO_DET_U = 1u << 8,
  INFO_DET_V = 1u << 9,
  INFO_EXT = 1u << 10,
  INFO_RSWAP = 1u << 11,
  INFO_TPSI_OVF = 1u << 12,
  INFO_PSIG = 1u << 13,
  INFO_DEGEN = 1u << 14,
  INFO_NONFINITE = 1u << 15,
};

template <class R> struct Res {
  M2<R> U, V;
  EF<R> s1, s2; /* backscaled sigma_1 >= sigma_2 */
  uint32_t info;
};

template <class R, bool CR = true> static Res<R> ksvd2(R g11, R g21, R g12, R g22) {
  Res<R> res;
  M2<R> G = {{{g11, g12}, {g21, g22}}};
  int t = type_of(G);
  if (!std::isfinite(g11) || !std::isfinite(g21) || !std::isfinite(g12) || !std::isfinite(g22)) {
    R nan = (R)NAN;
    res.U = M2<R>{{{nan, nan}, {nan, nan}}};
    res.V = res.U;
    res.s1.e = res.s2.e = 0;
    res.s1.f = res.s2.f = nan;
    res.info = (uint32_t)t | INFO_NONFINITE;
    return res;
  }
  /* Phase 1: prescaling (eqs. eG and s); matrices of class 9 are not
     scaled (Sect. 3.1) */
  Cls c = cls_of(t);
  int s = 0;
  if (c != Z9) {
    int eG = INT_MIN;
    for (int i = 0; i < 2; ++i)
      for (int j = 0; j < 2; ++j)
        if (G.a[i][j] != 0) eG = std::max(eG, std::ilogb(G.a[i][j]));
    s = Fmt<R>::e_nu - eG - scale_type(c);
  }
  M2<R> Gp;
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) Gp.a[i][j] = std::scalbn(G.a[i][j], s);
  /* the zero pattern is re-examined after the scaling */
  int t1 = type_of(Gp);
  Cls c1 = cls_of(t1);
  uint32_t info = (uint32_t)t | ((uint32_t)t1 << 4);

  Part<R> part;
  bool done = false;
  if (c1 == Z9) {
    part = svd_z9(Gp, t1);
    done = true;
  } else if (c1 == Z3) {
    part = svd_z3<CR>(Gp, t1);
    done = true;
  } else if (c1 == Z5) {
    part = svd_z5<CR>(Gp, t1);
    done = true;
  }

  /* Phase 2: the (pivoted) URV factorisation */
  R r11 = 0, r12 = 0, r22 = 0;
  M2<R> Uplus = m_id<R>(), Vplus = m_id<R>();
  /* Z15 keeps the factors of U_+ apart for the heuristic */
  M2<R> S1 = m_id<R>(), PU15 = m_id<R>();
  R tan_t = 0;
  bool s22neg = false;
  if (!done && c1 == Z13) {
    /* Sect. 3.2.1: permute into the upper triangular form, then three sign
       changes make the upper triangle positive; all error-free */
    M2<R> PU = m_id<R>(), PV = m_id<R>();
    if (t1 == 7) PV = m_x<R>();
    if (t1 == 14) PU = m_x<R>();
    if (t1 == 11) {
      PU = m_x<R>();
      PV = m_x<R>();
    }
    M2<R> H = m_mul(m_t(PU), m_mul(Gp, PV)); /* [x y; 0 z] */
    R x = H.a[0][0], y = H.a[0][1], z = H.a[1][1];
    M2<R> S11 = m_diag(sgn(x), (R)1);
    y = y * sgn(x);
    M2<R> S12 = m_diag((R)1, sgn(y));
    z = z * sgn(y);
    M2<R> S22 = m_diag((R)1, sgn(z));
    r11 = std::fabs(x);
    r12 = std::fabs(y);
    r22 = std::fabs(z);
    Uplus = m_mul(m_mul(PU, S11), S22);
    Vplus = m_mul(PV, S12);
  } else if (!done && c1 == Z15) {
    Urv15<R> q = urv15<CR>(Gp);
    if (q.ext) info |= INFO_EXT;
    M2<R> PV = q.PV;
    S1 = q.S1;
    PU15 = q.PU;
    tan_t = q.tan_t;
    r11 = q.r11;
    r12 = q.r12;
    r22 = q.r22;
    if (r12 == 0 || r22 == 0) {
      /* a zero appeared: R'' is of type 9 (or 1), or 5; it is processed as
         in Sect. 3.1, accounting for the transformations already applied */
      info |= INFO_DEGEN;
      M2<R> Rpp = {{{r11, r12}, {(R)0, r22}}};
      int t2 = type_of(Rpp);
      Part<R> sub = (cls_of(t2) == Z5) ? svd_z5<CR>(Rpp, t2) : svd_z9(Rpp, t2);
      part.U = m_mul(m_mul(m_mul(S1, PU15), givens<CR>(tan_t)), sub.U);
      part.V = m_mul(PV, sub.V);
      part.s1 = sub.s1;
      part.s2 = sub.s2;
      done = true;
    } else {
      M2<R> S12 = m_diag((R)1, sgn(r12));
      r22 = r22 * sgn(r12);
      r12 = std::fabs(r12);
      s22neg = r22 < 0;
      r22 = std::fabs(r22);
      Vplus = m_mul(PV, S12);
    }
  }

  if (!done) {
    /* Phase 3 (Sect. 3.3): swap the diagonal if r11 < r22 by permuting
       R^T symmetrically with X (eq. RT), compute the SVD of R~ and assemble */
    bool swapped = r11 < r22;
    if (swapped) info |= INFO_RSWAP;
    Tri<R> tr = swapped ? tri_svd<CR>(r22, r12, r11) : tri_svd<CR>(r11, r12, r22);
    if (tr.ovf) info |= INFO_TPSI_OVF;
    if (tr.psig) info |= INFO_PSIG;
    M2<R> S2 = swapped ? m_diag((R)1, (R)-1) : m_id<R>();
    /* eq. RT: U_bphi = rot(sin psi, cos psi) S2, V_bpsi = rot(sin phi,
       cos phi) S2, tan(bphi) = 1/tan(psi) when swapped */
    M2<R> Ubphi = swapped ? m_mul(m_rot(tr.spsi, tr.cpsi), S2) : m_rot(tr.cphi, tr.sphi);
    M2<R> Vbpsi = swapped ? m_mul(m_rot(tr.sphi, tr.cphi), S2) : m_rot(tr.cpsi, tr.spsi);
    R tbphi = swapped ? (R)1 / tr.tpsi : tr.tphi;
    M2<R> Psig = tr.psig ? m_x<R>() : m_id<R>();
    if (c1 == Z13) {
      part.U = m_mul(m_mul(Uplus, Ubphi), Psig);
    } else {
      /* Z15: the left-vector heuristic (eqs. p+t, p-t, tan+-, UV): the two
         rotations by theta and bphi are merged into one by the tangent of
         the sum (S22 = I) or of the difference (S22 = diag(1,-1)); the
         quadrant follows from the sign of the denominator */
      R num, den;
      if (!s22neg) {
        num = tbphi + tan_t;
        den = std::fma(-tbphi, tan_t, (R)1);
      } else {
        num = tbphi - tan_t;
        den = std::fma(tbphi, tan_t, (R)1);
      }
      R ca, sa;
      if (std::isinf(tbphi)) {
        /* tan(psi) underflowed to 0 in the swapped case: bphi = pi/2, and the
           merged angle is pi/2 + theta (S22 = I) or pi/2 - theta */
        R sec_t = hyp<CR>(tan_t, (R)1);
        R ct = (R)1 / sec_t, st = tan_t / sec_t;
        ca = s22neg ? st : -st;
        sa = ct;
      } else if (den == 0) {
        ca = 0;
        sa = sgn(num);
      } else {
        R ta = num / den;
        R sec_a = hyp<CR>(ta, (R)1);
        R sd = sgn(den);
        ca = sd * ((R)1 / sec_a);
        sa = sd * (ta / sec_a);
      }
      M2<R> Mrot = m_mul(m_rot(ca, sa), S2);
      if (s22neg) Mrot = m_mul(m_diag((R)1, (R)-1), Mrot);
      part.U = m_mul(m_mul(m_mul(S1, PU15), Mrot), Psig);
    }
    part.V = m_mul(m_mul(Vplus, Vbpsi), Psig);
    part.s1 = tr.s1;
    part.s2 = tr.s2;
  }

  /* Sect. 3.3.2: backscale, sigma_i = 2^-s (.) sigma~_i' */
  res.U = part.U;
  res.V = part.V;
  res.s1 = ef_pow2(-s, part.s1);
  res.s2 = ef_pow2(-s, part.s2);
  res.info = info | ((uint32_t)(uint16_t)(int16_t)s << 16);
  return res;
}

/* U (or V) is a signed permutation times a plane rotation, hence of the
   form [c -d s; s d c] with d = det = +-1.  Returns false if not. */
template <class R> static bool compact(const M2<R> &U, R &c, R &s, bool &neg) {
  R d = U.a[0][0] * U.a[1][1] - U.a[0][1] * U.a[1][0];
  neg = d < 0;
  R dd = neg ? (R)-1 : (R)1;
  c = U.a[0][0];
  s = U.a[1][0];
  bool ok = (U.a[0][1] == -dd * s) && (U.a[1][1] == dd * c);
  /* canonical zeros: -0 becomes +0 */
  c = c + (R)0;
  s = s + (R)0;
  return ok;
}

template <class R, bool CR = true>
static int batch_fwd(int64_t n, const R *g11, const R *g21, const R *g12, const R *g22, R *cu,
                     R *su, R *cv, R *sv, R *f1, R *f2, int32_t *e1, int32_t *e2, int32_t *info,
                     R *s1, R *s2, int nthreads) {
  int bad = 0;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(static) reduction(+ : bad)
#endif
  for (int64_t i = 0; i < n; ++i) {
    Res<R> r = ksvd2<R, CR>(g11[i], g21[i], g12[i], g22[i]);
    bool nu, nv;
    R c, s;
    bool okU = compact(r.U, c, s, nu);
    cu[i] = c;
    su[i] = s;
    bool okV = compact(r.V, c, s, nv);
    cv[i] = c;
    sv[i] = s;
    uint32_t inf = r.info;
    if (!(inf & INFO_NONFINITE)) {
      if (nu) inf |= INFO_DET_U;
      if (nv) inf |= INFO_DET_V;
      if (!okU || !okV) bad += 1;
    }
    f1[i] = r.s1.f;
    f2[i] = r.s2.f;
    e1[i] = r.s1.e;
    e2[i] = r.s2.e;
    info[i] = (int32_t)inf;
    if (s1) s1[i] = ef_fl(r.s1);
    if (s2) s2[i] = ef_fl(r.s2);
  }
  return bad;
}

/* ------------------------------------------------------------------------ */
/* 4b. The complex 2x2 SVD (Sect. 3.4): G = U diag(sigma) V^H.              */
/*    A real G is the real method; a purely imaginary G = i Im(G) is the    */
/*    real method on Im(G) with U multiplied by i.  Otherwise every element */
/*    made real and non-negative goes through a unit phase e^{i alpha} =    */
/*    g/|g| into a diagonal phase matrix (the complex "sign matrix") and is */
/*    replaced by |g|; the scale type is s_C = s + 1 (class 9 included, its */
/*    |g| could overflow); e_G takes the real and imaginary parts; U_+ is   */
/*    formed explicitly and multiplied by the real factors of the SVD of R; */
/*    no wider datatype (no eq. EXT), no merging of rotations.              */
/* ------------------------------------------------------------------------ */
template <class R> struct Cx {
  R re, im;
};
template <class R> static Cx<R> cx(R re, R im) { return Cx<R>{re, im}; }
template <class R> static Cx<R> c_conj(Cx<R> a) { return Cx<R>{a.re, -a.im}; }
/* (a + ib)(c + id) = (ac - bd) + i(ad + bc), each part one fma after one product */
template <class R> static Cx<R> c_mul(Cx<R> a, Cx<R> b) {
  return Cx<R>{std::fma(a.re, b.re, -(a.im * b.im)), std::fma(a.re, b.im, a.im * b.re)};
}
template <class R> static Cx<R> c_scale(Cx<R> a, R r) { return Cx<R>{a.re * r, a.im * r}; }
/* |g| (the correctly rounded hypot of the parts) and the phase g/|g| of a
   non-zero g, taken of g 2^-k with k the exponent of its larger part (exact),
   so that a subnormal g, whose modulus rounds coarsely, still has a phase of
   modulus one to working accuracy */
template <class R> static R c_abs(Cx<R> a) { return cr_hypot(a.re, a.im); }
template <class R> static Cx<R> c_phase(Cx<R> a) {
  int k = std::ilogb(std::max(std::fabs(a.re), std::fabs(a.im)));
  Cx<R> b = {std::scalbn(a.re, -k), std::scalbn(a.im, -k)};
  R m = cr_hypot(b.re, b.im);
  return Cx<R>{b.re / m, b.im / m};
}

template <class R> struct CM2 {
  Cx<R> a[2][2];
};
/* complex 2x2 times real 2x2: each entry is c_i0 r_0j + c_i1 r_1j, per part as
   fma(c_i0, r_0j, c_i1 r_1j) */
template <class R> static CM2<R> cm_mul_real(const CM2<R> &C, const M2<R> &B) {
  CM2<R> o;
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) {
      o.a[i][j].re = std::fma(C.a[i][0].re, B.a[0][j], C.a[i][1].re * B.a[1][j]);
      o.a[i][j].im = std::fma(C.a[i][0].im, B.a[0][j], C.a[i][1].im * B.a[1][j]);
    }
  return o;
}
/* diag(d1, d2) times a real matrix (row i scaled by d_i): every entry is a
   phase times a real, one rounding per part */
template <class R> static CM2<R> cm_diag_real(Cx<R> d1, Cx<R> d2, const M2<R> &B) {
  CM2<R> o;
  Cx<R> d[2] = {d1, d2};
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) o.a[i][j] = c_scale(d[i], B.a[i][j]);
  return o;
}
/* a real matrix times a complex one, entry by entry as for cm_mul_real */
template <class R> static CM2<R> real_mul_cm(const M2<R> &A, const CM2<R> &C) {
  CM2<R> o;
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) {
      o.a[i][j].re = std::fma(A.a[i][0], C.a[0][j].re, A.a[i][1] * C.a[1][j].re);
      o.a[i][j].im = std::fma(A.a[i][0], C.a[0][j].im, A.a[i][1] * C.a[1][j].im);
    }
  return o;
}
template <class R> static CM2<R> cm_of_real(const M2<R> &A) {
  CM2<R> o;
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) o.a[i][j] = Cx<R>{A.a[i][j], (R)0};
  return o;
}

template <class R> struct CRes {
  CM2<R> U, V;
  EF<R> s1, s2;
  uint32_t info;
};

/* the real factors of the SVD of R = [a b; 0 d] (a, b, d >= 0, b > 0, d > 0),
   with the swap of eq. RT when a < d: R = Ub diag(s1, s2) Vb^T, P_sigma
   included (Sect. 3.3; as in the real method's phase 3 without the heuristic) */
template <class R> struct TriUV {
  M2<R> Ub, Vb;
  EF<R> s1, s2;
  uint32_t flags;
};
template <class R> static TriUV<R> tri_uv(R a, R b, R d) {
  TriUV<R> o;
  o.flags = 0;
  bool swapped = a < d;
  if (swapped) o.flags |= INFO_RSWAP;
  Tri<R> tr = swapped ? tri_svd<true>(d, b, a) : tri_svd<true>(a, b, d);
  if (tr.ovf) o.flags |= INFO_TPSI_OVF;
  if (tr.psig) o.flags |= INFO_PSIG;
  M2<R> S2 = swapped ? m_diag((R)1, (R)-1) : m_id<R>();
  M2<R> Ubphi = swapped ? m_mul(m_rot(tr.spsi, tr.cpsi), S2) : m_rot(tr.cphi, tr.sphi);
  M2<R> Vbpsi = swapped ? m_mul(m_rot(tr.sphi, tr.cphi), S2) : m_rot(tr.cpsi, tr.spsi);
  M2<R> Psig = tr.psig ? m_x<R>() : m_id<R>();
  o.Ub = m_mul(Ubphi, Psig);
  o.Vb = m_mul(Vbpsi, Psig);
  o.s1 = tr.s1;
  o.s2 = tr.s2;
  return o;
}

template <class R> static CRes<R> ksvd2c(const Cx<R> g[4]) {
  /* g in the order g11, g21, g12, g22 */
  CRes<R> res;
  bool finite = true, all_re = true, all_im = true;
  for (int k = 0; k < 4; ++k) {
    finite = finite && std::isfinite(g[k].re) && std::isfinite(g[k].im);
    all_re = all_re && g[k].im == 0;
    all_im = all_im && g[k].re == 0;
  }
  int t = 0;
  for (int k = 0; k < 4; ++k) t |= (g[k].re != 0 || g[k].im != 0) << k;
  if (!finite) {
    R nan = (R)NAN;
    for (int i = 0; i < 2; ++i)
      for (int j = 0; j < 2; ++j) res.U.a[i][j] = res.V.a[i][j] = Cx<R>{nan, nan};
    res.s1.e = res.s2.e = 0;
    res.s1.f = res.s2.f = nan;
    res.info = (uint32_t)t | INFO_NONFINITE;
    return res;
  }
  if (all_re || all_im) {
    /* a real matrix, or i times one */
    Res<R> r = all_re ? ksvd2<R>(g[0].re, g[1].re, g[2].re, g[3].re)
                      : ksvd2<R>(g[0].im, g[1].im, g[2].im, g[3].im);
    res.V = cm_of_real(r.V);
    for (int i = 0; i < 2; ++i)
      for (int j = 0; j < 2; ++j)
        res.U.a[i][j] = all_re ? Cx<R>{r.U.a[i][j], (R)0} : Cx<R>{(R)0, r.U.a[i][j]};
    res.s1 = r.s1;
    res.s2 = r.s2;
    res.info = r.info;
    bool nu, nv;
    R c, sn;
    compact(r.U, c, sn, nu);
    compact(r.V, c, sn, nv);
    if (nu) res.info |= INFO_DET_U;
    if (nv) res.info |= INFO_DET_V;
    return res;
  }
  /* prescaling (eqs. eG, s) with s_C = s + 1 over all real and imaginary parts */
  Cls c = cls_of(t);
  int eG = INT_MIN;
  for (int k = 0; k < 4; ++k) {
    if (g[k].re != 0) eG = std::max(eG, std::ilogb(g[k].re));
    if (g[k].im != 0) eG = std::max(eG, std::ilogb(g[k].im));
  }
  int s = Fmt<R>::e_nu - eG - (scale_type(c) + 1);
  Cx<R> h[4];
  for (int k = 0; k < 4; ++k) h[k] = Cx<R>{std::scalbn(g[k].re, s), std::scalbn(g[k].im, s)};
  int t1 = 0;
  for (int k = 0; k < 4; ++k) t1 |= (h[k].re != 0 || h[k].im != 0) << k;
  Cls c1 = cls_of(t1);
  uint32_t info = (uint32_t)t | ((uint32_t)t1 << 4);
  R m[4];
  Cx<R> ph[4];
  for (int k = 0; k < 4; ++k) {
    m[k] = c_abs(h[k]);
    ph[k] = (m[k] != 0) ? c_phase(h[k]) : Cx<R>{(R)1, (R)0};
  }
  const Cx<R> one = {(R)1, (R)0};
  M2<R> Mg = {{{m[0], m[2]}, {m[1], m[3]}}}; /* |G'| */
  EF<R> s1, s2;
  if (c1 == Z9 || c1 == Z3) {
    /* row phases: the phase of the row's non-zero element (the non-zero
       column's element for class 3), 1 for a zero row */
    Cx<R> d1 = (m[0] != 0) ? ph[0] : (m[2] != 0) ? ph[2] : one;
    Cx<R> d2 = (m[1] != 0) ? ph[1] : (m[3] != 0) ? ph[3] : one;
    Part<R> p = (c1 == Z9) ? svd_z9(Mg, t1) : svd_z3<true>(Mg, t1);
    res.U = cm_diag_real(d1, d2, p.U);
    res.V = cm_of_real(p.V);
    s1 = p.s1;
    s2 = p.s2;
  } else if (c1 == Z5) {
    /* column phases conj(phase) of the non-zero row's elements go into V */
    Cx<R> d1 = c_conj((m[0] != 0) ? ph[0] : ph[1]);
    Cx<R> d2 = c_conj((m[2] != 0) ? ph[2] : ph[3]);
    Part<R> p = svd_z5<true>(Mg, t1);
    res.U = cm_of_real(p.U);
    res.V = cm_diag_real(d1, d2, p.V);
    s1 = p.s1;
    s2 = p.s2;
  } else if (c1 == Z13) {
    /* permute into [x y; 0 z] (types 7: columns, 14: rows, 11: both), then
       P_U^T G P_V = D_U [|x| |y|; 0 |z|] D_V^H with D_U = diag(px, pz b2),
       D_V = diag(1, b2), b2 = px conj(py) */
    M2<R> PU = m_id<R>(), PV = m_id<R>();
    if (t1 == 7) PV = m_x<R>();
    if (t1 == 14) PU = m_x<R>();
    if (t1 == 11) {
      PU = m_x<R>();
      PV = m_x<R>();
    }
    /* the positions (row, column) of x, y, z in G' */
    int rx = (PU.a[0][0] != 0) ? 0 : 1, ry = rx, rz = 1 - rx;
    int cx_ = (PV.a[0][0] != 0) ? 0 : 1, cy = 1 - cx_, cz = cy;
    int kx = rx + 2 * cx_, ky = ry + 2 * cy, kz = rz + 2 * cz;
    Cx<R> b2 = c_mul(ph[kx], c_conj(ph[ky]));
    Cx<R> a2 = c_mul(ph[kz], b2);
    TriUV<R> tu = tri_uv(m[kx], m[ky], m[kz]);
    info |= tu.flags;
    res.U = real_mul_cm(PU, cm_diag_real(ph[kx], a2, tu.Ub));
    res.V = real_mul_cm(PV, cm_diag_real(one, b2, tu.Vb));
    s1 = tu.s1;
    s2 = tu.s2;
  } else {
    /* class 15: column pivoting by the column norms, row phases making the
       first column real and non-negative, row pivoting, one real rotation by
       tan(theta) = |g21|/|g11|; T = [w1 r12; 0 r22] with complex r12, r22,
       T = D_a [w1 |r12|; 0 |r22|] D_b^H, D_a = diag(1, p22 conj(p12)),
       D_b = diag(1, conj(p12)) */
    R w1 = cr_hypot(m[0], m[1]), w2 = cr_hypot(m[2], m[3]);
    bool cswap = w1 < w2;
    if (cswap) std::swap(w1, w2);
    int k11 = cswap ? 2 : 0, k21 = cswap ? 3 : 1, k12 = cswap ? 0 : 2, k22 = cswap ? 1 : 3;
    /* row phases of the first column, applied to the second */
    Cx<R> q12 = c_mul(c_conj(ph[k11]), h[k12]);
    Cx<R> q22 = c_mul(c_conj(ph[k21]), h[k22]);
    R a = m[k11], b = m[k21];
    bool rswap = a < b;
    Cx<R> p1 = ph[k11], p2 = ph[k21]; /* D1 = diag(p1, p2) */
    if (rswap) {
      std::swap(a, b);
      std::swap(q12, q22);
    }
    R tan_t = b / a;
    R sec_t = cr_hypot(tan_t, (R)1);
    Cx<R> r12 = {std::fma(q22.re, tan_t, q12.re) / sec_t, std::fma(q22.im, tan_t, q12.im) / sec_t};
    Cx<R> r22 = {std::fma(-q12.re, tan_t, q22.re) / sec_t, std::fma(-q12.im, tan_t, q22.im) / sec_t};
    R m12 = c_abs(r12), m22 = c_abs(r22);
    Cx<R> p12 = (m12 != 0) ? c_phase(r12) : one;
    Cx<R> p22 = (m22 != 0) ? c_phase(r22) : one;
    Cx<R> beta2 = c_conj(p12);
    Cx<R> alpha2 = (m12 != 0) ? c_mul(p22, beta2) : p22;
    /* U_+ = D1 P_U U_theta D_a, formed explicitly */
    M2<R> PU = rswap ? m_x<R>() : m_id<R>();
    M2<R> W = m_mul(PU, givens<true>(tan_t)); /* P_U U_theta, exact */
    CM2<R> Up;
    Cx<R> d[2] = {p1, p2};
    for (int i = 0; i < 2; ++i) {
      Up.a[i][0] = c_scale(d[i], W.a[i][0]);
      Up.a[i][1] = c_mul(c_scale(d[i], W.a[i][1]), alpha2);
    }
    M2<R> PV = cswap ? m_x<R>() : m_id<R>();
    M2<R> Ub, Vb;
    if (m12 == 0 || m22 == 0) {
      /* a zero appeared: finished as in Sect. 3.1 */
      info |= INFO_DEGEN;
      M2<R> Rpp = {{{w1, m12}, {(R)0, m22}}};
      int t2 = type_of(Rpp);
      Part<R> sub = (cls_of(t2) == Z5) ? svd_z5<true>(Rpp, t2) : svd_z9(Rpp, t2);
      Ub = sub.U;
      Vb = sub.V;
      s1 = sub.s1;
      s2 = sub.s2;
    } else {
      TriUV<R> tu = tri_uv(w1, m12, m22);
      info |= tu.flags;
      Ub = tu.Ub;
      Vb = tu.Vb;
      s1 = tu.s1;
      s2 = tu.s2;
    }
    res.U = cm_mul_real(Up, Ub);
    res.V = real_mul_cm(PV, cm_diag_real(one, beta2, Vb));
  }
  /* backscale (Sect. 3.3.2) */
  res.s1 = ef_pow2(-s, s1);
  res.s2 = ef_pow2(-s, s2);
  res.info = info | ((uint32_t)(uint16_t)(int16_t)s << 16);
  return res;
}

/* batch driver: G, U, V are [n][2][2] complex (re, im interleaved, row-major
   2x2); S [n][2] plain sigma; f [n][2], e [n][2] the (e,f) pairs */
template <class R>
static void batch_c(int64_t n, const R *G, R *U, R *S, R *V, R *f, int32_t *e, int32_t *info,
                    int nthreads) {
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(static)
#endif
  for (int64_t b = 0; b < n; ++b) {
    const R *x = G + 8 * b;
    /* row-major (i, j) -> 2 (2 i + j); order g11, g21, g12, g22 */
    Cx<R> g[4] = {{x[0], x[1]}, {x[4], x[5]}, {x[2], x[3]}, {x[6], x[7]}};
    CRes<R> r = ksvd2c<R>(g);
    for (int i = 0; i < 2; ++i)
      for (int j = 0; j < 2; ++j) {
        int o = 8 * b + 2 * (2 * i + j);
        /* canonical zeros: -0 becomes +0 */
        U[o] = r.U.a[i][j].re + (R)0;
        U[o + 1] = r.U.a[i][j].im + (R)0;
        V[o] = r.V.a[i][j].re + (R)0;
        V[o + 1] = r.V.a[i][j].im + (R)0;
      }
    S[2 * b] = ef_fl(r.s1);
    S[2 * b + 1] = ef_fl(r.s2);
    if (f) {
      f[2 * b] = r.s1.f;
      f[2 * b + 1] = r.s2.f;
    }
    if (e) {
      e[2 * b] = r.s1.e;
      e[2 * b + 1] = r.s2.e;
    }
    if (info) info[b] = (int32_t)r.info;
  }
}

/* ------------------------------------------------------------------------ */
/* 5. Two-sided Kogbetliantz iteration over one n x n matrix (Sect. 1, eq.  */
/*    (SVD)): in each parallel step the n/2 disjoint pivot submatrices of a  */
/*    round-robin ordering are diagonalised by the 2x2 SVD above; the        */
/*    embedded U_k^T is applied to the pivot rows, then V_k to the pivot     */
/*    columns; the pivot off-diagonals become 0 and its diagonal sigma; U_k  */
/*    and V_k accumulate into U and V.  Matrices are column-major.           */
/*    G is first scaled by a power of two so that the two-sided updates      */
/*    cannot overflow (Sect. 4, on the order-n implementation; read as       */
/*    2^s_G with s_G = e_nu - 2 - e_G - ceil(lg n), applied only when        */
/*    negative) and scaled back at the end.                                   */
/* ------------------------------------------------------------------------ */

/* Round-robin (circle) ordering: position 0 is fixed, positions 1..n-1
   rotate by one each step; in step k the slot pairs (q, n-1-q) meet. */
static int rr_player(int n, int k, int q) {
  if (q == 0) return 0;
  return 1 + (q - 1 + k) % (n - 1);
}

/* The pivot pairs (i < j) of step k of a sweep, n/2 of them, in pi, pj.
   ordering 0: the round-robin pairs above, slot by slot.
   ordering 1: the modified modulus strategy (Sect. 4 names it for the order-n
   iteration), read as the modulus strategy for the odd order m = n - 1 -- step
   k pairs the indices i < j < m with i + j = k (mod m) and leaves idle the
   index c with 2c = k (mod m) -- with the idle index paired with m. */
static void step_pairs(int ordering, int n, int k, int *pi, int *pj) {
  int np = n / 2, t = 0;
  if (ordering == 0) {
    for (int q = 0; q < np; ++q) {
      int a = rr_player(n, k, q), b = rr_player(n, k, n - 1 - q);
      pi[q] = std::min(a, b);
      pj[q] = std::max(a, b);
    }
    return;
  }
  int m = n - 1;
  for (int c = 0; c < m; ++c)
    if ((2 * c) % m == k) {
      pi[t] = c;
      pj[t] = m;
      ++t;
    }
  for (int i = 0; i < m; ++i)
    for (int j = i + 1; j < m; ++j)
      if ((i + j) % m == k) {
        pi[t] = i;
        pj[t] = j;
        ++t;
      }
}

/* Dynamic ordering (ordering 2; Sect. 1 names dynamic orderings as candidates
   for parallel strategies that are not cyclic; read here as follows): the
   pivots of a step are chosen from the current iterate by a greedy matching on
   the weights w_ij = x_ij^2 + x_ji^2 (i < j, x = G 2^-t with t the norm
   exponent of the sweep, one fma in binary64: fma(x_ij, x_ij, x_ji * x_ji)):
   the pairs are taken in decreasing order of weight, equal weights by the
   smaller i and then the smaller j, each one when both of its indices are still
   free.  On the complete graph of an even order this pairs every index. */
struct DynEdge {
  double w;
  int i, j;
};

template <class R>
static void dynamic_pairs(int n, const R *G, double ns, int *pi, int *pj) {
  std::vector<DynEdge> e;
  e.reserve((size_t)n * (n - 1) / 2);
  for (int i = 0; i < n; ++i)
    for (int j = i + 1; j < n; ++j) {
      double a = (double)G[i + (int64_t)j * n] * ns, b = (double)G[j + (int64_t)i * n] * ns;
      e.push_back(DynEdge{std::fma(a, a, b * b), i, j});
    }
  std::sort(e.begin(), e.end(), [](const DynEdge &x, const DynEdge &y) {
    if (x.w != y.w) return x.w > y.w;
    if (x.i != y.i) return x.i < y.i;
    return x.j < y.j;
  });
  std::vector<char> used(n, 0);
  int t = 0;
  for (const DynEdge &x : e) {
    if (used[x.i] || used[x.j]) continue;
    used[x.i] = used[x.j] = 1;
    pi[t] = x.i;
    pj[t] = x.j;
    ++t;
  }
}

/* one element pair of a rotation: x' = a x + b y as fma(a, x, b*y) */
template <class R> static R rot_lin(R a, R x, R b, R y) { return std::fma(a, x, b * y); }

template <class R>
static int sweep_one(int n, R *G, R *U, R *V, int max_sweeps, double tol_factor, int accumulate,
                     int ordering, int *sweeps_done) {
  if (!accumulate) {
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < n; ++i) {
        U[i + (int64_t)j * n] = (i == j) ? (R)1 : (R)0;
        V[i + (int64_t)j * n] = (i == j) ? (R)1 : (R)0;
      }
  }
  /* the global scaling: e_G the largest exponent of a non-zero entry */
  int eg = INT_MIN;
  for (int64_t k = 0; k < (int64_t)n * n; ++k)
    if (G[k] != 0) eg = std::max(eg, std::ilogb(G[k]));
  int lgn = 0;
  while ((1 << lgn) < n) ++lgn;
  int sg = (eg == INT_MIN) ? 0 : std::min(0, Fmt<R>::e_nu - 2 - eg - lgn);
  if (sg < 0)
    for (int64_t k = 0; k < (int64_t)n * n; ++k) G[k] = std::scalbn(G[k], sg);
  /* ||G_0||_F in binary64 (the threshold of the stopping criterion), as the
     norm of G 2^-t with t the largest exponent after the scaling, so that no
     square overflows; the off-diagonal norm below is taken the same way (the
     stopping test compares the two, so the factor cancels) */
  int t = (eg == INT_MIN) ? 0 : eg + sg;
  double ns = std::scalbn(1.0, -t);
  double fro2 = 0;
  for (int64_t k = 0; k < (int64_t)n * n; ++k) {
    double x = (double)G[k] * ns;
    fro2 += x * x;
  }
  double tol = tol_factor * n * (double)Fmt<R>::eps() * std::sqrt(fro2);
  int np = n / 2;
  R *pc = new R[4 * np]; /* per pivot: u11 u21 u12 u22 */
  R *pv = new R[4 * np];
  int *pi = new int[np], *pj = new int[np];
  R *ps1 = new R[np], *ps2 = new R[np];
  int status = 1;
  int sw = 0;
  for (sw = 0; sw < max_sweeps; ++sw) {
    for (int k = 0; k < n - 1; ++k) {
      if (ordering == 2)
        dynamic_pairs(n, G, ns, pi, pj);
      else
        step_pairs(ordering, n, k, pi, pj);
      for (int q = 0; q < np; ++q) {
        int i = pi[q], j = pj[q];
        R gii = G[i + (int64_t)i * n], gji = G[j + (int64_t)i * n];
        R gij = G[i + (int64_t)j * n], gjj = G[j + (int64_t)j * n];
        Res<R> r = ksvd2<R>(gii, gji, gij, gjj);
        /* the pivot's U and V as delivered by the 2x2 SVD: [c -d s; s d c] */
        R c, sn;
        bool neg;
        compact(r.U, c, sn, neg);
        R d = neg ? (R)-1 : (R)1;
        pc[4 * q] = c;
        pc[4 * q + 1] = sn;
        pc[4 * q + 2] = -d * sn;
        pc[4 * q + 3] = d * c;
        compact(r.V, c, sn, neg);
        d = neg ? (R)-1 : (R)1;
        pv[4 * q] = c;
        pv[4 * q + 1] = sn;
        pv[4 * q + 2] = -d * sn;
        pv[4 * q + 3] = d * c;
        ps1[q] = ef_fl(r.s1);
        ps2[q] = ef_fl(r.s2);
      }
      /* rows: G <- U_k^T G; row i' = u11 row_i + u21 row_j, row j' = u12 row_i + u22 row_j */
      for (int q = 0; q < np; ++q) {
        int i = pi[q], j = pj[q];
        R u11 = pc[4 * q], u21 = pc[4 * q + 1], u12 = pc[4 * q + 2], u22 = pc[4 * q + 3];
        for (int c = 0; c < n; ++c) {
          R x = G[i + (int64_t)c * n], y = G[j + (int64_t)c * n];
          G[i + (int64_t)c * n] = rot_lin(u11, x, u21, y);
          G[j + (int64_t)c * n] = rot_lin(u12, x, u22, y);
        }
      }
      /* columns: G <- G V_k; col i' = col_i v11 + col_j v21, col j' = col_i v12 + col_j v22 */
      for (int q = 0; q < np; ++q) {
        int i = pi[q], j = pj[q];
        R v11 = pv[4 * q], v21 = pv[4 * q + 1], v12 = pv[4 * q + 2], v22 = pv[4 * q + 3];
        for (int r = 0; r < n; ++r) {
          R x = G[r + (int64_t)i * n], y = G[r + (int64_t)j * n];
          G[r + (int64_t)i * n] = rot_lin(v11, x, v21, y);
          G[r + (int64_t)j * n] = rot_lin(v12, x, v22, y);
        }
        /* the pivot block becomes diag(sigma1, sigma2) */
        G[i + (int64_t)i * n] = ps1[q];
        G[j + (int64_t)j * n] = ps2[q];
        G[i + (int64_t)j * n] = 0;
        G[j + (int64_t)i * n] = 0;
      }
      /* U <- U U_k, V <- V V_k (columns) */
      for (int q = 0; q < np; ++q) {
        int i = pi[q], j = pj[q];
        R u11 = pc[4 * q], u21 = pc[4 * q + 1], u12 = pc[4 * q + 2], u22 = pc[4 * q + 3];
        R v11 = pv[4 * q], v21 = pv[4 * q + 1], v12 = pv[4 * q + 2], v22 = pv[4 * q + 3];
        for (int r = 0; r < n; ++r) {
          R x = U[r + (int64_t)i * n], y = U[r + (int64_t)j * n];
          U[r + (int64_t)i * n] = rot_lin(u11, x, u21, y);
          U[r + (int64_t)j * n] = rot_lin(u12, x, u22, y);
          x = V[r + (int64_t)i * n];
          y = V[r + (int64_t)j * n];
          V[r + (int64_t)i * n] = rot_lin(v11, x, v21, y);
          V[r + (int64_t)j * n] = rot_lin(v12, x, v22, y);
        }
      }
    }
    /* off-diagonal Frobenius norm after the sweep, in binary64 */
    double off2 = 0;
    for (int c = 0; c < n; ++c)
      for (int r = 0; r < n; ++r)
        if (r != c) {
          double x = (double)G[r + (int64_t)c * n] * ns;
          off2 += x * x;
        }
    if (std::sqrt(off2) <= tol) {
      status = 0;
      ++sw;
      break;
    }
  }
  *sweeps_done = sw;
  if (sg < 0)
    for (int64_t k = 0; k < (int64_t)n * n; ++k) G[k] = std::scalbn(G[k], -sg);
  delete[] pc;
  delete[] pv;
  delete[] pi;
  delete[] pj;
  delete[] ps1;
  delete[] ps2;
  return status;
}

}  // namespace

/* ------------------------------------------------------------------------ */
/* 5b. Rectangular m x n inputs, m >= n (Sect. 1: preprocessed to a square  */
/*    triangular G_0 = U_0^T G V_0 by a URV-type factorization, the QR      */
/*    factorization with column pivoting).  Householder reflections         */
/*    H_k = I - tau_k v_k v_k^T (v_k(k) = 1), the pivot the trailing column */
/*    of largest norm (the first such on ties), the norms recomputed at     */
/*    every step.  G P = Q R; after the sweep R = U_R Sigma V_R^T,          */
/*    U = Q [U_R; 0] and V = P V_R.  Column-major arrays.                   */
/* ------------------------------------------------------------------------ */
template <class R>
static void qrcp_one(int m, int n, R *A, R *tau, int32_t *perm, R *Rsq) {
  auto a = [&](int i, int j) -> R & { return A[i + (int64_t)j * m]; };
  for (int j = 0; j < n; ++j) perm[j] = j;
  /* Scaling (a reading: the paper takes the QR preprocessing from LAPACK, whose
     norms avoid overflow): when the squared column norms could leave the normal
     range (2 |e_max| + ceil(lg m) + 2 >= e_nu, e_max the largest exponent of an
     entry), the matrix is multiplied by 2^-e_max first and R by 2^e_max at the
     end; the reflectors and tau are scale-free. */
  int emax = INT_MIN;
  for (int64_t x = 0; x < (int64_t)m * n; ++x)
    if (A[x] != 0) emax = std::max(emax, std::ilogb(A[x]));
  int lgm = 0;
  while ((1 << lgm) < m) ++lgm;
  int sc = 0;
  if (emax != INT_MIN && 2 * std::abs(emax) + lgm + 2 >= Fmt<R>::e_nu) sc = -emax;
  if (sc != 0)
    for (int64_t x = 0; x < (int64_t)m * n; ++x) A[x] = std::scalbn(A[x], sc);
  for (int k = 0; k < n; ++k) {
    /* pivot: the largest squared norm of the trailing columns (rows k..m-1) */
    int p = k;
    R best = (R)-1;
    for (int j = k; j < n; ++j) {
      R s = 0;
      for (int i = k; i < m; ++i) s += a(i, j) * a(i, j);
      if (s > best) {
        best = s;
        p = j;
      }
    }
    if (p != k) {
      for (int i = 0; i < m; ++i) std::swap(a(i, k), a(i, p));
      std::swap(perm[k], perm[p]);
    }
    /* the reflection that maps column k (rows k..m-1) onto beta e_k */
    R x0 = a(k, k), s = 0;
    for (int i = k + 1; i < m; ++i) s += a(i, k) * a(i, k);
    if (s == 0) {
      tau[k] = 0;
      continue;
    }
    R nrm = std::sqrt(x0 * x0 + s);
    R beta = x0 >= 0 ? -nrm : nrm;
    tau[k] = (beta - x0) / beta;
    R scal = (R)1 / (x0 - beta);
    for (int i = k + 1; i < m; ++i) a(i, k) *= scal;
    a(k, k) = beta;
    /* H_k on the trailing columns */
    for (int j = k + 1; j < n; ++j) {
      R w = a(k, j);
      for (int i = k + 1; i < m; ++i) w += a(i, k) * a(i, j);
      R tw = tau[k] * w;
      a(k, j) -= tw;
      for (int i = k + 1; i < m; ++i) a(i, j) -= tw * a(i, k);
    }
  }
  if (sc != 0)
    for (int j = 0; j < n; ++j)
      for (int i = 0; i <= j && i < m; ++i) a(i, j) = std::scalbn(a(i, j), -sc);
  /* the n x n triangular factor, zeros below the diagonal */
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i) Rsq[i + (int64_t)j * n] = (i <= j) ? a(i, j) : (R)0;
}

/* U = H_0 ... H_{n-1} [U_R; 0] (m x n) and V = P V_R (n x n) */
template <class R>
static void qapply_one(int m, int n, const R *A, const R *tau, const int32_t *perm, const R *UR,
                       const R *VR, R *U, R *V) {
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < m; ++i) U[i + (int64_t)j * m] = (i < n) ? UR[i + (int64_t)j * n] : (R)0;
  for (int k = n - 1; k >= 0; --k) {
    if (tau[k] == 0) continue;
    for (int j = 0; j < n; ++j) {
      R *u = U + (int64_t)j * m;
      const R *v = A + (int64_t)k * m;
      R w = u[k];
      for (int i = k + 1; i < m; ++i) w += v[i] * u[i];
      R tw = tau[k] * w;
      u[k] -= tw;
      for (int i = k + 1; i < m; ++i) u[i] -= tw * v[i];
    }
  }
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i) V[perm[i] + (int64_t)j * n] = VR[i + (int64_t)j * n];
}

/* ------------------------------------------------------------------------ */
/* 6. extern "C" entry points used by the test-suite (via ctypes).           */
/* ------------------------------------------------------------------------ */
extern "C" {

int orc_version(void) { return 1; }

double orc_hypot_f64(double x, double y) { return cr_hypot(x, y); }
float orc_hypot_f32(float x, float y) { return cr_hypot(x, y); }

void orc_hypot_batch_f64(int64_t n, const double *x, const double *y, double *out) {
#ifdef _OPENMP
#pragma omp parallel for schedule(static)
#endif
  for (int64_t i = 0; i < n; ++i) out[i] = cr_hypot(x[i], y[i]);
}

void orc_hypot_batch_f32(int64_t n, const float *x, const float *y, float *out) {
#ifdef _OPENMP
#pragma omp parallel for schedule(static)
#endif
  for (int64_t i = 0; i < n; ++i) out[i] = cr_hypot(x[i], y[i]);
}

void orc_hypot_fast_batch_f64(int64_t n, const double *x, const double *y, double *out) {
  for (int64_t i = 0; i < n; ++i) out[i] = fast_hypot(x[i], y[i]);
}

void orc_hypot_fast_batch_f32(int64_t n, const float *x, const float *y, float *out) {
  for (int64_t i = 0; i < n; ++i) out[i] = fast_hypot(x[i], y[i]);
}

/* (e,f) operations, exposed for their pins: op 0 = plus, 1 = minus,
   2 = mul, 3 = div (the last two on N(x), N(y)) */
void orc_ef_op_f64(int op, double x, double y, int *e, double *f) {
  EF<double> r;
  switch (op) {
    case 0:
      r = ef_plus(x, y);
      break;
    case 1:
      r = ef_minus(x, y);
      break;
    case 2:
      r = ef_mul(ef_of(x), ef_of(y));
      break;
    default:
      r = ef_div(ef_of(x), ef_of(y));
      break;
  }
  *e = r.e;
  *f = r.f;
}

void orc_ef_op_f32(int op, float x, float y, int *e, float *f) {
  EF<float> r;
  switch (op) {
    case 0:
      r = ef_plus(x, y);
      break;
    case 1:
      r = ef_minus(x, y);
      break;
    case 2:
      r = ef_mul(ef_of(x), ef_of(y));
      break;
    default:
      r = ef_div(ef_of(x), ef_of(y));
      break;
  }
  *e = r.e;
  *f = r.f;
}

double orc_ext_f64(double x1, double y1, double x2, double y2, int minus, double d) {
  return ext_f64(x1, y1, x2, y2, minus != 0, d);
}

float orc_ext_f32(float x1, float y1, float x2, float y2, int minus, float d) {
  return ext_f32(x1, y1, x2, y2, minus != 0, d);
}

/* The URV factorisation of a prescaled type-15 matrix (for the Theorem R
   checks): out = {r11, r12, r22, tan(theta)}, flags bit0 exact tan, bit1 EXT. */
void orc_urv15_f64(double g11, double g21, double g12, double g22, double *out, int *flags) {
  M2<double> G = {{{g11, g12}, {g21, g22}}};
  Urv15<double> q = urv15<true>(G);
  out[0] = q.r11;
  out[1] = q.r12;
  out[2] = q.r22;
  out[3] = q.tan_t;
  *flags = (q.exact ? 1 : 0) | (q.ext ? 2 : 0);
}

void orc_urv15_f32(float g11, float g21, float g12, float g22, float *out, int *flags) {
  M2<float> G = {{{g11, g12}, {g21, g22}}};
  Urv15<float> q = urv15<true>(G);
  out[0] = q.r11;
  out[1] = q.r12;
  out[2] = q.r22;
  out[3] = q.tan_t;
  *flags = (q.exact ? 1 : 0) | (q.ext ? 2 : 0);
}

/* returns the number of results whose U or V is not of the compact form
   (an internal consistency check; 0 expected) */
int orc_ksvd2_f64(int64_t n, const double *g11, const double *g21, const double *g12,
                  const double *g22, double *cu, double *su, double *cv, double *sv, double *f1,
                  double *f2, int32_t *e1, int32_t *e2, int32_t *info, double *s1, double *s2,
                  int nthreads) {
  return batch_fwd<double>(n, g11, g21, g12, g22, cu, su, cv, sv, f1, f2, e1, e2, info, s1, s2,
                           nthreads);
}

int orc_ksvd2_f32(int64_t n, const float *g11, const float *g21, const float *g12,
                  const float *g22, float *cu, float *su, float *cv, float *sv, float *f1,
                  float *f2, int32_t *e1, int32_t *e2, int32_t *info, float *s1, float *s2,
                  int nthreads) {
  return batch_fwd<float>(n, g11, g21, g12, g22, cu, su, cv, sv, f1, f2, e1, e2, info, s1, s2,
                          nthreads);
}

/* the variant for a hypot that is not correctly rounded (Algorithm tf) */
int orc_ksvd2_fast_f64(int64_t n, const double *g11, const double *g21, const double *g12,
                       const double *g22, double *cu, double *su, double *cv, double *sv,
                       double *f1, double *f2, int32_t *e1, int32_t *e2, int32_t *info,
                       double *s1, double *s2, int nthreads) {
  return batch_fwd<double, false>(n, g11, g21, g12, g22, cu, su, cv, sv, f1, f2, e1, e2, info,
                                  s1, s2, nthreads);
}

int orc_ksvd2_fast_f32(int64_t n, const float *g11, const float *g21, const float *g12,
                       const float *g22, float *cu, float *su, float *cv, float *sv, float *f1,
                       float *f2, int32_t *e1, int32_t *e2, int32_t *info, float *s1, float *s2,
                       int nthreads) {
  return batch_fwd<float, false>(n, g11, g21, g12, g22, cu, su, cv, sv, f1, f2, e1, e2, info,
                                 s1, s2, nthreads);
}

/* One n x n matrix (column-major, in place): returns 0 when converged,
   1 when max_sweeps ran out; tol_factor < 0 disables the stopping test. */
int orc_kog_sweep_f64(int n, double *G, double *U, double *V, int max_sweeps, double tol_factor,
                      int accumulate, int ordering, int *sweeps_done) {
  return sweep_one<double>(n, G, U, V, max_sweeps, tol_factor, accumulate, ordering,
                           sweeps_done);
}

int orc_kog_sweep_f32(int n, float *G, float *U, float *V, int max_sweeps, double tol_factor,
                      int accumulate, int ordering, int *sweeps_done) {
  return sweep_one<float>(n, G, U, V, max_sweeps, tol_factor, accumulate, ordering,
                          sweeps_done);
}

/* QR with column pivoting of one m x n column-major matrix (in place:
   reflectors below the diagonal, R on and above), tau[n], perm[n], and the
   n x n triangular factor */
void orc_qrcp_f64(int m, int n, double *A, double *tau, int32_t *perm, double *Rsq) {
  qrcp_one<double>(m, n, A, tau, perm, Rsq);
}
void orc_qrcp_f32(int m, int n, float *A, float *tau, int32_t *perm, float *Rsq) {
  qrcp_one<float>(m, n, A, tau, perm, Rsq);
}
void orc_qapply_f64(int m, int n, const double *A, const double *tau, const int32_t *perm,
                    const double *UR, const double *VR, double *U, double *V) {
  qapply_one<double>(m, n, A, tau, perm, UR, VR, U, V);
}
void orc_qapply_f32(int m, int n, const float *A, const float *tau, const int32_t *perm,
                    const float *UR, const float *VR, float *U, float *V) {
  qapply_one<float>(m, n, A, tau, perm, UR, VR, U, V);
}

/* the complex 2x2 SVD (Sect. 3.4), layouts as batch_c */
void orc_ksvd2c_f64(int64_t n, const double *G, double *U, double *S, double *V, double *f,
                    int32_t *e, int32_t *info, int nthreads) {
  batch_c<double>(n, G, U, S, V, f, e, info, nthreads);
}

void orc_ksvd2c_f32(int64_t n, const float *G, float *U, float *S, float *V, float *f,
                    int32_t *e, int32_t *info, int nthreads) {
  batch_c<float>(n, G, U, S, V, f, e, info, nthreads);
}

/* the pairs of the dynamic ordering for an n x n matrix (weights of G itself,
   t = 0): 2 * (n/2) ints, i then j, in the order they were taken */
void orc_dynamic_pairs_f64(int n, const double *G, int *out) {
  int np = n / 2;
  std::vector<int> pi(np), pj(np);
  dynamic_pairs(n, G, 1.0, pi.data(), pj.data());
  for (int q = 0; q < np; ++q) {
    out[2 * q] = pi[q];
    out[2 * q + 1] = pj[q];
  }
}

/* the pivot pairs of step k (for the ordering pins): 2 * (n/2) ints, i then j */
void orc_step_pairs(int ordering, int n, int k, int *out) {
  int np = n / 2;
  int *pi = new int[np], *pj = new int[np];
  step_pairs(ordering, n, k, pi, pj);
  for (int q = 0; q < np; ++q) {
    out[2 * q] = pi[q];
    out[2 * q + 1] = pj[q];
  }
  delete[] pi;
  delete[] pj;
}

}  // extern "C"
