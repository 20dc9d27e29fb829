// The complex 2x2 SVD (Sect. 3.4) on the GPU: G = U diag(sigma) V^H for a
// batch of complex matrices, one matrix per lane.  Entry point declared and
// documented in include/ksvd2.h (ksvd2c_batch).
//
// A real G is the real method (svd2); a purely imaginary G is the real method
// on Im(G) with U multiplied by i.  Otherwise each element that is made real
// goes through its unit phase g/|g| into a diagonal phase matrix (the complex
// counterpart of the sign matrices) and is replaced by its correctly rounded
// modulus; the scale type is s + 1 for every class; the exponents of the real
// and imaginary parts both enter e_G; U_+ is formed explicitly and multiplied
// by the real factors of the triangular SVD; no wider datatype (no eq. EXT) and
// no merging of rotations.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "abi_common.hpp"
#include "ksvd2_device.hpp"

namespace ksvd2 {

template <class R> struct Cx {
  R re, im;
};
template <class R> __device__ inline Cx<R> c_conj(Cx<R> a) { return Cx<R>{a.re, -a.im}; }
// (a + ib)(c + id) = (ac - bd) + i(ad + bc): one product, then one fma per part
template <class R> __device__ inline Cx<R> c_mul(Cx<R> a, Cx<R> b) {
  return Cx<R>{fma(a.re, b.re, -(a.im * b.im)), fma(a.re, b.im, a.im * b.re)};
}
template <class R> __device__ inline Cx<R> c_scale(Cx<R> a, R r) {
  return Cx<R>{a.re * r, a.im * r};
}
// the unit phase g/|g| of a non-zero g, taken of g 2^-k (k the exponent of its
// larger part, an exact scaling) so that a subnormal g keeps a unit phase
template <class R> __device__ inline Cx<R> c_phase(Cx<R> a) {
  int k = ilog2(fmax(fabs(a.re), fabs(a.im)));
  R br = scale2(a.re, -k), bi = scale2(a.im, -k);
  R m = hypot_cr(br, bi);
  return Cx<R>{br / m, bi / m};
}

// explicit real and complex 2x2 matrices, row-major
template <class R> struct RM {
  R a[2][2];
};
template <class R> struct CM {
  Cx<R> a[2][2];
};

template <class R> __device__ inline RM<R> rm_rot(R c, R s) {  // [c -s; s c]
  RM<R> m;
  m.a[0][0] = c;
  m.a[0][1] = -s;
  m.a[1][0] = s;
  m.a[1][1] = c;
  return m;
}
// exchange of the columns (right factor X) or of the rows (left factor X)
template <class R> __device__ inline RM<R> rm_swapcols(RM<R> m, bool on) {
  if (on) {
    for (int i = 0; i < 2; ++i) {
      R t = m.a[i][0];
      m.a[i][0] = m.a[i][1];
      m.a[i][1] = t;
    }
  }
  return m;
}
template <class R> __device__ inline RM<R> rm_swaprows(RM<R> m, bool on) {
  if (on) {
    for (int j = 0; j < 2; ++j) {
      R t = m.a[0][j];
      m.a[0][j] = m.a[1][j];
      m.a[1][j] = t;
    }
  }
  return m;
}
template <class R> __device__ inline CM<R> cm_swaprows(CM<R> m, bool on) {
  if (on) {
    for (int j = 0; j < 2; ++j) {
      Cx<R> t = m.a[0][j];
      m.a[0][j] = m.a[1][j];
      m.a[1][j] = t;
    }
  }
  return m;
}
// L rot(c, s) Rt of the real method, entries formed exactly (each is +-c, +-s or 0)
template <class R> __device__ inline RM<R> rm_of(const Fac<R> &f) {
  RM<R> r = rm_rot(f.c, f.s);
  // right factor Rt: column j of r Rt is (-1)^{n_j} column pi(j) of r
  r = rm_swapcols(r, f.Rt.x != 0);
  for (int i = 0; i < 2; ++i) {
    r.a[i][0] = neg_if(r.a[i][0], f.Rt.n0);
    r.a[i][1] = neg_if(r.a[i][1], f.Rt.n1);
  }
  // left factor L: row k of r lands in row pi_L(k) with the sign (-1)^{nL_k}
  for (int j = 0; j < 2; ++j) {
    r.a[0][j] = neg_if(r.a[0][j], f.L.n0);
    r.a[1][j] = neg_if(r.a[1][j], f.L.n1);
  }
  return rm_swaprows(r, f.L.x != 0);
}
// diag(d1, d2) B: row i scaled by the phase d_i
template <class R> __device__ inline CM<R> cm_diag_real(Cx<R> d1, Cx<R> d2, const RM<R> &B) {
  CM<R> o;
  for (int j = 0; j < 2; ++j) {
    o.a[0][j] = c_scale(d1, B.a[0][j]);
    o.a[1][j] = c_scale(d2, B.a[1][j]);
  }
  return o;
}
// C B for complex C and real B: per part fma(c_i0, b_0j, c_i1 b_1j)
template <class R> __device__ inline CM<R> cm_mul_real(const CM<R> &C, const RM<R> &B) {
  CM<R> o;
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) {
      o.a[i][j].re = fma(C.a[i][0].re, B.a[0][j], C.a[i][1].re * B.a[1][j]);
      o.a[i][j].im = fma(C.a[i][0].im, B.a[0][j], C.a[i][1].im * B.a[1][j]);
    }
  return o;
}
template <class R> __device__ inline CM<R> cm_real(const RM<R> &B) {
  CM<R> o;
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) o.a[i][j] = Cx<R>{B.a[i][j], (R)0};
  return o;
}

// the real factors of the SVD of [a b; 0 d] (a, b, d > 0), with the swap of
// eq. RT when a < d, P_sigma included: R = Ub diag(s1, s2) Vb^T (Sect. 3.3)
template <class R> struct TriUV {
  RM<R> Ub, Vb;
  EF<R> s1, s2;
  uint32_t flags;
};
template <class R> __device__ __attribute__((always_inline)) TriUV<R> tri_uv(R a, R b, R d) {
  TriUV<R> o;
  bool swapped = a < d;
  Tri<R> tr = tri_svd<R, true>(swapped ? d : a, b, swapped ? a : d);
  o.flags = (swapped ? I_RSWAP : 0u) | (tr.ovf ? I_TPSI_OVF : 0u) | (tr.psig ? I_PSIG : 0u);
  // U_bphi = rot(sin psi, cos psi) diag(1, -1) when swapped, else rot(cos phi, sin phi);
  // V_bpsi likewise with phi and psi exchanged
  RM<R> Ub = swapped ? rm_rot(tr.spsi, tr.cpsi) : rm_rot(tr.cphi, tr.sphi);
  RM<R> Vb = swapped ? rm_rot(tr.sphi, tr.cphi) : rm_rot(tr.cpsi, tr.spsi);
  if (swapped) {
    for (int i = 0; i < 2; ++i) {
      Ub.a[i][1] = -Ub.a[i][1];
      Vb.a[i][1] = -Vb.a[i][1];
    }
  }
  o.Ub = rm_swapcols(Ub, tr.psig);
  o.Vb = rm_swapcols(Vb, tr.psig);
  o.s1 = tr.s1;
  o.s2 = tr.s2;
  return o;
}

template <class R> struct Svd2c {
  CM<R> U, V;
  R f1, f2;
  int e1, e2;
  uint32_t info;
};

// a finite G whose elements are all real, or all imaginary
template <class R> __device__ inline bool real_or_imag(const Cx<R> g[4], bool &all_re) {
  bool re = true, im = true, fin = true;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    fin = fin && isfinite(g[k].re) && isfinite(g[k].im);
    re = re && g[k].im == (R)0;
    im = im && g[k].re == (R)0;
  }
  all_re = re;
  return fin && (re || im);
}

// a real matrix, or i times one: the real method (U multiplied by i for the latter)
template <class R>
__device__ __attribute__((always_inline)) Svd2c<R> svd2c_real(const Cx<R> g[4], bool all_re) {
  Svd2c<R> out;
  Svd2<R> r = all_re ? svd2<R>(g[0].re, g[1].re, g[2].re, g[3].re)
                     : svd2<R>(g[0].im, g[1].im, g[2].im, g[3].im);
  R du = (r.info & I_DETU) ? (R)-1 : (R)1, dv = (r.info & I_DETV) ? (R)-1 : (R)1;
  RM<R> Ur, Vr;
  Ur.a[0][0] = r.cu;
  Ur.a[0][1] = -du * r.su;
  Ur.a[1][0] = r.su;
  Ur.a[1][1] = du * r.cu;
  Vr.a[0][0] = r.cv;
  Vr.a[0][1] = -dv * r.sv;
  Vr.a[1][0] = r.sv;
  Vr.a[1][1] = dv * r.cv;
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j)
      out.U.a[i][j] = all_re ? Cx<R>{Ur.a[i][j], (R)0} : Cx<R>{(R)0, Ur.a[i][j]};
  out.V = cm_real(Vr);
  out.f1 = r.f1;
  out.f2 = r.f2;
  out.e1 = r.e1;
  out.e2 = r.e2;
  out.info = r.info;
  return out;
}

// g in the order g11, g21, g12, g22; a non-finite G or one with a complex
// element (real and purely imaginary matrices take svd2c_real)
template <class R> __device__ __attribute__((always_inline)) Svd2c<R> svd2c(const Cx<R> g[4]) {
  Svd2c<R> out;
  bool finite = true;
  int t = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    finite = finite && isfinite(g[k].re) && isfinite(g[k].im);
    t |= (g[k].re != (R)0 || g[k].im != (R)0) << k;
  }
  if (!finite) {
    R nan = (R)NAN;
    for (int i = 0; i < 2; ++i)
      for (int j = 0; j < 2; ++j) out.U.a[i][j] = out.V.a[i][j] = Cx<R>{nan, nan};
    out.f1 = out.f2 = nan;
    out.e1 = out.e2 = 0;
    out.info = (uint32_t)t | I_NONFINITE;
    return out;
  }
  // prescaling with s_C = s + 1 over all real and imaginary parts
  uint32_t tb = 1u << t;
  int stype = (tb & CL9) ? 0 : (t == 15) ? 2 : 1;
  int eg = -0x7fffffff;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    if (g[k].re != (R)0) eg = max(eg, ilog2(g[k].re));
    if (g[k].im != (R)0) eg = max(eg, ilog2(g[k].im));
  }
  int s = Lim<R>::e_nu - eg - (stype + 1);
  Cx<R> h[4];
  int t1 = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    h[k] = Cx<R>{scale2(g[k].re, s), scale2(g[k].im, s)};
    t1 |= (h[k].re != (R)0 || h[k].im != (R)0) << k;
  }
  uint32_t tb1 = 1u << t1;
  uint32_t info = (uint32_t)t | ((uint32_t)t1 << 4);
  R m[4];
  Cx<R> ph[4];
  const Cx<R> one = {(R)1, (R)0};
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    m[k] = hypot_cr(h[k].re, h[k].im);
    ph[k] = (m[k] != (R)0) ? c_phase(h[k]) : one;
  }
  M2<R> Mg = {m[0], m[2], m[1], m[3]};  // |G'|, row-major [a b; c d]
  // Each class prepares the operands of one of two shared bodies -- the simple
  // classes of Sect. 3.1 (part9 / part35) or the triangular SVD (tri_uv) -- and
  // the phase factors around it, so that lanes of one wave in different classes
  // run each body once:
  //   kind 0 (classes 9, 3): U = diag(d1, d2) Ub, V = Vb;
  //   kind 1 (class 5):      U = Ub, V = diag(d1, d2) Vb;
  //   kind 2 (classes 13, 15): U = Up Ub, V = rows exchanged if vsw of diag(1, vph) Vb.
  int kind = 2;
  bool use_tri = false;
  M2<R> Ms = Mg;
  int ts = t1;
  R ra = 0, rb = 0, rd = 0;  // the triangular factor [ra rb; 0 rd]
  EF<R> s1, s2;
  Cx<R> d1 = one, d2 = one, vph = one;
  bool vsw = false;
  CM<R> Up;
  if (tb1 & (CL9 | CL3)) {
    // row phases: the phase of the row's non-zero element, 1 for a zero row
    kind = 0;
    d1 = (m[0] != (R)0) ? ph[0] : (m[2] != (R)0) ? ph[2] : one;
    d2 = (m[1] != (R)0) ? ph[1] : (m[3] != (R)0) ? ph[3] : one;
  } else if (tb1 & CL5) {
    // column phases: conj of the phases of the non-zero row's elements, into V
    kind = 1;
    d1 = c_conj((m[0] != (R)0) ? ph[0] : ph[1]);
    d2 = c_conj((m[2] != (R)0) ? ph[2] : ph[3]);
  } else if (tb1 & CL13) {
    // permute into [x y; 0 z] (types 7: columns, 14: rows, 11: both); then
    // P_U^T G' P_V = D_U [|x| |y|; 0 |z|] D_V^H with D_U = diag(px, pz b2),
    // D_V = diag(1, b2), b2 = px conj(py); Up = P_U D_U
    bool pu = (t1 == 14 || t1 == 11), pv = (t1 == 7 || t1 == 11);
    int rx = pu ? 1 : 0, cx = pv ? 1 : 0;
    int kx = rx + 2 * cx, ky = rx + 2 * (1 - cx), kz = (1 - rx) + 2 * (1 - cx);
    Cx<R> b2 = c_mul(ph[kx], c_conj(ph[ky]));
    Cx<R> a2 = c_mul(ph[kz], b2);
    const Cx<R> zero = {(R)0, (R)0};
    Up.a[0][0] = pu ? zero : ph[kx];
    Up.a[0][1] = pu ? a2 : zero;
    Up.a[1][0] = pu ? ph[kx] : zero;
    Up.a[1][1] = pu ? zero : a2;
    vph = b2;
    vsw = pv;
    ra = m[kx];
    rb = m[ky];
    rd = m[kz];
    use_tri = true;
  } else {
    // class 15: column pivoting by the column norms, row phases making the
    // first column real and non-negative, row pivoting, one real rotation by
    // tan(theta) = |g21|/|g11|; T = [w1 r12; 0 r22] = D_a [w1 |r12|; 0 |r22|]
    // D_b^H, D_a = diag(1, p22 conj(p12)), D_b = diag(1, conj(p12))
    R w1 = hypot_cr(m[0], m[1]), w2 = hypot_cr(m[2], m[3]);
    bool cswap = w1 < w2;
    if (cswap) w1 = w2;
    int k11 = cswap ? 2 : 0, k21 = cswap ? 3 : 1, k12 = cswap ? 0 : 2, k22 = cswap ? 1 : 3;
    Cx<R> q12 = c_mul(c_conj(ph[k11]), h[k12]);
    Cx<R> q22 = c_mul(c_conj(ph[k21]), h[k22]);
    R a = m[k11], b = m[k21];
    bool rswap = a < b;
    Cx<R> p1 = ph[k11], p2 = ph[k21];
    if (rswap) {
      R tt = a;
      a = b;
      b = tt;
      Cx<R> tq = q12;
      q12 = q22;
      q22 = tq;
    }
    R tan_t = b / a;
    R sec_t = hypot1_le1(tan_t);  // 0 < tan(theta) <= 1
    R ct, st;
    cos_sin(tan_t, sec_t, ct, st);
    Cx<R> r12 = {fma(q22.re, tan_t, q12.re) / sec_t, fma(q22.im, tan_t, q12.im) / sec_t};
    Cx<R> r22 = {fma(-q12.re, tan_t, q22.re) / sec_t, fma(-q12.im, tan_t, q22.im) / sec_t};
    R m12 = hypot_cr(r12.re, r12.im), m22 = hypot_cr(r22.re, r22.im);
    Cx<R> p12 = (m12 != (R)0) ? c_phase(r12) : one;
    Cx<R> p22 = (m22 != (R)0) ? c_phase(r22) : one;
    Cx<R> beta2 = c_conj(p12);
    Cx<R> alpha2 = (m12 != (R)0) ? c_mul(p22, beta2) : p22;
    // U_+ = D1 P_U U_theta D_a, formed explicitly
    RM<R> W = rm_swaprows(rm_rot(ct, st), rswap);
    Up.a[0][0] = c_scale(p1, W.a[0][0]);
    Up.a[1][0] = c_scale(p2, W.a[1][0]);
    Up.a[0][1] = c_mul(c_scale(p1, W.a[0][1]), alpha2);
    Up.a[1][1] = c_mul(c_scale(p2, W.a[1][1]), alpha2);
    vph = beta2;
    vsw = cswap;
    if (m12 == (R)0 || m22 == (R)0) {
      // a zero appeared: finished as in Sect. 3.1
      info |= I_DEGEN;
      Ms = M2<R>{w1, m12, (R)0, m22};
      ts = ztype(Ms.a, Ms.c, Ms.b, Ms.d);
    } else {
      ra = w1;
      rb = m12;
      rd = m22;
      use_tri = true;
    }
  }
  RM<R> Ub, Vb;
  if (use_tri) {
    TriUV<R> tu = tri_uv(ra, rb, rd);
    info |= tu.flags;
    Ub = tu.Ub;
    Vb = tu.Vb;
    s1 = tu.s1;
    s2 = tu.s2;
  } else {
    Part<R> p = ((1u << ts) & CL9) ? part9(Ms, ts) : part35<R, true>(Ms, ts);
    Ub = rm_of(p.U);
    Vb = rm_of(p.V);
    s1 = p.s1;
    s2 = p.s2;
  }
  if (kind == 0) {
    out.U = cm_diag_real(d1, d2, Ub);
    out.V = cm_real(Vb);
  } else if (kind == 1) {
    out.U = cm_real(Ub);
    out.V = cm_diag_real(d1, d2, Vb);
  } else {
    out.U = cm_mul_real(Up, Ub);
    out.V = cm_swaprows(cm_diag_real(one, vph, Vb), vsw);
  }
  // backscale (Sect. 3.3.2); frexp form -> the paper's (e, f), f in [1, 2)
  out.f1 = s1.f * (R)2;
  out.f2 = s2.f * (R)2;
  out.e1 = (s1.f != (R)0) ? s1.e - 1 - s : 0;
  out.e2 = (s2.f != (R)0) ? s2.e - 1 - s : 0;
  out.info = info | ((uint32_t)(uint16_t)(int16_t)s << 16);
  return out;
}

template <class R>
__device__ inline void store_c(int64_t i, const Svd2c<R> &r, R *U, R *S, R *V, R *f, int32_t *e,
                               int32_t *info) {
  R *u = U + 8 * i, *v = V + 8 * i;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      int o = 2 * (2 * a + b);
      u[o] = r.U.a[a][b].re + (R)0;  // canonical zeros: -0 -> +0
      u[o + 1] = r.U.a[a][b].im + (R)0;
      v[o] = r.V.a[a][b].re + (R)0;
      v[o + 1] = r.V.a[a][b].im + (R)0;
    }
  S[2 * i] = scale2(r.f1, r.e1);
  S[2 * i + 1] = scale2(r.f2, r.e2);
  if (f) {
    f[2 * i] = r.f1;
    f[2 * i + 1] = r.f2;
  }
  if (e) {
    e[2 * i] = r.e1;
    e[2 * i + 1] = r.e2;
  }
  if (info) info[i] = (int32_t)r.info;
}

template <class R> __device__ inline void load_c(const R *G, int64_t i, Cx<R> g[4]) {
  const R *x = G + 8 * i;
  // row-major (r, c) at 2 (2 r + c); order g11, g21, g12, g22
  g[0] = Cx<R>{x[0], x[1]};
  g[1] = Cx<R>{x[4], x[5]};
  g[2] = Cx<R>{x[2], x[3]};
  g[3] = Cx<R>{x[6], x[7]};
}

// One matrix per lane; G, U, V are [n][2][2] complex (real and imaginary part
// interleaved), S [n][2] plain sigma, f [n][2] and e [n][2] the (e,f) pairs.
// Real and purely imaginary matrices are rare but would make every wave that
// holds one run the whole real method beside the complex path, so a workgroup
// collects them in LDS and its first lanes run the real method on them after
// the complex lanes are done (each matrix's result does not depend on which
// lane computes it).  At most 128 registers (4 waves per SIMD).
template <class R>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4, 8))) void k_fwd_c(
    int64_t n, const R *__restrict__ G, R *__restrict__ U, R *__restrict__ S,
    R *__restrict__ V, R *__restrict__ f, int32_t *__restrict__ e, int32_t *__restrict__ info) {
  __shared__ int s_cnt;
  __shared__ int s_list[kBlock];
  const int64_t base = (int64_t)blockIdx.x * kBlock;
  const int64_t i = base + threadIdx.x;
  const bool valid = i < n;
  Cx<R> g[4];
  bool all_re = false, rl = false;
  if (valid) {
    load_c(G, i, g);
    rl = real_or_imag(g, all_re);
  }
  if (threadIdx.x == 0) s_cnt = 0;
  __syncthreads();
  if (rl) s_list[atomicAdd(&s_cnt, 1)] = threadIdx.x;
  __syncthreads();
  if (valid && !rl) store_c(i, svd2c<R>(g), U, S, V, f, e, info);
  const int cnt = s_cnt;
  if ((int)threadIdx.x < cnt) {
    const int64_t j = base + s_list[threadIdx.x];
    Cx<R> h[4];
    load_c(G, j, h);
    bool hre;
    (void)real_or_imag(h, hre);
    store_c(j, svd2c_real<R>(h, hre), U, S, V, f, e, info);
  }
}

template <class R>
static int fwd_c(int64_t n, const R *G, R *U, R *S, R *V, R *f, int32_t *e, int32_t *info,
                 void *stream) {
  if (n < 0) return fail(KSVD2_EINVAL, "batch < 0");
  if (n == 0) return KSVD2_OK;
  const size_t w = sizeof(R);
  KSVD2_REQ(G, w); KSVD2_REQ(U, w); KSVD2_REQ(S, w); KSVD2_REQ(V, w);
  KSVD2_OPT(f, w); KSVD2_OPT(e, 4); KSVD2_OPT(info, 4);
  hipLaunchKernelGGL(k_fwd_c<R>, dim3(grid_for(n)), dim3(kBlock), 0, (hipStream_t)stream, n, G,
                     U, S, V, f, e, info);
  return launch_status("ksvd2c forward launch");
}

}  // namespace ksvd2

using namespace ksvd2;

extern "C" {

int ksvd2c_batch(int dtype, int64_t batch, const void *G, void *U, void *S, void *V, void *f,
                 int32_t *e, int32_t *info, void *stream) {
  if (dtype == 1)
    return fwd_c<double>(batch, (const double *)G, (double *)U, (double *)S, (double *)V,
                         (double *)f, e, info, stream);
  if (dtype == 0)
    return fwd_c<float>(batch, (const float *)G, (float *)U, (float *)S, (float *)V, (float *)f,
                        e, info, stream);
  return fail(KSVD2_EDTYPE, "dtype must be 0 (complex64) or 1 (complex128), got %d", dtype);
}

}  // extern "C"
