// Batched kernels of the 2x2 SVD and its adjoint, and their C ABI entry points
// (declared and documented in include/ksvd2.h).
//
// Launch shape: one matrix per lane, 256-lane workgroups (4 waves of 64), a
// 1-D grid of ceil(B/256) workgroups, so a 2^24 batch is 65,536 workgroups,
// far more than the 256 compute units.  Loads and stores are per-plane
// (structure of arrays) and therefore coalesced: lane i touches element i of
// every plane.
#include <hip/hip_runtime.h>

#include <initializer_list>
#include <string>

#include "abi_common.hpp"
#include "ksvd2_device.hpp"

namespace ksvd2 {

std::string &last_error_ref() {
  static thread_local std::string s;
  return s;
}

// element at byte offset `bo` of a plane: a 32-bit offset from the plane's base
// lets every load and store take the scalar-base addressing form instead of a
// 64-bit address per plane and lane (launches are split so that offsets fit)
template <class T> __device__ inline T &at(T *base, uint32_t bo) {
  return *reinterpret_cast<T *>(reinterpret_cast<char *>(base) + bo);
}
template <class T> __device__ inline const T &at(const T *base, uint32_t bo) {
  return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) + bo);
}
constexpr int64_t kMaxLaunch = int64_t(1) << 28;  // elements per launch: offsets < 2^31
constexpr int64_t kMaxLaunchFull = int64_t(1) << 26;  // [B,2,2] matrices per launch: 32 B each

// 6 waves per SIMD (at most 80 registers): the straight-line SVD code issues
// back-to-back dependent FP64 instructions, and one more resident wave hides
// more of their latency than the few registers given up cost (measured).
// CR: the correctly rounded hypot (the method as analysed) or the fast variant.
template <class R, bool CR>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(6, 8))) void k_fwd_soa(
    uint32_t n, const R *__restrict__ g11, const R *__restrict__ g21, const R *__restrict__ g12,
    const R *__restrict__ g22, R *__restrict__ cu, R *__restrict__ su, R *__restrict__ cv,
    R *__restrict__ sv, R *__restrict__ f1, R *__restrict__ f2, int32_t *__restrict__ e1,
    int32_t *__restrict__ e2, int32_t *__restrict__ info, R *__restrict__ s1,
    R *__restrict__ s2) {
  const uint32_t i = blockIdx.x * (uint32_t)kBlock + threadIdx.x;
  if (i >= n) return;
  const uint32_t bw = i * (uint32_t)sizeof(R), b4 = i * 4u;
  Svd2<R> r = svd2<R, CR>(at(g11, bw), at(g21, bw), at(g12, bw), at(g22, bw));
  at(cu, bw) = r.cu;
  at(su, bw) = r.su;
  at(cv, bw) = r.cv;
  at(sv, bw) = r.sv;
  at(f1, bw) = r.f1;
  at(f2, bw) = r.f2;
  at(e1, b4) = r.e1;
  at(e2, b4) = r.e2;
  at(info, b4) = (int32_t)r.info;
  if (s1) at(s1, bw) = scale2(r.f1, r.e1);
  if (s2) at(s2, bw) = scale2(r.f2, r.e2);
}

// [B,2,2] blocks (4 consecutive values) and [B,2] pairs, moved as 16-byte
// (binary32 pairs: 8-byte) vectors when every pointer of the launch is
// aligned for it (kVec), else value by value.
template <class R, bool kVec>
__device__ inline void ld4(const R *p, R &a, R &b, R &c, R &d) {
  if constexpr (kVec && sizeof(R) == 8) {
    double2 x = reinterpret_cast<const double2 *>(p)[0], y = reinterpret_cast<const double2 *>(p)[1];
    a = x.x; b = x.y; c = y.x; d = y.y;
  } else if constexpr (kVec) {
    float4 x = *reinterpret_cast<const float4 *>(p);
    a = x.x; b = x.y; c = x.z; d = x.w;
  } else {
    a = p[0]; b = p[1]; c = p[2]; d = p[3];
  }
}
// streaming loads for the backward pass, whose 2x2 operands are each read once:
// non-temporal loads let the memory system stream them (measured: 142 -> 123 us
// per 2^22 FP64 matrices; non-temporal loads of the sigma pairs and a
// non-temporal store of dG measured slower)
typedef double Nt2d __attribute__((ext_vector_type(2)));
typedef float Nt4f __attribute__((ext_vector_type(4)));
template <class R> __device__ inline void ld4s(const R *p, R &a, R &b, R &c, R &d) {
  if constexpr (sizeof(R) == 8) {
    Nt2d x = __builtin_nontemporal_load(reinterpret_cast<const Nt2d *>(p));
    Nt2d y = __builtin_nontemporal_load(reinterpret_cast<const Nt2d *>(p) + 1);
    a = x.x; b = x.y; c = y.x; d = y.y;
  } else {
    Nt4f x = __builtin_nontemporal_load(reinterpret_cast<const Nt4f *>(p));
    a = x.x; b = x.y; c = x.z; d = x.w;
  }
}
template <class R, bool kVec> __device__ inline void st4(R *p, R a, R b, R c, R d) {
  if constexpr (kVec && sizeof(R) == 8) {
    reinterpret_cast<double2 *>(p)[0] = double2{a, b};
    reinterpret_cast<double2 *>(p)[1] = double2{c, d};
  } else if constexpr (kVec) {
    *reinterpret_cast<float4 *>(p) = float4{a, b, c, d};
  } else {
    p[0] = a; p[1] = b; p[2] = c; p[3] = d;
  }
}
template <class R, bool kVec> __device__ inline void ld2(const R *p, R &a, R &b) {
  if constexpr (kVec && sizeof(R) == 8) {
    double2 x = *reinterpret_cast<const double2 *>(p);
    a = x.x; b = x.y;
  } else if constexpr (kVec) {
    float2 x = *reinterpret_cast<const float2 *>(p);
    a = x.x; b = x.y;
  } else {
    a = p[0]; b = p[1];
  }
}
template <class R, bool kVec> __device__ inline void st2(R *p, R a, R b) {
  if constexpr (kVec && sizeof(R) == 8) {
    *reinterpret_cast<double2 *>(p) = double2{a, b};
  } else if constexpr (kVec) {
    *reinterpret_cast<float2 *>(p) = float2{a, b};
  } else {
    p[0] = a; p[1] = b;
  }
}

// whether every non-null pointer is aligned for the vector forms above
static bool vec_aligned(size_t w, std::initializer_list<const void *> ps) {
  for (const void *p : ps)
    if (p && (reinterpret_cast<uintptr_t>(p) % 16 != 0)) return false;
  (void)w;
  return true;
}

// Autograd layout: G, U, V are [B,2,2] row-major, S is [B,2] (plain sigma).
// Addressed like k_fwd_soa: scalar bases and one 32-bit byte offset per lane
// (launches are split so that the offsets of G, U, V stay below 2^31).
template <class R, bool kVec>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(6, 8))) void k_fwd_full(
    uint32_t n, const R *__restrict__ G, R *__restrict__ U, R *__restrict__ S,
    R *__restrict__ V, int32_t *__restrict__ info) {
  const uint32_t i = blockIdx.x * (uint32_t)kBlock + threadIdx.x;
  if (i >= n) return;
  const uint32_t b4 = i * (uint32_t)(4 * sizeof(R)), b2 = i * (uint32_t)(2 * sizeof(R));
  R g11, g12, g21, g22;
  ld4<R, kVec>(&at(G, b4), g11, g12, g21, g22);
  Svd2<R> r = svd2<R>(g11, g21, g12, g22);
  R du = (r.info & I_DETU) ? (R)-1 : (R)1;
  R dv = (r.info & I_DETV) ? (R)-1 : (R)1;
  st4<R, kVec>(&at(U, b4), r.cu, -du * r.su, r.su, du * r.cu);
  st4<R, kVec>(&at(V, b4), r.cv, -dv * r.sv, r.sv, dv * r.cv);
  st2<R, kVec>(&at(S, b2), scale2(r.f1, r.e1), scale2(r.f2, r.e2));
  if (info) at(info, i * 4u) = (int32_t)r.info;
}

// Adjoint of G = U diag(S) V^T (2x2, square, full U and V):
//   a = (U^T dU)_12 - (U^T dU)_21,  b = (V^T dV)_12 - (V^T dV)_21,
//   p = (a + b)/2, q = (a - b)/2,
//   M = [[dS1, -p/(s1-s2) + q/(s1+s2)], [-p/(s1-s2) - q/(s1+s2), dS2]],
//   dG = U M V^T.
// 1/(s1-s2): with tau > 0 replaced by (s1-s2)/((s1-s2)^2 + (tau s1)^2);
// with tau = 0 taken as 0 when s1 == s2; 1/(s1+s2) taken as 0 when s1+s2 == 0.
template <class R, bool kVec>
__global__ __launch_bounds__(kBlock) void k_bwd(int64_t n, const R *__restrict__ U,
                                                const R *__restrict__ S,
                                                const R *__restrict__ V,
                                                const R *__restrict__ dS,
                                                const R *__restrict__ dU,
                                                const R *__restrict__ dV, R *__restrict__ dG,
                                                R tau) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  auto ldq = [](const R *p, R &a, R &b, R &c, R &d) {
    if constexpr (kVec) ld4s<R>(p, a, b, c, d); else ld4<R, kVec>(p, a, b, c, d);
  };
  auto ldp = [](const R *p, R &a, R &b) { ld2<R, kVec>(p, a, b); };
  R u11, u12, u21, u22, v11, v12, v21, v22, s1, s2;
  ldq(U + 4 * i, u11, u12, u21, u22);
  ldq(V + 4 * i, v11, v12, v21, v22);
  ldp(S + 2 * i, s1, s2);
  R a = 0, b = 0;
  if (dU) {
    R w11, w12, w21, w22;
    ldq(dU + 4 * i, w11, w12, w21, w22);
    // (U^T dU)_12 = u11 w12 + u21 w22 ; (U^T dU)_21 = u12 w11 + u22 w21
    a = fma(u11, w12, u21 * w22) - fma(u12, w11, u22 * w21);
  }
  if (dV) {
    R w11, w12, w21, w22;
    ldq(dV + 4 * i, w11, w12, w21, w22);
    b = fma(v11, w12, v21 * w22) - fma(v12, w11, v22 * w21);
  }
  R p = (R)0.5 * (a + b), q = (R)0.5 * (a - b);
  R dm = s1 - s2, sm = s1 + s2;
  R idm;
  if (tau > (R)0) {
    R eta = tau * s1;
    R den = fma(dm, dm, eta * eta);
    idm = (den > (R)0) ? dm / den : (R)0;
  } else {
    idm = (dm != (R)0) ? (R)1 / dm : (R)0;
  }
  R ism = (sm != (R)0) ? (R)1 / sm : (R)0;
  R m11 = 0, m22 = 0;
  if (dS) ldp(dS + 2 * i, m11, m22);
  R pd = p * idm, qs = q * ism;
  R m12 = qs - pd, m21 = -pd - qs;
  // T = U M, then dG = T V^T
  R t11 = fma(u11, m11, u12 * m21), t12 = fma(u11, m12, u12 * m22);
  R t21 = fma(u21, m11, u22 * m21), t22 = fma(u21, m12, u22 * m22);
  const R g11 = fma(t11, v11, t12 * v12), g12 = fma(t11, v21, t12 * v22);
  const R g21 = fma(t21, v11, t22 * v12), g22 = fma(t21, v21, t22 * v22);
  st4<R, kVec>(dG + 4 * i, g11, g12, g21, g22);
}

// The same adjoint on the structure-of-arrays planes of the forward entry
// points: U = [cu -dU su; su dU cu] and V likewise, with the determinant signs
// dU, dV from info bits 8 and 9, so a matrix reads 4 + 4 + 1 words of U, V and
// info instead of 8 full entries.  U and V are expanded into their four entries
// (sign changes only) and then go through exactly the operations of k_bwd in
// the same order: the result is bit for bit that of k_bwd on the expanded
// matrices.  Upstream gradients: ds1, ds2 (nullable: 0), dU, dV (nullable: 0)
// as plane pointers u11, u21, u12, u22; dG as four planes g11, g21, g12, g22.
template <class R> struct BwdSoaArgs {
  const R *cu, *su, *cv, *sv, *s1, *s2, *ds1, *ds2;
  const int32_t *info;
  const R *du[4], *dv[4];
  R *dg[4];
};

template <class R>
__global__ __launch_bounds__(kBlock) void k_bwd_soa(uint32_t n, BwdSoaArgs<R> A, R tau) {
  const uint32_t i = blockIdx.x * (uint32_t)kBlock + threadIdx.x;
  if (i >= n) return;
  const uint32_t bw = i * (uint32_t)sizeof(R);
  const uint32_t inf = (uint32_t)at(A.info, i * 4u);
  const R c_u = at(A.cu, bw), s_u = at(A.su, bw), c_v = at(A.cv, bw), s_v = at(A.sv, bw);
  const bool nu = (inf & I_DETU) != 0, nv = (inf & I_DETV) != 0;
  // U = [u11 u12; u21 u22] with u12 = -dU su, u22 = dU cu (likewise V)
  const R u11 = c_u, u21 = s_u, u12 = nu ? s_u : -s_u, u22 = nu ? -c_u : c_u;
  const R v11 = c_v, v21 = s_v, v12 = nv ? s_v : -s_v, v22 = nv ? -c_v : c_v;
  const R s1 = at(A.s1, bw), s2 = at(A.s2, bw);
  R a = 0, b = 0;
  if (A.du[0]) {
    const R w11 = at(A.du[0], bw), w21 = at(A.du[1], bw), w12 = at(A.du[2], bw),
            w22 = at(A.du[3], bw);
    a = fma(u11, w12, u21 * w22) - fma(u12, w11, u22 * w21);
  }
  if (A.dv[0]) {
    const R w11 = at(A.dv[0], bw), w21 = at(A.dv[1], bw), w12 = at(A.dv[2], bw),
            w22 = at(A.dv[3], bw);
    b = fma(v11, w12, v21 * w22) - fma(v12, w11, v22 * w21);
  }
  R p = (R)0.5 * (a + b), q = (R)0.5 * (a - b);
  R dm = s1 - s2, sm = s1 + s2;
  R idm;
  if (tau > (R)0) {
    R eta = tau * s1;
    R den = fma(dm, dm, eta * eta);
    idm = (den > (R)0) ? dm / den : (R)0;
  } else {
    idm = (dm != (R)0) ? (R)1 / dm : (R)0;
  }
  R ism = (sm != (R)0) ? (R)1 / sm : (R)0;
  const R m11 = A.ds1 ? at(A.ds1, bw) : (R)0, m22 = A.ds2 ? at(A.ds2, bw) : (R)0;
  R pd = p * idm, qs = q * ism;
  R m12 = qs - pd, m21 = -pd - qs;
  R t11 = fma(u11, m11, u12 * m21), t12 = fma(u11, m12, u12 * m22);
  R t21 = fma(u21, m11, u22 * m21), t22 = fma(u21, m12, u22 * m22);
  at(A.dg[0], bw) = fma(t11, v11, t12 * v12);
  at(A.dg[1], bw) = fma(t21, v11, t22 * v12);
  at(A.dg[2], bw) = fma(t11, v21, t12 * v22);
  at(A.dg[3], bw) = fma(t21, v21, t22 * v22);
}

template <class R, bool CR>
__global__ __launch_bounds__(kBlock) void k_hypot(int64_t n, const R *__restrict__ x,
                                                  const R *__restrict__ y, R *__restrict__ out) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  out[i] = hyp<CR>(x[i], y[i]);
}

template <class R, bool CR>
static int fwd_soa(int64_t n, const R *g11, const R *g21, const R *g12, const R *g22, R *cu, R *su,
                   R *cv, R *sv, R *f1, R *f2, int32_t *e1, int32_t *e2, int32_t *info, R *s1,
                   R *s2, void *stream) {
  if (n < 0) return fail(KSVD2_EINVAL, "batch < 0");
  if (n == 0) return KSVD2_OK;
  const size_t w = sizeof(R);
  KSVD2_REQ(g11, w); KSVD2_REQ(g21, w); KSVD2_REQ(g12, w); KSVD2_REQ(g22, w);
  KSVD2_REQ(cu, w); KSVD2_REQ(su, w); KSVD2_REQ(cv, w); KSVD2_REQ(sv, w);
  KSVD2_REQ(f1, w); KSVD2_REQ(f2, w); KSVD2_REQ(e1, 4); KSVD2_REQ(e2, 4); KSVD2_REQ(info, 4);
  KSVD2_OPT(s1, w); KSVD2_OPT(s2, w);
  for (int64_t o = 0; o < n; o += kMaxLaunch) {
    const uint32_t c = (uint32_t)(n - o < kMaxLaunch ? n - o : kMaxLaunch);
    R *s1o = s1 ? s1 + o : nullptr, *s2o = s2 ? s2 + o : nullptr;
    hipLaunchKernelGGL((k_fwd_soa<R, CR>), dim3(grid_for(c)), dim3(kBlock), 0,
                       (hipStream_t)stream, c, g11 + o, g21 + o, g12 + o, g22 + o, cu + o, su + o,
                       cv + o, sv + o, f1 + o, f2 + o, e1 + o, e2 + o, info + o, s1o, s2o);
  }
  return launch_status("ksvd2 forward launch");
}

template <class R>
static int fwd_full(int64_t n, const R *G, R *U, R *S, R *V, int32_t *info, void *stream) {
  if (n < 0) return fail(KSVD2_EINVAL, "batch < 0");
  if (n == 0) return KSVD2_OK;
  const size_t w = sizeof(R);
  KSVD2_REQ(G, w); KSVD2_REQ(U, w); KSVD2_REQ(S, w); KSVD2_REQ(V, w);
  KSVD2_OPT(info, 4);
  const bool vec = vec_aligned(w, {G, U, S, V});
  for (int64_t o = 0; o < n; o += kMaxLaunchFull) {
    const uint32_t c = (uint32_t)(n - o < kMaxLaunchFull ? n - o : kMaxLaunchFull);
    int32_t *io = info ? info + o : nullptr;
    if (vec)
      hipLaunchKernelGGL((k_fwd_full<R, true>), dim3(grid_for(c)), dim3(kBlock), 0,
                         (hipStream_t)stream, c, G + 4 * o, U + 4 * o, S + 2 * o, V + 4 * o, io);
    else
      hipLaunchKernelGGL((k_fwd_full<R, false>), dim3(grid_for(c)), dim3(kBlock), 0,
                         (hipStream_t)stream, c, G + 4 * o, U + 4 * o, S + 2 * o, V + 4 * o, io);
  }
  return launch_status("ksvd2 forward (full layout) launch");
}

template <class R>
static int bwd(int64_t n, const void *U, const void *S, const void *V, const void *dS,
               const void *dU, const void *dV, void *dG, double tau, void *stream) {
  if (n < 0) return fail(KSVD2_EINVAL, "batch < 0");
  if (!(tau >= 0.0)) return fail(KSVD2_EINVAL, "tau must be >= 0");
  if (n == 0) return KSVD2_OK;
  const size_t w = sizeof(R);
  KSVD2_REQ(U, w); KSVD2_REQ(S, w); KSVD2_REQ(V, w); KSVD2_REQ(dG, w);
  KSVD2_OPT(dS, w); KSVD2_OPT(dU, w); KSVD2_OPT(dV, w);
  if (vec_aligned(w, {U, S, V, dS, dU, dV, dG}))
    hipLaunchKernelGGL((k_bwd<R, true>), dim3(grid_for(n)), dim3(kBlock), 0, (hipStream_t)stream,
                       n, (const R *)U, (const R *)S, (const R *)V, (const R *)dS, (const R *)dU,
                       (const R *)dV, (R *)dG, (R)tau);
  else
    hipLaunchKernelGGL((k_bwd<R, false>), dim3(grid_for(n)), dim3(kBlock), 0,
                       (hipStream_t)stream, n, (const R *)U, (const R *)S, (const R *)V,
                       (const R *)dS, (const R *)dU, (const R *)dV, (R *)dG, (R)tau);
  return launch_status("ksvd2 backward launch");
}

template <class R>
static int bwd_soa(int64_t n, const void *cu, const void *su, const void *cv, const void *sv,
                   const int32_t *info, const void *s1, const void *s2, const void *ds1,
                   const void *ds2, const void *dU, const void *dV, void *dg11, void *dg21,
                   void *dg12, void *dg22, double tau, void *stream) {
  if (n < 0) return fail(KSVD2_EINVAL, "batch < 0");
  if (!(tau >= 0.0)) return fail(KSVD2_EINVAL, "tau must be >= 0");
  if (n == 0) return KSVD2_OK;
  const size_t w = sizeof(R);
  KSVD2_REQ(cu, w); KSVD2_REQ(su, w); KSVD2_REQ(cv, w); KSVD2_REQ(sv, w); KSVD2_REQ(info, 4);
  KSVD2_REQ(s1, w); KSVD2_REQ(s2, w);
  KSVD2_OPT(ds1, w); KSVD2_OPT(ds2, w); KSVD2_OPT(dU, w); KSVD2_OPT(dV, w);
  KSVD2_REQ(dg11, w); KSVD2_REQ(dg21, w); KSVD2_REQ(dg12, w); KSVD2_REQ(dg22, w);
  for (int64_t o = 0; o < n; o += kMaxLaunch) {
    const uint32_t c = (uint32_t)(n - o < kMaxLaunch ? n - o : kMaxLaunch);
    BwdSoaArgs<R> A;
    A.cu = (const R *)cu + o; A.su = (const R *)su + o;
    A.cv = (const R *)cv + o; A.sv = (const R *)sv + o;
    A.s1 = (const R *)s1 + o; A.s2 = (const R *)s2 + o;
    A.ds1 = ds1 ? (const R *)ds1 + o : nullptr;
    A.ds2 = ds2 ? (const R *)ds2 + o : nullptr;
    A.info = info + o;
    for (int k = 0; k < 4; ++k) {
      A.du[k] = dU ? (const R *)dU + (int64_t)k * n + o : nullptr;
      A.dv[k] = dV ? (const R *)dV + (int64_t)k * n + o : nullptr;
    }
    A.dg[0] = (R *)dg11 + o; A.dg[1] = (R *)dg21 + o;
    A.dg[2] = (R *)dg12 + o; A.dg[3] = (R *)dg22 + o;
    hipLaunchKernelGGL(k_bwd_soa<R>, dim3(grid_for(c)), dim3(kBlock), 0, (hipStream_t)stream, c,
                       A, (R)tau);
  }
  return launch_status("ksvd2 backward (planes) launch");
}

template <bool CR>
static int hypot_launch(int dtype, int64_t n, const void *x, const void *y, void *out,
                        void *stream) {
  if (n < 0) return fail(KSVD2_EINVAL, "n < 0");
  if (dtype != 0 && dtype != 1)
    return fail(KSVD2_EDTYPE, "dtype must be 0 (f32) or 1 (f64), got %d", dtype);
  if (n == 0) return KSVD2_OK;
  size_t w = dtype ? 8 : 4;
  KSVD2_REQ(x, w); KSVD2_REQ(y, w); KSVD2_REQ(out, w);
  if (dtype)
    hipLaunchKernelGGL((k_hypot<double, CR>), dim3(grid_for(n)), dim3(kBlock), 0,
                       (hipStream_t)stream, n, (const double *)x, (const double *)y,
                       (double *)out);
  else
    hipLaunchKernelGGL((k_hypot<float, CR>), dim3(grid_for(n)), dim3(kBlock), 0,
                       (hipStream_t)stream, n, (const float *)x, (const float *)y, (float *)out);
  return launch_status("ksvd2 hypot launch");
}

}  // namespace ksvd2

using namespace ksvd2;

extern "C" {

int ksvd2_version(void) { return 4; }

const char *ksvd2_last_error(void) { return last_error_ref().c_str(); }

int ksvd2_batch_f64(int64_t batch, const double *g11, const double *g21, const double *g12,
                    const double *g22, double *cu, double *su, double *cv, double *sv, double *f1,
                    double *f2, int32_t *e1, int32_t *e2, int32_t *info, double *s1_plain,
                    double *s2_plain, void *stream) {
  return fwd_soa<double, true>(batch, g11, g21, g12, g22, cu, su, cv, sv, f1, f2, e1, e2, info,
                         s1_plain, s2_plain, stream);
}

int ksvd2_batch_f32(int64_t batch, const float *g11, const float *g21, const float *g12,
                    const float *g22, float *cu, float *su, float *cv, float *sv, float *f1,
                    float *f2, int32_t *e1, int32_t *e2, int32_t *info, float *s1_plain,
                    float *s2_plain, void *stream) {
  return fwd_soa<float, true>(batch, g11, g21, g12, g22, cu, su, cv, sv, f1, f2, e1, e2, info, s1_plain,
                        s2_plain, stream);
}

int ksvd2_svd2x2(int dtype, int64_t batch, const void *G, void *U, void *S, void *V,
                 int32_t *info, void *stream) {
  if (dtype == 1)
    return fwd_full<double>(batch, (const double *)G, (double *)U, (double *)S, (double *)V, info,
                            stream);
  if (dtype == 0)
    return fwd_full<float>(batch, (const float *)G, (float *)U, (float *)S, (float *)V, info,
                           stream);
  return fail(KSVD2_EDTYPE, "dtype must be 0 (f32) or 1 (f64), got %d", dtype);
}

int ksvd2_svd2x2_backward(int dtype, int64_t batch, const void *U, const void *S, const void *V,
                          const void *dS, const void *dU, const void *dV, void *dG, double tau,
                          void *stream) {
  if (dtype == 1) return bwd<double>(batch, U, S, V, dS, dU, dV, dG, tau, stream);
  if (dtype == 0) return bwd<float>(batch, U, S, V, dS, dU, dV, dG, tau, stream);
  return fail(KSVD2_EDTYPE, "dtype must be 0 (f32) or 1 (f64), got %d", dtype);
}

int ksvd2_batch_backward(int dtype, int64_t batch, const void *cu, const void *su,
                         const void *cv, const void *sv, const int32_t *info, const void *s1,
                         const void *s2, const void *ds1, const void *ds2, const void *dU,
                         const void *dV, void *dg11, void *dg21, void *dg12, void *dg22,
                         double tau, void *stream) {
  if (dtype == 1)
    return bwd_soa<double>(batch, cu, su, cv, sv, info, s1, s2, ds1, ds2, dU, dV, dg11, dg21,
                           dg12, dg22, tau, stream);
  if (dtype == 0)
    return bwd_soa<float>(batch, cu, su, cv, sv, info, s1, s2, ds1, ds2, dU, dV, dg11, dg21,
                          dg12, dg22, tau, stream);
  return fail(KSVD2_EDTYPE, "dtype must be 0 (f32) or 1 (f64), got %d", dtype);
}

int ksvd2_batch_fast_f64(int64_t batch, const double *g11, const double *g21, const double *g12,
                         const double *g22, double *cu, double *su, double *cv, double *sv,
                         double *f1, double *f2, int32_t *e1, int32_t *e2, int32_t *info,
                         double *s1_plain, double *s2_plain, void *stream) {
  return fwd_soa<double, false>(batch, g11, g21, g12, g22, cu, su, cv, sv, f1, f2, e1, e2, info,
                                s1_plain, s2_plain, stream);
}

int ksvd2_batch_fast_f32(int64_t batch, const float *g11, const float *g21, const float *g12,
                         const float *g22, float *cu, float *su, float *cv, float *sv, float *f1,
                         float *f2, int32_t *e1, int32_t *e2, int32_t *info, float *s1_plain,
                         float *s2_plain, void *stream) {
  return fwd_soa<float, false>(batch, g11, g21, g12, g22, cu, su, cv, sv, f1, f2, e1, e2, info,
                               s1_plain, s2_plain, stream);
}

int ksvd2_hypot_batch(int dtype, int64_t n, const void *x, const void *y, void *out,
                      void *stream) {
  return hypot_launch<true>(dtype, n, x, y, out, stream);
}

int ksvd2_hypot_fast_batch(int dtype, int64_t n, const void *x, const void *y, void *out,
                           void *stream) {
  return hypot_launch<false>(dtype, n, x, y, out, stream);
}

}  // extern "C"
