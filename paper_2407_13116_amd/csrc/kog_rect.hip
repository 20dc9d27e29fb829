// Rectangular inputs for the Kogbetliantz iteration (Sect. 1): an m x n matrix
// with m >= n is reduced to a square triangular one by the QR factorization with
// column pivoting, G P = Q R, the iteration runs on R = U_R Sigma V_R^T, and the
// factors of G are U = Q [U_R; 0], V = P V_R.  Entry points declared and
// documented in include/ksvd2.h (kog_qrcp_batch, kog_qrcp_apply,
// kog_rect_workspace_size).
//
// One workgroup per matrix factorizes it in place (Householder reflections
// H_k = I - tau_k v_k v_k^T, v_k(k) = 1, stored below the diagonal as LAPACK's
// geqp3 does): per column the pivot (largest trailing norm, the first on ties),
// the column exchange, the reflector, and its application to the trailing
// columns, which also yields their norms for the next pivot; waves take whole
// columns and reduce over the rows with a fixed lane tree.  Q is applied to
// [U_R; 0] column by column, one wave per column through all n reflectors
// (columns are independent, so no workgroup barrier is needed there).
#include <hip/hip_runtime.h>

#include <climits>
#include <cstdint>
#include <cstring>
#include <vector>

#include "abi_common.hpp"

namespace ksvd2 {

constexpr int kRectMaxN = 4096;  // the column norms of a matrix live in LDS
constexpr int kQrcpBlock = 1024;
constexpr int kQapplyBlock = 256;
constexpr size_t kQapplyLds = 64 * 1024;  // the U columns of a workgroup, when they fit

struct RectDesc {
  const int32_t *m, *n;
  const int64_t *aoff, *roff, *toff;
};

template <class R> __device__ inline R wave_sum(R v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

template <class R> struct RectLim;
template <> struct RectLim<double> {
  static constexpr int e_nu = 1023;
};
template <> struct RectLim<float> {
  static constexpr int e_nu = 127;
};

// The power of two s by which the factorization scales the matrix first: the
// squared column norms (m terms up to 2^(2 e_max + 2)) stay in the normal range
// when 2 |e_max| + ceil(lg m) + 2 < e_nu; otherwise s = -e_max puts the largest
// entry into [1, 2).  The reflectors and tau do not depend on such a scaling, R
// scales by 2^s, so R is scaled back at the end; the pivots compare norms all
// scaled alike.  (Exact, except for entries that scaling down moves below the
// normal range.)
__host__ __device__ inline int qrcp_scale(int emax, int m, int e_nu) {
  if (emax == INT_MIN) return 0;
  int lgm = 0;
  while ((1 << lgm) < m) ++lgm;
  const int ae = emax < 0 ? -emax : emax;
  return (2 * ae + lgm + 2 < e_nu) ? 0 : -emax;
}

template <class R>
__global__ __launch_bounds__(kQrcpBlock) void k_qrcp(RectDesc d, R *A, R *tau, int32_t *perm,
                                                     R *Rsq) {
  __shared__ R s_nrm[kRectMaxN];
  __shared__ int s_piv, s_emax;
  __shared__ R s_tau, s_beta, s_scal;
  const int mat = blockIdx.x;
  const int m = d.m[mat], n = d.n[mat];
  R *a = A + d.aoff[mat];
  R *tu = tau + d.toff[mat];
  int32_t *pm = perm + d.toff[mat];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int j = threadIdx.x; j < n; j += blockDim.x) pm[j] = j;
  const int64_t tot = (int64_t)m * n;
  if (threadIdx.x == 0) s_emax = INT_MIN;
  __syncthreads();
  {
    int e = INT_MIN;
    for (int64_t x = threadIdx.x; x < tot; x += blockDim.x)
      if (a[x] != (R)0) e = max(e, ilogb(a[x]));
    atomicMax(&s_emax, e);  // LDS
  }
  __syncthreads();
  const int sc = qrcp_scale(s_emax, m, RectLim<R>::e_nu);
  if (sc != 0) {
    for (int64_t x = threadIdx.x; x < tot; x += blockDim.x) a[x] = ldexp(a[x], sc);
    __syncthreads();
  }
  // squared column norms over all rows; later steps take them from the update
  // pass of the step before (the same rows, summed by the same lanes in the same
  // order as a separate pass would)
  for (int j = wv; j < n; j += nw) {
    const R *c = a + (int64_t)j * m;
    R s = 0;
    for (int i = lane; i < m; i += 64) s += c[i] * c[i];
    s = wave_sum(s);
    if (lane == 0) s_nrm[j] = s;
  }
  __syncthreads();
  for (int k = 0; k < n; ++k) {
    // the pivot: the largest squared norm, the smallest index on ties
    if (wv == 0) {
      R best = (R)-1;
      int bi = n;
      for (int j = k + lane; j < n; j += 64) {
        R v = s_nrm[j];
        if (v > best) {
          best = v;
          bi = j;
        }
      }
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) {
        R ob = __shfl_xor(best, o, 64);
        int oi = __shfl_xor(bi, o, 64);
        if (ob > best || (ob == best && oi < bi)) {
          best = ob;
          bi = oi;
        }
      }
      if (lane == 0) s_piv = bi < n ? bi : k;  // no comparable norm (NaN): no exchange
    }
    __syncthreads();
    const int p = s_piv;
    if (p != k) {
      R *ck = a + (int64_t)k * m, *cp = a + (int64_t)p * m;
      for (int i = threadIdx.x; i < m; i += blockDim.x) {
        R t = ck[i];
        ck[i] = cp[i];
        cp[i] = t;
      }
      if (threadIdx.x == 0) {
        int32_t t = pm[k];
        pm[k] = pm[p];
        pm[p] = t;
      }
    }
    __syncthreads();
    // the reflector mapping column k (rows k..m-1) onto beta e_k
    R *ck = a + (int64_t)k * m;
    if (wv == 0) {
      R s = 0;
      for (int i = k + 1 + lane; i < m; i += 64) s += ck[i] * ck[i];
      s = wave_sum(s);
      if (lane == 0) {
        R x0 = ck[k];
        if (s == (R)0) {
          s_tau = 0;
        } else {
          R nrm = sqrt(x0 * x0 + s);
          R beta = x0 >= (R)0 ? -nrm : nrm;
          s_tau = (beta - x0) / beta;
          s_beta = beta;
          s_scal = (R)1 / (x0 - beta);
        }
        tu[k] = s_tau;
      }
    }
    __syncthreads();
    const R tk = s_tau;
    if (tk != (R)0) {
      const R scal = s_scal;
      for (int i = k + 1 + threadIdx.x; i < m; i += blockDim.x) ck[i] *= scal;
      __syncthreads();
      if (threadIdx.x == 0) ck[k] = s_beta;
      // H_k on the trailing columns, and their squared norms over rows k+1..m-1
      // for the next pivot
      for (int j = k + 1 + wv; j < n; j += nw) {
        R *cj = a + (int64_t)j * m;
        R w = 0;
        for (int i = k + 1 + lane; i < m; i += 64) w += ck[i] * cj[i];
        w = wave_sum(w) + cj[k];
        R tw = tk * w;
        if (lane == 0) cj[k] -= tw;
        R s = 0;
        for (int i = k + 1 + lane; i < m; i += 64) {
          R x = cj[i] - tw * ck[i];
          cj[i] = x;
          s += x * x;
        }
        s = wave_sum(s);
        if (lane == 0) s_nrm[j] = s;
      }
    } else {
      for (int j = k + 1 + wv; j < n; j += nw) {
        const R *cj = a + (int64_t)j * m;
        R s = 0;
        for (int i = k + 1 + lane; i < m; i += 64) s += cj[i] * cj[i];
        s = wave_sum(s);
        if (lane == 0) s_nrm[j] = s;
      }
    }
    __syncthreads();
  }
  // R scaled back (the reflectors below the diagonal are scale-free)
  if (sc != 0) {
    for (int64_t idx = threadIdx.x; idx < (int64_t)n * n; idx += blockDim.x) {
      int j = (int)(idx / n), i = (int)(idx - (int64_t)j * n);
      if (i <= j) a[i + (int64_t)j * m] = ldexp(a[i + (int64_t)j * m], -sc);
    }
    __syncthreads();
  }
  // the n x n triangular factor, zeros below the diagonal
  R *rs = Rsq + d.roff[mat];
  for (int64_t idx = threadIdx.x; idx < (int64_t)n * n; idx += blockDim.x) {
    int j = (int)(idx / n), i = (int)(idx - (int64_t)j * n);
    rs[idx] = (i <= j) ? a[i + (int64_t)j * m] : (R)0;
  }
}

// U = H_0 ... H_{n-1} [U_R; 0]: one wave per column of U; V = P V_R by rows.
// kLds: the wave's column lives in LDS while the reflectors are applied (the
// reflectors stream from L2/HBM); otherwise it is updated in place in U.  Both
// perform the same operations in the same order.
template <class R, bool kLds>
__global__ __launch_bounds__(kQapplyBlock) void k_qapply(RectDesc d, const R *A, const R *tau,
                                                         const int32_t *perm, const R *UR,
                                                         const R *VR, R *U, R *V, int ldsm) {
  extern __shared__ unsigned char s_raw[];
  const int mat = blockIdx.y;
  const int m = d.m[mat], n = d.n[mat];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int j = blockIdx.x * (kQapplyBlock >> 6) + wv;
  if (j >= n) return;  // whole waves leave; no barrier below
  const R *a = A + d.aoff[mat];
  const R *tu = tau + d.toff[mat];
  const R *ur = UR + d.roff[mat] + (int64_t)j * n;
  R *ug = U + d.aoff[mat] + (int64_t)j * m;
  R *u = kLds ? reinterpret_cast<R *>(s_raw) + (size_t)wv * ldsm : ug;
  for (int i = lane; i < m; i += 64) u[i] = (i < n) ? ur[i] : (R)0;
  if (kLds) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
  for (int k = n - 1; k >= 0; --k) {
    const R tk = tu[k];
    if (tk == (R)0) continue;
    const R *v = a + (int64_t)k * m;
    R w = 0;
    for (int i = k + 1 + lane; i < m; i += 64) w += v[i] * u[i];
    w = wave_sum(w) + u[k];
    R tw = tk * w;
    if (kLds) {
      // every lane has read u[k] before lane 0 rewrites it
      __builtin_amdgcn_wave_barrier();
    }
    if (lane == 0) u[k] -= tw;
    for (int i = k + 1 + lane; i < m; i += 64) u[i] -= tw * v[i];
    if (kLds) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
  }
  if (kLds)
    for (int i = lane; i < m; i += 64) ug[i] = u[i];
  const int32_t *pm = perm + d.toff[mat];
  const R *vr = VR + d.roff[mat] + (int64_t)j * n;
  R *vo = V + d.roff[mat] + (int64_t)j * n;
  for (int i = lane; i < n; i += 64) vo[pm[i]] = vr[i];
}

static size_t rect_align(size_t x) { return (x + 255) & ~(size_t)255; }

struct RectLayout {
  size_t m, n, aoff, roff, toff, total;
};
static RectLayout rect_layout(int64_t nmat) {
  RectLayout L;
  size_t p = 0;
  L.m = p;    p = rect_align(p + nmat * 4);
  L.n = p;    p = rect_align(p + nmat * 4);
  L.aoff = p; p = rect_align(p + nmat * 8);
  L.roff = p; p = rect_align(p + nmat * 8);
  L.toff = p; p = rect_align(p + nmat * 8);
  L.total = p;
  return L;
}

// validates the batch and uploads its descriptor into the workspace
static int rect_setup(int64_t nmat, const int32_t *m_host, const int32_t *n_host,
                      const int64_t *aoff_host, const int64_t *roff_host, void *ws,
                      size_t ws_bytes, hipStream_t st, RectDesc &d, int &maxn) {
  if (!m_host || !n_host || !aoff_host || !roff_host)
    return fail(KSVD2_EINVAL, "m_host, n_host, aoff_host and roff_host are required");
  if (nmat > 65535) return fail(KSVD2_EINVAL, "at most 65535 matrices per call");
  KSVD2_REQ(ws, 256);
  RectLayout L = rect_layout(nmat);
  if (ws_bytes < L.total)
    return fail(KSVD2_EWORKSPACE, "workspace of %zu bytes, %zu needed", ws_bytes, L.total);
  std::vector<int64_t> toff(nmat);
  int64_t acc = 0;
  maxn = 0;
  for (int64_t k = 0; k < nmat; ++k) {
    int m = m_host[k], n = n_host[k];
    if (n < 1 || n > kRectMaxN || m < n)
      return fail(KSVD2_EINVAL, "matrix %lld: need 1 <= n <= %d and m >= n (m = %d, n = %d)",
                  (long long)k, kRectMaxN, m, n);
    if (aoff_host[k] < 0 || roff_host[k] < 0)
      return fail(KSVD2_EINVAL, "matrix %lld: negative offset", (long long)k);
    toff[k] = acc;
    acc += n;
    maxn = n > maxn ? n : maxn;
  }
  std::vector<unsigned char> host(L.total, 0);
  std::memcpy(host.data() + L.m, m_host, nmat * 4);
  std::memcpy(host.data() + L.n, n_host, nmat * 4);
  std::memcpy(host.data() + L.aoff, aoff_host, nmat * 8);
  std::memcpy(host.data() + L.roff, roff_host, nmat * 8);
  std::memcpy(host.data() + L.toff, toff.data(), nmat * 8);
  unsigned char *w = static_cast<unsigned char *>(ws);
  hipError_t e = hipMemcpyAsync(w, host.data(), L.total, hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return fail(KSVD2_EHIP, "descriptor upload: %s", hipGetErrorString(e));
  d.m = reinterpret_cast<const int32_t *>(w + L.m);
  d.n = reinterpret_cast<const int32_t *>(w + L.n);
  d.aoff = reinterpret_cast<const int64_t *>(w + L.aoff);
  d.roff = reinterpret_cast<const int64_t *>(w + L.roff);
  d.toff = reinterpret_cast<const int64_t *>(w + L.toff);
  return KSVD2_OK;
}

template <class R>
static int qrcp_impl(int64_t nmat, const int32_t *m_host, const int32_t *n_host,
                     const int64_t *aoff_host, const int64_t *roff_host, R *A, R *tau,
                     int32_t *perm, R *Rsq, void *ws, size_t ws_bytes, hipStream_t st) {
  if (nmat < 0) return fail(KSVD2_EINVAL, "nmat < 0");
  if (nmat == 0) return KSVD2_OK;
  const size_t w = sizeof(R);
  KSVD2_REQ(A, w); KSVD2_REQ(tau, w); KSVD2_REQ(perm, 4); KSVD2_REQ(Rsq, w);
  RectDesc d;
  int maxn;
  int rc = rect_setup(nmat, m_host, n_host, aoff_host, roff_host, ws, ws_bytes, st, d, maxn);
  if (rc) return rc;
  hipLaunchKernelGGL(k_qrcp<R>, dim3((unsigned)nmat), dim3(kQrcpBlock), 0, st, d, A, tau, perm,
                     Rsq);
  return launch_status("kog_qrcp launch");
}

template <class R>
static int qapply_impl(int64_t nmat, const int32_t *m_host, const int32_t *n_host,
                       const int64_t *aoff_host, const int64_t *roff_host, const R *A,
                       const R *tau, const int32_t *perm, const R *UR, const R *VR, R *U, R *V,
                       void *ws, size_t ws_bytes, hipStream_t st) {
  if (nmat < 0) return fail(KSVD2_EINVAL, "nmat < 0");
  if (nmat == 0) return KSVD2_OK;
  const size_t w = sizeof(R);
  KSVD2_REQ(A, w); KSVD2_REQ(tau, w); KSVD2_REQ(perm, 4); KSVD2_REQ(UR, w); KSVD2_REQ(VR, w);
  KSVD2_REQ(U, w); KSVD2_REQ(V, w);
  RectDesc d;
  int maxn;
  int rc = rect_setup(nmat, m_host, n_host, aoff_host, roff_host, ws, ws_bytes, st, d, maxn);
  if (rc) return rc;
  const int cols = kQapplyBlock >> 6;
  int maxm = 0;
  for (int64_t k = 0; k < nmat; ++k) maxm = m_host[k] > maxm ? m_host[k] : maxm;
  const size_t lds = (size_t)cols * maxm * sizeof(R);
  dim3 grid((unsigned)((maxn + cols - 1) / cols), (unsigned)nmat);
  if (lds <= kQapplyLds)
    hipLaunchKernelGGL((k_qapply<R, true>), grid, dim3(kQapplyBlock), lds, st, d, A, tau, perm,
                       UR, VR, U, V, maxm);
  else
    hipLaunchKernelGGL((k_qapply<R, false>), grid, dim3(kQapplyBlock), 0, st, d, A, tau, perm,
                       UR, VR, U, V, 0);
  return launch_status("kog_qrcp_apply launch");
}

}  // namespace ksvd2

using namespace ksvd2;

extern "C" {

size_t kog_rect_workspace_size(int64_t nmat) {
  return nmat <= 0 ? 256 : rect_layout(nmat).total;
}

int kog_qrcp_batch(int dtype, int64_t nmat, const int32_t *m_host, const int32_t *n_host,
                   const int64_t *aoff_host, const int64_t *roff_host, void *A, void *tau,
                   int32_t *perm, void *Rsq, void *workspace, size_t ws_bytes, void *stream) {
  hipStream_t st = (hipStream_t)stream;
  if (dtype == 1)
    return qrcp_impl<double>(nmat, m_host, n_host, aoff_host, roff_host, (double *)A,
                             (double *)tau, perm, (double *)Rsq, workspace, ws_bytes, st);
  if (dtype == 0)
    return qrcp_impl<float>(nmat, m_host, n_host, aoff_host, roff_host, (float *)A,
                            (float *)tau, perm, (float *)Rsq, workspace, ws_bytes, st);
  return fail(KSVD2_EDTYPE, "dtype must be 0 (f32) or 1 (f64), got %d", dtype);
}

int kog_qrcp_apply(int dtype, int64_t nmat, const int32_t *m_host, const int32_t *n_host,
                   const int64_t *aoff_host, const int64_t *roff_host, const void *A,
                   const void *tau, const int32_t *perm, const void *UR, const void *VR, void *U,
                   void *V, void *workspace, size_t ws_bytes, void *stream) {
  hipStream_t st = (hipStream_t)stream;
  if (dtype == 1)
    return qapply_impl<double>(nmat, m_host, n_host, aoff_host, roff_host, (const double *)A,
                               (const double *)tau, perm, (const double *)UR,
                               (const double *)VR, (double *)U, (double *)V, workspace,
                               ws_bytes, st);
  if (dtype == 0)
    return qapply_impl<float>(nmat, m_host, n_host, aoff_host, roff_host, (const float *)A,
                              (const float *)tau, perm, (const float *)UR, (const float *)VR,
                              (float *)U, (float *)V, workspace, ws_bytes, st);
  return fail(KSVD2_EDTYPE, "dtype must be 0 (f32) or 1 (f64), got %d", dtype);
}

}  // extern "C"
