// Batched two-sided Kogbetliantz iteration (Sect. 1, eq. SVD) over many square
// matrices of possibly different even orders, built on the 2x2 SVD of
// ksvd2_device.hpp.
//
// One parallel step k of a sweep (n/2 disjoint pivots from the round-robin or
// the modified modulus ordering):
//   1. every pivot (i, j) of step k is diagonalised by the 2x2 SVD of
//      [g_ii g_ij; g_ji g_jj] (U_p, sigma, V_p; sigma rounded to W);
//   2. rows i, j of G are rotated by U_p^T, then columns i, j by V_p:
//      x' = fma(a, x, b*y) for every element pair;
//   3. the pivot block becomes diag(sigma_1, sigma_2) exactly;
//   4. columns i, j of U and V are rotated by U_p and V_p.
// A sweep is n - 1 steps; after each sweep the off-diagonal Frobenius norm
// is compared with tol_factor * n * eps * ||G_0||_F.  G is first scaled by
// 2^s_G, s_G = e_nu - 2 - e_G - ceil(lg n) when that is negative (e_G the
// largest exponent of an entry), so that the two-sided updates cannot
// overflow (Sect. 4, on the order-n implementation), and scaled back at the
// end.
//
// Only G feeds the next step's pivots, so step 4 is deferred: the rotations of
// kChunk consecutive steps are kept in a table, and U and V are brought up to
// date once per chunk, a tile of rows at a time in LDS.  Each row of U or V
// receives exactly the same rotations in the same order as with per-step
// updates; deferring changes the memory traffic, not a single bit.  Under both
// cyclic orderings (round-robin is the modified modulus ordering with its
// indices relabeled) the persistent modes also update G two steps per pass
// (the pairs of consecutive steps interlock; see g_fused_pair) and rotate the
// U/V tiles two steps per LDS pass (tile_rotate_pair), again with the same
// operations on every element.
//
// Executions of exactly the same arithmetic:
//   mode 0  plain per-step launches: a pivot kernel and a G kernel per step,
//           a U/V kernel per chunk, a check kernel per sweep, the host polls
//           convergence;
//   mode 1  persistent: one workgroup per matrix runs all its sweeps (step
//           parameters and the U/V tile in LDS, workgroup barriers between
//           phases), one launch per size bucket, no host round trips;
//   mode 2  mode 1 captured once into a hipGraph and replayed.
// The reductions use a fixed order, so the results are bitwise identical.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstring>
#include <map>
#include <mutex>
#include <numeric>
#include <tuple>
#include <vector>

#include "abi_common.hpp"
#include "ksvd2_device.hpp"

namespace ksvd2 {

constexpr int kRed = 256;        // lanes of the fixed-order reductions
constexpr int kMaxOrder = 8192;  // pair indices are stored as int16
constexpr int kChunk = 128;      // default and largest count of steps whose U/V rotations
                                 // are applied together (a power of two)
constexpr int kApplyBlock = 256; // workgroup of the mode-0 U/V kernel
constexpr size_t kApplyLds = 64 * 1024;

struct SweepDesc {
  const int32_t *n;      // order of matrix m
  const int64_t *off;    // element offset of matrix m in G, U, V
  const int64_t *soff;   // offset of matrix m in sigma
  const int64_t *poff;   // sum of n/2 over the matrices before m
  double *fro2;          // ||G_0||_F^2
  int32_t *sweeps;       // sweeps done so far
  int32_t *done;         // converged flag
  int32_t *scale;        // s_G of matrix m (0: not scaled)
  int32_t *nexp;         // t of matrix m: the norms are taken of G 2^-t
  int ord;               // pivot ordering: 0 round-robin, 1 modified modulus
  const int64_t *aoff;   // offset of matrix m in galt
  void *galt;            // a second buffer of G's size (the two-step G updates)
  int chunk;             // steps per U/V update, a power of two in [2, kChunk]
  int16_t *pairs;        // pair table of the chunk's steps (mode 0, dynamic ordering)
};

// Pivot orderings.  Modified modulus (ord = 1; the parallel strategy Sect. 4
// names for the order-n iteration): with m = n - 1 odd, step k pairs the
// indices below m whose sum is k modulo m, and the one index c with 2c = k
// (mod m), which the modulus strategy for odd orders leaves idle, with m.  Slot
// 0 holds (c, m), slot q >= 1 the pair A_q = c + q, B_q = c - q (mod m).  Every
// pair meets once in the m steps of a sweep.
//
// Round-robin (ord = 0; the circle method: index 0 fixed, 1..n-1 rotating by
// one position per step, positions s and n-1-s meeting) is the same
// 1-factorization under a fixed relabeling: with x the modulus label, the
// round-robin index is lambda(x) = 1 + (2x mod m) for x < m and lambda(m) = 0,
// and round-robin step k is modulus step k - 1 (mod m).  (Player 1 + ((s - 1 +
// k) mod m) at position s meets 1 + ((m - 1 - s + k) mod m); halving the
// labels minus one turns their sum 2k - 2 into k - 1.)  So both orderings run
// through the same slot structure, and the two-step passes below serve both:
// only the indices are mapped.  The slots of a step may be numbered in any
// order without changing a bit (disjoint pivots).
__device__ inline int ord_index(int ord, int m, int x) {
  if (ord == 1) return x;
  const int y = 2 * x;
  return x == m ? 0 : 1 + (y >= m ? y - m : y);
}

// the centre c of step k (2c = k' mod m, k' the modulus step)
__device__ inline int mm_center(int n, int k, int ord) {
  const int m = n - 1;
  const int kk = ord == 1 ? k : (k == 0 ? m - 1 : k - 1);
  return (kk & 1) ? (kk + m) >> 1 : kk >> 1;
}

// the indices A and B of slot q of the step with centre c
__device__ inline void mm_ab(int m, int c, int q, int &A, int &B, int ord) {
  int a = c + q, b = c - q;
  a = a >= m ? a - m : a;
  b = b < 0 ? b + m : b;
  A = ord_index(ord, m, q == 0 ? m : a);
  B = ord_index(ord, m, q == 0 ? c : b);
}

// the pivot pair of slot q in step k of the ordering `ord` (0 or 1), i < j
__device__ inline void piv_pair(int ord, int n, int k, int q, int &i, int &j) {
  int A, B;
  mm_ab(n - 1, mm_center(n, k, ord), q, A, B, ord);
  i = A < B ? A : B;
  j = A < B ? B : A;
}

// Dynamic ordering (ord = 2): the pivots of a step are a greedy matching on the
// weights w = fma(x_ij, x_ij, x_ji * x_ji) (binary64, x = G 2^-t with t the norm
// exponent), taken by decreasing weight, equal weights by the smaller index and
// then the larger.  With that strict total order on the pairs, the greedy
// matching is found in rounds of locally dominant pairs: each free index v
// points to the first pair (v, u) among free u; pairs whose two ends point to
// each other are the first at both ends, are taken by the greedy matching, and
// leave the greedy matching of what remains; every round takes at least the
// first remaining pair.  A pointer stays valid while its target is free (the
// candidates only shrink), so only indices whose target was taken scan again.
template <class R>
__device__ inline double dyn_weight(const R *G, int n, int a, int b, double sc) {
  double x = (double)G[a + (int64_t)b * n] * sc, y = (double)G[b + (int64_t)a * n] * sc;
  return fma(x, x, y * y);
}

// pair (w1; a1 < b1) before pair (w2; a2 < b2) in the order of the matching
__device__ inline bool dyn_before(double w1, int a1, int b1, double w2, int a2, int b2) {
  if (w1 != w2) return w1 > w2;
  if (a1 != a2) return a1 < a2;
  return b1 < b2;
}

// The matching of the current G by the whole workgroup; mate and best are n
// entries of LDS each, flag one int of LDS.  The pairs go to spair (i < j) in
// increasing order of i.  Every thread of the block calls it.
template <class R>
__device__ void dyn_match(const R *G, int n, double sc, int16_t *mate, int16_t *best, int *flag,
                          int16_t *spair) {
  for (int v = threadIdx.x; v < n; v += blockDim.x) {
    mate[v] = -1;
    best[v] = -1;
  }
  if (threadIdx.x == 0) *flag = 0;
  __syncthreads();
  for (;;) {
    for (int v = threadIdx.x; v < n; v += blockDim.x) {
      if (mate[v] >= 0) continue;
      int b = best[v];
      if (b >= 0 && mate[b] < 0) continue;
      double bw = 0.0;
      int bu = -1, ba = 0, bb = 0;
      for (int u = 0; u < n; ++u) {
        if (u == v || mate[u] >= 0) continue;
        int a = min(u, v), c = max(u, v);
        double w = dyn_weight(G, n, a, c, sc);
        if (bu < 0 || dyn_before(w, a, c, bw, ba, bb)) {
          bw = w;
          bu = u;
          ba = a;
          bb = c;
        }
      }
      best[v] = (int16_t)bu;
    }
    __syncthreads();
    // each index writes only its own entry: a mutual pair is taken by both ends
    for (int v = threadIdx.x; v < n; v += blockDim.x) {
      if (mate[v] >= 0) continue;
      int u = best[v];
      if (best[u] == v)
        mate[v] = (int16_t)u;
      else
        *flag = 1;
    }
    __syncthreads();
    int more = *flag;
    __syncthreads();
    if (!more) break;
    if (threadIdx.x == 0) *flag = 0;
    __syncthreads();
  }
  // the pairs in increasing order of their smaller index (wave 0)
  if (threadIdx.x < 64) {
    const int lane = threadIdx.x;
    int base = 0;
    for (int v0 = 0; v0 < n; v0 += 64) {
      int v = v0 + lane;
      bool lead = v < n && v < mate[v];
      uint64_t bal = __ballot(lead);
      int pos = base + __popcll(bal & ((1ull << lane) - 1ull));
      if (lead) {
        spair[2 * pos] = (int16_t)v;
        spair[2 * pos + 1] = mate[v];
      }
      base += __popcll(bal);
    }
  }
  __syncthreads();
}

template <class R> struct Piv {
  R u11, u21, u12, u22, v11, v21, v12, v22, s1, s2;
};

template <class R> __device__ inline Piv<R> pivot_svd_of(R gii, R gji, R gij, R gjj) {
  Svd2<R> r = svd2<R>(gii, gji, gij, gjj);
  R du = (r.info & I_DETU) ? (R)-1 : (R)1, dv = (r.info & I_DETV) ? (R)-1 : (R)1;
  Piv<R> p;
  p.u11 = r.cu;
  p.u21 = r.su;
  p.u12 = -du * r.su;
  p.u22 = du * r.cu;
  p.v11 = r.cv;
  p.v21 = r.sv;
  p.v12 = -dv * r.sv;
  p.v22 = dv * r.cv;
  p.s1 = scale2(r.f1, r.e1);
  p.s2 = scale2(r.f2, r.e2);
  return p;
}

template <class R> __device__ inline Piv<R> pivot_svd(const R *G, int n, int i, int j) {
  return pivot_svd_of(G[i + (int64_t)i * n], G[j + (int64_t)i * n], G[i + (int64_t)j * n],
                      G[j + (int64_t)j * n]);
}

template <class R> __device__ inline R lin(R a, R x, R b, R y) { return fma(a, x, b * y); }

// Step tables are stored by component: a slot of np pivots holds the np values
// of u11, then of u21, u12, u22, v11, v21, v12, v22, s1, s2, so that lanes
// reading consecutive pivots read consecutive addresses.
constexpr int kPivComp = 10;
enum { C_U11, C_U21, C_U12, C_U22, C_V11, C_V21, C_V12, C_V22, C_S1, C_S2 };

template <class R> __device__ inline void piv_store(R *slot, int np, int q, const Piv<R> &P) {
  slot[C_U11 * np + q] = P.u11;
  slot[C_U21 * np + q] = P.u21;
  slot[C_U12 * np + q] = P.u12;
  slot[C_U22 * np + q] = P.u22;
  slot[C_V11 * np + q] = P.v11;
  slot[C_V21 * np + q] = P.v21;
  slot[C_V12 * np + q] = P.v12;
  slot[C_V22 * np + q] = P.v22;
  slot[C_S1 * np + q] = P.s1;
  slot[C_S2 * np + q] = P.s2;
}

// ------------------------------------------------------------- the G update
//
// Block (p, q) of step k: rows (i_p, j_p) x columns (i_q, j_q).  Rows first
// (row_i' = u11 row_i + u21 row_j, row_j' = u12 row_i + u22 row_j), then
// columns (col_i' = col_i v11 + col_j v21, col_j' = col_i v12 + col_j v22);
// the diagonal blocks become diag(sigma_1, sigma_2).

// the four elements of a block, by row (i_p or j_p) and column (i_q or j_q)
template <class R> struct Blk {
  R ii, ji, ij, jj;
};

// block (p, q) of a step rotated: a = g(i_p, i_q), b = g(j_p, i_q), c = g(i_p, j_q),
// d = g(j_p, j_q) before it
template <class R>
__device__ inline Blk<R> blk_rot(R u11, R u21, R u12, R u22, R v11, R v21, R v12, R v22, R a,
                                 R b, R c, R d) {
  R a1 = lin(u11, a, u21, b), b1 = lin(u12, a, u22, b);
  R c1 = lin(u11, c, u21, d), d1 = lin(u12, c, u22, d);
  Blk<R> o;
  o.ii = lin(v11, a1, v21, c1);
  o.ij = lin(v12, a1, v22, c1);
  o.ji = lin(v11, b1, v21, d1);
  o.jj = lin(v12, b1, v22, d1);
  return o;
}
template <class R>
__device__ inline Blk<R> blk_rotate(const R *S, int np, int p, int q, R a, R b, R c, R d) {
  return blk_rot(S[C_U11 * np + p], S[C_U21 * np + p], S[C_U12 * np + p], S[C_U22 * np + p],
                 S[C_V11 * np + q], S[C_V21 * np + q], S[C_V12 * np + q], S[C_V22 * np + q], a,
                 b, c, d);
}

template <class R>
__device__ inline void g_block_store(R *G, int n, int ip, int jp, int iq, int jq, const R *S,
                                     int np, int p, int q, R a, R b, R c, R d) {
  Blk<R> o = blk_rotate(S, np, p, q, a, b, c, d);
  R *ci = G + (int64_t)iq * n, *cj = G + (int64_t)jq * n;
  ci[ip] = o.ii;
  cj[ip] = o.ij;
  ci[jp] = o.ji;
  cj[jp] = o.jj;
}

template <class R>
__device__ inline void g_diag_store(R *G, int n, int i, int j, const R *S, int np, int p) {
  G[i + (int64_t)i * n] = S[C_S1 * np + p];
  G[j + (int64_t)j * n] = S[C_S2 * np + p];
  G[i + (int64_t)j * n] = (R)0;
  G[j + (int64_t)i * n] = (R)0;
}

// all np^2 blocks of one step by one workgroup of BS lanes, D blocks per lane
// in flight: the loads are issued without branches (a lane past the end reads
// block (0, 0) and stores nothing), so none of them waits for another.  Reads
// Gin and writes G (the same buffer, or another one of the same layout: every
// element is written).
template <class R, int BS, int D>
__device__ __attribute__((always_inline)) void g_step_block(const R *Gin, R *G, int n, const R *S,
                                                             const int16_t *pr) {
  const int np = n >> 1;
  const int dp = BS % np, dq = BS / np;
  // block w = p + q np, walked with stride BS by carries
  int p = threadIdx.x % np, q = threadIdx.x / np;
  while (q < np) {
    R a[D], b[D], c[D], d[D];
    int ip[D], jp[D], iq[D], jq[D], pp[D], qq[D];
#pragma unroll
    for (int u = 0; u < D; ++u) {
      bool ok = q < np;
      pp[u] = ok ? p : -1;
      qq[u] = ok ? q : 0;
      int ps = ok ? p : 0, qs = ok ? q : 0;
      ip[u] = pr[2 * ps];
      jp[u] = pr[2 * ps + 1];
      iq[u] = pr[2 * qs];
      jq[u] = pr[2 * qs + 1];
      const R *ci = Gin + (int64_t)iq[u] * n, *cj = Gin + (int64_t)jq[u] * n;
      a[u] = ci[ip[u]];
      b[u] = ci[jp[u]];
      c[u] = cj[ip[u]];
      d[u] = cj[jp[u]];
      p += dp;
      q += dq;
      bool carry = p >= np;
      p = carry ? p - np : p;
      q = carry ? q + 1 : q;
    }
#pragma unroll
    for (int u = 0; u < D; ++u) {
      if (pp[u] < 0) continue;
      if (pp[u] == qq[u])
        g_diag_store(G, n, ip[u], jp[u], S, np, pp[u]);
      else
        g_block_store(G, n, ip[u], jp[u], iq[u], jq[u], S, np, pp[u], qq[u], a[u], b[u], c[u],
                      d[u]);
    }
  }
}

// ------------------------------------------------ two steps of G in one pass
//
// Under the modified modulus ordering (m = n - 1, c = c_k with 2c = k mod m),
// slot q >= 1 of step k pairs A_q = c + q with B_q = c - q (mod m), and slot 0
// pairs A_0 = m with B_0 = c.  As 2 c_(k+1) = 2c + 1 (mod m), the pairs of step
// k + 1 are {A_d, B_(d-1)}: slot np - d for d = 1 .. np - 1, and {A_0,
// B_(np-1)} in slot 0.  So block (d, e) of step k + 1 (rows {A_d, B_(d-1)},
// columns {A_e, B_(e-1)}) holds one element of each of the step-k blocks
// (d, e), (d, e-1), (d-1, e) and (d-1, e-1) after step k.  One pass over G
// forms every step-k block and, from four of them, every block of step k + 1:
// G is read once and written once per two steps instead of twice, and every
// element goes through exactly the operations of two separate steps, in the
// same order (the same bits).  The pivots of step k + 1 are formed first, by
// the same element formulas.

// a 2x2 block given by A/B row and A/B column (xAB = element (A row, B column))
// to its i/j form (a = (i, i), b = (j, i), c = (i, j), d = (j, j)); rai: the A
// row is the smaller index of its pair, cai likewise for the columns
template <class R>
__device__ inline void ab_to_ij(bool rai, bool cai, R xAA, R xAB, R xBA, R xBB, R &a, R &b,
                                R &c, R &d) {
  R rAi = cai ? xAA : xAB, rAj = cai ? xAB : xAA;  // row A at columns i, j
  R rBi = cai ? xBA : xBB, rBj = cai ? xBB : xBA;
  a = rai ? rAi : rBi;
  b = rai ? rBi : rAi;
  c = rai ? rAj : rBj;
  d = rai ? rBj : rAj;
}

template <class R> struct Wab {
  R AA, AB, BA, BB;
};

// step-k block (p, q) after step k by A/B row and column (aip, aiq: A is the
// smaller index of slot p, q), from its elements before it (a = (i_p, i_q),
// b = (j_p, i_q), c = (i_p, j_q), d = (j_p, j_q))
template <class R>
__device__ inline Wab<R> blk_after(const R *S, int np, int p, int q, bool aip, bool aiq, R a,
                                   R b, R c, R d) {
  Blk<R> o;
  if (p == q) {  // the pivot block becomes diag(sigma_1, sigma_2)
    o.ii = S[C_S1 * np + p];
    o.jj = S[C_S2 * np + p];
    o.ij = (R)0;
    o.ji = (R)0;
  } else {
    o = blk_rotate(S, np, p, q, a, b, c, d);
  }
  R rAi = aip ? o.ii : o.ji, rAj = aip ? o.ij : o.jj;
  R rBi = aip ? o.ji : o.ii, rBj = aip ? o.jj : o.ij;
  Wab<R> w;
  w.AA = aiq ? rAi : rAj;
  w.AB = aiq ? rAj : rAi;
  w.BA = aiq ? rBi : rBj;
  w.BB = aiq ? rBj : rBi;
  return w;
}

// the pivots of step k + 1 from G before step k and the parameters S1 of step
// k: pair d = {A_d, B_(d-1)} has the diagonal elements sigma of A_d (slot d)
// and of B_(d-1) (slot d - 1), and its off-diagonal elements in the step-k
// blocks (d, d-1) and (d-1, d).  Parameters to S2 (LDS) and slot2 (table).
template <class R, int BS>
__device__ __attribute__((always_inline)) void g_pivots_next(const R *Gin, int n, int k,
                                                              const R *S1, R *S2, R *slot2,
                                                              int ord) {
  const int np = n >> 1, m = n - 1, c = mm_center(n, k, ord);
  for (int dd = threadIdx.x; dd < np; dd += BS) {
    const int dm = dd == 0 ? np - 1 : dd - 1;
    int Ad, Bd, Am, Bm;
    mm_ab(m, c, dd, Ad, Bd, ord);
    mm_ab(m, c, dm, Am, Bm, ord);
    const bool aid = Ad < Bd, aim = Am < Bm;
    const R gAA = aid ? S1[C_S1 * np + dd] : S1[C_S2 * np + dd];
    const R gBB = aim ? S1[C_S2 * np + dm] : S1[C_S1 * np + dm];
    const int id = min(Ad, Bd), jd = max(Ad, Bd), im = min(Am, Bm), jm = max(Am, Bm);
    const R *cim = Gin + (int64_t)im * n, *cjm = Gin + (int64_t)jm * n;
    const R *cid = Gin + (int64_t)id * n, *cjd = Gin + (int64_t)jd * n;
    Wab<R> w1 = blk_after(S1, np, dd, dm, aid, aim, cim[id], cim[jd], cjm[id], cjm[jd]);
    Wab<R> w2 = blk_after(S1, np, dm, dd, aim, aid, cid[im], cid[jm], cjd[im], cjd[jm]);
    const R gAB = w1.AB, gBA = w2.BA;  // (A_d, B_(d-1)) and (B_(d-1), A_d)
    const bool rai = Ad < Bm;
    const R gii = rai ? gAA : gBB, gjj = rai ? gBB : gAA;
    const R gij = rai ? gAB : gBA, gji = rai ? gBA : gAB;
    Piv<R> P = pivot_svd_of(gii, gji, gij, gjj);
    const int q2 = dd == 0 ? 0 : np - dd;
    piv_store(S2, np, q2, P);
    piv_store(slot2, np, q2, P);
  }
}

// Raw buffer access to one matrix: byte offsets as a per-lane part and a
// wave-uniform (column) part; an offset at or past the end (kOff) reads zero
// and stores nothing, without a memory access.  The descriptor's last word
// (kBufWord3) selects 32-bit raw data access on this GPU family; the range is
// the matrix's size in bytes, with no stride.  The base and size are the same
// in every lane; taking them from the first lane says so to the compiler,
// which otherwise wraps every access in a loop over distinct descriptors when
// it cannot prove that (the two G buffers of a pass swap roles every pass).
constexpr int kOff = 0x40000000;
constexpr int kBufWord3 = 0x00020000;
template <class T> __device__ inline T *wave_uniform(T *p) {
  const uint64_t v = reinterpret_cast<uint64_t>(p);
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return reinterpret_cast<T *>(((uint64_t)hi << 32) | lo);
}
template <class R> struct Buf;
template <> struct Buf<double> {
  typedef unsigned int V __attribute__((ext_vector_type(2)));
  __amdgpu_buffer_rsrc_t r;
  __device__ Buf(const double *p, int bytes)
      : r(__builtin_amdgcn_make_buffer_rsrc(wave_uniform(const_cast<double *>(p)), (short)0,
                                            __builtin_amdgcn_readfirstlane(bytes), kBufWord3)) {}
  __device__ double ld(int vo, int so) const {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, vo, so, 0));
  }
  __device__ void st(double x, int vo, int so) const {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V, x), r, vo, so, 0);
  }
};
template <> struct Buf<float> {
  __amdgpu_buffer_rsrc_t r;
  __device__ Buf(const float *p, int bytes)
      : r(__builtin_amdgcn_make_buffer_rsrc(wave_uniform(const_cast<float *>(p)), (short)0,
                                            __builtin_amdgcn_readfirstlane(bytes), kBufWord3)) {}
  __device__ float ld(int vo, int so) const {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, vo, so, 0));
  }
  __device__ void st(float x, int vo, int so) const {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, x), r, vo, so, 0);
  }
};

// lane l receives lane l - 1's value (a wave shift; every lane active)
__device__ inline float lane_up(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x138, 0xf, 0xf, false));
}
__device__ inline double lane_up(double x) {
  int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), 0x138, 0xf, 0xf, false);
  int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), 0x138, 0xf, 0xf, false);
  return __hiloint2double(hi, lo);
}

// Steps k and k + 1 from Gin to G (another buffer: blocks of step k + 1 read
// elements that other lanes write).  A wave takes up to 63 consecutive row
// slots p and a segment of column slots: lane l forms the step-k blocks of
// row slot p = d0 + l - 1 one column slot e after the other, e from e0 - 1
// on; lanes 1.. own the output row pairs p, whose B row (B_(p-1)) the lane
// below formed, and column e's B column (B_(e-1)) comes from the previous
// column slot.  Row and column halos are formed twice (one row slot per 63,
// one column slot per segment).  Loads run kAhead column slots ahead; the
// walk is padded to a multiple of kAhead (the padding re-reads the last
// column and stores nothing), so its body has no branches but the wave-
// uniform one around the stores.  Pivot blocks take their diag(sigma) by
// selection, inactive lanes load and store nothing through the buffer's
// range check.
template <class R, int BS, int kAhead>
__device__ __attribute__((always_inline)) void g_fused_pair(const R *Gin, R *G, int n, int k,
                                                             const R *S1, const R *S2, int ord) {
  constexpr int NW = BS / 64;
  constexpr int W = (int)sizeof(R);
  const int np = n >> 1, m = n - 1, c = mm_center(n, k, ord);
  // the wave index is the same for all lanes of a wave: saying so keeps the
  // column offsets in scalar registers
  const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int rw = (np + 62) / 63;  // row chunks of at most 63 output pairs
  const int lr = (np + rw - 1) / rw;
  const int cs = max(1, min(NW / rw, np / 8));  // column segments
  const int ls = (np + cs - 1) / cs;
  const int cb = n * W;  // bytes per column
  const Buf<R> in(Gin, n * cb), out(G, n * cb);
  for (int u = wv; u < rw * cs; u += NW) {
    const int d0 = (u % rw) * lr, e0 = (u / rw) * ls;
    const int dn = min(lr, np - d0), e1 = min(np, e0 + ls);
    if (dn <= 0 || e0 >= e1) continue;  // the same for the whole wave
    const bool act = lane <= dn, own = act && lane >= 1;
    int p = d0 + lane - 1;
    p = act ? (p < 0 ? p + np : p) : 0;
    int Ap, Bp, Aq, Bq;
    mm_ab(m, c, p, Ap, Bp, ord);
    mm_ab(m, c, p == 0 ? np - 1 : p - 1, Aq, Bq, ord);
    const bool aip = Ap < Bp;
    const int rA = Ap, rB = Bq;  // output row pair p of step k + 1
    const bool rai = rA < rB;
    const int q2r = p == 0 ? 0 : np - p;
    const int vip = act ? min(Ap, Bp) * W : kOff, vjp = act ? max(Ap, Bp) * W : kOff;
    const int vi2 = own ? min(rA, rB) * W : kOff, vj2 = own ? max(rA, rB) * W : kOff;
    // the lane's row parameters: step k, slot p; step k + 1, slot q2r
    const R u11 = S1[C_U11 * np + p], u21 = S1[C_U21 * np + p];
    const R u12 = S1[C_U12 * np + p], u22 = S1[C_U22 * np + p];
    const R s1p = S1[C_S1 * np + p], s2p = S1[C_S2 * np + p];
    const R y11 = S2[C_U11 * np + q2r], y21 = S2[C_U21 * np + q2r];
    const R y12 = S2[C_U12 * np + q2r], y22 = S2[C_U22 * np + q2r];
    const R t1p = S2[C_S1 * np + q2r], t2p = S2[C_S2 * np + q2r];
    const int cnt = e1 - e0 + 1;
    const int nt = (cnt + kAhead - 1) / kAhead * kAhead;
    auto slot_of = [&](int t) {
      int e = e0 - 1 + min(t, cnt - 1);
      return e < 0 ? e + np : e;
    };
    auto load = [&](int t, R *x) {
      int Ae, Be;
      mm_ab(m, c, slot_of(t), Ae, Be, ord);
      const int si = min(Ae, Be) * cb, sj = max(Ae, Be) * cb;
      x[0] = in.ld(vip, si);
      x[1] = in.ld(vjp, si);
      x[2] = in.ld(vip, sj);
      x[3] = in.ld(vjp, sj);
    };
    R f[kAhead][4];
#pragma unroll
    for (int z = 0; z < kAhead; ++z) load(z, f[z]);
    R pAB = (R)0, pBB = (R)0;
    int pB = 0;
    for (int t0 = 0; t0 < nt; t0 += kAhead) {
#pragma unroll
      for (int z = 0; z < kAhead; ++z) {
        const int t = t0 + z;
        const R x0 = f[z][0], x1 = f[z][1], x2 = f[z][2], x3 = f[z][3];
        load(t + kAhead, f[z]);
        const int e = slot_of(t);
        int Ae, Be;
        mm_ab(m, c, e, Ae, Be, ord);
        const bool aie = Ae < Be;
        // step-k block (p, e) after step k, by A/B row and column
        Blk<R> o = blk_rot(u11, u21, u12, u22, S1[C_V11 * np + e], S1[C_V21 * np + e],
                           S1[C_V12 * np + e], S1[C_V22 * np + e], x0, x1, x2, x3);
        const bool dg = p == e;
        const R oii = dg ? s1p : o.ii, ojj = dg ? s2p : o.jj;
        const R oij = dg ? (R)0 : o.ij, oji = dg ? (R)0 : o.ji;
        const R rAi = aip ? oii : oji, rAj = aip ? oij : ojj;
        const R rBi = aip ? oji : oii, rBj = aip ? ojj : oij;
        const R wAA = aie ? rAi : rAj, wAB = aie ? rAj : rAi;
        const R wBA = aie ? rBi : rBj, wBB = aie ? rBj : rBi;
        const R uBA = lane_up(wBA), uBB = lane_up(wBB);
        if (t > 0 && t < cnt) {
          // output block (p, e) of step k + 1: columns A_e and B_(e-1)
          const int cA = Ae, cB = pB;
          const bool cai = cA < cB;
          const int siq = min(cA, cB) * cb, sjq = max(cA, cB) * cb;
          const int q2c = e == 0 ? 0 : np - e;
          R a, b, cc, dd;
          ab_to_ij(rai, cai, wAA, pAB, uBA, pBB, a, b, cc, dd);
          Blk<R> o2 = blk_rot(y11, y21, y12, y22, S2[C_V11 * np + q2c], S2[C_V21 * np + q2c],
                              S2[C_V12 * np + q2c], S2[C_V22 * np + q2c], a, b, cc, dd);
          out.st(dg ? t1p : o2.ii, vi2, siq);
          out.st(dg ? (R)0 : o2.ij, vi2, sjq);
          out.st(dg ? (R)0 : o2.ji, vj2, siq);
          out.st(dg ? t2p : o2.jj, vj2, sjq);
        }
        pAB = wAB;
        pBB = uBB;
        pB = Be;
      }
    }
  }
}

// The same two steps in place, for orders up to 256 (np <= 128 slots): one
// wave holds every row slot (lane l the S consecutive slots l S .. l S + S - 1;
// the B row of a lane's first output pair comes from the lane before it, that
// of lane 0 from the last slot np - 1), and the waves split the column slots
// into segments.  A wave's loads then only read columns that no other wave
// writes, and it writes a column only after its own last read of it, except
// for the boundary column slot between two segments (the last of one, read
// before the next one's first output pair writes its B column; the pre-step
// of the next, whose A column the first writes): both waves take that slot
// from a copy in LDS made before the pass.  kAhead S = 4 blocks are loaded
// ahead per lane.
struct FusedGeo {
  int cs, ls;  // column segments and slots per segment
};
__device__ inline FusedGeo fused_geo(int n, int nw, int snap_elems) {
  const int np = n >> 1;
  FusedGeo g;
  g.cs = max(1, min(min(nw, max(1, np / 4)), snap_elems / (2 * n)));
  g.ls = (np + g.cs - 1) / g.cs;
  g.cs = (np + g.ls - 1) / g.ls;
  return g;
}

// columns A and B of each boundary slot (the pre-step slot of each segment)
template <class R, int BS>
__device__ __attribute__((always_inline)) void g_fused_snapshot(const R *G, int n, int k,
                                                                 FusedGeo g, R *snap, int ord) {
  const int np = n >> 1, m = n - 1, c = mm_center(n, k, ord);
  for (int x = threadIdx.x; x < g.cs * 2 * n; x += BS) {
    const int sg = x / (2 * n), r = x - sg * 2 * n, side = r / n, row = r - side * n;
    int b = sg * g.ls - 1;
    b = b < 0 ? b + np : b;
    int A, B;
    mm_ab(m, c, b, A, B, ord);
    snap[x] = G[row + (int64_t)(side ? B : A) * n];
  }
}

template <class R, int BS, int S>
__device__ __attribute__((always_inline)) void g_fused_inplace(R *G, int n, int k, const R *S1,
                                                                const R *S2, FusedGeo g,
                                                                const R *snap, int ord) {
  constexpr int W = (int)sizeof(R);
  constexpr int kAhead = 4 / S;
  const int np = n >> 1, m = n - 1, c = mm_center(n, k, ord);
  const int lane = threadIdx.x & 63, sg = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (sg >= g.cs) return;  // this wave has no segment (the same for all its lanes)
  const int L = (np + S - 1) / S;  // lanes holding slots
  const int cb = n * W;
  const Buf<R> buf(G, n * cb);
  const int e0 = sg * g.ls, e1 = min(np, e0 + g.ls), cnt = e1 - e0 + 1;
  const int sgn = sg + 1 == g.cs ? 0 : sg + 1;
  const int pred = lane == 0 ? L - 1 : lane - 1;
  const int slast = lane == L - 1 ? np - 1 - (L - 1) * S : S - 1;
  int pp[S], vip[S], vjp[S], vi2[S], vj2[S], sip[S], sjp[S], q2r[S];
  bool aip[S], rai[S], val[S];
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const int p = lane * S + s;
    val[s] = lane < L && p < np;
    pp[s] = val[s] ? p : 0;
    int Ap, Bp, Aq, Bq;
    mm_ab(m, c, pp[s], Ap, Bp, ord);
    mm_ab(m, c, pp[s] == 0 ? np - 1 : pp[s] - 1, Aq, Bq, ord);
    aip[s] = Ap < Bp;
    rai[s] = Ap < Bq;  // output pair p: rows A_p and B_(p-1)
    sip[s] = min(Ap, Bp);
    sjp[s] = max(Ap, Bp);
    vip[s] = val[s] ? sip[s] * W : kOff;
    vjp[s] = val[s] ? sjp[s] * W : kOff;
    vi2[s] = val[s] ? min(Ap, Bq) * W : kOff;
    vj2[s] = val[s] ? max(Ap, Bq) * W : kOff;
    q2r[s] = pp[s] == 0 ? 0 : np - pp[s];
  }
  const int nt = (cnt + kAhead - 1) / kAhead * kAhead;
  auto slot_of = [&](int t) {
    int e = e0 - 1 + min(t, cnt - 1);
    return e < 0 ? e + np : e;
  };
  // the blocks of column slot t (nothing is read for the boundary slots)
  auto load = [&](int t, R (*x)[4]) {
    int Ae, Be;
    mm_ab(m, c, slot_of(t), Ae, Be, ord);
    const bool edge = t == 0 || t >= cnt - 1;
    const int si = min(Ae, Be) * cb, sj = max(Ae, Be) * cb;
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const int oi = edge ? kOff : vip[s], oj = edge ? kOff : vjp[s];
      x[s][0] = buf.ld(oi, si);
      x[s][1] = buf.ld(oj, si);
      x[s][2] = buf.ld(oi, sj);
      x[s][3] = buf.ld(oj, sj);
    }
  };
  R f[kAhead][S][4];
#pragma unroll
  for (int z = 0; z < kAhead; ++z) load(z, f[z]);
  R pAB[S], pBB[S], pBBu = (R)0;
#pragma unroll
  for (int s = 0; s < S; ++s) pAB[s] = pBB[s] = (R)0;
  int pB = 0;
  for (int t0 = 0; t0 < nt; t0 += kAhead) {
#pragma unroll
    for (int z = 0; z < kAhead; ++z) {
      const int t = t0 + z;
      R x[S][4];
#pragma unroll
      for (int s = 0; s < S; ++s)
#pragma unroll
        for (int q = 0; q < 4; ++q) x[s][q] = f[z][s][q];
      load(t + kAhead, f[z]);
      const int e = slot_of(t);
      int Ae, Be;
      mm_ab(m, c, e, Ae, Be, ord);
      const bool aie = Ae < Be;
      if (t == 0 || t == cnt - 1) {  // a boundary slot: from the copy
        const R *sa = snap + (size_t)(t == 0 ? sg : sgn) * 2 * n, *sb = sa + n;
        const R *ci = aie ? sa : sb, *cj = aie ? sb : sa;
#pragma unroll
        for (int s = 0; s < S; ++s) {
          x[s][0] = ci[sip[s]];
          x[s][1] = ci[sjp[s]];
          x[s][2] = cj[sip[s]];
          x[s][3] = cj[sjp[s]];
        }
      }
      const R v11 = S1[C_V11 * np + e], v21 = S1[C_V21 * np + e];
      const R v12 = S1[C_V12 * np + e], v22 = S1[C_V22 * np + e];
      R wAA[S], wAB[S], wBA[S], wBB[S];
#pragma unroll
      for (int s = 0; s < S; ++s) {
        const int p = pp[s];
        Blk<R> o = blk_rot(S1[C_U11 * np + p], S1[C_U21 * np + p], S1[C_U12 * np + p],
                           S1[C_U22 * np + p], v11, v21, v12, v22, x[s][0], x[s][1], x[s][2],
                           x[s][3]);
        const bool dg = p == e;
        const R oii = dg ? S1[C_S1 * np + p] : o.ii, ojj = dg ? S1[C_S2 * np + p] : o.jj;
        const R oij = dg ? (R)0 : o.ij, oji = dg ? (R)0 : o.ji;
        const R rAi = aip[s] ? oii : oji, rAj = aip[s] ? oij : ojj;
        const R rBi = aip[s] ? oji : oii, rBj = aip[s] ? ojj : oij;
        wAA[s] = aie ? rAi : rAj;
        wAB[s] = aie ? rAj : rAi;
        wBA[s] = aie ? rBi : rBj;
        wBB[s] = aie ? rBj : rBi;
      }
      // the B row of the lane's first output pair: the previous lane's last slot
      R lBA = wBA[0], lBB = wBB[0];
#pragma unroll
      for (int s = 1; s < S; ++s) {
        lBA = slast == s ? wBA[s] : lBA;
        lBB = slast == s ? wBB[s] : lBB;
      }
      const R uBA = __shfl(lBA, pred), uBB = __shfl(lBB, pred);
      if (t > 0 && t < cnt) {
        // output blocks (p, e) of step k + 1: columns A_e and B_(e-1)
        const int cA = Ae, cB = pB;
        const bool cai = cA < cB;
        const int siq = min(cA, cB) * cb, sjq = max(cA, cB) * cb;
        const int q2c = e == 0 ? 0 : np - e;
        const R y11 = S2[C_V11 * np + q2c], y21 = S2[C_V21 * np + q2c];
        const R y12 = S2[C_V12 * np + q2c], y22 = S2[C_V22 * np + q2c];
#pragma unroll
        for (int s = 0; s < S; ++s) {
          const R bBA = s == 0 ? uBA : wBA[s > 0 ? s - 1 : 0];
          const R bBB = s == 0 ? pBBu : pBB[s > 0 ? s - 1 : 0];
          R a, b, cc, dd;
          ab_to_ij(rai[s], cai, wAA[s], pAB[s], bBA, bBB, a, b, cc, dd);
          const int q = q2r[s];
          Blk<R> o2 = blk_rot(S2[C_U11 * np + q], S2[C_U21 * np + q], S2[C_U12 * np + q],
                              S2[C_U22 * np + q], y11, y21, y12, y22, a, b, cc, dd);
          const bool dg = pp[s] == e;
          buf.st(dg ? S2[C_S1 * np + q] : o2.ii, vi2[s], siq);
          buf.st(dg ? (R)0 : o2.ij, vi2[s], sjq);
          buf.st(dg ? (R)0 : o2.ji, vj2[s], siq);
          buf.st(dg ? S2[C_S2 * np + q] : o2.jj, vj2[s], sjq);
        }
      }
#pragma unroll
      for (int s = 0; s < S; ++s) {
        pAB[s] = wAB[s];
        pBB[s] = wBB[s];
      }
      pBBu = uBB;
      pB = Be;
    }
  }
}

// ------------------------------------------------------------ the U/V update
//
// Rows [r0, r0 + nr) of M (U or V, column-major n x n) are copied into an LDS
// tile T (row-major, row stride n + 1), rotated by the pivots of steps
// k0..k1 (whose parameters are in `tab`, slot k % kChunk, np per slot), and
// copied back.  Each wave owns whole rows of the tile (rows w, w + nw, ...),
// its lanes split a step's pivots, so a step only needs the wave's own
// preceding LDS writes: waves never wait for each other inside a chunk.

// element e = r + c nr of the tile, walked with stride blockDim.x (one
// division per thread, then carries), D elements per lane in flight; the
// loads carry no branches (a lane past the end reads element (0, 0)), only
// the stores are predicated
template <class R, bool kLoad, int D>
__device__ void tile_copy(R *T, R *M, int n, int r0, int nr) {
  const int ldt = n + 1;
  const int bs = blockDim.x, dr = bs % nr, dc = bs / nr;
  int r = threadIdx.x % nr, c = threadIdx.x / nr;
  while (c < n) {
    R v[D];
    int lr[D], lc[D];
#pragma unroll
    for (int u = 0; u < D; ++u) {
      bool ok = c < n;
      lr[u] = ok ? r : -1;
      lc[u] = ok ? c : 0;
      int rs = ok ? r : 0;
      v[u] = kLoad ? M[r0 + rs + (int64_t)lc[u] * n] : T[rs * ldt + lc[u]];
      r += dr;
      c += dc;
      bool carry = r >= nr;
      r = carry ? r - nr : r;
      c = carry ? c + 1 : c;
    }
#pragma unroll
    for (int u = 0; u < D; ++u) {
      if (lr[u] < 0) continue;
      if (kLoad)
        T[lr[u] * ldt + lc[u]] = v[u];
      else
        M[r0 + lr[u] + (int64_t)lc[u] * n] = v[u];
    }
  }
}
// D: 8 elements in flight per lane for small workgroups, 4 for 1024 lanes
// (16 waves per CU already overlap their loads, and 128 registers is the cap)
template <class R, int D = 8> __device__ void tile_load(R *T, const R *M, int n, int r0, int nr) {
  tile_copy<R, true, D>(T, const_cast<R *>(M), n, r0, nr);
}
template <class R, int D = 8> __device__ void tile_store(const R *T, R *M, int n, int r0, int nr) {
  tile_copy<R, false, D>(const_cast<R *>(T), M, n, r0, nr);
}

// NG of the lane's pivots (q = q0 + 64 u, u < NG) per pass; a slot past the
// last pivot rotates the padding column n of the tile (never copied back), so
// the loop body has no branches
template <class R, int NG>
__device__ __attribute__((always_inline)) void tile_rotate_ng(R *T, int n, int nr, int k0, int k1,
                                                               const R *tab, bool isv, int ord,
                                                               int cm, const int16_t *ptab) {
  const int ldt = n + 1;
  const int np = n >> 1;
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int k = k0; k <= k1; ++k) {
    const R *S = tab + (size_t)(k & cm) * kPivComp * np + (isv ? C_V11 : C_U11) * np;
    for (int q0 = lane; q0 < np; q0 += 64 * NG) {
      R e1[NG], e2[NG], e3[NG], e4[NG];
      int ii[NG], jj[NG];
#pragma unroll
      for (int u = 0; u < NG; ++u) {
        int q = q0 + 64 * u;
        bool ok = q < np;
        int qs = ok ? q : 0;
        int i, j;
        if (ord == 2) {
          const int16_t *pp = ptab + 2 * ((size_t)(k & cm) * np + qs);
          i = pp[0];
          j = pp[1];
        } else {
          piv_pair(ord, n, k, qs, i, j);
        }
        ii[u] = ok ? i : n;
        jj[u] = ok ? j : n;
        e1[u] = S[qs];           // u11 or v11
        e2[u] = S[np + qs];      // u21 or v21
        e3[u] = S[2 * np + qs];  // u12 or v12
        e4[u] = S[3 * np + qs];  // u22 or v22
      }
      for (int r = wv; r < nr; r += nw) {
        R *row = T + r * ldt;
        R x[NG], y[NG];
#pragma unroll
        for (int u = 0; u < NG; ++u) {
          x[u] = row[ii[u]];
          y[u] = row[jj[u]];
        }
#pragma unroll
        for (int u = 0; u < NG; ++u) {
          row[ii[u]] = lin(e1[u], x[u], e2[u], y[u]);
          row[jj[u]] = lin(e3[u], x[u], e4[u], y[u]);
        }
      }
    }
    // the next step reads what other lanes of this wave wrote in this one
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
}

// wave rotation by one lane (lane l receives lane l - 1's value, lane 0 lane
// 63's) and a read of one lane's value; every lane active (every lane has a
// source, so no previous value of the destination is kept)
__device__ inline float lane_ror(float x) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), 0x13c, 0xf, 0xf, true));
}
__device__ inline double lane_ror(double x) {
  int lo = __builtin_amdgcn_mov_dpp(__double2loint(x), 0x13c, 0xf, 0xf, true);
  int hi = __builtin_amdgcn_mov_dpp(__double2hiint(x), 0x13c, 0xf, 0xf, true);
  return __hiloint2double(hi, lo);
}
__device__ inline float lane_read(float x, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), l));
}
__device__ inline double lane_read(double x, int l) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(x), l),
                          __builtin_amdgcn_readlane(__double2loint(x), l));
}

// Steps k and k + 1 of the modified modulus ordering on the wave's rows of the
// tile in one pass (the chain of the two-step G update, in one dimension):
// lane l holds the slots l + 64 s (s < S); per row it reads the two elements
// of each of its step-k pairs, rotates them, forms its step-(k+1) pairs
// {A_p, B_(p-1)} (B_(p-1) from the lane before it, or for lane 0 from lane 63's
// previous slot, or from the last slot np - 1) and writes them: each element
// is read and written once per two steps.  Slots past np use the padding
// column n, which is never copied back.
template <class R, int S>
__device__ __attribute__((always_inline)) void tile_rotate_pair(R *T, int n, int nr, int k,
                                                                 const R *tab, bool isv, int cm,
                                                                 int ord) {
  const int ldt = n + 1, np = n >> 1, m = n - 1, c = mm_center(n, k, ord);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int comp = isv ? C_V11 : C_U11;
  const R *S1 = tab + (size_t)(k & cm) * kPivComp * np + comp * np;
  const R *S2 = tab + (size_t)((k + 1) & cm) * kPivComp * np + comp * np;
  const int wl = (np - 1) & 63, ws = (np - 1) >> 6;  // lane and slot of slot np - 1
  int ia[S], ib[S], i2[S], j2[S];
  bool rai[S];
  R pA1[S], pA2[S], pB1[S], pB2[S], b11[S], b21[S], b12[S], b22[S];
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const int p = lane + 64 * s;
    const bool ok = p < np;
    const int ps = ok ? p : 0;
    int A, B, Aq, Bq;
    mm_ab(m, c, ps, A, B, ord);
    mm_ab(m, c, ps == 0 ? np - 1 : ps - 1, Aq, Bq, ord);
    const bool aip = A < B;
    rai[s] = A < Bq;
    ia[s] = ok ? min(A, B) : n;  // the step-k pair (i, j) of slot p
    ib[s] = ok ? max(A, B) : n;
    i2[s] = ok ? min(A, Bq) : n;
    j2[s] = ok ? max(A, Bq) : n;
    const int q2 = ps == 0 ? 0 : np - ps;
    // step k: row A of the pair takes the rotation's first output when A < B,
    // else its second (choosing the coefficients once per pass is the same
    // operation, on the same operands, as choosing between the two outputs)
    const R a11 = S1[ps], a21 = S1[np + ps], a12 = S1[2 * np + ps], a22 = S1[3 * np + ps];
    pA1[s] = aip ? a11 : a12;
    pA2[s] = aip ? a21 : a22;
    pB1[s] = aip ? a12 : a11;
    pB2[s] = aip ? a22 : a21;
    b11[s] = S2[q2];
    b21[s] = S2[np + q2];
    b12[s] = S2[2 * np + q2];
    b22[s] = S2[3 * np + q2];
  }
  for (int r = wv; r < nr; r += nw) {
    R *row = T + r * ldt;
    R xa[S], xb[S];
#pragma unroll
    for (int s = 0; s < S; ++s) {
      xa[s] = row[ia[s]];
      xb[s] = row[ib[s]];
    }
    R nA[S], nB[S];
#pragma unroll
    for (int s = 0; s < S; ++s) {
      nA[s] = lin(pA1[s], xa[s], pA2[s], xb[s]);
      nB[s] = lin(pB1[s], xa[s], pB2[s], xb[s]);
    }
    // the B element of slot np - 1 (lane wl, slot ws) for lane 0's first pair
    R wsel = nB[0];
#pragma unroll
    for (int s = 1; s < S; ++s) wsel = ws == s ? nB[s] : wsel;
    const R wrap = lane_read(wsel, wl);
#pragma unroll
    for (int s = 0; s < S; ++s) {
      // lane 63 passes its previous slot to lane 0 of the next slot
      const R give = (s > 0 && lane == 63) ? nB[s > 0 ? s - 1 : 0] : nB[s];
      const R got = lane_ror(give);
      const R bv = (s == 0 && lane == 0) ? wrap : got;
      const R xi = rai[s] ? nA[s] : bv, xj = rai[s] ? bv : nA[s];
      row[i2[s]] = lin(b11[s], xi, b21[s], xj);
      row[j2[s]] = lin(b12[s], xi, b22[s], xj);
    }
  }
}

// PS: take consecutive steps of the modified modulus ordering in pairs with up
// to PS slots per lane (0: never; 2: orders up to 256; 4: up to 512), as the
// register budget of the calling kernel allows.  The rotations are inlined
// into their kernels, whose compiler then knows the tile is in LDS (an
// outlined copy would reach it through generic addresses).
template <class R, int PS>
__device__ __attribute__((always_inline)) void tile_rotate(R *T, int n, int nr, int k0, int k1,
                                                            const R *tab, bool isv, int ord,
                                                            int cm, const int16_t *ptab) {
  if ((int)(threadIdx.x >> 6) >= nr) return;  // more waves than rows: this wave has none
  const int np = n >> 1;
  if (PS > 0 && ord != 2 && n >= 4 && np <= 64 * PS) {
    // consecutive steps in pairs (the rows of a wave are its own: a wave
    // barrier orders one pass after the previous)
    int k = k0;
    for (; k + 1 <= k1; k += 2) {
      if (np <= 64)
        tile_rotate_pair<R, 1>(T, n, nr, k, tab, isv, cm, ord);
      else if (PS < 4 || np <= 128)
        tile_rotate_pair<R, 2>(T, n, nr, k, tab, isv, cm, ord);
      else
        tile_rotate_pair<R, (PS < 4 ? 2 : 4)>(T, n, nr, k, tab, isv, cm, ord);
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    if (k <= k1) {
      if (np <= 64)
        tile_rotate_ng<R, 1>(T, n, nr, k, k, tab, isv, ord, cm, ptab);
      else if (PS < 4 || np <= 128 || sizeof(R) == 8)
        tile_rotate_ng<R, 2>(T, n, nr, k, k, tab, isv, ord, cm, ptab);
      else
        tile_rotate_ng<R, (PS < 4 ? 2 : 4)>(T, n, nr, k, k, tab, isv, ord, cm, ptab);
    }
    return;
  }
  // binary32 lanes take up to four pivots per pass when there are more than 128
  // (one round of parameter loads per step instead of two); binary64 stays at two,
  // whose registers the 1,024-lane kernels already need for their other phases
  if (np <= 64)
    tile_rotate_ng<R, 1>(T, n, nr, k0, k1, tab, isv, ord, cm, ptab);
  else if (np <= 128 || sizeof(R) == 8)
    tile_rotate_ng<R, 2>(T, n, nr, k0, k1, tab, isv, ord, cm, ptab);
  else
    tile_rotate_ng<R, 4>(T, n, nr, k0, k1, tab, isv, ord, cm, ptab);
}

// Fixed-order sum of squares (in binary64) of G's entries (or of its off-
// diagonal ones): lane t < 256 sums rows t, t+256, ... of every column in
// column order; then a fixed halving tree.  Every thread of the block calls it.
// The entries are multiplied by sc = 2^-t (t the largest exponent of G_0
// after the global scaling), so no square overflows; the stopping test
// compares two such sums, so the factor cancels.
template <class R>
__device__ double block_sumsq(const R *G, int n, bool offdiag, double *red, double sc) {
  int t = threadIdx.x;
  if (t < kRed) {
    double acc = 0.0;
    for (int c = 0; c < n; ++c) {
      const R *col = G + (int64_t)c * n;
      for (int r = t; r < n; r += kRed) {
        if (offdiag && r == c) continue;
        double x = (double)col[r] * sc;
        acc = fma(x, x, acc);
      }
    }
    red[t] = acc;
  }
  __syncthreads();
  for (int s = kRed / 2; s > 0; s >>= 1) {
    if (t < s) red[t] += red[t + s];
    __syncthreads();
  }
  double v = red[0];
  __syncthreads();
  return v;
}

// The largest exponent of a non-zero entry (INT_MIN for a zero matrix); every
// thread of the block (a multiple of kRed lanes) calls it: the block folds into
// kRed slots one group of kRed lanes at a time, then a halving tree.  This and
// scale_matrix run once per matrix and stay out of line, so they do not add to
// the persistent kernel's registers.
template <class R>
__device__ __attribute__((noinline)) int max_exponent(const R *G, int n, double *red) {
  int *ired = reinterpret_cast<int *>(red);
  int64_t tot = (int64_t)n * n;
  int eg = INT_MIN;
  for (int64_t e = threadIdx.x; e < tot; e += blockDim.x)
    if (G[e] != (R)0) eg = max(eg, ilog2(G[e]));
  const int t = threadIdx.x, groups = blockDim.x / kRed;
  for (int g = 0; g < groups; ++g) {
    if (t / kRed == g) ired[t % kRed] = (g == 0) ? eg : max(ired[t % kRed], eg);
    __syncthreads();
  }
  for (int st = kRed / 2; st > 0; st >>= 1) {
    if (t < st) ired[t] = max(ired[t], ired[t + st]);
    __syncthreads();
  }
  int emax = ired[0];
  __syncthreads();
  return emax;
}

template <class R> __device__ __attribute__((noinline)) void scale_matrix(R *G, int n, int s) {
  int64_t tot = (int64_t)n * n;
  for (int64_t e = threadIdx.x; e < tot; e += blockDim.x) G[e] = scale2(G[e], s);
}

// identity U, V (unless continuing), the global scaling of G: s_G = e_nu - 2 -
// e_G - ceil(lg n) when negative (returned in sg), the exponent t of the norm
// factor (returned in nt), and ||G_0 2^-t||_F^2 of the scaled G
template <class R>
__device__ double init_matrix(R *G, R *U, R *V, int n, bool accumulate, double *red, int &sg,
                              int &nt) {
  if (!accumulate) {
    int64_t tot = (int64_t)n * n;
    for (int64_t e = threadIdx.x; e < tot; e += blockDim.x) {
      int r = (int)(e % n), c = (int)(e / n);
      R v = (r == c) ? (R)1 : (R)0;
      U[e] = v;
      V[e] = v;
    }
  }
  int emax = __builtin_amdgcn_readfirstlane(max_exponent(G, n, red));  // uniform: scalar
  int lgn = 32 - __clz(n - 1);                                          // ceil(lg n), n >= 2
  sg = (emax == INT_MIN) ? 0 : min(0, Lim<R>::e_nu - 2 - emax - lgn);
  nt = (emax == INT_MIN) ? 0 : emax + sg;
  if (sg < 0) {
    scale_matrix(G, n, sg);
    __syncthreads();
  }
  return block_sumsq(G, n, false, red, ldexp(1.0, -nt));
}

__device__ inline bool converged(double off2, double fro2, int n, double tolf, double eps) {
  if (tolf < 0.0) return false;
  double tol = tolf * (double)n * eps;
  return off2 <= tol * tol * fro2;
}

// undo the global scaling, then the singular values off the diagonal
template <class R>
__device__ void finish_matrix(R *G, int n, int sg, R *sig, int32_t *sweeps_out, int sweeps,
                              bool conv) {
  if (sg < 0) {
    scale_matrix(G, n, -sg);
    __syncthreads();
  }
  if (sig)
    for (int i = threadIdx.x; i < n; i += blockDim.x) sig[i] = G[i + (int64_t)i * n];
  if (threadIdx.x == 0 && sweeps_out) *sweeps_out = conv ? sweeps : -sweeps;
}

// the first step of the chunk (of cm + 1 steps) that ends with step k
__device__ inline int chunk_begin(int k, int cm) { return k - (k & cm); }

// ----------------------------------------------------------- mode 0 kernels

template <class R>
__global__ __launch_bounds__(kRed) void k_sw_init(SweepDesc d, R *G, R *U, R *V,
                                                  int accumulate) {
  __shared__ double red[kRed];
  int m = blockIdx.x;
  int64_t o = d.off[m];
  int sg, nt;
  double f2 = init_matrix(G + o, U + o, V + o, d.n[m], accumulate != 0, red, sg, nt);
  if (threadIdx.x == 0) {
    d.fro2[m] = f2;
    d.sweeps[m] = 0;
    d.done[m] = 0;
    d.scale[m] = sg;
    d.nexp[m] = nt;
  }
}

// the dynamic ordering's pairs of step k (one workgroup per matrix) into the
// pair table; LDS: the matching's two index arrays of the largest order
template <class R>
__global__ __launch_bounds__(kRed) void k_sw_match(SweepDesc d, const R *G, int16_t *pairs,
                                                   int k) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int flag;
  int m = blockIdx.x;
  int n = d.n[m];
  if (k >= n - 1 || d.done[m]) return;  // uniform over the block
  int np = n >> 1;
  int16_t *mate = reinterpret_cast<int16_t *>(smem), *best = mate + n;
  int64_t slot = d.chunk * d.poff[m] + (int64_t)(k & (d.chunk - 1)) * np;
  dyn_match(G + d.off[m], n, ldexp(1.0, -d.nexp[m]), mate, best, &flag, pairs + 2 * slot);
}

template <class R>
__global__ __launch_bounds__(kBlock) void k_sw_pivots(SweepDesc d, const R *G, R *par,
                                                      int16_t *pairs, int k) {
  int m = blockIdx.y;
  int n = d.n[m];
  int np = n >> 1;
  int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= np || k >= n - 1 || d.done[m]) return;
  int i, j;
  int64_t slot = d.chunk * d.poff[m] + (int64_t)(k & (d.chunk - 1)) * np;
  if (d.ord == 2) {  // written by k_sw_match
    i = pairs[2 * (slot + q)];
    j = pairs[2 * (slot + q) + 1];
  } else {
    piv_pair(d.ord, n, k, q, i, j);
    pairs[2 * (slot + q)] = (int16_t)i;
    pairs[2 * (slot + q) + 1] = (int16_t)j;
  }
  piv_store(par + slot * kPivComp, np, q, pivot_svd(G + d.off[m], n, i, j));
}

template <class R>
__global__ __launch_bounds__(kBlock) void k_sw_update(SweepDesc d, R *G, const R *par,
                                                      const int16_t *pairs, int k) {
  int m = blockIdx.y;
  int n = d.n[m];
  if (k >= n - 1 || d.done[m]) return;
  int np = n >> 1;
  int w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= np * np) return;
  int64_t slot = d.chunk * d.poff[m] + (int64_t)(k & (d.chunk - 1)) * np;
  const int16_t *pt = pairs + 2 * slot;
  const R *S = par + slot * kPivComp;
  R *Gm = G + d.off[m];
  int p = w % np, q = w / np;
  int ip = pt[2 * p], jp = pt[2 * p + 1];
  if (p == q) {
    g_diag_store(Gm, n, ip, jp, S, np, p);
    return;
  }
  int iq = pt[2 * q], jq = pt[2 * q + 1];
  const R *ci = Gm + (int64_t)iq * n, *cj = Gm + (int64_t)jq * n;
  R a = ci[ip], b = ci[jp], c = cj[ip], dd = cj[jp];
  g_block_store(Gm, n, ip, jp, iq, jq, S, np, p, q, a, b, c, dd);
}

// U/V of the chunk that ends at global step k (blockIdx.y: 0 = U, 1 = V;
// blockIdx.x: the row tile); matrices whose last step came earlier were
// brought up to date at their own last chunk.
template <class R>
__global__ __launch_bounds__(kApplyBlock) void k_sw_apply(SweepDesc d, R *U, R *V,
                                                          const R *par, int k,
                                                          int tile_elems) {
  extern __shared__ __align__(16) unsigned char smem[];
  R *T = reinterpret_cast<R *>(smem);
  int m = blockIdx.z;
  int n = d.n[m];
  if (d.done[m]) return;
  int k0 = chunk_begin(k, d.chunk - 1), k1 = min(k, n - 2);
  if (k0 > k1) return;
  int rows = min(n, tile_elems / (n + 1));
  int r0 = blockIdx.x * rows;
  if (r0 >= n) return;
  int nr = min(rows, n - r0);
  R *M = (blockIdx.y ? V : U) + d.off[m];
  tile_load(T, M, n, r0, nr);
  __syncthreads();
  tile_rotate<R, 0>(T, n, nr, k0, k1, par + d.chunk * d.poff[m] * kPivComp, blockIdx.y != 0,
                        d.ord, d.chunk - 1, d.pairs + 2 * d.chunk * d.poff[m]);
  __syncthreads();
  tile_store(T, M, n, r0, nr);
}

template <class R>
__global__ __launch_bounds__(kRed) void k_sw_check(SweepDesc d, const R *G, double tolf) {
  __shared__ double red[kRed];
  int m = blockIdx.x;
  if (d.done[m]) return;  // uniform over the block
  int n = d.n[m];
  double off2 = block_sumsq(G + d.off[m], n, true, red, ldexp(1.0, -d.nexp[m]));
  if (threadIdx.x == 0) {
    d.sweeps[m] += 1;
    if (converged(off2, d.fro2[m], n, tolf, (double)Lim<R>::eps())) d.done[m] = 1;
  }
}

template <class R>
__global__ __launch_bounds__(kRed) void k_sw_finish(SweepDesc d, R *G, R *sigma,
                                                    int32_t *sweeps_out) {
  int m = blockIdx.x;
  finish_matrix(G + d.off[m], d.n[m], d.scale[m], sigma ? sigma + d.soff[m] : nullptr,
                sweeps_out ? sweeps_out + m : nullptr, d.sweeps[m], d.done[m] != 0);
}

// ------------------------------------------------------- mode 1: persistent
//
// One workgroup per matrix (the launch covers the matrices listed in `mats`,
// longest first).  LDS holds the reduction buffer, the pivot parameters of
// one or two steps and the pair table, and the U/V row tile (which during a
// U/V update also spreads over the parameters and the pair table); G stays in
// global memory (two steps at a time go from G to a second buffer in the
// workspace and back); the chunk's rotation table is in the workspace.

// two: LDS holds the parameters of two steps, for the two-step passes (orders
// whose two steps' parameters leave no room for 16 U/V tile rows go one step
// per pass, which keeps room for a tile row up to the largest orders)
// the in-place two-step pass: orders up to 256 in workgroups of up to 512 lanes
// (their registers hold that path), with the boundary columns in the tile
__host__ __device__ inline bool uses_inplace(int bs, int n, int tile_elems) {
  return bs <= 512 && (n >> 1) <= 128 && tile_elems >= 2 * n;
}

template <class R> __host__ __device__ inline size_t persistent_fixed_lds(int maxn, bool two) {
  size_t b = kRed * sizeof(double) + (two ? 2 : 1) * (size_t)(maxn / 2) * kPivComp * sizeof(R) +
             (size_t)maxn * 2;
  return (b + 15) & ~(size_t)15;
}

// PS: pair slots per lane of the U/V rotations (see tile_rotate); the host takes
// 4 only for launches with orders above 256, so that the kernels of smaller
// orders keep the register allocation of 2
template <class R, int BS, int PS>
__global__ __launch_bounds__(BS) void k_sw_persistent(SweepDesc d, const int32_t *mats, R *G,
                                                      R *U, R *V, R *par, R *sigma,
                                                      int32_t *sweeps_out, int max_sweeps,
                                                      double tolf, int accumulate, int maxn,
                                                      int tile_elems, int two,
                                                      int inplace_ok) {
  extern __shared__ __align__(16) unsigned char smem[];
  double *red = reinterpret_cast<double *>(smem);
  R *spar = reinterpret_cast<R *>(smem + kRed * sizeof(double));
  R *spar2 = two ? spar + (size_t)(maxn / 2) * kPivComp : nullptr;
  int16_t *spair =
      reinterpret_cast<int16_t *>(spar + (size_t)(two ? 2 : 1) * (maxn / 2) * kPivComp);
  R *T = reinterpret_cast<R *>(smem + persistent_fixed_lds<R>(maxn, two != 0));
  int m = mats[blockIdx.x];
  int n = d.n[m];
  int np = n >> 1;
  int64_t o = d.off[m];
  R *Gm = G + o, *Um = U + o, *Vm = V + o;
  R *tab = par + d.chunk * d.poff[m] * kPivComp;
  const int cm = d.chunk - 1;
  // the U/V tiles also take the LDS of the step parameters and the pair list,
  // which no phase reads across a U/V update (each step writes them afresh)
  R *Tuv = reinterpret_cast<R *>(smem + kRed * sizeof(double));
  const int uv_elems =
      tile_elems +
      (int)((persistent_fixed_lds<R>(maxn, two != 0) - kRed * sizeof(double)) / sizeof(R));
  // U/V tiles of equal height, as few as fit, rounded up to a whole number of
  // rows per wave when that still fits
  const int rows_max = min(n, uv_elems / (n + 1));
  const int ntl = (n + rows_max - 1) / rows_max;
  int rows = (n + ntl - 1) / ntl;
  if ((rows + BS / 64 - 1) / (BS / 64) * (BS / 64) <= rows_max)
    rows = (rows + BS / 64 - 1) / (BS / 64) * (BS / 64);
  int sg, nt;
  double fro2 = init_matrix(Gm, Um, Vm, n, accumulate != 0, red, sg, nt);
  const double nsc = ldexp(1.0, -nt);
  __syncthreads();
  // under the modified modulus ordering steps go in pairs through G and a
  // second buffer; the sweep's last step (n - 1 steps, an odd count) lands in G
  const bool pairs2 = d.ord != 2 && n >= 4 && two;
  R *Ga = pairs2 ? reinterpret_cast<R *>(d.galt) + d.aoff[m] : Gm;
  // orders up to 256 update G in place when the boundary columns fit the tile
  // (in workgroups of up to 512 lanes, whose registers hold that path)
  const FusedGeo geo = fused_geo(n, BS / 64, tile_elems);
  const bool inplace = inplace_ok && uses_inplace(BS, n, tile_elems) && pairs2;
  int sw = 0;
  bool conv = false;
  // dynamic ordering: the chunk's pairs go to the pair table (for the U/V
  // update); the matching's index arrays use the U/V tile, its flag the
  // reduction buffer (both idle during a step's pivots)
  int16_t *ptab = d.ord == 2 ? d.pairs + 2 * d.chunk * d.poff[m] : nullptr;
  for (; sw < max_sweeps && !conv; ++sw) {
    const R *cur = Gm;
    for (int k = 0; k < n - 1;) {
      R *slot = tab + (size_t)(k & cm) * kPivComp * np;
      if (d.ord == 2) {
        int16_t *mate = reinterpret_cast<int16_t *>(T);
        dyn_match(cur, n, nsc, mate, mate + n, reinterpret_cast<int *>(red), spair);
      }
      for (int q = threadIdx.x; q < np; q += BS) {
        int i, j;
        if (d.ord == 2) {
          i = spair[2 * q];
          j = spair[2 * q + 1];
          int16_t *pp = ptab + 2 * ((size_t)(k & cm) * np + q);
          pp[0] = (int16_t)i;
          pp[1] = (int16_t)j;
        } else {
          piv_pair(d.ord, n, k, q, i, j);
          spair[2 * q] = (int16_t)i;
          spair[2 * q + 1] = (int16_t)j;
        }
        Piv<R> P = pivot_svd(cur, n, i, j);
        piv_store(spar, np, q, P);
        piv_store(slot, np, q, P);
      }
      __syncthreads();
      if (pairs2 && k + 2 <= n - 2) {
        R *slot2 = tab + (size_t)((k + 1) & cm) * kPivComp * np;
        g_pivots_next<R, BS>(cur, n, k, spar, spar2, slot2, d.ord);
        if (inplace) g_fused_snapshot<R, BS>(Gm, n, k, geo, T, d.ord);
        __syncthreads();
        if (inplace) {
          if constexpr (BS <= 512) {
            if (np <= 64)
              g_fused_inplace<R, BS, 1>(Gm, n, k, spar, spar2, geo, T, d.ord);
            else
              g_fused_inplace<R, BS, 2>(Gm, n, k, spar, spar2, geo, T, d.ord);
          }
        } else {
          R *nxt = cur == Gm ? Ga : Gm;
          g_fused_pair<R, BS, sizeof(R) == 8 ? 4 : 6>(cur, nxt, n, k, spar, spar2, d.ord);
          cur = nxt;
        }
        k += 2;
      } else {
        // 1024 lanes keep 16 waves per CU in flight: two blocks each suffice and
        // stay within the 128 registers that size allows
        g_step_block<R, BS, (BS >= 1024 ? 2 : 4)>(cur, Gm, n, spar, spair);
        cur = Gm;
        k += 1;
      }
      __syncthreads();
      const int kl = k - 1;  // the last step done
      if ((kl & cm) == cm || kl == n - 2) {
        int k0 = chunk_begin(kl, cm);
        for (int side = 0; side < 2; ++side) {
          R *M = side ? Vm : Um;
          for (int r0 = 0; r0 < n; r0 += rows) {
            int nr = min(rows, n - r0);
            tile_load<R, (BS >= 1024 ? 4 : 8)>(Tuv, M, n, r0, nr);
            __syncthreads();
            tile_rotate<R, PS>(Tuv, n, nr, k0, kl, tab, side != 0, d.ord, cm, ptab);
            __syncthreads();
            tile_store<R, (BS >= 1024 ? 4 : 8)>(Tuv, M, n, r0, nr);
            __syncthreads();
          }
        }
      }
    }
    double off2 = block_sumsq(Gm, n, true, red, nsc);
    conv = converged(off2, fro2, n, tolf, (double)Lim<R>::eps());
  }
  __syncthreads();
  finish_matrix(Gm, n, sg, sigma ? sigma + d.soff[m] : nullptr,
                sweeps_out ? sweeps_out + m : nullptr, sw, conv);
}

// ------------------------------------------------------------ sigma gradient
//
// dG = U diag(dsigma) V^T per matrix (d sigma_i / dG = u_i v_i^T, summed with
// weights dsigma_i): a dense contraction over k, run on the matrix cores.  A
// 128 x 128 output tile per 256-lane workgroup, 64 x 64 per wave as 4 x 4 MFMA
// blocks of 16 x 16 x 4: per step of four k, each lane supplies one element
// of A = U diag(dsigma) (row l mod 16, column k0 + l / 16) per row block and
// one of B = V^T (row k0 + l / 16, column l mod 16) per column block, i.e. 16
// consecutive rows of a column of U or V per quarter wave; the sixteen
// products of a step share those eight operands.  Rows and columns past the
// matrix read row or column n - 1 and feed only outputs that are not stored;
// k past the matrix contributes zero.  Result element (i, j) of a block sits
// in lane j + 16 (i mod 4), register i / 4 for binary64 and in lane
// j + 16 (i / 4), register i mod 4 for binary32 (as the instructions lay them
// out on gfx950).

template <class R> struct Mfma;
template <> struct Mfma<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  __device__ static v4 mma(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static int row(int lane, int v) { return 4 * v + (lane >> 4); }
};
template <> struct Mfma<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  __device__ static v4 mma(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static int row(int lane, int v) { return 4 * (lane >> 4) + v; }
};

constexpr int kSgWR = 4, kSgWC = 4;                   // 16 x 16 blocks per wave
constexpr int kSgTR = 32 * kSgWR, kSgTC = 32 * kSgWC;  // workgroup tile (2 x 2 waves)

// Workgroups are handed to the 8 XCDs (each with its own L2) in turn, so
// workgroup b runs on XCD b mod 8.  The host deals the matrices to the XCDs,
// largest first, each to the XCD with the least work so far, and lists each
// XCD's tiles matrix by matrix, largest matrices first: sched[b] = (matrix,
// tile) of workgroup b, or matrix -1 where an XCD's list is shorter than the
// longest.  The tiles of one matrix, which share its U and V panels, meet in
// one L2.  Every output element accumulates its k in ascending order, four per
// instruction, whatever the tile shape.
template <class R>
__global__ __launch_bounds__(256) void k_sigma_grad(SweepDesc d, const int2 *sched,
                                                    const R *U, const R *V, const R *ds, R *dG) {
  typedef typename Mfma<R>::v4 v4;
  const int2 e = sched[blockIdx.x];
  if (e.x < 0) return;  // padding of a shorter XCD list
  const int m = e.x, t = e.y;
  int n = d.n[m];
  int tr = (n + kSgTR - 1) / kSgTR;
  int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  int r0 = (t % tr) * kSgTR + (w & 1) * 16 * kSgWR, c0 = (t / tr) * kSgTC + (w >> 1) * 16 * kSgWC;
  if (r0 >= n || c0 >= n) return;  // the whole wave is outside the matrix
  int64_t o = d.off[m];
  const R *Um = U + o, *Vm = V + o, *dsm = ds + d.soff[m];
  const int li = lane & 15, lk = lane >> 4;
  // element indices within the matrix (at most 2^26 of them, so byte offsets
  // fit 32 bits and every load is a scalar base plus one 32-bit offset)
  uint32_t ra[kSgWR], cb[kSgWC];
#pragma unroll
  for (int x = 0; x < kSgWR; ++x) ra[x] = (uint32_t)min(r0 + 16 * x + li, n - 1);
#pragma unroll
  for (int y = 0; y < kSgWC; ++y) cb[y] = (uint32_t)min(c0 + 16 * y + li, n - 1);
  const uint32_t col = (uint32_t)n;
  auto at = [](const R *base, uint32_t idx) {
    return *reinterpret_cast<const R *>(reinterpret_cast<const char *>(base) +
                                        (size_t)(idx * (uint32_t)sizeof(R)));
  };
  v4 acc[kSgWR][kSgWC];
#pragma unroll
  for (int x = 0; x < kSgWR; ++x)
#pragma unroll
    for (int y = 0; y < kSgWC; ++y) acc[x][y] = v4{0, 0, 0, 0};
  // the operands of the four k of one step; `masked` for the steps that may
  // reach past the matrix
  auto load = [&](int k, bool masked, R *a, R *bv) {
    const bool kin = !masked || k < n;
    const uint32_t ks = (uint32_t)(kin ? k : n - 1), kc = ks * col;
    const R s = at(dsm, ks);
#pragma unroll
    for (int x = 0; x < kSgWR; ++x) {
      const R u = at(Um, kc + ra[x]);
      a[x] = kin ? u * s : (R)0;
    }
#pragma unroll
    for (int y = 0; y < kSgWC; ++y) {
      const R v = at(Vm, kc + cb[y]);
      bv[y] = kin ? v : (R)0;
    }
  };
  R a[kSgWR], bv[kSgWC];
  // one step: issue the matrix instructions of the operands in hand, then take
  // the next step's operands, which were loaded before them
  auto step = [&](const R *na, const R *nb) {
#pragma unroll
    for (int x = 0; x < kSgWR; ++x)
#pragma unroll
      for (int y = 0; y < kSgWC; ++y) acc[x][y] = Mfma<R>::mma(a[x], bv[y], acc[x][y]);
#pragma unroll
    for (int x = 0; x < kSgWR; ++x) a[x] = na[x];
#pragma unroll
    for (int y = 0; y < kSgWC; ++y) bv[y] = nb[y];
  };
  load(lk, true, a, bv);
  int k0 = 0;
  // every k of step k0 + 4 lies inside the matrix while k0 + 8 <= n
  for (; k0 + 8 <= n; k0 += 4) {
    R na[kSgWR], nb[kSgWC];
    load(k0 + 4 + lk, false, na, nb);
    step(na, nb);
  }
  for (; k0 < n; k0 += 4) {
    R na[kSgWR], nb[kSgWC];
    load(k0 + 4 + lk, true, na, nb);
    step(na, nb);
  }
  R *out = dG + o;
#pragma unroll
  for (int x = 0; x < kSgWR; ++x)
#pragma unroll
    for (int y = 0; y < kSgWC; ++y)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        int r = r0 + 16 * x + Mfma<R>::row(lane, v), c = c0 + 16 * y + li;
        if (r < n && c < n) out[r + (int64_t)c * n] = acc[x][y][v];
      }
}

// ------------------------------------------------------- sorted convention
//
// sigma of matrix m in descending order (equal values keep their index order)
// with the columns of U and V permuted to match, so that G0 = U diag(sigma) V^T
// holds with sigma_1 >= sigma_2 >= ...  One workgroup per matrix: the rank of
// every value is counted in LDS (stable, so the ranks are a permutation), then
// U and V are rewritten a tile of whole rows at a time (a row's columns move
// within the tile, so the permutation is in place).

template <class R>
__global__ __launch_bounds__(kRed) void k_sw_sort(SweepDesc d, R *U, R *V, R *sigma,
                                                 int tile_elems) {
  extern __shared__ __align__(16) unsigned char smem[];
  int m = blockIdx.x;
  int n = d.n[m];
  R *sv = reinterpret_cast<R *>(smem);
  int *rk = reinterpret_cast<int *>(smem + (size_t)n * sizeof(R));
  size_t fixed = ((size_t)n * (sizeof(R) + sizeof(int)) + 15) & ~(size_t)15;
  R *T = reinterpret_cast<R *>(smem + fixed);
  R *sg = sigma + d.soff[m];
  for (int i = threadIdx.x; i < n; i += blockDim.x) sv[i] = sg[i];
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    R x = sv[i];
    int r = 0;
    for (int j = 0; j < n; ++j) {
      R y = sv[j];
      r += (y > x) || (y == x && j < i);
    }
    rk[i] = r;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += blockDim.x) sg[rk[i]] = sv[i];
  const int ldt = n + 1;
  int rows = min(n, (tile_elems - (int)(fixed / sizeof(R))) / ldt);
  for (int side = 0; side < 2; ++side) {
    R *M = (side ? V : U) + d.off[m];
    for (int r0 = 0; r0 < n; r0 += rows) {
      int nr = min(rows, n - r0);
      tile_load(T, M, n, r0, nr);
      __syncthreads();
      // column c of the tile goes to column rank(c)
      for (int e = threadIdx.x; e < nr * n; e += blockDim.x) {
        int r = e % nr, c = e / nr;
        M[r0 + r + (int64_t)rk[c] * n] = T[r * ldt + c];
      }
      __syncthreads();
    }
  }
}

// ----------------------------------------------------------------- host side

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct WsLayout {
  size_t n, off, soff, poff, order, fro2, sweeps, done, scale, nexp, aoff, par, pairs, galt,
      total;
};

// npiv: the sum of n/2; chunk: steps per U/V update (rows of the step table);
// pairs: mode 0's pair table; galt_elems: the second G buffer (only the
// matrices whose two-step passes go through it)
static WsLayout ws_layout(int64_t nmat, int64_t npiv, int chunk, bool pairs, int64_t galt_elems,
                          size_t w) {
  WsLayout L;
  size_t p = 0;
  L.n = p;      p = align256(p + nmat * 4);
  L.off = p;    p = align256(p + nmat * 8);
  L.soff = p;   p = align256(p + nmat * 8);
  L.poff = p;   p = align256(p + nmat * 8);
  L.order = p;  p = align256(p + nmat * 4);
  L.fro2 = p;   p = align256(p + nmat * 8);
  L.sweeps = p; p = align256(p + nmat * 4);
  L.done = p;   p = align256(p + nmat * 4);
  L.scale = p;  p = align256(p + nmat * 4);
  L.nexp = p;   p = align256(p + nmat * 4);
  L.aoff = p;   p = align256(p + nmat * 8);
  L.par = p;    p = align256(p + (size_t)chunk * npiv * kPivComp * w);
  L.pairs = p;  p = align256(p + (pairs ? (size_t)chunk * npiv * 4 : 0));
  L.galt = p;   p = align256(p + (size_t)galt_elems * w);
  L.total = p;
  return L;
}

// Tuning table of the persistent sweep, per dtype and order bucket (0: n <= 64,
// 1: n <= 128, 2: n <= 256, 3: n <= 512, 4: larger).  No entry changes a bit
// of the results: every choice performs the same operations in the same order.
//   block    lanes per workgroup (one workgroup per matrix): 256, 512, 1024
//   chunk    steps per U/V update (power of two, 2..128); a call takes the
//            entry of the bucket of its largest order
//   two      two steps of G per pass under the modified modulus ordering
//   inplace  the in-place form of that pass (orders up to 256, up to 512 lanes)
//   rows     the U/V tile's own LDS for at most this many rows of the largest
//            order (0: as many as fit); fewer rows leave LDS for a second
//            workgroup on a compute unit (a U/V update also spreads over the
//            step parameters' LDS)
enum Knob { K_BLOCK = 0, K_CHUNK = 1, K_TWO = 2, K_INPLACE = 3, K_ROWS = 4, K_NKNOB = 5 };
struct Tune {
  int v[2][5][K_NKNOB];
};
static Tune default_tune() {
  Tune t;
  // binary64 orders 257-512 take 512 lanes (four pair slots per lane in the U/V
  // rotations), binary32 ones 1,024 (measured on the uneven batch)
  const int blocks[2][5] = {{256, 512, 512, 1024, 1024}, {256, 512, 512, 512, 1024}};
  for (int d = 0; d < 2; ++d)
    for (int b = 0; b < 5; ++b) {
      t.v[d][b][K_BLOCK] = blocks[d][b];
      t.v[d][b][K_CHUNK] = kChunk;
      t.v[d][b][K_TWO] = 1;
      t.v[d][b][K_INPLACE] = 1;
      t.v[d][b][K_ROWS] = 0;
    }
  return t;
}
static Tune g_tune = default_tune();
static std::mutex g_mu;

static int bucket_of(int n) {
  if (n <= 64) return 0;
  if (n <= 128) return 1;
  if (n <= 256) return 2;
  if (n <= 512) return 3;
  return 4;
}

static int tune_check(int knob, int value) {
  switch (knob) {
    case K_BLOCK:
      if (value != 256 && value != 512 && value != 1024)
        return fail(KSVD2_EINVAL, "block must be 256, 512 or 1024");
      return KSVD2_OK;
    case K_CHUNK:
      if (value < 2 || value > kChunk || (value & (value - 1)))
        return fail(KSVD2_EINVAL, "chunk must be a power of two in [2, %d]", kChunk);
      return KSVD2_OK;
    case K_TWO:
    case K_INPLACE:
      if (value != 0 && value != 1) return fail(KSVD2_EINVAL, "this knob is 0 or 1");
      return KSVD2_OK;
    case K_ROWS:
      if (value < 0 || value > kMaxOrder) return fail(KSVD2_EINVAL, "rows must be in [0, %d]", kMaxOrder);
      return KSVD2_OK;
    default:
      return fail(KSVD2_EINVAL, "unknown knob %d", knob);
  }
}

// LDS a workgroup may allocate on the current device (queried once per device)
static size_t device_lds_limit() {
  static std::mutex mu;
  static std::map<int, size_t> cache;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  std::lock_guard<std::mutex> lk(mu);
  auto it = cache.find(dev);
  if (it != cache.end()) return it->second;
  int v = 0;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
    v = 0;
  cache[dev] = (size_t)v;
  return (size_t)v;
}

// LDS of a persistent launch over matrices of order <= maxn: the fixed part
// plus the largest U/V tile that fits (at least one row of maxn + 1, at most
// max_rows rows when max_rows > 0); the parameters of two steps when allowed
// and when that leaves room for 16 tile rows, else of one (one step per pass)
template <class R> static size_t persistent_lds(int maxn, size_t limit, bool allow_two,
                                                int max_rows, int &tile_elems, int &two) {
  tile_elems = 0;
  for (two = allow_two ? 1 : 0; two >= 0; --two) {
    size_t fixed = persistent_fixed_lds<R>(maxn, two != 0);
    size_t rows = two ? std::min(16, maxn) : 1;
    if (limit <= fixed || (limit - fixed) / sizeof(R) < rows * ((size_t)maxn + 1)) continue;
    size_t te = (limit - fixed) / sizeof(R);
    size_t cap = max_rows > 0 ? std::min(max_rows, maxn) : maxn;
    te = std::min(te, cap * (size_t)(maxn + 1));  // never more than the whole matrix
    tile_elems = (int)std::min<size_t>(te, (size_t)1 << 30);
    return fixed + (size_t)tile_elems * sizeof(R);
  }
  two = 0;
  return 0;
}

template <class R, int BS, int PS> static void set_lds_attr(size_t lds) {
  (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&k_sw_persistent<R, BS, PS>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

// one persistent launch: matrices order[begin .. begin + count) (longest
// first), their largest order, workgroup size and LDS partition
struct Seg {
  int begin, count, maxn, block, tile_elems, two, inplace_ok;
  size_t lds;
};

// Everything a call needs on the host before it touches the device: the
// per-matrix offsets, the order of processing, the launches and the exact
// workspace layout.
struct Plan {
  int maxn = 0, chunk = kChunk;
  int64_t npiv = 0, galt = 0;
  std::vector<int64_t> soff, poff, aoff;
  std::vector<int32_t> order;
  std::vector<Seg> segs;
  WsLayout L;
};

template <class R>
static int make_plan(int64_t nmat, const int32_t *n_host, const int64_t *off_host, int mode,
                     int ordering, const Tune &tune, int chunk, Plan &P) {
  const size_t w = sizeof(R);
  const int di = (w == 8) ? 1 : 0;
  P.soff.assign(nmat, 0);
  P.poff.assign(nmat, 0);
  P.aoff.assign(nmat, 0);
  int64_t stot = 0;
  for (int64_t m = 0; m < nmat; ++m) {
    int n = n_host[m];
    if (n < 2 || (n & 1) || n > kMaxOrder)
      return fail(KSVD2_EINVAL, "matrix %lld: order %d must be even, in [2, %d]", (long long)m,
                  n, kMaxOrder);
    if (off_host[m] < 0) return fail(KSVD2_EINVAL, "matrix %lld: negative offset", (long long)m);
    P.soff[m] = stot;
    P.poff[m] = P.npiv;
    stot += n;
    P.npiv += n / 2;
    P.maxn = std::max(P.maxn, n);
  }
  P.chunk = chunk;
  // longest matrices first (they have the most steps)
  P.order.resize(nmat);
  std::iota(P.order.begin(), P.order.end(), 0);
  std::stable_sort(P.order.begin(), P.order.end(),
                   [&](int a, int b) { return n_host[a] > n_host[b]; });
  P.segs.clear();
  P.galt = 0;
  if (mode != 0) {
    // one persistent launch per order bucket, longest first
    for (int64_t a = 0; a < nmat;) {
      int b0 = bucket_of(n_host[P.order[a]]);
      int64_t bb = a;
      while (bb < nmat && bucket_of(n_host[P.order[bb]]) == b0) ++bb;
      const int *t = tune.v[di][b0];
      Seg s{(int)a, (int)(bb - a), n_host[P.order[a]], t[K_BLOCK], 0, t[K_TWO], t[K_INPLACE], 0};
      s.tile_elems = t[K_ROWS];  // the row cap until the LDS is partitioned
      P.segs.push_back(s);
      a = bb;
    }
    // one launch over all matrices, longest first, when the buckets agree on
    // the launch: the dispatcher then starts each next matrix as soon as a CU
    // frees up, with no drain between buckets
    bool same = std::all_of(P.segs.begin(), P.segs.end(), [&](const Seg &x) {
      const Seg &y = P.segs[0];
      return x.block == y.block && x.two == y.two && x.inplace_ok == y.inplace_ok &&
             x.tile_elems == y.tile_elems;
    });
    if (same && P.segs.size() > 1) {
      Seg s = P.segs[0];
      s.begin = 0;
      s.count = (int)nmat;
      P.segs = {s};
    }
    const size_t lds_limit = device_lds_limit();
    if (lds_limit == 0) return fail(KSVD2_EHIP, "cannot read the device's LDS limit");
    for (Seg &s : P.segs) {
      int te = 0, two = 0;
      s.lds = persistent_lds<R>(s.maxn, lds_limit, s.two != 0, s.tile_elems, te, two);
      if (s.lds == 0)
        return fail(KSVD2_EINVAL,
                    "order %d needs more LDS than a workgroup may allocate (%zu bytes) in the "
                    "persistent modes; use mode 0",
                    s.maxn, lds_limit);
      s.tile_elems = te;
      s.two = two;
      // the matrices whose two-step passes go through the second buffer
      for (int x = s.begin; x < s.begin + s.count; ++x) {
        const int m = P.order[x], n = n_host[m];
        const bool pairs2 = ordering != 2 && n >= 4 && two;
        const bool inplace = s.inplace_ok && uses_inplace(s.block, n, te) && pairs2;
        if (pairs2 && !inplace) {
          P.aoff[m] = P.galt;
          P.galt += (int64_t)n * n;
        }
      }
    }
  }
  P.L = ws_layout(nmat, P.npiv, chunk, mode == 0 || ordering == 2, P.galt, w);
  return KSVD2_OK;
}

template <class R>
static int launch_persistent(const SweepDesc &d, const int32_t *mats_dev, const Seg &s, R *G,
                             R *U, R *V, R *par, R *sigma, int32_t *sweeps_out, int max_sweeps,
                             double tolf, int accumulate, hipStream_t st) {
  const unsigned cnt = (unsigned)s.count;
  switch (s.block) {
    case 256:
      set_lds_attr<R, 256, 2>(s.lds);
      hipLaunchKernelGGL((k_sw_persistent<R, 256, 2>), dim3(cnt), dim3(256), s.lds, st, d,
                         mats_dev, G, U, V, par, sigma, sweeps_out, max_sweeps, tolf,
                         accumulate, s.maxn, s.tile_elems, s.two, s.inplace_ok);
      break;
    case 512:
      // four pair slots per lane only where an order above 256 needs them
      if (s.maxn > 256) {
        set_lds_attr<R, 512, 4>(s.lds);
        hipLaunchKernelGGL((k_sw_persistent<R, 512, 4>), dim3(cnt), dim3(512), s.lds, st, d,
                           mats_dev, G, U, V, par, sigma, sweeps_out, max_sweeps, tolf,
                           accumulate, s.maxn, s.tile_elems, s.two, s.inplace_ok);
      } else {
        set_lds_attr<R, 512, 2>(s.lds);
        hipLaunchKernelGGL((k_sw_persistent<R, 512, 2>), dim3(cnt), dim3(512), s.lds, st, d,
                           mats_dev, G, U, V, par, sigma, sweeps_out, max_sweeps, tolf,
                           accumulate, s.maxn, s.tile_elems, s.two, s.inplace_ok);
      }
      break;
    case 1024:
      set_lds_attr<R, 1024, 0>(s.lds);
      hipLaunchKernelGGL((k_sw_persistent<R, 1024, 0>), dim3(cnt), dim3(1024), s.lds, st, d,
                         mats_dev, G, U, V, par, sigma, sweeps_out, max_sweeps, tolf,
                         accumulate, s.maxn, s.tile_elems, s.two, s.inplace_ok);
      break;
    default:
      return fail(KSVD2_EINVAL, "unsupported block size %d", s.block);
  }
  return launch_status("kog_sweep persistent launch");
}

// Executable graphs of mode 2, one per argument set, at most kGraphCache per
// process: the least recently used one is destroyed (after its device has
// finished its work) to make room.
constexpr size_t kGraphCache = 16;
struct GraphKey {
  int dev, dtype, ordering;
  int64_t nmat;
  const void *G, *U, *V, *sigma, *sweeps, *ws;
  int max_sweeps, accumulate;
  double tolf;
  hipStream_t st;
  std::vector<int32_t> n;
  std::vector<int64_t> off;
  std::vector<int> tune;
  bool operator<(const GraphKey &o) const {
    return std::tie(dev, dtype, ordering, nmat, G, U, V, sigma, sweeps, ws, max_sweeps,
                    accumulate, tolf, st, n, off, tune) <
           std::tie(o.dev, o.dtype, o.ordering, o.nmat, o.G, o.U, o.V, o.sigma, o.sweeps, o.ws,
                    o.max_sweeps, o.accumulate, o.tolf, o.st, o.n, o.off, o.tune);
  }
};
struct GraphEntry {
  hipGraphExec_t exec;
  uint64_t used;
};
static std::map<GraphKey, GraphEntry> g_graphs;
static uint64_t g_graph_clock = 0;

// room for one more graph (caller holds g_mu)
static void graph_evict_one() {
  if (g_graphs.size() < kGraphCache) return;
  auto lru = g_graphs.begin();
  for (auto it = g_graphs.begin(); it != g_graphs.end(); ++it)
    if (it->second.used < lru->second.used) lru = it;
  int cur = 0;
  (void)hipGetDevice(&cur);
  if (lru->first.dev != cur) (void)hipSetDevice(lru->first.dev);
  (void)hipDeviceSynchronize();  // the graph may still run
  (void)hipGraphExecDestroy(lru->second.exec);
  if (lru->first.dev != cur) (void)hipSetDevice(cur);
  g_graphs.erase(lru);
}

// The iteration on one batch.  ws_bytes must cover the plan's layout; with
// shrink_chunk the chunk is halved (down to 2) until it does.
template <class R>
static int sweep_impl(int dtype, int64_t nmat, const int32_t *n_host, const int64_t *off_host,
                      R *G, R *U, R *V, R *sigma, int32_t *sweeps_out, int max_sweeps,
                      double tolf, int accumulate, int mode, int ordering, void *ws,
                      size_t ws_bytes, hipStream_t st, bool shrink_chunk) {
  if (nmat < 0) return fail(KSVD2_EINVAL, "nmat < 0");
  if (nmat == 0) return KSVD2_OK;
  if (!n_host || !off_host) return fail(KSVD2_EINVAL, "n_host and off_host are required");
  if (max_sweeps < 0) return fail(KSVD2_EINVAL, "max_sweeps < 0");
  if (mode < 0 || mode > 2) return fail(KSVD2_EINVAL, "mode must be 0, 1 or 2");
  if (ordering < 0 || ordering > 2)
    return fail(KSVD2_EINVAL,
                "ordering must be 0 (round-robin), 1 (modified modulus) or 2 (dynamic)");
  if (nmat > 65535) return fail(KSVD2_EINVAL, "at most 65535 matrices per call");
  if (mode == 2 && st == nullptr)
    return fail(KSVD2_EINVAL, "mode 2 (hipGraph) needs a non-null stream");
  const size_t w = sizeof(R);
  KSVD2_REQ(G, w); KSVD2_REQ(U, w); KSVD2_REQ(V, w); KSVD2_REQ(ws, 256);
  KSVD2_OPT(sigma, w); KSVD2_OPT(sweeps_out, 4);
  Tune tune;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    tune = g_tune;
  }
  const int di = (w == 8) ? 1 : 0;
  int maxn0 = 0;
  for (int64_t m = 0; m < nmat; ++m) maxn0 = std::max(maxn0, n_host[m]);
  int chunk = tune.v[di][bucket_of(maxn0)][K_CHUNK];
  Plan P;
  for (;;) {
    int rc = make_plan<R>(nmat, n_host, off_host, mode, ordering, tune, chunk, P);
    if (rc) return rc;
    if (P.L.total <= ws_bytes) break;
    if (!shrink_chunk || chunk <= 2)
      return fail(KSVD2_EWORKSPACE, "workspace of %zu bytes, %zu needed", ws_bytes, P.L.total);
    chunk >>= 1;
  }
  const WsLayout &L = P.L;
  const int maxn = P.maxn;
  // stage the descriptor into the workspace (one host buffer, one copy); the
  // zeros also clear the counters and flags
  std::vector<unsigned char> host(L.par, 0);
  std::memcpy(host.data() + L.n, n_host, nmat * 4);
  std::memcpy(host.data() + L.off, off_host, nmat * 8);
  std::memcpy(host.data() + L.soff, P.soff.data(), nmat * 8);
  std::memcpy(host.data() + L.poff, P.poff.data(), nmat * 8);
  std::memcpy(host.data() + L.order, P.order.data(), nmat * 4);
  std::memcpy(host.data() + L.aoff, P.aoff.data(), nmat * 8);
  unsigned char *wsb = static_cast<unsigned char *>(ws);
  hipError_t e = hipMemcpyAsync(wsb, host.data(), L.par, hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return fail(KSVD2_EHIP, "descriptor upload: %s", hipGetErrorString(e));
  SweepDesc d;
  d.n = reinterpret_cast<const int32_t *>(wsb + L.n);
  d.off = reinterpret_cast<const int64_t *>(wsb + L.off);
  d.soff = reinterpret_cast<const int64_t *>(wsb + L.soff);
  d.poff = reinterpret_cast<const int64_t *>(wsb + L.poff);
  d.fro2 = reinterpret_cast<double *>(wsb + L.fro2);
  d.sweeps = reinterpret_cast<int32_t *>(wsb + L.sweeps);
  d.done = reinterpret_cast<int32_t *>(wsb + L.done);
  d.scale = reinterpret_cast<int32_t *>(wsb + L.scale);
  d.nexp = reinterpret_cast<int32_t *>(wsb + L.nexp);
  d.ord = ordering;
  d.aoff = reinterpret_cast<const int64_t *>(wsb + L.aoff);
  d.galt = wsb + L.galt;
  d.chunk = P.chunk;
  d.pairs = reinterpret_cast<int16_t *>(wsb + L.pairs);
  const int32_t *order_dev = reinterpret_cast<const int32_t *>(wsb + L.order);

  R *par = reinterpret_cast<R *>(wsb + L.par);
  if (mode == 0) {
    int16_t *pairs = reinterpret_cast<int16_t *>(wsb + L.pairs);
    hipLaunchKernelGGL(k_sw_init<R>, dim3((unsigned)nmat), dim3(kRed), 0, st, d, G, U, V,
                       accumulate);
    int rc = launch_status("kog_sweep init");
    if (rc) return rc;
    int maxnp = maxn / 2;
    int64_t maxblocks = (int64_t)maxnp * maxnp;
    // U/V tiles of the mode-0 kernel: 64 KB, or as much LDS as a workgroup may
    // take when one row of the largest order needs more; the rows of the
    // smallest order set the tile count
    size_t apply_lds = std::max(kApplyLds, (size_t)(maxn + 1) * sizeof(R));
    if (apply_lds > kApplyLds) {
      apply_lds = device_lds_limit();
      (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&k_sw_apply<R>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)apply_lds);
    }
    const int apply_elems = (int)(apply_lds / sizeof(R));
    int minrows = maxn;
    for (int64_t m = 0; m < nmat; ++m)
      minrows = std::min(minrows, std::min(n_host[m], apply_elems / (n_host[m] + 1)));
    if (minrows < 1)
      return fail(KSVD2_EINVAL, "order %d too large for the U/V tile", maxn);
    unsigned apply_tiles = (unsigned)((maxn + minrows - 1) / minrows);
    const int cm = P.chunk - 1;
    std::vector<int32_t> done(nmat);
    for (int sw = 0; sw < max_sweeps; ++sw) {
      for (int k = 0; k < maxn - 1; ++k) {
        if (ordering == 2)
          hipLaunchKernelGGL(k_sw_match<R>, dim3((unsigned)nmat), dim3(kRed),
                             (size_t)4 * maxn, st, d, G, pairs, k);
        hipLaunchKernelGGL(k_sw_pivots<R>, dim3(grid_for(maxnp), (unsigned)nmat), dim3(kBlock), 0,
                           st, d, G, par, pairs, k);
        hipLaunchKernelGGL(k_sw_update<R>, dim3(grid_for(maxblocks), (unsigned)nmat),
                           dim3(kBlock), 0, st, d, G, par, pairs, k);
        if ((k & cm) == cm || k == maxn - 2)
          hipLaunchKernelGGL(k_sw_apply<R>, dim3(apply_tiles, 2, (unsigned)nmat),
                             dim3(kApplyBlock), apply_lds, st, d, U, V, par, k, apply_elems);
      }
      hipLaunchKernelGGL(k_sw_check<R>, dim3((unsigned)nmat), dim3(kRed), 0, st, d, G, tolf);
      rc = launch_status("kog_sweep step");
      if (rc) return rc;
      e = hipMemcpyAsync(done.data(), d.done, nmat * 4, hipMemcpyDeviceToHost, st);
      if (e == hipSuccess) e = hipStreamSynchronize(st);
      if (e != hipSuccess) return fail(KSVD2_EHIP, "convergence poll: %s", hipGetErrorString(e));
      if (std::all_of(done.begin(), done.end(), [](int32_t v) { return v != 0; })) break;
    }
    hipLaunchKernelGGL(k_sw_finish<R>, dim3((unsigned)nmat), dim3(kRed), 0, st, d, G, sigma,
                       sweeps_out);
    return launch_status("kog_sweep finish");
  }

  auto launch_all = [&]() -> int {
    for (const Seg &s : P.segs) {
      int rc = launch_persistent<R>(d, order_dev + s.begin, s, G, U, V, par, sigma, sweeps_out,
                                    max_sweeps, tolf, accumulate, st);
      if (rc) return rc;
    }
    return KSVD2_OK;
  };
  if (mode == 1) return launch_all();

  // mode 2: capture the launches once per argument set, then replay
  int dev = 0;
  e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(KSVD2_EHIP, "hipGetDevice: %s", hipGetErrorString(e));
  GraphKey key{dev, dtype, ordering, nmat, G, U, V, sigma, sweeps_out, ws, max_sweeps,
               accumulate, tolf, st, std::vector<int32_t>(n_host, n_host + nmat),
               std::vector<int64_t>(off_host, off_host + nmat), {}};
  for (const Seg &s : P.segs)
    key.tune.insert(key.tune.end(), {s.block, s.two, s.inplace_ok, s.tile_elems});
  key.tune.push_back(P.chunk);
  hipGraphExec_t exec = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_graphs.find(key);
    if (it != g_graphs.end()) {
      exec = it->second.exec;
      it->second.used = ++g_graph_clock;
    }
  }
  if (!exec) {
    e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return fail(KSVD2_EHIP, "graph capture: %s", hipGetErrorString(e));
    int rc = launch_all();
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(st, &graph);
    if (rc) {
      if (graph) (void)hipGraphDestroy(graph);
      return rc;
    }
    if (e != hipSuccess) return fail(KSVD2_EHIP, "graph capture end: %s", hipGetErrorString(e));
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return fail(KSVD2_EHIP, "graph instantiate: %s", hipGetErrorString(e));
    std::lock_guard<std::mutex> lk(g_mu);
    graph_evict_one();
    g_graphs[key] = GraphEntry{exec, ++g_graph_clock};
  }
  e = hipGraphLaunch(exec, st);
  if (e != hipSuccess) return fail(KSVD2_EHIP, "graph launch: %s", hipGetErrorString(e));
  return KSVD2_OK;
}

// Scratch of kog_sweep_batch_noalloc: a file-scope device array in place of the
// caller's workspace, so that the call allocates no device memory.  Every GPU the
// library runs on holds its own copy for the life of the process.  In host code
// the array's name stands for no device address: the address comes from
// hipGetSymbolAddress, once per device with that device current, and only that
// address is handed to the copies and kernels.
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
constexpr int kMaxDevices = 64;
static void *g_scratch_ptr[kMaxDevices];

static int scratch_address(void **out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(KSVD2_EHIP, "hipGetDevice: %s", hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices)
    return fail(KSVD2_EINVAL, "device %d: the static scratch serves devices 0..%d", dev,
                kMaxDevices - 1);
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(KSVD2_EHIP, "address of the static scratch on device %d: %s", dev,
                  hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return KSVD2_OK;
}

template <class R>
static int sigma_grad_impl(int64_t nmat, const int32_t *n_host, const int64_t *off_host,
                           const R *U, const R *V, const R *ds, R *dG, void *ws, size_t ws_bytes,
                           hipStream_t st) {
  if (nmat < 0) return fail(KSVD2_EINVAL, "nmat < 0");
  if (nmat == 0) return KSVD2_OK;
  if (!n_host || !off_host) return fail(KSVD2_EINVAL, "n_host and off_host are required");
  if (nmat > 65535) return fail(KSVD2_EINVAL, "at most 65535 matrices per call");
  const size_t w = sizeof(R);
  KSVD2_REQ(U, w); KSVD2_REQ(V, w); KSVD2_REQ(ds, w); KSVD2_REQ(dG, w); KSVD2_REQ(ws, 256);
  int maxn = 0;
  int64_t stot = 0;
  std::vector<int64_t> soff(nmat);
  for (int64_t m = 0; m < nmat; ++m) {
    int n = n_host[m];
    if (n < 1 || n > kMaxOrder) return fail(KSVD2_EINVAL, "bad order %d", n);
    soff[m] = stot;
    stot += n;
    maxn = std::max(maxn, n);
  }
  // the workgroup schedule: matrices by decreasing order, each dealt to the
  // XCD with the least work so far (work of a tile ~ n)
  std::vector<int> ord(nmat);
  std::iota(ord.begin(), ord.end(), 0);
  std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return n_host[x] > n_host[y]; });
  std::vector<std::vector<int2>> bins(8);
  double load[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int m : ord) {
    const int n = n_host[m];
    const int tl = ((n + kSgTR - 1) / kSgTR) * ((n + kSgTC - 1) / kSgTC);
    const int x = (int)(std::min_element(load, load + 8) - load);
    for (int t = 0; t < tl; ++t) bins[x].push_back(make_int2(m, t));
    load[x] += (double)tl * n;
  }
  size_t longest = 0;
  for (auto &v : bins) longest = std::max(longest, v.size());
  const size_t nwg = 8 * longest;
  if (nwg > (size_t)(UINT32_MAX / 256))
    return fail(KSVD2_EINVAL, "%lld matrices of order up to %d are too many tiles for one call",
                (long long)nmat, maxn);
  size_t o_n = 0, o_off = align256(nmat * 4), o_soff = o_off + align256(nmat * 8);
  size_t o_sched = o_soff + align256(nmat * 8);
  size_t need = o_sched + align256(nwg * sizeof(int2));
  if (ws_bytes < need) return fail(KSVD2_EWORKSPACE, "workspace of %zu bytes, %zu needed", ws_bytes, need);
  std::vector<unsigned char> host(need, 0);
  std::memcpy(host.data() + o_n, n_host, nmat * 4);
  std::memcpy(host.data() + o_off, off_host, nmat * 8);
  std::memcpy(host.data() + o_soff, soff.data(), nmat * 8);
  int2 *sc = reinterpret_cast<int2 *>(host.data() + o_sched);
  for (size_t j = 0; j < longest; ++j)
    for (int x = 0; x < 8; ++x) sc[8 * j + x] = j < bins[x].size() ? bins[x][j] : make_int2(-1, 0);
  unsigned char *wsb = static_cast<unsigned char *>(ws);
  hipError_t e = hipMemcpyAsync(wsb, host.data(), need, hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return fail(KSVD2_EHIP, "descriptor upload: %s", hipGetErrorString(e));
  SweepDesc d{};
  d.n = reinterpret_cast<const int32_t *>(wsb + o_n);
  d.off = reinterpret_cast<const int64_t *>(wsb + o_off);
  d.soff = reinterpret_cast<const int64_t *>(wsb + o_soff);
  hipLaunchKernelGGL(k_sigma_grad<R>, dim3((unsigned)nwg), dim3(256), 0, st, d,
                     reinterpret_cast<const int2 *>(wsb + o_sched), U, V, ds, dG);
  return launch_status("kog_sigma_grad launch");
}

template <class R>
static int sort_impl(int64_t nmat, const int32_t *n_host, const int64_t *off_host, R *U, R *V,
                     R *sigma, void *ws, size_t ws_bytes, hipStream_t st) {
  if (nmat < 0) return fail(KSVD2_EINVAL, "nmat < 0");
  if (nmat == 0) return KSVD2_OK;
  if (!n_host || !off_host) return fail(KSVD2_EINVAL, "n_host and off_host are required");
  if (nmat > 65535) return fail(KSVD2_EINVAL, "at most 65535 matrices per call");
  const size_t w = sizeof(R);
  KSVD2_REQ(U, w); KSVD2_REQ(V, w); KSVD2_REQ(sigma, w); KSVD2_REQ(ws, 256);
  int maxn = 0;
  int64_t stot = 0;
  std::vector<int64_t> soff(nmat);
  for (int64_t m = 0; m < nmat; ++m) {
    int n = n_host[m];
    if (n < 1 || n > kMaxOrder) return fail(KSVD2_EINVAL, "bad order %d", n);
    if (off_host[m] < 0) return fail(KSVD2_EINVAL, "matrix %lld: negative offset", (long long)m);
    soff[m] = stot;
    stot += n;
    maxn = std::max(maxn, n);
  }
  size_t need = align256(nmat * 4) + align256(nmat * 8) * 2;
  if (ws_bytes < need)
    return fail(KSVD2_EWORKSPACE, "workspace of %zu bytes, %zu needed", ws_bytes, need);
  // LDS: the values and ranks of the largest order, plus at least one tile row
  size_t fixed = ((size_t)maxn * (w + sizeof(int)) + 15) & ~(size_t)15;
  size_t lds = std::max((size_t)64 * 1024, fixed + (size_t)(maxn + 1) * w);
  if (lds > 64 * 1024) {
    size_t lim = device_lds_limit();
    if (lds > lim)
      return fail(KSVD2_EINVAL, "order %d needs %zu bytes of LDS, %zu available", maxn, lds, lim);
    lds = lim;
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&k_sw_sort<R>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  }
  std::vector<unsigned char> host(need, 0);
  size_t o_n = 0, o_off = align256(nmat * 4), o_soff = o_off + align256(nmat * 8);
  std::memcpy(host.data() + o_n, n_host, nmat * 4);
  std::memcpy(host.data() + o_off, off_host, nmat * 8);
  std::memcpy(host.data() + o_soff, soff.data(), nmat * 8);
  unsigned char *wsb = static_cast<unsigned char *>(ws);
  hipError_t e = hipMemcpyAsync(wsb, host.data(), need, hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return fail(KSVD2_EHIP, "descriptor upload: %s", hipGetErrorString(e));
  SweepDesc d{};
  d.n = reinterpret_cast<const int32_t *>(wsb + o_n);
  d.off = reinterpret_cast<const int64_t *>(wsb + o_off);
  d.soff = reinterpret_cast<const int64_t *>(wsb + o_soff);
  hipLaunchKernelGGL(k_sw_sort<R>, dim3((unsigned)nmat), dim3(kRed), lds, st, d, U, V, sigma,
                     (int)(lds / w));
  return launch_status("kog_sweep_sort launch");
}

}  // namespace ksvd2

using namespace ksvd2;

extern "C" {

size_t kog_sweep_workspace_size(int dtype, int64_t nmat, const int32_t *n_host) {
  if (nmat <= 0 || !n_host || (dtype != 0 && dtype != 1)) return 0;
  int64_t npiv = 0, nsq = 0, tiles = 0;
  for (int64_t m = 0; m < nmat; ++m) {
    int64_t nm = std::max(n_host[m], 0);
    npiv += nm / 2;
    nsq += nm * nm;
    tiles += ((nm + kSgTR - 1) / kSgTR) * ((nm + kSgTC - 1) / kSgTC);
  }
  // every mode, ordering and tuning: the longest chunk, the pair table and a
  // second buffer for every matrix
  size_t a = ws_layout(nmat, npiv, kChunk, true, nsq, dtype ? 8 : 4).total;
  // kog_sigma_grad: the descriptors and its workgroup schedule (at most eight
  // lists as long as all the tiles together)
  size_t b = align256(nmat * 4) + align256(nmat * 8) * 2 + align256((size_t)tiles * 8 * 8);
  return std::max(a, b);
}

int kog_sweep_batch(int dtype, int64_t nmat, const int32_t *n_host, const int64_t *off_host,
                    void *G, void *U, void *V, void *sigma, int32_t *sweeps_out,
                    int32_t max_sweeps, double tol_factor, int accumulate, int mode,
                    int ordering, void *workspace, size_t ws_bytes, void *stream) {
  hipStream_t st = (hipStream_t)stream;
  if (dtype == 1)
    return sweep_impl<double>(1, nmat, n_host, off_host, (double *)G, (double *)U, (double *)V,
                              (double *)sigma, sweeps_out, max_sweeps, tol_factor, accumulate,
                              mode, ordering, workspace, ws_bytes, st, false);
  if (dtype == 0)
    return sweep_impl<float>(0, nmat, n_host, off_host, (float *)G, (float *)U, (float *)V,
                             (float *)sigma, sweeps_out, max_sweeps, tol_factor, accumulate, mode,
                             ordering, workspace, ws_bytes, st, false);
  return fail(KSVD2_EDTYPE, "dtype must be 0 (f32) or 1 (f64), got %d", dtype);
}

int kog_sweep_batch_noalloc(int dtype, int64_t nmat, const int32_t *n_host,
                            const int64_t *off_host, void *G, void *U, void *V, void *sigma,
                            int32_t *sweeps_out, int32_t max_sweeps, double tol_factor,
                            int accumulate, int mode, int ordering, void *stream) {
  if (mode == 2)
    return fail(KSVD2_EINVAL, "kog_sweep_batch_noalloc takes modes 0 and 1 (a graph of "
                              "mode 2 would be instantiated, which may allocate)");
  if (dtype != 0 && dtype != 1)
    return fail(KSVD2_EDTYPE, "dtype must be 0 (f32) or 1 (f64), got %d", dtype);
  if (nmat == 0) return KSVD2_OK;
  void *ws = nullptr;
  int rc = scratch_address(&ws);
  if (rc) return rc;
  hipStream_t st = (hipStream_t)stream;
  // the step table shrinks (fewer steps per U/V update, the same results) until the
  // call's workspace fits the scratch; a batch that does not fit even then is refused
  if (dtype == 1)
    rc = sweep_impl<double>(1, nmat, n_host, off_host, (double *)G, (double *)U, (double *)V,
                            (double *)sigma, sweeps_out, max_sweeps, tol_factor, accumulate,
                            mode, ordering, ws, kScratchBytes, st, true);
  else
    rc = sweep_impl<float>(0, nmat, n_host, off_host, (float *)G, (float *)U, (float *)V,
                           (float *)sigma, sweeps_out, max_sweeps, tol_factor, accumulate, mode,
                           ordering, ws, kScratchBytes, st, true);
  if (rc == KSVD2_EWORKSPACE)
    return fail(KSVD2_EWORKSPACE,
                "kog_sweep_batch_noalloc: the batch needs more than the %zu bytes of static "
                "scratch (%s); use kog_sweep_batch with a workspace",
                kScratchBytes, last_error_ref().c_str());
  return rc;
}

int kog_sweep_set_tuning(int dtype, int bucket, int knob, int value) {
  if (dtype != 0 && dtype != 1) return fail(KSVD2_EDTYPE, "dtype must be 0 or 1");
  if (bucket < -1 || bucket > 4) return fail(KSVD2_EINVAL, "bucket must be in [-1, 4]");
  int rc = tune_check(knob, value);
  if (rc) return rc;
  std::lock_guard<std::mutex> lk(g_mu);
  for (int b = 0; b < 5; ++b)
    if (bucket == -1 || bucket == b) g_tune.v[dtype][b][knob] = value;
  return KSVD2_OK;
}

int kog_sweep_tune(int dtype, int bucket, int block) {
  if (bucket < 0) return fail(KSVD2_EINVAL, "bucket must be in [0, 4]");
  return kog_sweep_set_tuning(dtype, bucket, K_BLOCK, block);
}

int kog_sweep_get_tuning(int dtype, int bucket, int knob) {
  if (dtype != 0 && dtype != 1) return fail(KSVD2_EDTYPE, "dtype must be 0 or 1");
  if (bucket < 0 || bucket > 4) return fail(KSVD2_EINVAL, "bucket must be in [0, 4]");
  if (knob < 0 || knob >= K_NKNOB) return fail(KSVD2_EINVAL, "unknown knob %d", knob);
  std::lock_guard<std::mutex> lk(g_mu);
  return g_tune.v[dtype][bucket][knob];
}

int kog_sweep_reset_tuning(void) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_tune = default_tune();
  return KSVD2_OK;
}

int kog_sigma_grad(int dtype, int64_t nmat, const int32_t *n_host, const int64_t *off_host,
                   const void *U, const void *V, const void *dsigma, void *dG, void *workspace,
                   size_t ws_bytes, void *stream) {
  hipStream_t st = (hipStream_t)stream;
  if (dtype == 1)
    return sigma_grad_impl<double>(nmat, n_host, off_host, (const double *)U, (const double *)V,
                                   (const double *)dsigma, (double *)dG, workspace, ws_bytes, st);
  if (dtype == 0)
    return sigma_grad_impl<float>(nmat, n_host, off_host, (const float *)U, (const float *)V,
                                  (const float *)dsigma, (float *)dG, workspace, ws_bytes, st);
  return fail(KSVD2_EDTYPE, "dtype must be 0 (f32) or 1 (f64), got %d", dtype);
}

int kog_sweep_sort(int dtype, int64_t nmat, const int32_t *n_host, const int64_t *off_host,
                   void *U, void *V, void *sigma, void *workspace, size_t ws_bytes, void *stream) {
  hipStream_t st = (hipStream_t)stream;
  if (dtype == 1)
    return sort_impl<double>(nmat, n_host, off_host, (double *)U, (double *)V, (double *)sigma,
                             workspace, ws_bytes, st);
  if (dtype == 0)
    return sort_impl<float>(nmat, n_host, off_host, (float *)U, (float *)V, (float *)sigma,
                            workspace, ws_bytes, st);
  return fail(KSVD2_EDTYPE, "dtype must be 0 (f32) or 1 (f64), got %d", dtype);
}

}  // extern "C"
