/*
 * ksvd2.h -- C ABI of libksvd2.so: the enhanced Kogbetliantz SVD of real 2x2
 * matrices (V. Novakovic, "Arithmetical enhancements of the Kogbetliantz
 * method for the SVD of order two", arXiv 2407.13116), batched on an AMD
 * Instinct MI355X (gfx950), its adjoint, and a batched two-sided Kogbetliantz
 * sweep built on it.
 *
 * Conventions common to every entry point
 * ---------------------------------------
 *  - G = U Sigma V^T with U, V orthogonal and sigma_1 >= sigma_2 >= 0
 *    (Sect. 1, the definition of the SVD).
 *  - Every pointer argument is device memory owned by the caller (for example
 *    the storage of a torch tensor), aligned to its element size, and the
 *    arrays must not overlap unless stated.  The library allocates nothing
 *    per call and keeps no reference to the arrays after the call returns.
 *  - `stream` is a hipStream_t (NULL selects the null stream).  Calls only
 *    enqueue work: they are asynchronous and ordered on that stream; results
 *    are valid once the stream has been synchronised.
 *  - dtype codes: 0 = binary32 (float), 1 = binary64 (double).
 *  - Return value: 0 on success, or a negative status; the matching message
 *    is available from ksvd2_last_error() (per host thread):
 *      KSVD2_EINVAL (-1)  invalid argument (negative size, null or misaligned
 *                         required pointer, tau < 0, ...), nothing enqueued
 *      KSVD2_EDTYPE (-2)  unsupported dtype code, nothing enqueued
 *      KSVD2_EHIP   (-3)  the HIP runtime reported an error at launch
 *      KSVD2_EWORKSPACE (-4) a workspace is smaller than required
 *    A batch of size 0 is a no-op that returns 0.
 *  - Inputs must be finite (Sect. 2).  A non-finite matrix is not an error:
 *    its info word gets bit 15 and its outputs are NaN.
 *  - Results are bitwise reproducible (Sect. 3.3.2, the reproducibility
 *    remark): they depend only on the input bits, not on the launch.
 */
#ifndef KSVD2_H
#define KSVD2_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define KSVD2_OK 0
#define KSVD2_EINVAL (-1)
#define KSVD2_EDTYPE (-2)
#define KSVD2_EHIP (-3)
#define KSVD2_EWORKSPACE (-4)

/* Bits of the per-matrix info word written by the forward entry points. */
#define KSVD2_INFO_TYPE_MASK 0x0000000Fu      /* t: zero pattern before scaling (eq. ts)  */
#define KSVD2_INFO_TYPE1_SHIFT 4              /* t': zero pattern after scaling (Sect. 3.1) */
#define KSVD2_INFO_DET_U (1u << 8)            /* det U = -1                               */
#define KSVD2_INFO_DET_V (1u << 9)            /* det V = -1                               */
#define KSVD2_INFO_EXT (1u << 10)             /* an element of R by eq. (EXT)             */
#define KSVD2_INFO_RSWAP (1u << 11)           /* r11 < r22: R^T permuted (eq. RT)         */
#define KSVD2_INFO_TPSI_OVF (1u << 12)        /* tan(psi) overflowed (eq. tp')            */
#define KSVD2_INFO_PSIGMA (1u << 13)          /* sigma~'' reordered, P_sigma = X (Alg. tp) */
#define KSVD2_INFO_DEGENERATE (1u << 14)      /* r12 or r22 became 0 in the URV (Sect. 3.2.2) */
#define KSVD2_INFO_NONFINITE (1u << 15)       /* non-finite input; outputs are NaN         */
#define KSVD2_INFO_SCALE_SHIFT 16             /* bits 16..31: s of eq. (s) as int16        */

/* Library version (incremented on ABI changes). */
int ksvd2_version(void);

/* Message of the last failed call on this host thread ("" if none). */
const char *ksvd2_last_error(void);

/*
 * ksvd2_batch_f64 / ksvd2_batch_f32 -- the enhanced Kogbetliantz SVD of `batch`
 * independent real 2x2 matrices (Sect. 3: prescaling and the simple classes,
 * Sect. 3.1; the URV factorisation, Sect. 3.2 and eq. EXT; the SVD of the
 * triangular factor, Algorithms tf and tp; assembly with the left-vector
 * heuristic and backscaling, Sect. 3.3.2).
 *
 * Layout: structure of arrays.  Each argument is a plane of `batch` elements;
 * matrix k is G_k = [g11[k] g12[k]; g21[k] g22[k]].
 * Outputs (all required except the two plain-sigma planes):
 *   cu, su   U_k = [cu -d su; su d cu] with d = -1 if info bit 8 else +1
 *   cv, sv   V_k = [cv -d sv; sv d cv] with d = -1 if info bit 9 else +1
 *   f1, e1   sigma_1 = f1 * 2^e1 with 1 <= f1 < 2, or f1 = 0 and e1 = 0
 *   f2, e2   sigma_2 likewise, sigma_1 >= sigma_2 >= 0.  The (e,f) form of
 *            Sect. 2 cannot overflow or underflow (Sect. 3.3.2).
 *   info     the bits above
 *   s1_plain, s2_plain (nullable): sigma_i rounded once to the working
 *            precision (may overflow to +inf or underflow).
 * Zeros in cu, su, cv, sv are +0.
 * Outputs must not alias inputs.
 */
int ksvd2_batch_f64(int64_t batch, const double *g11, const double *g21, const double *g12,
                    const double *g22, double *cu, double *su, double *cv, double *sv,
                    double *f1, double *f2, int32_t *e1, int32_t *e2, int32_t *info,
                    double *s1_plain, double *s2_plain, void *stream);
int ksvd2_batch_f32(int64_t batch, const float *g11, const float *g21, const float *g12,
                    const float *g22, float *cu, float *su, float *cv, float *sv, float *f1,
                    float *f2, int32_t *e1, int32_t *e2, int32_t *info, float *s1_plain,
                    float *s2_plain, void *stream);

/*
 * ksvd2_batch_fast_f64 / ksvd2_batch_fast_f32 -- the variant of the method for
 * a hypot that is not correctly rounded (Algorithm tf's branch for that case,
 * Sect. 3.2): every hypot is hi * sqrt(1 + (lo/hi)^2) with each operation
 * correctly rounded (a few ulps from the exact value; see ksvd2_hypot_fast_batch),
 * and tan(2 phi) of the triangular factor is formed from the quotients of
 * r12 (or r11) and r22 by the larger of r11, r12, without squaring.  The paper
 * gives no relative error bound for this variant.  Arguments, layout, ownership,
 * info words and errors as for ksvd2_batch_f64 / ksvd2_batch_f32.
 */
int ksvd2_batch_fast_f64(int64_t batch, const double *g11, const double *g21, const double *g12,
                         const double *g22, double *cu, double *su, double *cv, double *sv,
                         double *f1, double *f2, int32_t *e1, int32_t *e2, int32_t *info,
                         double *s1_plain, double *s2_plain, void *stream);
int ksvd2_batch_fast_f32(int64_t batch, const float *g11, const float *g21, const float *g12,
                         const float *g22, float *cu, float *su, float *cv, float *sv, float *f1,
                         float *f2, int32_t *e1, int32_t *e2, int32_t *info, float *s1_plain,
                         float *s2_plain, void *stream);

/*
 * ksvd2c_batch -- the complex 2x2 SVD (Sect. 3.4): G = U diag(sigma) V^H for
 * `batch` complex matrices.  A real G takes the real method above (U, V real);
 * a purely imaginary G the real method on Im(G), with U multiplied by i.
 * Otherwise every element that is made real goes through its unit phase g/|g|
 * into a diagonal phase matrix (the complex counterpart of the sign matrices)
 * and is replaced by its correctly rounded modulus; the prescaling uses s + 1
 * for the scale type of every class and the exponents of both parts; the
 * triangular factor is the real [|r11| |r12|; 0 |r22|] handled by Algorithms
 * tf and tp; U_+ is formed explicitly; no wider datatype is used (no eq. EXT),
 * so sigma_2 of a general complex matrix is accurate relative to sigma_1, not
 * to itself.
 * Layout: G, U, V are [batch][2][2] complex row-major arrays with the real and
 * imaginary parts interleaved (element (i,j) of matrix k at 8k + 2(2i + j)),
 * as complex64 / complex128 tensors store them; S is [batch][2] plain sigma
 * (sigma_1 >= sigma_2 >= 0, rounded once; may overflow where the (e,f) pair
 * does not); f, e (nullable) [batch][2] the pairs sigma = f 2^e, f in [1,2);
 * info (nullable) [batch]: bits 0-3 the type t of the complex zero pattern,
 * 4-7 t', bits 11-15 as for ksvd2_batch_*, bits 16-31 the prescaling exponent
 * s (real and imaginary inputs: the real method's info word).  Entries of U and
 * V that are zero are +0.  Non-finite input: NaN outputs, bit 15, status 0.
 * dtype: 0 = complex64 (float parts), 1 = complex128 (double parts).  All
 * pointers are caller-owned device memory aligned to the part type (4 or 8
 * bytes); status codes as for ksvd2_batch_*.
 */
int ksvd2c_batch(int dtype, int64_t batch, const void *G, void *U, void *S, void *V, void *f,
                 int32_t *e, int32_t *info, void *stream);

/*
 * ksvd2_svd2x2 -- the same SVD in the layout of an autograd graph: G, U, V are
 * [batch,2,2] row-major arrays (element (i,j) of matrix k at 4k + 2i + j), S is
 * [batch,2] with the plain singular values (rounded once to the working
 * precision).  `info` (nullable) receives the info words.  U and V are the full
 * matrices of ksvd2_batch_*, bit for bit.  dtype: 0 = float, 1 = double.
 */
int ksvd2_svd2x2(int dtype, int64_t batch, const void *G, void *U, void *S, void *V,
                 int32_t *info, void *stream);

/*
 * ksvd2_batch_backward -- the adjoint of G = U diag(sigma) V^T on the planes of
 * ksvd2_batch_f64 / ksvd2_batch_f32 (the standard SVD adjoint,
 *   dG = U [diag(dsigma) + (F o (J - J^T)) Sigma + Sigma (F o (K - K^T))] V^T,
 *   J = U^T dU, K = V^T dV, F_ij = 1/(s_j^2 - s_i^2) (i != j),
 * written out for order two with a = J12 - J21, b = K12 - K21, p = (a+b)/2,
 * q = (a-b)/2:  M12 = -p/(s1-s2) + q/(s1+s2), M21 = -p/(s1-s2) - q/(s1+s2),
 * dG = U [[ds1, M12], [M21, ds2]] V^T).  The paper defines the forward map
 * (Sect. 1, G = U Sigma V^T; Sect. 3.3.2 for the delivered factors); the adjoint
 * is textbook calculus on it.
 * Inputs (planes of `batch` elements, as the forward entry points write them):
 *   cu, su, cv, sv, info  U = [cu -d su; su d cu], d = -1 if info bit 8 else
 *                         +1; V likewise with info bit 9 (the other info bits
 *                         are ignored)
 *   s1, s2                the plain singular values (s1_plain, s2_plain)
 *   ds1, ds2              upstream gradient of sigma (each nullable: 0)
 *   dU, dV                upstream gradients of U and V (nullable: 0), each
 *                         four consecutive planes [4][batch] holding the
 *                         entries (1,1), (2,1), (1,2), (2,2) of every matrix
 * Outputs: dg11, dg21, dg12, dg22, the four planes of dG (required; they must
 * not alias the inputs).
 * Degenerate singular values: with tau > 0, 1/(s1-s2) is replaced by
 * (s1-s2)/((s1-s2)^2 + (tau s1)^2) (Lorentzian broadening); with tau = 0 the
 * exact formula is used and the p-term is dropped only when s1 - s2 == 0.  The
 * q-term needs 1/(s1+s2) only, so s2 = 0 < s1 is finite; s1 = s2 = 0 gives
 * M = diag(ds).  tau < 0 is KSVD2_EINVAL.  dtype: 0 = float, 1 = double.
 * The result equals, bit for bit, ksvd2_svd2x2_backward on the full matrices.
 */
int ksvd2_batch_backward(int dtype, int64_t batch, const void *cu, const void *su,
                         const void *cv, const void *sv, const int32_t *info, const void *s1,
                         const void *s2, const void *ds1, const void *ds2, const void *dU,
                         const void *dV, void *dg11, void *dg21, void *dg12, void *dg22,
                         double tau, void *stream);

/*
 * ksvd2_svd2x2_backward -- the same adjoint in the layout of ksvd2_svd2x2 (the
 * layout of an autograd graph): U, V, dU, dV, dG are [batch,2,2] row-major,
 * S and dS are [batch,2].  dS, dU, dV are nullable (a null pointer means a
 * zero upstream gradient).  Degenerate handling, tau and errors as for
 * ksvd2_batch_backward.  dtype: 0 = float, 1 = double.
 */
int ksvd2_svd2x2_backward(int dtype, int64_t batch, const void *U, const void *S, const void *V,
                          const void *dS, const void *dU, const void *dV, void *dG, double tau,
                          void *stream);

/*
 * ksvd2_hypot_batch -- the correctly rounded hypot(x, y) = fl(sqrt(x^2 + y^2))
 * of Sect. 2 (never overflows spuriously, zero iff both arguments are zero),
 * elementwise over n elements, as used inside the SVD.  Exposed so that the
 * primitive itself can be checked on the device.  dtype: 0 = float, 1 = double.
 */
int ksvd2_hypot_batch(int dtype, int64_t n, const void *x, const void *y, void *out,
                      void *stream);

/*
 * ksvd2_hypot_fast_batch -- the hypot of the fast variant: with hi = max(|x|,
 * |y|) and lo = min(|x|, |y|), fl(hi * fl(sqrt(fl(fma(r, r, 1))))) where r =
 * fl(lo / hi); hi itself when hi is 0 or infinite.  Not correctly rounded (its
 * error is a few ulps), and it may overflow when hi is within a few ulps of the
 * largest finite value.  Arguments and errors as for ksvd2_hypot_batch.
 */
int ksvd2_hypot_fast_batch(int dtype, int64_t n, const void *x, const void *y, void *out,
                           void *stream);

/*
 * kog_sweep_batch -- the two-sided Kogbetliantz iteration (Sect. 1, eq. SVD) on
 * `nmat` independent square matrices of even orders n_k (2 <= n_k <= 8192, at
 * most 65535 matrices): in each parallel step the n_k/2 disjoint pivots of the
 * chosen ordering are diagonalised by the 2x2 SVD above (U_p, sigma,
 * V_p; sigma rounded once to W), U_p^T is applied to the pivot rows of G, then
 * V_p to the pivot columns (each element pair as fma(a, x, b*y)), the pivot
 * block is set to diag(sigma_1, sigma_2), and U <- U U_p, V <- V V_p on the
 * pivot columns.  A sweep is n_k - 1 steps (every pair meets once); after each
 * sweep the iteration stops once ||offdiag(G)||_F <= tol_factor n_k eps ||G_0||_F
 * (eps = 2^-53 or 2^-24; tol_factor < 0 disables the test), or after
 * max_sweeps sweeps.
 *
 * Layout: matrix k is column-major at element offset off_host[k] of G, U and
 * V (the caller packs them; the matrices must not overlap).  n_host and
 * off_host are host arrays of nmat entries.
 *   G        in: the matrices; out: the final iteration matrices (their
 *            diagonals are the singular values, unsorted, non-negative)
 *   U, V     out: the accumulated transformations (in/out when accumulate != 0:
 *            the iteration then continues from the given U, V, e.g. to resume)
 *   sigma    (nullable) out: diag(G) of matrix k at offset n_0 + ... + n_{k-1}
 *   sweeps_out (nullable, device int32[nmat]): sweeps performed, negated when
 *            the stopping test was not met within max_sweeps
 * mode: 0 = plain per-step launches (the host polls convergence once per sweep,
 *           so the call returns after the work is done);
 *       1 = persistent kernels (one workgroup per matrix, one launch per order
 *           bucket), asynchronous; a workgroup keeps the step's parameters in
 *           LDS, which bounds the order (on MI355X, with 160 KB per workgroup:
 *           n <= 3,200 in binary64, n <= 6,200 in binary32); larger orders
 *           return KSVD2_EINVAL naming mode 0, which takes every order;
 *       2 = mode 1 captured into a hipGraph on first use and replayed on later
 *           calls with identical arguments (needs a non-null stream).
 * ordering: 0 = round-robin (circle method: index 0 fixed, 1..n-1 rotate by one
 *           position per step, positions s and n-1-s meet);
 *           1 = modified modulus (the strategy Sect. 4 names for the order-n
 *           iteration): with m = n-1, step k pairs the indices below m whose sum
 *           is k mod m, and the index c with 2c = k mod m with m.
 *           Both visit every pair once per sweep, in different step orders.
 *           2 = dynamic (Sect. 1 names dynamic orderings for non-cyclic parallel
 *           strategies): every step takes a greedy matching of the current G on
 *           the weights w_ij = fma(x_ij, x_ij, x_ji * x_ji) (binary64, x = G
 *           2^-t as for the stopping test), pairs by decreasing weight, equal
 *           weights by the smaller index, then the larger; a sweep is n-1 such
 *           steps.  One step per pass of G (the two-step passes need ordering 1).
 * All modes perform the same arithmetic in the same order: bitwise identical.
 * workspace: device memory of at least kog_sweep_workspace_size() bytes (an
 * amount that covers every mode, ordering and tuning; a call checks only what
 * it uses), 256-byte aligned, owned by the caller, used only during the call's
 * work: the batch descriptor, the counters, the step table (the parameters of
 * up to 128 steps of every pivot), the pair table (mode 0, ordering 2), and a second buffer,
 * of G's size at most, through which the persistent modes update G two steps
 * at a time under the modified modulus ordering.
 * Overflow: G is first multiplied by 2^s_G with s_G = e_nu - 2 - e_G - ceil(lg n)
 * when that is negative (e_G the largest exponent of its entries, e_nu that of
 * the largest finite value), so no two-sided update can overflow, and scaled
 * back on exit; the stopping test takes its norms of G 2^-t (t the largest
 * exponent after the scaling).  Status codes as above; an invalid mode or
 * ordering is KSVD2_EINVAL.
 */
int kog_sweep_batch(int dtype, int64_t nmat, const int32_t *n_host, const int64_t *off_host,
                    void *G, void *U, void *V, void *sigma, int32_t *sweeps_out,
                    int32_t max_sweeps, double tol_factor, int accumulate, int mode,
                    int ordering, void *workspace, size_t ws_bytes, void *stream);

/*
 * kog_sweep_batch_noalloc -- kog_sweep_batch for callers that cannot allocate
 * device memory (code under graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): the same iteration, bit for bit the same results, with the
 * workspace taken from a static device array of KOG_SWEEP_NOALLOC_SCRATCH_BYTES
 * (64 MiB) that each GPU holds from the library's first call on it until the
 * process ends.  The call allocates nothing; the caller still owns G, U, V,
 * sigma and sweeps_out.  Arguments as for kog_sweep_batch without the workspace;
 * modes 0 and 1 only (mode 2 is KSVD2_EINVAL: instantiating its graph may
 * allocate).  When the step table of 128 steps does not fit, fewer steps per U/V
 * update are used (down to 2; the results do not change); a batch whose
 * workspace exceeds the scratch even then returns KSVD2_EWORKSPACE with a
 * message naming kog_sweep_batch.  Every call on one GPU shares that GPU's
 * scratch and leaves its contents behind (the next call re-initialises what it
 * reads): calls that overlap on one GPU (other streams or host threads) race
 * and must be serialised by the caller.
 */
#define KOG_SWEEP_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int kog_sweep_batch_noalloc(int dtype, int64_t nmat, const int32_t *n_host,
                            const int64_t *off_host, void *G, void *U, void *V, void *sigma,
                            int32_t *sweeps_out, int32_t max_sweeps, double tol_factor,
                            int accumulate, int mode, int ordering, void *stream);

/*
 * kog_sweep_sort -- the delivered singular values in the usual order: for each
 * matrix of a kog_sweep_batch result, sigma (packed as kog_sweep_batch writes
 * it, on entry the iterate's diagonal) is put in descending order, equal values
 * keeping their index order, and the columns of U and V are permuted the same
 * way, all in place, so that G_0 = U diag(sigma) V^T with sigma_1 >= sigma_2 >=
 * ... >= 0.  The paper takes sigma_i as the diagonal of the final iterate (Sect.
 * 1, eq. SVD) without ordering them; this is the ordering convention on top.
 * G is not touched, so an iteration resumed with `accumulate` needs the U and V
 * from before this call.  Layouts and workspace as for kog_sweep_batch; orders
 * up to 8192 (an order's values, ranks and one row of U must fit a workgroup's
 * LDS).  Status codes as above.
 */
int kog_sweep_sort(int dtype, int64_t nmat, const int32_t *n_host, const int64_t *off_host,
                   void *U, void *V, void *sigma, void *workspace, size_t ws_bytes, void *stream);

/*
 * Rectangular inputs (Sect. 1): an m x n matrix with m >= n is reduced to a
 * square triangular one by the QR factorization with column pivoting, G P =
 * Q R; kog_sweep_batch then takes R (n even) and kog_qrcp_apply forms the
 * factors of G, U = Q [U_R; 0] (m x n, orthonormal columns) and V = P V_R.
 * (For m < n, factor G^T.)
 *
 * kog_qrcp_batch -- in place on A (matrix k column-major m_k x n_k at element
 * offset aoff_host[k]; 1 <= n_k <= 4096, m_k >= n_k): Householder reflections
 * H_j = I - tau_j v_j v_j^T with v_j(j) = 1, v_j stored below the diagonal of
 * column j and R on and above it (the layout of LAPACK's geqp3).  At step j
 * the trailing column of largest norm (rows j..m-1, recomputed at every step;
 * the first one on ties) is exchanged into place; the reflector maps it onto
 * beta e_j with beta = -sign(x_j) ||x||.  tau and perm are packed by matrix
 * at n_0 + ... + n_{k-1}; perm[j] is the column of G that became column j of
 * G P.  Rsq receives the n_k x n_k triangular factor, zeros below the diagonal,
 * column-major at element offset roff_host[k] (ready for kog_sweep_batch).
 * Entries must keep the squared column norms finite.
 *
 * kog_qrcp_apply -- from kog_qrcp_batch's A, tau, perm and the SVD factors
 * U_R, V_R of R (n_k x n_k at roff_host[k], e.g. from kog_sweep_batch and
 * kog_sweep_sort), writes U = H_0 ... H_{n-1} [U_R; 0] (m_k x n_k at
 * aoff_host[k] of U) and V = P V_R (n_k x n_k at roff_host[k] of V).  perm must
 * be the one kog_qrcp_batch wrote.
 *
 * Both: m_host, n_host, aoff_host, roff_host are host arrays of nmat entries
 * (at most 65535 matrices); every other pointer is caller-owned device memory;
 * workspace: at least kog_rect_workspace_size(nmat) bytes, 256-byte aligned;
 * stream-ordered; status codes as above.
 */
size_t kog_rect_workspace_size(int64_t nmat);
int kog_qrcp_batch(int dtype, int64_t nmat, const int32_t *m_host, const int32_t *n_host,
                   const int64_t *aoff_host, const int64_t *roff_host, void *A, void *tau,
                   int32_t *perm, void *Rsq, void *workspace, size_t ws_bytes, void *stream);
int kog_qrcp_apply(int dtype, int64_t nmat, const int32_t *m_host, const int32_t *n_host,
                   const int64_t *aoff_host, const int64_t *roff_host, const void *A,
                   const void *tau, const int32_t *perm, const void *UR, const void *VR, void *U,
                   void *V, void *workspace, size_t ws_bytes, void *stream);

/* Bytes of workspace kog_sweep_batch and kog_sigma_grad need for this batch
   (0 for invalid arguments). */
size_t kog_sweep_workspace_size(int dtype, int64_t nmat, const int32_t *n_host);

/*
 * Tuning table of kog_sweep_batch's persistent modes, per dtype and order
 * bucket (0: n <= 64, 1: n <= 128, 2: n <= 256, 3: n <= 512, 4: larger).
 * Process-wide; set by the autotuner.  Results do not depend on it: every
 * setting performs the same arithmetic in the same order.  Knobs:
 *   KOG_TUNE_BLOCK   (0) lanes per workgroup (one workgroup per matrix): 256,
 *                        512 or 1024; defaults 256, 512, 512, 512, 1024
 *                        (binary64) and 256, 512, 512, 1024, 1024 (binary32)
 *   KOG_TUNE_CHUNK   (1) steps whose U/V rotations are applied together, a
 *                        power of two in [2, 128] (default 128); a call uses
 *                        the entry of the bucket of its largest order; it sets
 *                        the size of the step table in the workspace
 *   KOG_TUNE_TWO     (2) 1 (default): two steps of G per pass under the
 *                        modified modulus ordering; 0: one step per pass
 *   KOG_TUNE_INPLACE (3) 1 (default): that pass in place for orders up to 256
 *                        in workgroups of up to 512 lanes; 0: through the
 *                        second buffer
 *   KOG_TUNE_ROWS    (4) size the U/V tile's own LDS for at most this many
 *                        rows of the largest order (0, the default: as many as
 *                        fit), which leaves LDS for more workgroups per compute
 *                        unit; a U/V update also spreads over the LDS of the
 *                        step parameters
 * kog_sweep_set_tuning sets `knob` of `bucket` (-1: of every bucket) and returns
 * KSVD2_EINVAL for a value out of range; kog_sweep_get_tuning returns the entry
 * (or a negative status); kog_sweep_reset_tuning restores the defaults;
 * kog_sweep_tune(dtype, bucket, block) is kog_sweep_set_tuning(dtype, bucket,
 * KOG_TUNE_BLOCK, block).
 */
#define KOG_TUNE_BLOCK 0
#define KOG_TUNE_CHUNK 1
#define KOG_TUNE_TWO 2
#define KOG_TUNE_INPLACE 3
#define KOG_TUNE_ROWS 4
int kog_sweep_set_tuning(int dtype, int bucket, int knob, int value);
int kog_sweep_get_tuning(int dtype, int bucket, int knob);
int kog_sweep_reset_tuning(void);
int kog_sweep_tune(int dtype, int bucket, int block);

/*
 * kog_sigma_grad -- the gradient of sum_i dsigma_i sigma_i with respect to G
 * for the SVD G = U diag(sigma) V^T delivered by kog_sweep_batch:
 * dG = U diag(dsigma) V^T (d sigma_i / dG = u_i v_i^T).  Layouts as in
 * kog_sweep_batch (U, V, dG column-major at off_host[k]; dsigma packed like
 * sigma); workspace as for kog_sweep_batch.
 */
int kog_sigma_grad(int dtype, int64_t nmat, const int32_t *n_host, const int64_t *off_host,
                   const void *U, const void *V, const void *dsigma, void *dG, void *workspace,
                   size_t ws_bytes, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* KSVD2_H */
