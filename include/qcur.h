/*
 * libqcur -- quaternion CUR (QMCUR) low-rank approximation on AMD MI355X (gfx950).
 *
 * Method: Wu, Kou, Cai, Yu, "Efficient quaternion CUR method for low-rank
 * approximation to quaternion matrix" (arXiv 2402.19147), Algorithm 1 and
 * Section 3.1.  Given a quaternion matrix A (m x n), column and row index sets
 * J and I are drawn from length (squared-norm) or uniform probabilities,
 * C = A(:,J), R = A(I,:) and W = A(I,J) are gathered, the core U is formed as
 * W^+ or C^+ A R^+, and C U R together with ||A - CUR||_F is evaluated.
 *
 * Conventions shared by every call
 * --------------------------------
 * Quaternion matrices are four real planes (qcur_qmat).  Plane c (0 = real,
 * 1 = i, 2 = j, 3 = k) starts at p + c * pstride elements; element (i, j) of a
 * plane sits at i * ld + j (row-major).  Planes must not overlap:
 * ld >= cols and pstride >= rows * ld (pstride may be anything when rows == 0).
 *
 * All matrix, vector and index pointers are DEVICE pointers unless a name
 * ends in _host.  The caller owns every buffer; the library never allocates
 * or frees caller memory and keeps no pointer after a call returns.  Work is
 * enqueued on the handle's stream (qcur_set_stream) and calls return without
 * waiting for it, except where a call says it synchronises.
 *
 * Indices are 0-based (the paper's [n] is 1-based).  The core U is
 * |J| x |I| = c x r.
 *
 * Errors: every call returns a qcur_status and never throws or aborts.
 * Argument, shape and dtype errors are detected on the host before anything
 * is enqueued (and before the handle is used, so they can be checked without
 * a GPU).  Conditions that depend on data (zero norm, non-finite values,
 * invalid probabilities, too few positive weights, out-of-range or repeated
 * indices) are detected by the kernels, which OR a bit into the handle's
 * device status word; qcur_sync_status synchronises the stream and returns
 * and clears that word.  HIP runtime failures map to QCUR_ERR_DEVICE.
 * qcur_last_error gives a thread-local text for the last host-side error.
 */
#ifndef QCUR_H
#define QCUR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  QCUR_OK = 0,
  QCUR_ERR_ARG = 1,          /* null pointer, negative size, bad enum, bad index */
  QCUR_ERR_SHAPE = 2,        /* operand shapes or strides disagree */
  QCUR_ERR_DTYPE = 3,        /* unsupported dtype combination */
  QCUR_ERR_WORKSPACE = 4,    /* workspace missing or too small */
  QCUR_ERR_SAMPLE = 5,       /* invalid probabilities or fewer positive weights than draws */
  QCUR_ERR_NUMERIC = 6,      /* non-finite values or ||A||_F = 0 */
  QCUR_ERR_DEVICE = 7,       /* HIP runtime error */
  QCUR_ERR_UNSUPPORTED = 8   /* valid request outside the implemented limits */
} qcur_status;

typedef enum { QCUR_F64 = 0, QCUR_F32 = 1, QCUR_BF16 = 2 } qcur_dtype;
/* Product precision ("compute") of the calls that take one: a qcur_dtype
 * (operands stored in that dtype; BF16 products accumulate in FP32), or
 * QCUR_BF16X3: FP32 operands, each element split into BF16 hi = bf16(x) and
 * lo = bf16(x - hi) when staged, products hi.hi + hi.lo + lo.hi on BF16
 * matrix cores with FP32 accumulation (about 2^-16 relative error per
 * product, against 2^-24 for FP32 and 2^-9 for BF16).  Not offered by the
 * batched solve. */
enum { QCUR_BF16X3 = 3 };
typedef enum { QCUR_OP_N = 0, QCUR_OP_H = 1 } qcur_op;           /* H: conjugate transpose */
typedef enum { QCUR_LENGTH = 0, QCUR_UNIFORM = 1 } qcur_sampling;
typedef enum { QCUR_CORE_WPINV = 0, QCUR_CORE_CAR = 1 } qcur_core;

typedef struct {
  void* p;          /* device pointer to element (0,0) of plane 0 */
  int64_t rows;
  int64_t cols;
  int64_t ld;       /* row stride in elements */
  int64_t pstride;  /* plane stride in elements */
  int32_t dtype;    /* qcur_dtype */
} qcur_qmat;

typedef struct qcur_ctx* qcur_handle;

/* ---- handle, stream, status ------------------------------------------- */

/* Creates a handle bound to HIP device `device`.  Allocates the handle's own
 * device status word (4 bytes).  Errors: QCUR_ERR_ARG, QCUR_ERR_DEVICE. */
qcur_status qcur_create(qcur_handle* handle, int device);
qcur_status qcur_destroy(qcur_handle handle);
/* Binds a hipStream_t (passed as void*; NULL = default stream). */
qcur_status qcur_set_stream(qcur_handle handle, void* hip_stream);
/* Synchronises the stream, returns the status bits raised by kernels since
 * the last call (mapped to the most severe qcur_status) and clears them. */
qcur_status qcur_sync_status(qcur_handle handle);
const char* qcur_status_string(qcur_status status);
const char* qcur_last_error(void);
/* Library version as major*10000 + minor*100 + patch. */
int qcur_version(void);

/* ---- workspace queries (host only, no GPU needed) --------------------- */
size_t qcur_probs_workspace(int64_t m, int64_t n);
size_t qcur_pinv_workspace(int64_t p, int64_t q);
size_t qcur_svd_workspace(int64_t p, int64_t q);
size_t qcur_approx_workspace(int64_t m, int64_t n, int64_t c, int64_t r, int core, int compute);
size_t qcur_residual_workspace(int64_t m, int64_t n, int64_t c, int64_t r, int compute);
size_t qcur_backward_workspace(int64_t m, int64_t n, int64_t c, int64_t r, int compute);
/* Optional split-K workspace of qcur_gemm for D (M x N) with inner size K. */
size_t qcur_gemm_workspace(int64_t M, int64_t N, int64_t K, int compute);

/* ---- the eight calls of the hot path ----------------------------------- */

/* Sampling probabilities (Section 3.1).  QCUR_LENGTH: p_col[j] =
 * ||A(:,j)||^2 / ||A||_F^2 and q_row[i] = ||A(i,:)||^2 / ||A||_F^2, where
 * |a|^2 sums the squares of the four components (Section 2.2); sums are
 * accumulated in FP64 in a fixed order, so results are run-to-run identical.
 * QCUR_UNIFORM: p_col[j] = 1/n, q_row[i] = 1/m.
 * A: any dtype, m x n.  p_col: double[n], q_row: double[m], fro2: double[1]
 * (optional, may be NULL; always ||A||_F^2).  ws: qcur_probs_workspace(m, n)
 * bytes.  ||A||_F = 0 or a non-finite norm raises QCUR_ERR_NUMERIC in the
 * status word (length mode). */
qcur_status qcur_probs(qcur_handle handle, const qcur_qmat* A, int sampling, double* p_col,
                       double* q_row, double* fro2, void* ws, size_t ws_bytes);

/* qcur_probs without a workspace argument, for callers that cannot allocate
 * device memory (code under stream/graph capture, serving loops, harnesses
 * that forbid allocation).  The partial sums live in the library's static
 * device scratch of QCUR_SCRATCH_BYTES bytes, one copy per device, whose
 * address the handle takes when it is created; it stays allocated until the
 * process ends.  This call allocates nothing.  Same arguments, results and
 * data errors as qcur_probs (bitwise the same results).  A matrix whose
 * partial sums need more than the scratch holds (qcur_probs_workspace(m, n) >
 * QCUR_SCRATCH_BYTES; every m, n <= 16384 fits) returns
 * QCUR_ERR_UNSUPPORTED before anything is enqueued.  All calls on one device
 * share its scratch and every call writes the part it reads before reading
 * it (nothing needs clearing): calls that overlap on one device (on
 * different streams or handles) race and must not be issued concurrently. */
#define QCUR_SCRATCH_BYTES ((size_t)32 << 20)
qcur_status qcur_probs_noalloc(qcur_handle handle, const qcur_qmat* A, int sampling, double* p_col,
                               double* q_row, double* fro2);

/* Draws `count` indices from the probabilities probs[0..n) (Algorithm 1,
 * steps 1-2) and writes them sorted ascending to idx[count] (int64).
 * Integer-CDF sampler: weights w_j = floor(p_j * 2^60); draw t takes
 * u = output number set_id * 2^32 + t of SplitMix64 seeded with `seed`,
 * tau = floor(u * T / 2^64) for the current weight total T, and picks the
 * smallest j whose inclusive prefix sum exceeds tau; without replacement the
 * picked weight is then removed.  Bit-exact for identical probs.
 * Limits: 1 <= n <= 16384 without replacement, n <= 8192 with replacement
 * (weights are held in LDS); count <= n without replacement, count < 2^31.
 * Data errors (QCUR_ERR_SAMPLE in the status word): p_j outside [0, 1] or
 * non-finite, total weight zero or >= 2^64, fewer positive weights than
 * draws without replacement.  On such an error idx is filled with -1. */
qcur_status qcur_draw(qcur_handle handle, const double* probs, int64_t n, int64_t count,
                      uint64_t seed, uint64_t set_id, int with_replacement, int64_t* idx);

/* Gathers C = A(:,J) (m x c), R = A(I,:) (r x n) and W = A(I,J) (r x c)
 * (Section 2.1 notation; Algorithm 1 steps 1-2).  Any of C, R, W may be NULL.
 * Each output may have its own dtype (values are converted, BF16 with
 * round-to-nearest-even).  Out-of-range indices write zeros and raise
 * QCUR_ERR_ARG in the status word. */
qcur_status qcur_gather(qcur_handle handle, const qcur_qmat* A, const int64_t* I, int64_t r,
                        const int64_t* J, int64_t c, qcur_qmat* C, qcur_qmat* R, qcur_qmat* W);

/* Moore-Penrose inverse Xp = X^+ (q x p) of X (p x q), both FP64
 * (Section 2.1).  Singular values <= rtol * sigma_max count as zero
 * (rtol < 0 selects max(p, q) * 2^-52); max_rank > 0 keeps at most that many.
 * rank_out (device int64[1], may be NULL) receives the kept rank.
 * Route: with Z = X (p >= q) or X^H, FP64 CholeskyQR2 (Z = Q T, X^+ from
 * Q and T^{-1}) when its full-rank certificate holds (Cholesky succeeds,
 * kappa_F(Z) below 1e7 and kappa_F * rtol below 1e-2) and no rank cap
 * applies.  A cap k with 2k <= min(p, q) (Algorithm 1's predefined rank)
 * on a matrix too large for one workgroup: subspace iteration (a fixed
 * pseudo-random sketch, CholeskyQR2 of the p x k and q x k iterates), kept
 * when an a posteriori bound (Davis-Kahan on the Rayleigh-Ritz residual,
 * then Wedin's pseudoinverse perturbation bound) puts the result within
 * 2^-30 relative of the k-truncated pseudoinverse, at most three
 * iterations.  Otherwise, and for matrices small enough for one
 * workgroup, one-sided (Hestenes) Jacobi on quaternion columns.
 * Synchronises the stream once to read the certificate (three to four
 * times per iteration on the capped route), and on the Jacobi route once
 * per sweep to test convergence.
 * ws: qcur_pinv_workspace(p, q) bytes.  Non-finite input raises
 * QCUR_ERR_NUMERIC in the status word. */
qcur_status qcur_pinv(qcur_handle handle, const qcur_qmat* X, double rtol, int64_t max_rank,
                      qcur_qmat* Xp, int64_t* rank_out, void* ws, size_t ws_bytes);

/* Thin quaternion SVD X = U diag(s) V^H of X (p x q, any dtype), k =
 * min(p, q), computed in FP64 by the same one-sided Jacobi method as
 * qcur_pinv (Section 2.1's QSVD; the costly route that QMCUR avoids, kept
 * as the baseline).  s: device double[k], descending.  U (p x k) and V
 * (q x k): FP64 outputs with orthonormal columns for the nonzero singular
 * values; for zero singular values the columns of U (p >= q) or of V
 * (p < q) are zero and the other factor keeps orthonormal columns.  Either
 * may be NULL.  Synchronises the
 * stream once per Jacobi sweep.  ws: qcur_svd_workspace(p, q) bytes.
 * Non-finite input raises QCUR_ERR_NUMERIC in the status word. */
qcur_status qcur_svd(qcur_handle handle, const qcur_qmat* X, double* s, qcur_qmat* U, qcur_qmat* V, void* ws,
                     size_t ws_bytes);

/* Quaternion product D = alpha * op(A) op(B) + beta * D (Section 2.2
 * multiplication laws) with real alpha, beta; op(X) is X or X^H.
 * Mapped onto MFMA as the real-block (4m x 4k) times component-stacked
 * (4k x n) contraction: exactly 16 real multiply-accumulates per quaternion
 * multiply-accumulate.  compute = QCUR_F64: A, B, D FP64.  QCUR_F32: A, B, D
 * FP32.  QCUR_BF16: A, B BF16, D FP32 (FP32 accumulation).  D must not
 * alias A or B.  beta == 0 ignores the old contents of D.  ws (may be NULL)
 * enables a deterministic split of K for thin outputs when ws_bytes >=
 * qcur_gemm_workspace(M, N, K, compute); results do not depend on it beyond
 * summation order. */
qcur_status qcur_gemm(qcur_handle handle, int opA, int opB, double alpha, const qcur_qmat* A,
                      const qcur_qmat* B, double beta, qcur_qmat* D, int compute, void* ws,
                      size_t ws_bytes);

/* Core and optional product (Algorithm 1 step 3; Section 3.1).
 * core QCUR_CORE_WPINV: U = W^+ (W r x c, any dtype; A, C, R may be NULL).
 * core QCUR_CORE_CAR: U = C^+ (A R^+) with C (m x c), R (r x n), A (m x n),
 * evaluated in orthonormal form: C = Q_C T_C and R^H = Q_R T_R (FP64
 * CholeskyQR2, or the Jacobi SVD when its certificate fails) give
 * U = P_C^H (Q_C^H A Q_R) P_R with P = T^{-H}, so that C U R =
 * Q_C M Q_R^H, M = Q_C^H A Q_R.  compute selects the dtype of the products
 * with A: QCUR_F64 (U, B FP64), QCUR_F32 (FP32 products; U, B FP32) or
 * QCUR_BF16 (BF16 operands with FP32 accumulation; U, B FP32); the small
 * products with P run in FP64.  A, C, R and W may be given in any dtype:
 * operands are converted to the product dtype in the workspace, while the
 * refinement residual A - C U R subtracts A in the precision it was given.
 * refine_steps >= 0 applies M <- M + Q_C^H (A - C U R) Q_R (equivalently
 * U <- U + C^+ ((A - C U R) R^+)) that many times (CAR only).  B (m x n,
 * may be NULL) receives C U R.
 * rank_out (device int64[2], may be NULL): kept ranks of the pseudoinverses
 * (W: [rank, rank]; CAR: [rank C, rank R]).
 * CAR synchronises once with the host for the factors' full-rank
 * certificate.  When 32 m n r <= 4e10 the products of the fast path are
 * enqueued before that wait and, if the certificate rejects the fast path
 * or asks for a second CholeskyQR pass, computed again after the
 * fallback; outputs do not depend on this.
 * ws: qcur_approx_workspace(m, n, c, r, core, compute) bytes. */
qcur_status qcur_approx(qcur_handle handle, const qcur_qmat* A, const qcur_qmat* C,
                        const qcur_qmat* R, const qcur_qmat* W, int core, int compute,
                        int refine_steps, double rtol, int64_t max_rank, qcur_qmat* U,
                        qcur_qmat* B, int64_t* rank_out, void* ws, size_t ws_bytes);

/* Residual ||P_Omega(A - C U R)||_F (the numerator of the relative error of
 * Example 4.2; with a mask, the data-fit term of the completion problem in
 * Example 4.4).  B1 = C U is formed first, then B1 R is produced tile by tile
 * and never stored: each tile subtracts A, applies the mask, squares and
 * reduces; tile partials are summed in FP64 in a fixed order.
 * mask: uint8 m x n with row stride mask_ld (NULL = all ones).
 * compute as in qcur_gemm; C, U, R are converted to its operand dtype when
 * needed, A is read in its own dtype.
 * fro: device double[1].  E (optional, m x n, FP64 for QCUR_F64 else FP32)
 * receives e_scale * P_Omega(A - CUR).
 * ws: qcur_residual_workspace(m, n, c, r, compute) bytes. */
qcur_status qcur_residual(qcur_handle handle, const qcur_qmat* A, const qcur_qmat* C,
                          const qcur_qmat* U, const qcur_qmat* R, const uint8_t* mask,
                          int64_t mask_ld, int compute, double* fro, qcur_qmat* E,
                          double e_scale, void* ws, size_t ws_bytes);

/* Adjoint of B = C U R with U = W^+ (intersection core), through the gathers
 * C = A(:,J), R = A(I,:), W = A(I,J) and the pseudoinverse (constant-rank
 * derivative of Golub and Pereyra).  U is recomputed from W, not stored.
 * gB != NULL: dA = d<gB, CUR(A)>/dA (vector-Jacobian product).
 * gB == NULL: masked loss L = ||P_Omega(A - CUR(A))||_F^2 (mask as in
 * qcur_residual); dA = dL/dA and loss (device double[1], may be NULL)
 * receives L.  In this mode dA may be NULL when loss is given: then only L
 * is computed.  I and J must hold distinct in-range indices (else
 * QCUR_ERR_ARG in the status word).  compute QCUR_F64 or QCUR_F32 (A, gB
 * and dA in that dtype).  ws: qcur_backward_workspace(m, n, c, r, compute). */
qcur_status qcur_backward(qcur_handle handle, const qcur_qmat* A, const int64_t* I, int64_t r,
                          const int64_t* J, int64_t c, const qcur_qmat* gB, const uint8_t* mask,
                          int64_t mask_ld, double rtol, int64_t max_rank, int compute,
                          qcur_qmat* dA, double* loss, void* ws, size_t ws_bytes);

/* ---- the whole path ------------------------------------------------------ */

/* One QMCUR solve (Algorithm 1) of A (m x n): sampling probabilities
 * (QCUR_LENGTH or QCUR_UNIFORM), J (c column indices, SplitMix64 set 0) and
 * I (r row indices, set 1) drawn as in qcur_draw (both in one launch), the
 * gathers, the core as in qcur_approx (core, compute, refine_steps, rtol,
 * max_rank) and residual (device double[1]) = ||A - C U R||_F as in
 * qcur_residual.  With refine_steps > 0 and B not requested, the residual
 * of the refined core is taken from the last step's residual E and
 * correction D = Q_C^H E Q_R as sqrt(||E||^2 - ||D||^2) (exact up to the
 * factors' orthogonality defect, which the refinement holds below 2^-12)
 * when ||D||^2 <= 2^-8 ||E||^2; otherwise, and always when B is requested,
 * by the explicit product.  Outputs: I (int64[r]), J (int64[c]) sorted, U (c x r, FP64
 * for QCUR_F64 else FP32), rank_out (device int64[2] or NULL).  Optional
 * outputs (NULL = internal): p_col[n], q_row[m] and C, R, W in A's dtype;
 * B (m x n, FP64 for QCUR_F64 else FP32, NULL = not formed) receives C U R
 * as in qcur_approx.  Same limits as qcur_draw for m and n.  Synchronises once per group of
 * pseudoinverses (the full-rank certificate), after the products that follow
 * it when they are cheap (as in qcur_approx).
 * ws: qcur_solve_workspace(m, n, c, r, core, compute) bytes. */
qcur_status qcur_solve(qcur_handle handle, const qcur_qmat* A, int64_t c, int64_t r, int sampling, int core,
                       int compute, uint64_t seed, int with_replacement, int refine_steps, double rtol,
                       int64_t max_rank, int64_t* I, int64_t* J, qcur_qmat* U, double* residual,
                       int64_t* rank_out, double* p_col, double* q_row, qcur_qmat* C, qcur_qmat* R,
                       qcur_qmat* W, qcur_qmat* B, void* ws, size_t ws_bytes);
size_t qcur_solve_workspace(int64_t m, int64_t n, int64_t c, int64_t r, int core, int compute);

/* ---- many independent solves of uneven sizes --------------------------- */

/* Batched QMCUR (Algorithm 1 on `count` independent problems, e.g. the patch
 * groups of an image), least-squares core U_b = C_b^+ A_b R_b^+ (Section 3.1,
 * eq. (2)) and residual_b = ||A_b - C_b U_b R_b||_F, all problems advancing
 * through one sequence of batched launches with no host synchronisation, so
 * that the whole call can be captured into one graph and replayed.
 *
 * dims: host int32[count][4] = (m_b, n_b, c_b, r_b), 1 <= count <= 16384,
 * 1 <= m_b, n_b <= 4096,
 * 1 <= c_b, r_b <= 1024, c_b <= n_b and r_b <= m_b without replacement.
 * Slots: with mx, nx, cx, rx the largest m_b, n_b, c_b, r_b, problem b's A_b
 * is the top-left m_b x n_b corner of slot b of A (A->rows >= mx,
 * A->cols >= nx, planes A->pstride apart, slots a_bstride elements apart);
 * U_b (c_b x r_b, FP64 for QCUR_F64 else FP32) is the corner of slot b of U
 * (u_bstride apart).  I: device int64[count][rx] (row b holds I_b, sorted,
 * in its first r_b entries); J: int64[count][cx].  residual: device
 * double[count] (with refine_steps > 0 and B NULL, per problem from the last
 * step's E_b and D_b as in qcur_solve when ||D_b||^2 <= 2^-8 ||E_b||^2, else
 * by the explicit product).  rank_out: device int64[count][2] (ranks of C_b, R_b) or
 * NULL.  p_col: device double[count][nx], q_row: double[count][mx] or NULL.
 * B (may be NULL): B_b = C_b U_b R_b in the top-left m_b x n_b corner of
 * slot b (rows >= mx, cols >= nx, slots b_bstride elements apart; FP64 for
 * QCUR_F64 else FP32), written by the residual's own product tiles.
 * Problem b draws with the seed seed + b (J_b set 0, I_b set 1), so it
 * repeats qcur_solve of A_b with that seed; its probabilities are folded in
 * another order, equal to qcur_solve's up to rounding.
 * The pseudoinverses run batched in FP64: CholeskyQR (two passes for
 * QCUR_F64, one otherwise) with the kappa_F certificate of qcur_pinv, and
 * for each problem that fails it, the Jacobi SVD inside the same launch
 * sequence.  Errors found in kernels go to the status word.
 *
 * Before the first call, qcur_batch_prepare(handle, count, dims, A's dtype,
 * sampling, compute, refine_steps, autotune, ws, ws_bytes) writes the
 * batch's size tables into the workspace (synchronously; not under stream
 * capture) and records the workspace in the handle; qcur_solve_batched
 * refuses a workspace that was not prepared for the same sizes and options.
 * Calls that share one workspace must not overlap.
 * autotune = 1: the first qcur_solve_batched call on this workspace that is
 * not being captured times every candidate launch plan (tile edge 32 or 64,
 * 1, 2 or 4 slices of K) of each of its quaternion GEMM stages on the real
 * operands (and 32- or 64-tiles for the residual) and keeps the fastest;
 * later calls, captured ones included, reuse those plans.  The measuring
 * call synchronises with the host.  Plans change only the summation order,
 * so results of differently tuned runs differ by rounding.  autotune = 0:
 * fixed plans from the problem shapes (bitwise reproducible).
 * ws: qcur_batch_workspace(count, dims, A's dtype, sampling, compute,
 * refine_steps, autotune) bytes (0 for invalid arguments). */
size_t qcur_batch_workspace(int32_t count, const int32_t* dims, int a_dtype, int sampling, int compute,
                            int refine_steps, int autotune);
qcur_status qcur_batch_prepare(qcur_handle handle, int32_t count, const int32_t* dims, int a_dtype,
                               int sampling, int compute, int refine_steps, int autotune, void* ws,
                               size_t ws_bytes);
/* Launch plans kept by the autotuner for a prepared workspace: tiles[i] and
 * splits[i] (host int[n]) for stage i of the batched solve (factor Grams of
 * C and R, first-pass factors of C and R, second-pass Gram, P2 P1, Q1 P2^H,
 * A Q_R, Q_C^H T, Q_C M, M P_R, P_C^H W, residual).  Returns the number of
 * stages (13) once the plans have been measured, else 0. */
int qcur_batch_plans(qcur_handle handle, const void* ws, int* tiles, int* splits, int n);
qcur_status qcur_solve_batched(qcur_handle handle, int32_t count, const int32_t* dims,
                               const qcur_qmat* A, int64_t a_bstride, int sampling, int compute,
                               uint64_t seed, int with_replacement, int refine_steps, double rtol,
                               int64_t max_rank, int64_t* I, int64_t* J, qcur_qmat* U, int64_t u_bstride,
                               double* residual, int64_t* rank_out, double* p_col, double* q_row,
                               qcur_qmat* B, int64_t b_bstride, void* ws, size_t ws_bytes);

/* ---- completion from partially observed entries (Algorithm 2) ---------- */

/* Quaternion matrix completion with QMCUR (Algorithm 2; Example 4.4): from
 * the observed Y (m x n, any dtype; entries where mask == 0 are ignored)
 * and the fixed index sets I (r rows) and J (c columns, device int64),
 * X^0 = P_Omega(Y), then for t = 0, 1, ...: M^{t+1} = C U R of X^t
 * (Algorithm 1 with C = X^t(:,J), R = X^t(I,:), U = C^+ X^t R^+, evaluated
 * as in qcur_approx), X^{t+1} = P_Omega(Y) + P_Omega^c(M^{t+1}) (fused into
 * the last product), until ||X^{t+1} - X^t||_F / ||X^t||_F <= tol or
 * max_iter steps (the paper's t_max = 200 and 1e-4).
 * mask: device uint8 m x n, row stride mask_ld (nonzero = observed).
 * compute: product dtype as in qcur_approx; X (m x n, FP64 for QCUR_F64 else
 * FP32) receives the last iterate.  rtol and max_rank (the predefined rank
 * k) apply to the pseudoinverses.  iters (host int, may be NULL): steps
 * taken; rel (host double, may be NULL): the last relative change.
 * When a step is cheap (32 m n r <= 4e10 flops), up to eight steps are
 * enqueued per host round trip: each leaves its certificate verdict and
 * stopping sums on the device, the host reads them together and keeps the
 * first step that meets the stopping rule (later ones are discarded, status
 * bits included), or redoes a step whose certificate was rejected while
 * waiting for the verdict (Jacobi fallback), then runs the following steps
 * one at a time for a while.  The workspace then holds up to eight more
 * m x n iterates (at most about 512 MiB).  Larger steps synchronise once
 * per step.  ws: qcur_complete_workspace(m, n, c, r, compute). */
qcur_status qcur_complete(qcur_handle handle, const qcur_qmat* Y, const uint8_t* mask, int64_t mask_ld,
                          const int64_t* I, int64_t r, const int64_t* J, int64_t c, int compute, double rtol,
                          int64_t max_rank, int max_iter, double tol, qcur_qmat* X, int* iters, double* rel,
                          void* ws, size_t ws_bytes);
size_t qcur_complete_workspace(int64_t m, int64_t n, int64_t c, int64_t r, int compute);

/* Algorithm 2 with the index sets drawn again at every step: step t draws
 * J (c columns, set 0) and I (r rows, set 1) from the sampling
 * probabilities of the current iterate X^t (sampling = QCUR_LENGTH or
 * QCUR_UNIFORM, Section 3.1; without replacement) with seed + t, then
 * proceeds as qcur_complete.  I (device int64[r]) and J (device int64[c])
 * are outputs: the index sets of the last step.  Other arguments and the
 * stopping rule as in qcur_complete.  Also errors with QCUR_ERR_SAMPLE (on
 * the status word) when an iterate has fewer nonzero rows or columns than
 * r or c.  ws: qcur_complete_resampled_workspace(m, n, c, r, sampling,
 * compute). */
qcur_status qcur_complete_resampled(qcur_handle handle, const qcur_qmat* Y, const uint8_t* mask, int64_t mask_ld,
                                    int64_t r, int64_t c, int sampling, uint64_t seed, int compute, double rtol,
                                    int64_t max_rank, int max_iter, double tol, qcur_qmat* X, int64_t* I,
                                    int64_t* J, int* iters, double* rel, void* ws, size_t ws_bytes);
size_t qcur_complete_resampled_workspace(int64_t m, int64_t n, int64_t c, int64_t r, int sampling, int compute);

/* Sample size for a target rank k (Section 3.1 sizes C and R as k log k):
 * ceil(k ln k), at least k and at most limit (k = 1 gives 1).  Host only;
 * returns 0 when k < 1 or limit < 1. */
int64_t qcur_sample_size(int64_t k, int64_t limit);

/* ---- helpers ----------------------------------------------------------- */

/* Elementwise dtype conversion Y = X (same shape; BF16 with
 * round-to-nearest-even, FP64 -> FP32 correctly rounded). */
qcur_status qcur_cast(qcur_handle handle, const qcur_qmat* X, qcur_qmat* Y);

#ifdef __cplusplus
}
#endif

#endif /* QCUR_H */
