// Internal declarations shared by the libqcur kernels and its C ABI layer.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/qcur.h"

namespace qcur {

// ---- device status word bits (OR-ed by kernels, read by qcur_sync_status)
enum StatusBit : unsigned {
  ST_ARG = 1u << 0,
  ST_SAMPLE = 1u << 1,
  ST_NUMERIC = 1u << 2,
};

// A quaternion matrix view: four planes of rows x cols, row stride ld,
// plane stride ps, all in elements of the view's dtype.
struct QView {
  void* p;
  int64_t rows, cols, ld, ps;
  int dt;
};

inline QView view_of(const qcur_qmat& m) {
  return QView{m.p, m.rows, m.cols, m.ld, m.pstride, (int)m.dtype};
}

__host__ __device__ inline size_t dtype_size(int dt) { return dt == QCUR_F64 ? 8 : dt == QCUR_F32 ? 4 : 2; }

struct Ctx {
  int device;
  hipStream_t stream;
  unsigned* status;  // device word
  void* pinned;      // small pinned host buffer (fast-path verdicts)
  hipEvent_t done;   // marks the arrival of those verdicts
  void* scratch;     // this device's copy of the static scratch (SCRATCH_BYTES)
};

// Static device scratch of the entry points that allocate nothing.  Its
// device address on `device` (which must be current at the first call for
// that device).
constexpr size_t SCRATCH_BYTES = (size_t)32 << 20;
hipError_t scratch_address(int device, void** out);

// ---- element conversions --------------------------------------------------
// BF16 is stored as raw uint16 bits.  float -> bf16 rounds to nearest even
// (the usual add-0x7FFF-plus-lsb method); NaN maps to a quiet NaN.
__host__ __device__ inline uint16_t f32_to_bf16(float f) {
  union { float f; uint32_t u; } v;
  v.f = f;
  if ((v.u & 0x7F800000u) == 0x7F800000u && (v.u & 0x007FFFFFu)) return (uint16_t)((v.u >> 16) | 0x40u);
  uint32_t lsb = (v.u >> 16) & 1u;
  return (uint16_t)((v.u + 0x7FFFu + lsb) >> 16);
}
__host__ __device__ inline float bf16_to_f32(uint16_t b) {
  union { float f; uint32_t u; } v;
  v.u = ((uint32_t)b) << 16;
  return v.f;
}

template <int DT> struct Elem;
template <> struct Elem<QCUR_F64> { typedef double T; };
template <> struct Elem<QCUR_F32> { typedef float T; };
template <> struct Elem<QCUR_BF16> { typedef uint16_t T; };

__device__ inline double load_as_double(const void* p, int dt, int64_t off) {
  if (dt == QCUR_F64) return ((const double*)p)[off];
  if (dt == QCUR_F32) return (double)((const float*)p)[off];
  return (double)bf16_to_f32(((const uint16_t*)p)[off]);
}
__device__ inline void store_from_double(void* p, int dt, int64_t off, double v) {
  if (dt == QCUR_F64) ((double*)p)[off] = v;
  else if (dt == QCUR_F32) ((float*)p)[off] = (float)v;
  else ((uint16_t*)p)[off] = f32_to_bf16((float)v);
}

// ---- launchers (implemented in the kernel sources) ------------------------
hipError_t launch_probs_partials(const Ctx& c, QView A, double* colpart, double* rowpart, int rb, int ncb);
hipError_t launch_probs_finish(const Ctx& c, int64_t m, int64_t n, const double* colpart,
                               const double* rowpart, int nrb, int ncb, int sampling, double* p,
                               double* q, double* fro2, double* scratch);
void probs_grid(int64_t m, int64_t n, int* rb, int* nrb, int* ncb);

hipError_t launch_draw(const Ctx& c, const double* probs, int64_t n, int64_t count, uint64_t seed,
                       uint64_t set_id, int with_replacement, int64_t* idx);
hipError_t launch_draw_pair(const Ctx& c, const double* p0, int64_t n0, int64_t count0, uint64_t set0,
                            int64_t* idx0, const double* p1, int64_t n1, int64_t count1, uint64_t set1,
                            int64_t* idx1, uint64_t seed, int with_replacement);

hipError_t launch_gather(const Ctx& c, QView A, const int64_t* I, int64_t r, const int64_t* J,
                         int64_t cc, const QView* C, const QView* R, const QView* W);
// mode bit 1: transpose, bit 2: conjugate (quaternion conjugate of every entry)
// CAST_CHECK: also raise ST_NUMERIC in the status word for an element that is not finite
enum { CAST_COPY = 0, CAST_T = 1, CAST_CONJ = 2, CAST_H = 3, CAST_CHECK = 4 };
hipError_t launch_cast(const Ctx& c, QView X, QView Y, int mode);
// n <= MAXB casts in one launch when they share the input and the output dtype
hipError_t launch_cast_set(const Ctx& c, int n, const QView* X, const QView* Y, const int* modes);

// qGEMM: D = alpha * op(A) op(B) + beta * D.  ws may be NULL (no split-K).
// A batch runs `count` products in one launch: problem b uses the views'
// pointers advanced by b * stride (elements) and, when the dims arrays (device
// int[count]) are given, its own M, N, K, at most those of the views.
struct BatchSpec {
  int count = 1;
  int64_t sA = 0, sB = 0, sD = 0;
  const int* M = nullptr;
  const int* N = nullptr;
  const int* K = nullptr;
  int tile = 0;    // launch plan override: tile edge 32 or 64 (0: automatic)
  int splits = 0;  // K slices (0: automatic; reduced to 1 without enough workspace)
  int tri = 0;     // TRI_* flags: zero triangles of op(A), op(B), lower output only
  // with M or N given: the problems in the order a persistent launch hands
  // out their tiles (device int[count], largest first; NULL: one workgroup
  // per tile of the padded grid)
  const int* order = nullptr;
  // per-problem device flags: problem b's product is not written when
  // skip[b] != 0 (the k_qgemm and split-K routes; the thin and tall routes
  // compute it regardless)
  const int* skip = nullptr;
};
// op(A) / op(B) lower or upper triangular (exact zeros elsewhere): K steps
// that meet only zeros are skipped.  TRI_LOWER_OUT: only the lower triangle
// of D is wanted; tiles wholly above the diagonal are not written.
enum { TRI_LOWER_OUT = 1, TRI_A_LOWER = 2, TRI_A_UPPER = 4, TRI_B_LOWER = 8, TRI_B_UPPER = 16 };
size_t gemm_workspace(int64_t M, int64_t N, int64_t K, int compute, int batch = 1);
// Thin FP64 / FP32 products D = alpha A^H B + beta D (A: K x M, B: K x N,
// both K-major; M, N <= 512, K >= 4 max(M, N), equal sizes over a batch):
// one wave per 16 x 16 block of D streaming its fragments from global
// memory.  Needs no more workspace than gemm_workspace gives the tiled plan
// (fewer K splits); lower_only computes the blocks on and below the diagonal.
bool thin_hn_applies(int compute, int opA, int opB, int64_t M, int64_t N, int64_t K, int tri, bool per_problem_dims);
// With bM / bN / bK (device int[batch], may be NULL) problem b has its own
// M, N, K within the extents (D.rows, D.cols, K); no K split then.
hipError_t launch_thin_hn(const Ctx& c, int compute, double alpha, QView A, QView B, double beta, QView D,
                          int64_t K, int batch, int64_t sA, int64_t sB, int64_t sD, bool lower_only, void* ws,
                          size_t ws_bytes, const int* bM = nullptr, const int* bN = nullptr,
                          const int* bK = nullptr);
// Tall FP64 products D = alpha A B^H + beta D with both operands contiguous
// in k (M >= 512, N <= 512, K <= 512 a multiple of 4, 16-byte aligned rows;
// equal sizes over a batch; op(B) may be upper triangular): one wave per
// 16 x 16 block of D over the whole K range, no workspace.
bool tall_nh_applies(int compute, int opA, int opB, QView A, QView B, int64_t M, int64_t N, int64_t K, int tri,
                     bool per_problem_dims, int64_t sA, int64_t sB);
// With bM / bN / bK as for launch_thin_hn; the extent K must be a multiple
// of 4 and the operands' rows hold at least that many elements.  copy: D
// also stored (or only stored, when D.p is NULL and beta is 0) in dtype
// copy->dt, problems b < copy->split in slot b of p[0], the others in slot
// b - split of p[1] (row stride ld, plane stride ps, slot stride slab, in
// elements).
struct TallCopy {
  void* p[2];
  int64_t ld[2], ps[2], slab[2];
  int dt, split;
};
hipError_t launch_tall_nh(const Ctx& c, double alpha, QView A, QView B, double beta, QView D, int64_t K, int batch,
                          int64_t sA, int64_t sB, int64_t sD, bool b_upper, const int* bM = nullptr,
                          const int* bN = nullptr, const int* bK = nullptr, const TallCopy* copy = nullptr);
// Workspace for any plan with at most max_splits K slices.
size_t gemm_workspace_splits(int64_t M, int64_t N, int compute, int batch, int max_splits);
hipError_t launch_gemm(const Ctx& c, int opA, int opB, double alpha, QView A, QView B, double beta,
                       QView D, int compute, void* ws, size_t ws_bytes);
hipError_t launch_gemm_batched(const Ctx& c, int opA, int opB, double alpha, QView A, QView B, double beta,
                               QView D, int compute, void* ws, size_t ws_bytes, const BatchSpec& bs);
// Residual: partial sums of squares of e_scale-free P_Omega(A - B1 R) per tile,
// then a fixed-order final sum into fro (sqrt).  Optional E output and
// optional Bout = B1 op(R) itself (the product tile before the subtraction).
size_t residual_tiles(int64_t m, int64_t n, int compute);
hipError_t launch_residual_gemm(const Ctx& c, QView A, QView B1, QView R, const uint8_t* mask,
                                int64_t mask_ld, int compute, double* partials, QView* E,
                                double e_scale, int opR = QCUR_OP_N, const QView* Bout = nullptr,
                                const int* skip = nullptr);
hipError_t launch_sum_partials(const Ctx& c, const double* partials, int64_t count, double* out,
                               int take_sqrt, const int* skip = nullptr);
// Refinement's core update M += D (same shape and dtype, F32 or F64), with
// FP64 sums of squares of D per workgroup into dpart[CORE_PARTS].
constexpr int CORE_PARTS = 64;
hipError_t launch_core_correct(const Ctx& c, QView M, QView D, double* dpart);
// Residual of a refined core from the refinement's own residual E and
// correction D = Q_C^H E Q_R: ||E - Q_C D Q_R^H||^2 = ||E||^2 - 2 ||D||^2 +
// ||Q_C D Q_R^H||^2, the last term ||D||^2 (1 + e) with |e| <= 3 delta for
// factors whose orthogonality defect delta meets the refinement's bound
// 2^-12.  Taken when ||D||^2 <= gate ||E||^2: out = sqrt(||E||^2 - ||D||^2)
// and *skip = 1; otherwise *skip = 0 and out is left for the explicit
// residual product.  resid_identity_gate gives the gate per product dtype.
hipError_t launch_resid_identity(const Ctx& c, const double* epart, int64_t ecount, const double* dpart, double gate,
                                 double* out, int* skip);
// 2^-8 for FP32 and FP64 products (no cancellation, the defect term below
// 2^-21 of the result, under the rounding of an FP32 residual product);
// 1/2 for BF16 operands, whose own rounding (a relative 2^-8 per product,
// so D carries about 4e-3 of E) would fail the tighter gate: the result's
// square is then at least half of ||E||^2 and the defect term at most
// 3 * 2^-12 of it (a relative 4e-4 on the residual), against a BF16
// residual product's error of about 1e-3 of ||A||.
inline double resid_identity_gate(int compute) { return compute == QCUR_BF16 ? 0.5 : 0x1p-8; }
// Completion step (Algorithm 2): X1 = P_Omega(Y) + P_Omega^c(B1 op(R)) with
// per-tile sums of |X1 - X0|^2 (partials) and |X0|^2 (partials2), 64 x 64
// tiles (residual_tiles(m, n) of each).
hipError_t launch_merge_gemm(const Ctx& c, QView Y, const uint8_t* mask, int64_t mask_ld, QView X0, QView B1,
                             QView R, int opR, int compute, QView X1, double* partials, double* partials2);
// X = P_Omega(Y) (zeros where mask is 0), X in its own dtype.
hipError_t launch_mask_init(const Ctx& c, QView Y, const uint8_t* mask, int64_t mask_ld, QView X);

// Jacobi pseudoinverse pieces.
hipError_t launch_jacobi_round(const Ctx& c, double* Y, int64_t p, int64_t q, double* V, int64_t qpad, int round,
                               double tol, unsigned* rotated, double drop2, double* cmax, int slot);
hipError_t launch_deflation_check(const Ctx& c, const double* Y, int64_t p, int64_t q, double drop2, double rtol2q,
                                  unsigned* bad);
hipError_t launch_jacobi_small(const Ctx& c, double* Y, int64_t p, int64_t q, double* V,
                               double tol, int max_sweeps, unsigned* rotated);
bool jacobi_small_fits(int64_t p, int64_t q);
hipError_t launch_svd_out(const Ctx& c, const double* Y, int64_t pp, int64_t qq, const double* V, double* sig2,
                          int32_t* rank, double* s, bool tall, double* U, int64_t uld, int64_t ups, double* Vo,
                          int64_t vld, int64_t vps);
hipError_t launch_pinv_scale(const Ctx& c, double* Y, int64_t p, int64_t q, double rtol,
                             int64_t max_rank, int64_t* rank_out, double* sig);
hipError_t launch_check_finite(const Ctx& c, QView X);
hipError_t launch_fill_identity(const Ctx& c, double* V, int64_t q);
// Fixed pseudo-random sketch: every entry of the four planes of S (FP64,
// contiguous rows, plane stride rows * cols) uniform in [-1, 1), a function
// of the seed and the entry's flat index only.
hipError_t launch_sketch(const Ctx& c, QView S, uint64_t seed);
hipError_t launch_pinv_apply(const Ctx& c, double* Y, int64_t p, int64_t q, double* V, const double* dsc);
// Orthonormal-form output of the Jacobi pseudoinverse: Z^+ = P^H Q^H with
// Q (p x q, orthonormal or zero columns) and P (q x q), both FP64.
hipError_t launch_pinv_qp(const Ctx& c, const double* Y, int64_t p, int64_t q, const double* V, const double* dsc,
                          QView Q, QView P);

// Fast pseudoinverse pieces (CholeskyQR2), batched over up to MAXB matrices.
constexpr int CHOL_BLOCK = 64;
constexpr int MAXB = 4;
// CholeskyQR2 of a batch's factors in one launch (one workgroup per factor,
// orders q_t <= 64): Gram matrix, Cholesky factor and inverse P1,
// Q1 = Z P1^H (and its product-dtype copy), ||Z||_F^2 and ||P1||_F^2 into
// norms[4t], norms[4t+1]; with `adaptive` a factor whose first pass
// succeeded with ||Q1^H Q1 - I||_F^2 <= tol2 keeps it (q2 = 0, P = P1),
// every other one takes the second pass in place (q2 = q_t, P = P2 P1,
// Q = Q1 P2^H into Q (FP64, may be NULL) and the copy).  order (may be
// NULL): the factors in the order their workgroups start (largest first).
hipError_t launch_cholqr_batch(const Ctx& c, int count, const double* Z, double* Q1, double* Q, int64_t zld,
                               int64_t zps, int64_t zslab, double* P1, double* P, int64_t gld, int64_t gps,
                               int64_t gslab, const int* zp, const int* zq, int* fail, double* norms, int* q2,
                               int* skip, double tol2, int adaptive, const TallCopy* copy, const int* order);
hipError_t launch_chol_block(const Ctx& c, const double* G, double* P, int w, int64_t ld, int64_t ps, int* fail,
                             int batch, int64_t sbatch, const int* dims = nullptr);
// Factorisation and inverse of nb Hermitian positive definite n x n Gram
// matrices (matrix b at G + b * slab, lower triangle read) in one graph of
// 32 x 32 tile tasks: P = L^{-1} (lower; the upper part zeroed), the
// off-diagonal tiles of L in L.  flags: chol_dag_flag_ints(nb, n) ints of
// workspace (zeroed by the call).  A failed pivot sets fail[b].
size_t chol_dag_flag_ints(int nb, int64_t n);
hipError_t launch_chol_dag(const Ctx& c, const double* G, double* L, double* P, int64_t n, int64_t slab, int nb,
                           int* flags, int* fail);
hipError_t launch_sumsq(const Ctx& c, QView X, double* partials, double* out);
hipError_t launch_sumsq_batch(const Ctx& c, int nb, const QView* X, double* partials, double* out, int ostride);
hipError_t launch_pad_identity(const Ctx& c, double* G, int64_t n, int64_t sbatch, int nb, const int64_t* q);
hipError_t launch_pinv_decide(const Ctx& c, const double* norms, const int* fail, double rtol, int64_t max_rank,
                              int nb, const int64_t* q, int64_t* const* rank_out, int* ok);
hipError_t launch_defect_batch(const Ctx& c, int nb, const double* G, int64_t n, int64_t sbatch, const int64_t* q,
                               double* partials, double* out, int ostride);
hipError_t launch_zero(const Ctx& c, double* p, int64_t n);
hipError_t launch_zero_i32(const Ctx& c, int* p, int64_t n);

// Backward assembly: dA = G + scatter(gC, gR, gW).
hipError_t launch_inverse_map(const Ctx& c, const int64_t* idx, int64_t cnt, int64_t n, int32_t* inv);
hipError_t launch_backward_assemble(const Ctx& c, QView dA, QView G, int has_G, QView gC, QView gR,
                                    QView gW, const int32_t* iinv, const int32_t* jinv);
hipError_t launch_axpby(const Ctx& c, double alpha, QView X, double beta, QView Y);
hipError_t launch_identity_minus(const Ctx& c, QView X);

// ---- batched solve (many independent problems of uneven sizes) ------------
// Problem b owns slot b of every batched array: its matrix is the top-left
// corner of the slot, with the slot's row stride.  Sizes live in device int
// arrays (dm, dn, dc, dr: m_b, n_b, c_b, r_b); zp/zq hold the tall shapes
// p x q of the 2*count pseudoinverse problems (C_b, then R_b^H).
constexpr int JB_MAXQ = 1024;
struct JacobiBatch {
  const int* ok;
  const double* Cz;
  int64_t cld, cps, cslab;
  const double* Rz;
  int64_t rld, rps, rslab;
  const int *dm, *dn, *dc, *dr;
  double* Y;
  double* V;
  int64_t yslab, vslab;
  double* Q;  // [2*count] slots: p_t x q_t orthonormal factor
  int64_t qld, qps, qslab;
  double* P;  // [2*count] slots: q_t x q_t, Z^+ = P^H Q^H
  int64_t pld, pps, pslab;
  int64_t* rank_out;  // [count][2]
  double rtol;
  int64_t max_rank;
  int count;
  int max_sweeps;
};
hipError_t launch_jacobi_pinv_batch(const Ctx& c, const JacobiBatch& jb, int count2);

// A slot array: element (i, j) of plane k of problem b at
// p + b*slab + k*ps + i*ld + j (elements of dt).
struct Slots {
  void* p;
  int64_t ld, ps, slab;
  int dt;
};
constexpr int BATCH_RB = 32;  // rows per tile of the batched norm pass
constexpr int BATCH_CB = 64;  // columns per tile of the batched norm pass
hipError_t launch_norms_batch(const Ctx& c, int count, Slots A, const int* dm, const int* dn, int64_t mx,
                              int64_t nx, double* colpart, double* rowpart, const Slots* Ax);
struct DrawBatch {
  const int *dm, *dn, *dc, *dr;
  const double* colpart;  // [count][ceil(mx/BATCH_RB)][nx]
  const double* rowpart;  // [count][ceil(nx/256)][mx]
  int64_t mx, nx, cx, rx;
  double* p;  // [count][nx]
  double* q;  // [count][mx]
  int64_t* I;  // [count][rx]
  int64_t* J;  // [count][cx]
  uint64_t seed;
  int sampling, repl;
};
size_t draw_lds(int64_t n, int repl);
hipError_t launch_draw_batch(const Ctx& c, int count, const DrawBatch& d);
// out_b = A_b(rows idx, cols idx) with NULL index lists meaning the identity;
// written in FP64 (O) and, if Ox is given, in its dtype.
hipError_t launch_gather_batch(const Ctx& c, int count, Slots A, const int* dm, const int* dn,
                               const int64_t* ridx, int64_t ris, const int64_t* cidx, int64_t cis,
                               const int* orows, const int* ocols, int64_t rowsx, int64_t colsx, Slots O,
                               const Slots* Ox, int tconj = 0);
// skip_if (device int[count], may be NULL): problems b with skip_if[b] != 0
// are left alone
hipError_t launch_cast_batch(const Ctx& c, int count, Slots X, Slots Y, const int* rows, const int* cols,
                             int64_t rowsx, int64_t colsx, int mode, const int* skip_if = nullptr);
// Second-pass plan of a batch of CholeskyQR factors from G = Q1^H Q1 (n x n
// slots, leading q_t x q_t block of factor t, lower triangle): factor t
// keeps its first pass when that pass did not fail and
// ||Q1^H Q1 - I||_F^2 <= tol2; then q2[t] = 0, skip[t] = 1 and P1 is copied
// to P; otherwise q2[t] = q_t and skip[t] = 0.
hipError_t launch_defect_plan_batch(const Ctx& c, int count, const double* G, int64_t n, int64_t slab, const int* zq,
                                    const int* fail, double tol2, const double* P1, double* P, int* q2, int* skip);
hipError_t launch_pad_gram_batch(const Ctx& c, int count, double* G, int64_t n, int64_t slab, const int* zq);
hipError_t launch_sumsq_ragged(const Ctx& c, int count, Slots X, const int* rows, const int* cols, double* out,
                               int ostride);
hipError_t launch_decide_batch(const Ctx& c, int count2, int count, const double* norms, const int* fail,
                               double rtol, int64_t max_rank, const int* zp, const int* zq, int64_t* rank_out,
                               int* ok);
// residual_b = sqrt(sum of problem b's tile partials) over its own tiles:
// rows ceil(m_b / tile) and columns ceil(n_b / tile) of the gx-wide tile
// grid (tiles = partials per problem)
hipError_t launch_resid_sum_batch(const Ctx& c, int count, const double* part, int64_t tiles, int64_t gx, int tile,
                                  const int* dm, const int* dn, double* out, const int* skip = nullptr);
// The refinement's core update and the residual identity of
// launch_core_correct / launch_resid_identity, per problem of a batch
// (dpart: CORE_PARTS per problem; out and skip: one per problem).
hipError_t launch_core_correct_batch(const Ctx& c, int count, Slots M, Slots D, const int* rows, const int* cols,
                                     double* dpart);
hipError_t launch_resid_identity_batch(const Ctx& c, int count, const double* part, int64_t tiles, int64_t gx,
                                       int tile, const int* dm, const int* dn, const double* dpart, double gate,
                                       double* out, int* skip);
// Batched residual A_b - B1_b op(R_b) (op = QCUR_OP_N or QCUR_OP_H).
// tile: 64 or 32 (partials per problem: ceil(mx/tile) * ceil(nx/tile); only
// those of the problem's own tiles are written).  order: as BatchSpec::order.
hipError_t launch_residual_gemm_batched(const Ctx& c, int count, Slots A, Slots B1, Slots R, int opR, int64_t mx,
                                        int64_t nx, int64_t kx, const int* bM, const int* bN, const int* bK,
                                        int compute, double* partials, const Slots* E, double e_scale,
                                        int tile = 64, const Slots* Bout = nullptr, const int* order = nullptr,
                                        const int* skip = nullptr);

}  // namespace qcur
