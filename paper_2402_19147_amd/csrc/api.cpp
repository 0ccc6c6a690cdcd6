// libqcur C ABI: argument validation, workspace layout and the orchestration
// of the QMCUR steps (Algorithm 1) on top of the kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstddef>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "qcur_internal.hpp"

using namespace qcur;

// Launch plans of the GEMM stages of a batched solve, chosen by timing the
// candidates on the first eager call (the autotuner) or left automatic.
enum BatchStage {
  BS_GRAM_C, BS_GRAM_R, BS_Q1_C, BS_Q1_R, BS_G2, BS_P, BS_Q, BS_T, BS_M, BS_B1, BS_W1, BS_U, BS_RESID, BS_COUNT
};
struct StagePlan {
  int tile = 0, splits = 0;  // 0: automatic
};
struct BatchTuning {
  bool measure = false;  // time the candidates during this call
  hipEvent_t e0 = nullptr, e1 = nullptr;
  StagePlan plan[BS_COUNT];
};

// A prepared batch layout: the workspace it was uploaded into, a key of the
// sizes and options it was prepared for, and its stage plans.
struct BatchRecord {
  const void* ws = nullptr;
  uint64_t key = 0;
  int autotune = 0;
  bool tuned = false;
  BatchTuning tun;
};

struct qcur_ctx {
  Ctx c;
  BatchRecord batches[8];
  int next_batch = 0;
};

namespace {

thread_local std::string g_last_error;

qcur_status fail(qcur_status s, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
qcur_status fail(qcur_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return s;
}

#define HIPCHK(expr)                                                                    \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess)                                                               \
      return fail(QCUR_ERR_DEVICE, "%s: %s", #expr, hipGetErrorString(e_));             \
  } while (0)

#define CHK(expr)                       \
  do {                                  \
    qcur_status s_ = (expr);            \
    if (s_ != QCUR_OK) return s_;       \
  } while (0)

bool valid_dtype(int dt) { return dt == QCUR_F64 || dt == QCUR_F32 || dt == QCUR_BF16; }
bool valid_compute(int c) { return valid_dtype(c) || c == QCUR_BF16X3; }

// Shape/stride/dtype checks of one operand.
qcur_status check_qmat(const qcur_qmat* m, const char* name) {
  if (!m) return fail(QCUR_ERR_ARG, "%s is NULL", name);
  if (m->rows < 0 || m->cols < 0) return fail(QCUR_ERR_ARG, "%s has a negative size", name);
  if (!valid_dtype(m->dtype)) return fail(QCUR_ERR_DTYPE, "%s has an unknown dtype %d", name, (int)m->dtype);
  if (m->rows > 0 && m->cols > 0) {
    if (!m->p) return fail(QCUR_ERR_ARG, "%s has a NULL data pointer", name);
    if (m->ld < m->cols) return fail(QCUR_ERR_SHAPE, "%s: ld < cols", name);
    if (m->pstride < (m->rows - 1) * m->ld + m->cols)
      return fail(QCUR_ERR_SHAPE, "%s: planes overlap (pstride too small)", name);
  }
  return QCUR_OK;
}

qcur_status check_dims(const qcur_qmat* m, const char* name, int64_t rows, int64_t cols) {
  if (m->rows != rows || m->cols != cols)
    return fail(QCUR_ERR_SHAPE, "%s is %lldx%lld, expected %lldx%lld", name, (long long)m->rows,
                (long long)m->cols, (long long)rows, (long long)cols);
  return QCUR_OK;
}

qcur_status check_handle(qcur_handle h) {
  if (!h) return fail(QCUR_ERR_ARG, "handle is NULL");
  return QCUR_OK;
}

// ---- workspace: a bump allocator used both to size and to carve buffers.
struct Bump {
  char* base;
  size_t used;
  explicit Bump(void* b) : base((char*)b), used(0) {}
  void* take(size_t bytes) {
    used = (used + 255) & ~(size_t)255;
    void* p = base ? base + used : nullptr;
    used += bytes;
    return p;
  }
  QView mat(int64_t rows, int64_t cols, int dt) {
    QView v;
    v.p = take((size_t)4 * rows * cols * dtype_size(dt));
    v.rows = rows;
    v.cols = cols;
    v.ld = cols;
    v.ps = rows * cols;
    v.dt = dt;
    return v;
  }
};

int acc_dt(int compute) { return compute == QCUR_F64 ? QCUR_F64 : QCUR_F32; }
int in_dt(int compute) { return compute == QCUR_BF16X3 ? QCUR_F32 : compute; }

// ---- pseudoinverse -------------------------------------------------------
struct PinvPlan {
  int64_t p, q;     // X is p x q
  int64_t pp, qq;   // working tall shape: pp >= qq
  bool tall;
};

PinvPlan pinv_plan(int64_t p, int64_t q) {
  PinvPlan pl;
  pl.p = p;
  pl.q = q;
  pl.tall = p >= q;
  pl.pp = std::max(p, q);
  pl.qq = std::min(p, q);
  return pl;
}

// Jacobi (general) path buffers for one matrix.
struct PinvWs {
  double* Y;
  double* V;
  double* sig;
  unsigned* flag;
  void* gws;
  size_t gws_bytes;
};

PinvWs pinv_carve(Bump& b, int64_t p, int64_t q) {
  PinvPlan pl = pinv_plan(p, q);
  const int64_t pp = pl.pp, qq = pl.qq;
  PinvWs w;
  w.Y = (double*)b.take((size_t)4 * qq * pp * 8);
  w.V = (double*)b.take((size_t)4 * qq * qq * 8);
  w.sig = (double*)b.take((size_t)2 * std::max<int64_t>(qq, 1) * 8);
  w.flag = (unsigned*)b.take(256);
  const int64_t M = pl.tall ? qq : pp;
  const int64_t N = pl.tall ? pp : qq;
  w.gws_bytes = gemm_workspace(M, N, qq, QCUR_F64);
  w.gws = b.take(w.gws_bytes);
  return w;
}

// CholeskyQR path buffers for a group of nb matrices padded to pp x qq.
// The certificate inputs and verdicts of a group, one block of device
// memory laid out like the start of the pinned HostVerdict so that a single
// copy reads them back.
struct DevVerdict {
  int ok[MAXB];
  double nrm[4 * MAXB];
};

struct GroupWs {
  int nb;
  int64_t pp, qq;
  double *Z, *Q1, *Q, *G, *L, *P1, *P2, *P, *S, *part, *norms;
  int *fail, *ok;
  void* verdict;  // DevVerdict holding ok and norms
  void* gws;
  size_t gws_bytes;
  // per-matrix orders (device int[nb], may be NULL) for Gram matrices that
  // fit one diagonal block: matrix b is factored over its leading dims[b]
  // rows and columns only (0: skipped, P left as it is)
  const int* dims = nullptr;
};

GroupWs group_carve(Bump& b, int nb, int64_t pp, int64_t qq) {
  GroupWs w;
  w.nb = nb;
  w.pp = pp;
  w.qq = qq;
  const size_t zb = (size_t)nb * 4 * pp * qq * 8, gb = (size_t)nb * 4 * qq * qq * 8;
  w.Z = (double*)b.take(zb);
  w.Q1 = (double*)b.take(zb);
  w.Q = (double*)b.take(zb);
  w.G = (double*)b.take(gb);
  w.L = (double*)b.take(gb);
  w.P1 = (double*)b.take(gb);
  w.P2 = (double*)b.take(gb);
  w.P = (double*)b.take(gb);
  w.S = (double*)b.take((size_t)nb * 4 * CHOL_BLOCK * qq * 8);
  w.part = (double*)b.take((size_t)nb * 256 * 8);
  char* vb = (char*)b.take(sizeof(DevVerdict));  // nb <= MAXB
  w.verdict = vb;
  w.norms = vb ? (double*)(vb + offsetof(DevVerdict, nrm)) : nullptr;
  w.ok = vb ? (int*)(vb + offsetof(DevVerdict, ok)) : nullptr;
  w.fail = (int*)b.take((size_t)nb * 4);
  w.gws_bytes = std::max({gemm_workspace(qq, qq, pp, QCUR_F64, nb), gemm_workspace(pp, qq, qq, QCUR_F64, nb),
                          gemm_workspace(qq, qq, qq, QCUR_F64, nb), gemm_workspace(qq, pp, qq, QCUR_F64),
                          gemm_workspace(pp, qq, qq, QCUR_F64)});
  w.gws = b.take(w.gws_bytes);
  return w;
}

size_t pinv_ws_size(int64_t p, int64_t q) {
  Bump b(nullptr);
  pinv_carve(b, p, q);
  PinvPlan pl = pinv_plan(p, q);
  group_carve(b, 1, pl.pp, pl.qq);
  return b.used + 256;
}

constexpr int MAX_SWEEPS = 40;

// view of the (rows x cols) block at (r0, c0) of a dense n x n FP64 matrix
QView sq_view(double* base, int64_t n, int64_t r0, int64_t c0, int64_t rows, int64_t cols) {
  return QView{base + r0 * n + c0, rows, cols, n, n * n, QCUR_F64};
}

BatchSpec same_stride(int nb, int64_t s) {
  BatchSpec bs;
  bs.count = nb;
  bs.sA = bs.sB = bs.sD = s;
  return bs;
}

// Blocked Cholesky G = L L^H with the explicit inverse P = L^{-1} for the
// group's nb matrices (n x n, back to back; G is overwritten).  Diagonal
// blocks are factored and inverted in LDS; panels, trailing updates and the
// block rows of P are batched quaternion GEMMs on the matrix cores.
qcur_status chol_inv(const Ctx& c, GroupWs& w, double* P) {
  const int64_t n = w.qq, nb = CHOL_BLOCK;
  const int64_t slab = 4 * n * n;
  BatchSpec bs = same_stride(w.nb, slab);
  BatchSpec bs_up = bs, bs_low = bs;
  bs_up.tri = TRI_B_UPPER;     // op(B) = P_kk^H
  bs_low.tri = TRI_LOWER_OUT;  // the trailing Gram block: lower triangle only
  double *G = w.G, *L = w.L;
  if (n > nb) {
    // larger than one diagonal block: the tile-task graph in one launch
    HIPCHK(launch_chol_dag(c, G, L, P, n, slab, w.nb, (int*)w.S, w.fail));
    return QCUR_OK;
  }
  if (w.dims) {
    HIPCHK(launch_chol_block(c, G, P, (int)n, n, n * n, w.fail, w.nb, slab, w.dims));
    return QCUR_OK;
  }
  HIPCHK(launch_zero(c, P, w.nb * slab));
  for (int64_t kb = 0; kb < n; kb += nb) {
    const int64_t wd = std::min(nb, n - kb);
    const int64_t rest = n - kb - wd;
    HIPCHK(launch_chol_block(c, G + kb * n + kb, P + kb * n + kb, (int)wd, n, n * n, w.fail, w.nb, slab));
    if (rest > 0) {
      QView L21 = sq_view(L, n, kb + wd, kb, rest, wd);
      HIPCHK(launch_gemm_batched(c, QCUR_OP_N, QCUR_OP_H, 1.0, sq_view(G, n, kb + wd, kb, rest, wd),
                                 sq_view(P, n, kb, kb, wd, wd), 0.0, L21, QCUR_F64, w.gws, w.gws_bytes, bs_up));
      HIPCHK(launch_gemm_batched(c, QCUR_OP_N, QCUR_OP_H, -1.0, L21, L21, 1.0,
                                 sq_view(G, n, kb + wd, kb + wd, rest, rest), QCUR_F64, w.gws, w.gws_bytes, bs_low));
    }
  }
  BatchSpec bsS{w.nb, slab, slab, 4 * nb * n};
  bsS.tri = TRI_B_LOWER;  // op(B) = P[0:kb, 0:kb], lower triangular
  for (int64_t kb = nb; kb < n; kb += nb) {
    const int64_t wd = std::min(nb, n - kb);
    QView Sv{w.S, wd, kb, kb, wd * kb, QCUR_F64};
    HIPCHK(launch_gemm_batched(c, QCUR_OP_N, QCUR_OP_N, 1.0, sq_view(L, n, kb, 0, wd, kb), sq_view(P, n, 0, 0, kb, kb),
                               0.0, Sv, QCUR_F64, w.gws, w.gws_bytes, bsS));
    BatchSpec bsP{w.nb, slab, 4 * nb * n, slab};
    bsP.tri = TRI_A_LOWER;  // op(A) = P_kk, lower triangular
    HIPCHK(launch_gemm_batched(c, QCUR_OP_N, QCUR_OP_N, -1.0, sq_view(P, n, kb, kb, wd, wd), Sv, 0.0,
                               sq_view(P, n, kb, 0, wd, kb), QCUR_F64, w.gws, w.gws_bytes, bsP));
  }
  return QCUR_OK;
}

// CholeskyQR attempt on a group: Z_b = X_b (tall) or X_b^H (wide), padded
// with zero rows/columns to pp x qq (the padded Gram gets an identity block,
// which leaves the factors of the real block unchanged).  Two passes give Q
// orthonormal to working precision (CholeskyQR2); passes == 0 keeps one pass
// when its measured orthogonality defect is below orth_tol; one pass (the normal
// equations, error ~ eps * kappa^2) is used when the products downstream are
// FP32 or BF16.  done[b] reports whether the certificate of matrix b held;
// for those Xp_b and rank_out[b] are written.
// Fast-path verdicts of a CholeskyQR group, copied to the handle's pinned
// buffer.
struct HostVerdict {
  int ok[MAXB];
  double nrm[4 * MAXB];
  double aux[4];  // other small read-backs (the completion's stopping sums)
};
static_assert(offsetof(HostVerdict, ok) == offsetof(DevVerdict, ok) &&
                  offsetof(HostVerdict, nrm) == offsetof(DevVerdict, nrm) &&
                  sizeof(DevVerdict) <= offsetof(HostVerdict, aux),
              "one copy moves a DevVerdict into the head of a HostVerdict, short of aux");

// A verdict left pending by pinv_fast_group: the decision kernel has run and
// its result is on its way to pinned host memory (c.done marks its arrival).
// The factors of the fast path (the first pass when `adaptive`, which then
// also requires the orthogonality defect to be small) are in place, so the
// caller can enqueue the work that follows before it waits; if the verdict
// rejects the fast path, the caller recomputes without speculation.
// Largest orthogonality defect ||Q1^H Q1 - I||_F of a first CholeskyQR
// pass that the products of a solve accept in place of a second pass.  A
// defect delta (Q^H Q = I + Delta) moves the orthogonal projectors Q Q^H by
// O(delta), and so C U R.  FP64 products: 0 (always two passes).  FP32
// products: 2^-22, a fraction of the relative error the FP32 products
// themselves leave in C U R (sqrt(K) rounding units, about 1e-6 on the
// benchmark shapes).  BF16 operands, or a refinement step after the first
// core: 2^-12, since the refined core M1 is off the least-squares core by
// O(delta^2) only (and BF16 rounding is 2^-8).
double orth_bound(int compute, int refine) {
  if (compute == QCUR_F64) return 0.0;
  return (compute == QCUR_BF16 || refine > 0) ? 0x1p-12 : 0x1p-22;
}

struct PinvSpec {
  bool pending = false;
  int nb = 0;
  bool adaptive = false;
  double orth_tol = 0.0;
  void* dev_dst = nullptr;  // when set: the verdict is copied there (device), not to the pinned buffer
};

// Whether a verdict confirms the fast path (as pinv_spec_resolve decides).
bool verdict_valid(const PinvSpec& spec, const int* ok, const double* nrm) {
  bool valid = true;
  for (int b = 0; b < spec.nb; ++b)
    valid = valid && ok[b] && (!spec.adaptive || nrm[4 * b + 3] <= spec.orth_tol * spec.orth_tol);
  return valid;
}

// Did the pending verdict confirm the fast path?  Waits for it.
qcur_status pinv_spec_resolve(const Ctx& c, const PinvSpec& spec, bool* valid) {
  *valid = true;
  if (!spec.pending) return QCUR_OK;
  HIPCHK(hipEventSynchronize(c.done));
  const HostVerdict* hv = (const HostVerdict*)c.pinned;
  *valid = verdict_valid(spec, hv->ok, hv->nrm);
  return QCUR_OK;
}


qcur_status pinv_fast_group(const Ctx& c, int nb, const QView* X, double rtol, int64_t max_rank, const QView* Xp,
                            int64_t* const* rank_out, GroupWs& w, int passes, bool* done, double orth_tol = 0.0,
                            int* final_pass = nullptr, PinvSpec* spec = nullptr) {
  const int64_t pp = w.pp, qq = w.qq;
  const int64_t zslab = 4 * pp * qq, gslab = 4 * qq * qq;
  int64_t pb[MAXB], qb[MAXB];
  bool tall[MAXB];
  for (int b = 0; b < nb; ++b) {
    PinvPlan pl = pinv_plan(X[b].rows, X[b].cols);
    pb[b] = pl.pp;
    qb[b] = pl.qq;
    tall[b] = pl.tall;
    done[b] = false;
  }
  bool padded = false;
  for (int b = 0; b < nb; ++b) padded |= (pb[b] != pp || qb[b] != qq);
  HIPCHK(launch_zero_i32(c, w.fail, nb));
  if (padded) HIPCHK(launch_zero(c, w.Z, nb * zslab));
  QView Zr[MAXB], Pr[MAXB];
  int cmode[MAXB];
  for (int b = 0; b < nb; ++b) {
    Zr[b] = QView{w.Z + b * zslab, pb[b], qb[b], qq, pp * qq, QCUR_F64};
    cmode[b] = (tall[b] ? CAST_COPY : CAST_H) | CAST_CHECK;  // also checks for non-finite entries
  }
  HIPCHK(launch_cast_set(c, nb, X, Zr, cmode));
  HIPCHK(launch_sumsq_batch(c, nb, Zr, w.part, w.norms + 0, 4));
  BatchSpec bzg;  // Gram matrices: lower triangle only (all the Cholesky reads)
  bzg.count = nb;
  bzg.sA = zslab;
  bzg.sB = zslab;
  bzg.sD = gslab;
  bzg.tri = TRI_LOWER_OUT;
  QView Z{w.Z, pp, qq, qq, pp * qq, QCUR_F64};
  QView Q1{w.Q1, pp, qq, qq, pp * qq, QCUR_F64};
  QView Q{w.Q, pp, qq, qq, pp * qq, QCUR_F64};
  QView G{w.G, qq, qq, qq, qq * qq, QCUR_F64};
  QView P1{w.P1, qq, qq, qq, qq * qq, QCUR_F64};
  QView P2{w.P2, qq, qq, qq, qq * qq, QCUR_F64};
  QView P{w.P, qq, qq, qq, qq * qq, QCUR_F64};
  BatchSpec bzp;  // (pp x qq) . (qq x qq)^H -> pp x qq, op(B) = P^H upper triangular
  bzp.count = nb;
  bzp.sA = zslab;
  bzp.sB = gslab;
  bzp.sD = zslab;
  bzp.tri = TRI_B_UPPER;
  BatchSpec bg = same_stride(nb, gslab);  // P2 P1: both lower triangular
  bg.tri = TRI_A_LOWER | TRI_B_LOWER;
  // pass 1: G = Z^H Z = L1 L1^H, P1 = L1^{-1}, Q1 = Z L1^{-H}
  HIPCHK(launch_gemm_batched(c, QCUR_OP_H, QCUR_OP_N, 1.0, Z, Z, 0.0, G, QCUR_F64, w.gws, w.gws_bytes, bzg));
  if (padded) HIPCHK(launch_pad_identity(c, w.G, qq, gslab, nb, qb));
  CHK(chol_inv(c, w, w.P1));
  for (int b = 0; b < nb; ++b) Pr[b] = QView{w.P1 + b * gslab, qb[b], qb[b], qq, qq * qq, QCUR_F64};
  HIPCHK(launch_sumsq_batch(c, nb, Pr, w.part, w.norms + 1, 4));
  HIPCHK(launch_gemm_batched(c, QCUR_OP_N, QCUR_OP_H, 1.0, Z, P1, 0.0, Q1, QCUR_F64, w.gws, w.gws_bytes, bzp));
  double* Pf = w.P1;
  double* Qf = w.Q1;
  int ok[MAXB] = {0, 0, 0, 0};
  // one host synchronisation: the fast-path verdicts and, when given, the
  // norms behind them
  auto decide_and_read = [&](double* nrm_out = nullptr) -> qcur_status {
    HIPCHK(launch_pinv_decide(c, w.norms, w.fail, rtol, max_rank, nb, qb, rank_out, w.ok));
    HIPCHK(hipMemcpyAsync(ok, w.ok, sizeof(int) * nb, hipMemcpyDeviceToHost, c.stream));
    if (nrm_out) HIPCHK(hipMemcpyAsync(nrm_out, w.norms, sizeof(double) * 4 * nb, hipMemcpyDeviceToHost, c.stream));
    HIPCHK(hipStreamSynchronize(c.stream));
    return QCUR_OK;
  };
  // speculation (orthonormal-form output only): launch the verdict, copy it
  // to pinned memory and return the fast path's factors without waiting
  auto decide_async = [&](bool adaptive, int fp) -> qcur_status {
    HIPCHK(launch_pinv_decide(c, w.norms, w.fail, rtol, max_rank, nb, qb, rank_out, w.ok));
    if (spec->dev_dst) {
      HIPCHK(hipMemcpyAsync(spec->dev_dst, w.verdict, sizeof(DevVerdict), hipMemcpyDeviceToDevice, c.stream));
    } else {
      HIPCHK(hipMemcpyAsync(c.pinned, w.verdict, sizeof(DevVerdict), hipMemcpyDeviceToHost, c.stream));
      HIPCHK(hipEventRecord(c.done, c.stream));
    }
    spec->pending = true;
    spec->nb = nb;
    spec->adaptive = adaptive;
    spec->orth_tol = orth_tol;
    if (final_pass) *final_pass = fp;
    for (int b = 0; b < nb; ++b) done[b] = true;
    return QCUR_OK;
  };
  if (spec && Xp) spec = nullptr;
  bool second = passes >= 2;
  bool have_g2 = false;
  if (passes == 0) {
    // adaptive: keep the first pass when its orthogonality defect
    // ||Q1^H Q1 - I||_F is below orth_tol, else run the second
    HIPCHK(launch_gemm_batched(c, QCUR_OP_H, QCUR_OP_N, 1.0, Q1, Q1, 0.0, G, QCUR_F64, w.gws, w.gws_bytes, bzg));
    have_g2 = true;
    HIPCHK(launch_defect_batch(c, nb, w.G, qq, gslab, qb, w.part, w.norms + 3, 4));
    HIPCHK(launch_sumsq_batch(c, nb, Pr, w.part, w.norms + 2, 4));
    if (spec) return decide_async(true, 1);
    double nrm[4 * MAXB];
    CHK(decide_and_read(nrm));
    for (int b = 0; b < nb; ++b) second |= ok[b] && !(nrm[4 * b + 3] <= orth_tol * orth_tol);
  }
  if (second) {
    // pass 2: G = Q1^H Q1 = L2 L2^H;  P = L2^{-1} L1^{-1} = T^{-H} with Z = Q T
    if (!have_g2)
      HIPCHK(launch_gemm_batched(c, QCUR_OP_H, QCUR_OP_N, 1.0, Q1, Q1, 0.0, G, QCUR_F64, w.gws, w.gws_bytes, bzg));
    if (padded) HIPCHK(launch_pad_identity(c, w.G, qq, gslab, nb, qb));
    CHK(chol_inv(c, w, w.P2));
    HIPCHK(launch_gemm_batched(c, QCUR_OP_N, QCUR_OP_N, 1.0, P2, P1, 0.0, P, QCUR_F64, w.gws, w.gws_bytes, bg));
    for (int b = 0; b < nb; ++b) Pr[b] = QView{w.P + b * gslab, qb[b], qb[b], qq, qq * qq, QCUR_F64};
    HIPCHK(launch_sumsq_batch(c, nb, Pr, w.part, w.norms + 2, 4));
    HIPCHK(launch_gemm_batched(c, QCUR_OP_N, QCUR_OP_H, 1.0, Q1, P2, 0.0, Q, QCUR_F64, w.gws, w.gws_bytes, bzp));
    Pf = w.P;
    Qf = w.Q;
    if (spec && passes == 2) return decide_async(false, 2);
    CHK(decide_and_read());
  } else if (passes == 1) {
    HIPCHK(launch_sumsq_batch(c, nb, Pr, w.part, w.norms + 2, 4));
    if (spec) return decide_async(false, 1);
    CHK(decide_and_read());
  }
  if (final_pass) *final_pass = second ? 2 : 1;
  // Z^+ = T^{-1} Q^H = P^H Q^H;  for a wide X, X^+ = (Z^+)^H = Q P.  Without
  // Xp the factors stay in the group's Q and P slots (orthonormal form).
  for (int b = 0; b < nb; ++b) {
    if (!ok[b]) continue;
    if (!Xp) {
      done[b] = true;
      continue;
    }
    QView Pv{Pf + b * gslab, qb[b], qb[b], qq, qq * qq, QCUR_F64};
    QView Qv{Qf + b * zslab, pb[b], qb[b], qq, pp * qq, QCUR_F64};
    BatchSpec one;
    if (tall[b]) {
      one.tri = TRI_A_UPPER;  // op(A) = P^H
      HIPCHK(launch_gemm_batched(c, QCUR_OP_H, QCUR_OP_H, 1.0, Pv, Qv, 0.0, Xp[b], QCUR_F64, w.gws, w.gws_bytes, one));
    } else {
      one.tri = TRI_B_LOWER;  // op(B) = P
      HIPCHK(launch_gemm_batched(c, QCUR_OP_N, QCUR_OP_N, 1.0, Qv, Pv, 0.0, Xp[b], QCUR_F64, w.gws, w.gws_bytes, one));
    }
    done[b] = true;
  }
  return QCUR_OK;
}

// Cyclic one-sided Jacobi sweeps on the working matrix (too large for the
// single-workgroup kernel), one launch per round of disjoint pairs, until a
// sweep makes no rotation.  Pairs of negligible columns (below the
// truncation threshold set by rtol) are left alone.
qcur_status jacobi_sweeps(const Ctx& c, const PinvWs& w, int64_t pp, int64_t qq, double tol, double rtol) {
  double* cmax = (double*)((char*)w.flag + 64);
  unsigned* bad = (unsigned*)((char*)w.flag + 128);
  HIPCHK(launch_zero(c, cmax, 2));  // the two alternating slots of the running maximum
  const int64_t qpad = (qq + 1) / 2 * 2;
  // negligible pairs: first the per-column bound rtol sigma_max / 2, checked
  // on the result; if the skipped columns add up to more, sweeps go on with
  // the bound divided by sqrt(q)
  double drop2 = rtol > 0.0 ? rtol * rtol / 4.0 : 0.0;
  int launches = 0;  // round launches so far: selects the slot each one reads
  for (int attempt = 0; attempt < 2; ++attempt) {
    unsigned host_flag = 1;
    for (int sweep = 0; sweep < MAX_SWEEPS && host_flag; ++sweep) {
      HIPCHK(launch_zero_i32(c, (int*)w.flag, 1));
      for (int round = 0; round < qpad - 1; ++round)
        HIPCHK(launch_jacobi_round(c, w.Y, pp, qq, w.V, qpad, round, tol, w.flag, drop2, cmax, launches++));
      HIPCHK(hipMemcpyAsync(&host_flag, w.flag, sizeof(unsigned), hipMemcpyDeviceToHost, c.stream));
      HIPCHK(hipStreamSynchronize(c.stream));
    }
    if (drop2 == 0.0 || attempt == 1) break;
    unsigned host_bad = 0;
    HIPCHK(launch_deflation_check(c, w.Y, pp, qq, drop2, rtol * rtol / 4.0, bad));
    HIPCHK(hipMemcpyAsync(&host_bad, bad, sizeof(unsigned), hipMemcpyDeviceToHost, c.stream));
    HIPCHK(hipStreamSynchronize(c.stream));
    if (!host_bad) break;
    drop2 = rtol * rtol / (4.0 * (double)qq);
  }
  return QCUR_OK;
}

// Jacobi path: X (any dtype) -> Xp (F64, q x p).
qcur_status pinv_jacobi(const Ctx& c, QView X, double rtol, int64_t max_rank, QView Xp, int64_t* rank_out,
                        PinvWs w) {
  PinvPlan pl = pinv_plan(X.rows, X.cols);
  const int64_t pp = pl.pp, qq = pl.qq;
  // column rows of the tall working matrix Z (Z = X or X^H)
  QView Yv{w.Y, qq, pp, pp, qq * pp, QCUR_F64};
  HIPCHK(launch_cast(c, X, Yv, pl.tall ? CAST_T : CAST_CONJ));
  HIPCHK(launch_fill_identity(c, w.V, qq));
  const double tol = std::sqrt((double)pp) * std::ldexp(1.0, -53);
  if (jacobi_small_fits(pp, qq)) {
    HIPCHK(launch_jacobi_small(c, w.Y, pp, qq, w.V, tol, MAX_SWEEPS, w.flag));
  } else {
    CHK(jacobi_sweeps(c, w, pp, qq, tol, rtol));
  }
  HIPCHK(launch_pinv_scale(c, w.Y, pp, qq, rtol, max_rank, rank_out, w.sig));
  HIPCHK(launch_pinv_apply(c, w.Y, pp, qq, w.V, w.sig + qq));
  // Ydc = conj(D Yc) (qq x pp), Vcc = conj(Vc) (qq x qq)
  QView Ydc{w.Y, qq, pp, pp, qq * pp, QCUR_F64};
  QView Vcc{w.V, qq, qq, qq, qq * qq, QCUR_F64};
  if (pl.tall) {
    HIPCHK(launch_gemm(c, QCUR_OP_H, QCUR_OP_N, 1.0, Vcc, Ydc, 0.0, Xp, QCUR_F64, w.gws, w.gws_bytes));
  } else {
    HIPCHK(launch_gemm(c, QCUR_OP_H, QCUR_OP_N, 1.0, Ydc, Vcc, 0.0, Xp, QCUR_F64, w.gws, w.gws_bytes));
  }
  return QCUR_OK;
}

// Jacobi path in orthonormal form: Z^+ = P^H Q^H written into the views
// Q (pp x qq) and P (qq x qq).
qcur_status pinv_jacobi_qp(const Ctx& c, QView X, double rtol, int64_t max_rank, QView Qv, QView Pv,
                           int64_t* rank_out, PinvWs w) {
  PinvPlan pl = pinv_plan(X.rows, X.cols);
  const int64_t pp = pl.pp, qq = pl.qq;
  QView Yv{w.Y, qq, pp, pp, qq * pp, QCUR_F64};
  HIPCHK(launch_cast(c, X, Yv, pl.tall ? CAST_T : CAST_CONJ));
  HIPCHK(launch_fill_identity(c, w.V, qq));
  const double tol = std::sqrt((double)pp) * std::ldexp(1.0, -53);
  if (jacobi_small_fits(pp, qq)) {
    HIPCHK(launch_jacobi_small(c, w.Y, pp, qq, w.V, tol, MAX_SWEEPS, w.flag));
  } else {
    CHK(jacobi_sweeps(c, w, pp, qq, tol, rtol));
  }
  HIPCHK(launch_pinv_scale(c, w.Y, pp, qq, rtol, max_rank, rank_out, w.sig));
  HIPCHK(launch_pinv_qp(c, w.Y, pp, qq, w.V, w.sig + qq, Qv, Pv));
  return QCUR_OK;
}

// Orthonormal factors of nb matrices (any dtype), FP64: for each X_b with
// Z_b = X_b (tall) or X_b^H (wide), Z_b^+ = P_b^H Q_b^H with Q_b
// (pp_b x qq_b, orthonormal or zero columns) and P_b (qq_b x qq_b) left in
// the views Qv[b], Pv[b] inside the group workspace.  CholeskyQR2 where its
// certificate holds, else the Jacobi SVD.
// Matrices that skip the CholeskyQR attempt and go straight to the Jacobi
// SVD: those that fit one workgroup's LDS and whose rank is capped below
// their order (the certificate would reject the fast path anyway).  Small
// matrices without a cap take the fast path first: the one-workgroup Jacobi
// costs about a millisecond at 300 x 16, the CholeskyQR group tens of
// microseconds.
bool jacobi_direct(const PinvPlan& pl, int64_t max_rank) {
  return jacobi_small_fits(pl.pp, pl.qq) && max_rank > 0 && max_rank < pl.qq;
}

// Rank-capped pseudoinverse (cap k, 2k <= min(p, q), FP64) by subspace
// iteration in place of the Jacobi SVD of the whole matrix (Algorithm 1's
// predefined rank k; the truncated pseudoinverse X_k^+ of Section 2.1):
//   Q = orth(X S)   (S a fixed pseudo-random q x k sketch, one CholeskyQR pass)
//   repeat:  V = orth(X^H Q) (CholeskyQR2),  Y = X V = Q T (CholeskyQR2), P = T^{-H}
// and X^+ ~ V Y^+ = V (Q P)^H, the pseudoinverse of X V V^H.  Each iteration
// ends in an a posteriori bound on the relative distance of that result from
// X_k^+: with G = X^H X, the Rayleigh-Ritz residual R = G V - V (Y^H Y) and
// the separation delta = 1/||P||_F^2 - (||X||_F^2 - ||Y||_F^2) (a lower
// bound on the smallest eigenvalue of Y^H Y minus an upper bound on the
// (k+1)-th of G), the Davis-Kahan theorem gives ||sin Theta(V, V_k)||_F <=
// ||R||_F / delta; then ||X V V^H - X_k||_F <= 2 sigma_1 ||sin Theta||_F, and
// pseudoinverses of equal-rank matrices move by at most sqrt(2) ||A^+||_2
// ||B^+||_2 ||A - B||_F (Wedin), so the relative distance is at most
//   2 sqrt(2) ||X||_F ||P||_F ||R||_F / delta.
// Accepted below 2^-30 (CholeskyQR's own certificates holding too); up to
// three iterations while the bound at least halves, else the Jacobi SVD.  A
// rank below k, a small gap sigma_k / sigma_{k+1} or a cap that cuts
// through a cluster of singular values all end there.
constexpr double LOWRANK_TOL = 0x1p-30;
constexpr int LOWRANK_ITERS = 3;
constexpr uint64_t LOWRANK_SEED = 0x2402191470ull;

struct LowrankWs {
  GroupWs g;  // CholeskyQR of the p x k and q x k matrices
  double *A1, *A2, *A3, *A4, *sums;
};

bool lowrank_route(const PinvPlan& pl, int64_t max_rank, int dt) {
  return dt == QCUR_F64 && max_rank > 0 && 2 * max_rank <= pl.qq;
}

// The route's buffers lie over the Jacobi buffers Y and V and over the
// CholeskyQR group of the whole matrix, neither of which is in use while it
// runs.  False when they do not fit.
bool lowrank_carve(const PinvPlan& pl, int64_t k, const PinvWs& jw, const GroupWs& gw, LowrankWs* w) {
  Bump cg(nullptr), cl(nullptr);
  group_carve(cg, 1, pl.pp, pl.qq);
  group_carve(cl, 1, pl.pp, k);
  if (cl.used > cg.used) return false;
  Bump gb(gw.Z);
  w->g = group_carve(gb, 1, pl.pp, k);
  const size_t avail = (size_t)((char*)jw.V - (char*)jw.Y) + (size_t)4 * pl.qq * pl.qq * 8;
  Bump ab(jw.Y);
  w->A1 = (double*)ab.take((size_t)4 * pl.pp * k * 8);
  w->A2 = (double*)ab.take((size_t)4 * pl.q * k * 8);
  w->A3 = (double*)ab.take((size_t)4 * pl.p * k * 8);
  w->A4 = (double*)ab.take((size_t)4 * k * k * 8);
  w->sums = (double*)ab.take(4 * 8);
  return ab.used <= avail;
}

qcur_status pinv_lowrank(const Ctx& c, QView X, double rtol, int64_t k, QView Xp, int64_t* rank_out,
                         const PinvWs& jw, const GroupWs& gw, bool* accepted) {
  *accepted = false;
  const PinvPlan pl = pinv_plan(X.rows, X.cols);
  LowrankWs w;
  if (!lowrank_carve(pl, k, jw, gw, &w)) return QCUR_OK;
  const int64_t p = X.rows, q = X.cols, slot = pl.pp * k;
  auto mat = [](double* base, int64_t rows, int64_t cols) {
    return QView{base, rows, cols, cols, rows * cols, QCUR_F64};
  };
  const QView S = mat(w.A1, q, k), R = mat(w.A1, q, k), T1 = mat(w.A1, p, k);
  const QView V = mat(w.A2, q, k), Y = mat(w.A3, p, k), Hm = mat(w.A4, k, k);
  void* gws = jw.gws;
  const size_t gwb = jw.gws_bytes;
  int64_t* none[1] = {nullptr};
  int64_t* ro[1] = {rank_out};
  bool done = false;
  HIPCHK(launch_check_finite(c, X));
  HIPCHK(launch_sumsq_batch(c, 1, &X, w.g.part, w.sums + 0, 1));
  HIPCHK(launch_sketch(c, S, LOWRANK_SEED));
  HIPCHK(launch_gemm(c, QCUR_OP_N, QCUR_OP_N, 1.0, X, S, 0.0, Y, QCUR_F64, gws, gwb));
  CHK(pinv_fast_group(c, 1, &Y, rtol, 0, nullptr, none, w.g, 1, &done));
  if (!done) return QCUR_OK;
  QView Qc{w.g.Q1, p, k, k, slot, QCUR_F64};
  double last = INFINITY;
  for (int it = 0; it < LOWRANK_ITERS; ++it) {
    // V = orth(X^H Q), moved out of the group, which Y's factorisation reuses
    HIPCHK(launch_gemm(c, QCUR_OP_H, QCUR_OP_N, 1.0, X, Qc, 0.0, V, QCUR_F64, gws, gwb));
    CHK(pinv_fast_group(c, 1, &V, rtol, 0, nullptr, none, w.g, 2, &done));
    if (!done) return QCUR_OK;
    HIPCHK(launch_cast(c, QView{w.g.Q, q, k, k, slot, QCUR_F64}, V, CAST_COPY));
    // Y = X V, H = Y^H Y, R = X^H Y - V H and their norms
    HIPCHK(launch_gemm(c, QCUR_OP_N, QCUR_OP_N, 1.0, X, V, 0.0, Y, QCUR_F64, gws, gwb));
    HIPCHK(launch_gemm(c, QCUR_OP_H, QCUR_OP_N, 1.0, Y, Y, 0.0, Hm, QCUR_F64, gws, gwb));
    HIPCHK(launch_gemm(c, QCUR_OP_H, QCUR_OP_N, 1.0, X, Y, 0.0, R, QCUR_F64, gws, gwb));
    HIPCHK(launch_gemm(c, QCUR_OP_N, QCUR_OP_N, -1.0, V, Hm, 1.0, R, QCUR_F64, gws, gwb));
    HIPCHK(launch_sumsq_batch(c, 1, &R, w.g.part, w.sums + 1, 1));
    HIPCHK(launch_sumsq_batch(c, 1, &Y, w.g.part, w.sums + 2, 1));
    // Y = Q T with its certificate (this waits for the stream)
    CHK(pinv_fast_group(c, 1, &Y, rtol, 0, nullptr, ro, w.g, 2, &done));
    if (!done) return QCUR_OK;
    double h[3], nrm[4];
    HIPCHK(hipMemcpyAsync(h, w.sums, sizeof(h), hipMemcpyDeviceToHost, c.stream));
    HIPCHK(hipMemcpyAsync(nrm, w.g.norms, sizeof(nrm), hipMemcpyDeviceToHost, c.stream));
    HIPCHK(hipStreamSynchronize(c.stream));
    const double nx2 = h[0], rho2 = h[1], ny2 = h[2], pf2 = nrm[2];
    // the tail ||X||_F^2 - ||Y||_F^2 with room for the rounding of both sums
    const double eta2 = std::max(0.0, nx2 - ny2) + 0x1p-46 * (double)(p + q) * nx2;
    const double delta = 1.0 / pf2 - eta2;
    const double bound = delta > 0.0 ? 2.0 * std::sqrt(2.0) * std::sqrt(nx2 * pf2 * rho2) / delta : INFINITY;
    if (bound <= LOWRANK_TOL) {
      // X^+ = V (Q P)^H
      BatchSpec lo;
      lo.tri = TRI_B_LOWER;
      HIPCHK(launch_gemm_batched(c, QCUR_OP_N, QCUR_OP_N, 1.0, QView{w.g.Q, p, k, k, slot, QCUR_F64},
                                 QView{w.g.P, k, k, k, k * k, QCUR_F64}, 0.0, T1, QCUR_F64, gws, gwb, lo));
      HIPCHK(launch_gemm(c, QCUR_OP_N, QCUR_OP_H, 1.0, V, T1, 0.0, Xp, QCUR_F64, gws, gwb));
      *accepted = true;
      return QCUR_OK;
    }
    if (!(bound < 0.5 * last)) return QCUR_OK;
    last = bound;
    Qc = QView{w.g.Q, p, k, k, slot, QCUR_F64};
  }
  return QCUR_OK;
}

qcur_status pinv_group_qp(const Ctx& c, int nb, const QView* X, double rtol, int64_t max_rank,
                          int64_t* const* rank_out, GroupWs& gw, PinvWs jw, QView* Qv, QView* Pv,
                          double orth_tol, PinvSpec* spec = nullptr) {
  const int64_t pp = gw.pp, qq = gw.qq;
  const int64_t zslab = 4 * pp * qq, gslab = 4 * qq * qq;
  QView fx[MAXB];
  int64_t* fr[MAXB];
  int idx[MAXB], small[MAXB];
  int nf = 0, ns = 0;
  double rt[MAXB];
  for (int b = 0; b < nb; ++b) {
    PinvPlan pl = pinv_plan(X[b].rows, X[b].cols);
    rt[b] = rtol < 0 ? (double)std::max(pl.p, pl.q) * std::ldexp(1.0, -52) : rtol;
    if (pl.qq == 0) {
      if (rank_out[b]) HIPCHK(launch_zero(c, (double*)rank_out[b], 1));
      Qv[b] = QView{gw.Q, pl.pp, 0, 1, 1, QCUR_F64};
      Pv[b] = QView{gw.P, 0, 0, 1, 1, QCUR_F64};
      continue;
    }
    if (jacobi_direct(pl, max_rank)) {
      HIPCHK(launch_check_finite(c, X[b]));  // the CholeskyQR group checks in its cast
      small[ns++] = b;
      continue;
    }
    fx[nf] = X[b];
    fr[nf] = rank_out[b];
    idx[nf] = b;
    ++nf;
  }
  // slots: the CholeskyQR problems first, then the small ones; the factors
  // live in the buffers of the last CholeskyQR pass that ran
  int final_pass = 2;
  auto slot = [&](int s, int b) {
    PinvPlan pl = pinv_plan(X[b].rows, X[b].cols);
    double* qb = final_pass == 2 ? gw.Q : gw.Q1;
    double* pb = final_pass == 2 ? gw.P : gw.P1;
    Qv[b] = QView{qb + s * zslab, pl.pp, pl.qq, qq, pp * qq, QCUR_F64};
    Pv[b] = QView{pb + s * gslab, pl.qq, pl.qq, qq, qq * qq, QCUR_F64};
  };
  if (nf > 0) {
    bool done[MAXB];
    double rg = 0.0;
    for (int f = 0; f < nf; ++f) rg = std::max(rg, rt[idx[f]]);
    GroupWs w = gw;
    w.nb = nf;
    CHK(pinv_fast_group(c, nf, fx, rg, max_rank, nullptr, fr, w, orth_tol > 0.0 ? 0 : 2, done, orth_tol,
                        &final_pass, spec));
    for (int f = 0; f < nf; ++f) {
      slot(f, idx[f]);
      if (!done[f]) CHK(pinv_jacobi_qp(c, fx[f], rt[idx[f]], max_rank, Qv[idx[f]], Pv[idx[f]], fr[f], jw));
    }
  }
  for (int k = 0; k < ns; ++k) {
    const int b = small[k];
    slot(nf + k, b);
    CHK(pinv_jacobi_qp(c, X[b], rt[b], max_rank, Qv[b], Pv[b], rank_out[b], jw));
  }
  return QCUR_OK;
}

// Pseudoinverses of nb matrices (any dtype) into Xp (F64): small ones by
// single-workgroup Jacobi, the rest by the CholeskyQR group with a Jacobi
// fallback for each matrix whose certificate fails.
qcur_status pinv_group(const Ctx& c, int nb, const QView* X, double rtol, int64_t max_rank, const QView* Xp,
                       int64_t* const* rank_out, GroupWs& gw, PinvWs jw, int passes) {
  QView fx[MAXB], fxp[MAXB];
  int64_t* fr[MAXB];
  int idx[MAXB];
  int nf = 0;
  double rt[MAXB];
  for (int b = 0; b < nb; ++b) {
    PinvPlan pl = pinv_plan(X[b].rows, X[b].cols);
    rt[b] = rtol < 0 ? (double)std::max(pl.p, pl.q) * std::ldexp(1.0, -52) : rtol;
    if (pl.qq == 0) {
      if (rank_out[b]) HIPCHK(launch_zero(c, (double*)rank_out[b], 1));
      continue;
    }
    if (jacobi_direct(pl, max_rank)) {
      HIPCHK(launch_check_finite(c, X[b]));  // the CholeskyQR group checks in its cast
      CHK(pinv_jacobi(c, X[b], rt[b], max_rank, Xp[b], rank_out[b], jw));
      continue;
    }
    if (lowrank_route(pl, max_rank, X[b].dt) && nb == 1) {
      // a rank cap: subspace iteration, else the Jacobi SVD (the CholeskyQR
      // certificate of the whole matrix would reject it)
      bool ok = false;
      CHK(pinv_lowrank(c, X[b], rt[b], max_rank, Xp[b], rank_out[b], jw, gw, &ok));
      if (!ok) CHK(pinv_jacobi(c, X[b], rt[b], max_rank, Xp[b], rank_out[b], jw));
      continue;
    }
    fx[nf] = X[b];
    fxp[nf] = Xp[b];
    fr[nf] = rank_out[b];
    idx[nf] = b;
    ++nf;
  }
  if (nf == 0) return QCUR_OK;
  bool done[MAXB];
  // the certificate uses the largest default tolerance of the group
  double rg = 0.0;
  for (int f = 0; f < nf; ++f) rg = std::max(rg, rt[idx[f]]);
  GroupWs w = gw;
  w.nb = nf;
  CHK(pinv_fast_group(c, nf, fx, rg, max_rank, fxp, fr, w, passes, done));
  for (int f = 0; f < nf; ++f)
    if (!done[f]) CHK(pinv_jacobi(c, fx[f], rt[idx[f]], max_rank, fxp[f], fr[f], jw));
  return QCUR_OK;
}

qcur_status pinv_impl(const Ctx& c, QView X, double rtol, int64_t max_rank, QView Xp, int64_t* rank_out,
                      PinvWs jw, GroupWs gw, int passes = 2) {
  int64_t* ro[1] = {rank_out};
  return pinv_group(c, 1, &X, rtol, max_rank, &Xp, ro, gw, jw, passes);
}

// Returns X itself when it already has dtype dt, else a converted copy.
QView as_dtype(const Ctx& c, QView X, int dt, Bump& b, bool count_only, hipError_t* err) {
  if (X.dt == dt) return X;
  QView Y = b.mat(X.rows, X.cols, dt);
  if (!count_only) *err = launch_cast(c, X, Y, CAST_COPY);
  return Y;
}

// ---- approx -----------------------------------------------------------------
struct ApproxArgs {
  QView A, C, R, W, U, B;
  bool hasA, hasC, hasR, hasW, hasB;
  double* fro;  // least-squares core: ||A - CUR||_F (device double[1]) or NULL
  int core, compute, refine;
  double rtol;
  int64_t max_rank;
  int64_t* rank_out;
};

// Runs (or, with a null workspace base, only sizes) the approx pipeline.
qcur_status approx_run(const Ctx& c, const ApproxArgs& a, int64_t m, int64_t n, int64_t cc, int64_t r, Bump& b,
                       bool count_only) {
  hipError_t err = hipSuccess;
  const int idt = in_dt(a.compute), adt = acc_dt(a.compute);
  if (a.core == QCUR_CORE_WPINV) {
    // U = W^+ (c x r), FP64, then converted to the output dtype
    QView U64 = a.U.dt == QCUR_F64 ? a.U : b.mat(cc, r, QCUR_F64);
    PinvWs w = pinv_carve(b, r, cc);
    PinvPlan pl = pinv_plan(r, cc);
    GroupWs gw = group_carve(b, 1, pl.pp, pl.qq);
    if (!count_only) {
      CHK(pinv_impl(c, a.W, a.rtol, a.max_rank, U64, a.rank_out, w, gw));
      if (a.rank_out) HIPCHK(hipMemcpyAsync(a.rank_out + 1, a.rank_out, 8, hipMemcpyDeviceToDevice, c.stream));
      if (U64.p != a.U.p) HIPCHK(launch_cast(c, U64, a.U, CAST_COPY));
    }
  } else {
    // Least-squares core in orthonormal form.  C = Q_C T_C and R^H = Q_R T_R
    // (CholeskyQR2 or Jacobi, FP64) give C^+ = P_C^H Q_C^H and
    // R^+ = Q_R P_R with P = T^{-H}; then
    //   U = P_C^H M P_R,  M = Q_C^H A Q_R,  C U R = Q_C M Q_R^H.
    // The products that touch A use the orthonormal Q's in the product
    // dtype, so their rounding stays near u ||A|| whatever the conditioning
    // of C and R; only the small factors P meet M, in FP64.
    QView Qv[2], Pv[2];
    PinvPlan pc = pinv_plan(m, cc), pr = pinv_plan(r, n);
    const int64_t pp = std::max(pc.pp, pr.pp), qq = std::max(pc.qq, pr.qq);
    Bump pb = b;
    PinvWs jw = pinv_carve(pb, pp, qq);
    GroupWs gw = group_carve(pb, 2, pp, qq);
    b.used = pb.used;
    QView xs[2] = {a.C, a.R};
    int64_t* ro[2] = {a.rank_out, a.rank_out ? a.rank_out + 1 : nullptr};
    // FP64 products: CholeskyQR2; FP32/BF16 products: a second pass only
    // when the first leaves Q^H Q - I above the bound orth_bound gives
    const double orth_tol = orth_bound(a.compute, a.refine);
    // operands in the product dtype (Q_C, Q_R are cast into fixed buffers,
    // so that a recomputation reuses them)
    QView Ax = as_dtype(c, a.A, idt, b, count_only, &err);
    if (err != hipSuccess) return fail(QCUR_ERR_DEVICE, "cast: %s", hipGetErrorString(err));
    QView QcB = idt == QCUR_F64 ? QView{} : b.mat(m, cc, idt);
    QView QrB = idt == QCUR_F64 ? QView{} : b.mat(n, r, idt);
    QView T = b.mat(m, r, adt);
    QView Tx = (idt == adt) ? T : b.mat(m, r, idt);
    QView M = b.mat(cc, r, adt);
    QView Mx = (idt == adt) ? M : b.mat(cc, r, idt);
    QView B1 = b.mat(m, r, adt);
    QView B1x = (idt == adt) ? B1 : b.mat(m, r, idt);
    QView M64 = adt == QCUR_F64 ? M : b.mat(cc, r, QCUR_F64);
    QView W1 = b.mat(cc, r, QCUR_F64);
    QView U64 = a.U.dt == QCUR_F64 ? a.U : b.mat(cc, r, QCUR_F64);
    const bool need_E = a.refine > 0;
    QView E = need_E ? b.mat(m, n, adt) : QView{};
    QView Ex = need_E ? ((idt == adt) ? E : b.mat(m, n, idt)) : QView{};
    // the last refinement step's correction, its sums of squares and the
    // flag that tells the residual product it is not needed
    const bool ident = need_E && a.fro && !a.hasB && (adt == QCUR_F32 || adt == QCUR_F64);
    QView Dm = ident ? b.mat(cc, r, adt) : QView{};
    double* dpart = ident ? (double*)b.take(CORE_PARTS * 8) : nullptr;
    int* rskip = ident ? (int*)b.take(8) : nullptr;
    double* part = (double*)b.take(std::max<size_t>(residual_tiles(m, n, a.compute), 1) * 8);
    size_t gw_bytes = std::max({gemm_workspace(m, r, n, a.compute), gemm_workspace(cc, r, m, a.compute),
                                gemm_workspace(m, r, cc, a.compute), gemm_workspace(m, n, r, a.compute),
                                gemm_workspace(cc, r, r, QCUR_F64), gemm_workspace(cc, r, cc, QCUR_F64)});
    void* gws = b.take(gw_bytes);
    if (count_only) return QCUR_OK;
    // Everything after the factors: M = Q_C^H (A Q_R), refinement, residual,
    // B and U = P_C^H M P_R.
    auto products = [&]() -> qcur_status {
      QView Qc = Qv[0], Qr = Qv[1];
      if (idt != QCUR_F64) {
        // dense copies with the factors' shapes (same element counts as the
        // buffers carved above)
        const QView Qc2{QcB.p, Qc.rows, Qc.cols, Qc.cols, Qc.rows * Qc.cols, idt};
        const QView Qr2{QrB.p, Qr.rows, Qr.cols, Qr.cols, Qr.rows * Qr.cols, idt};
        const QView qs[2] = {Qc, Qr}, qd[2] = {Qc2, Qr2};
        const int cm[2] = {CAST_COPY, CAST_COPY};
        HIPCHK(launch_cast_set(c, 2, qs, qd, cm));
        Qc = Qc2;
        Qr = Qr2;
      }
      const size_t gw = gw_bytes;
      HIPCHK(launch_gemm(c, QCUR_OP_N, QCUR_OP_N, 1.0, Ax, Qr, 0.0, T, a.compute, gws, gw));
      if (Tx.p != T.p) HIPCHK(launch_cast(c, T, Tx, CAST_COPY));
      HIPCHK(launch_gemm(c, QCUR_OP_H, QCUR_OP_N, 1.0, Qc, Tx, 0.0, M, a.compute, gws, gw));
      // B1 = Q_C M in the product dtype (not written when *skip is set)
      auto left_factor = [&](const int* skip) -> qcur_status {
        if (Mx.p != M.p) HIPCHK(launch_cast(c, M, Mx, CAST_COPY));
        BatchSpec one;
        one.skip = skip;
        HIPCHK(launch_gemm_batched(c, QCUR_OP_N, QCUR_OP_N, 1.0, Qc, Mx, 0.0, B1, a.compute, gws, gw, one));
        if (B1x.p != B1.p) HIPCHK(launch_cast(c, B1, B1x, CAST_COPY));
        return QCUR_OK;
      };
      const int* skip_final = nullptr;
      for (int st = 0; st < a.refine; ++st) {
        // E = A - Q_C M Q_R^H (A in the precision it was given);  M += Q_C^H (E Q_R)
        CHK(left_factor(nullptr));
        HIPCHK(launch_residual_gemm(c, a.A, B1x, Qr, nullptr, 0, a.compute, part, &E, 1.0, QCUR_OP_H));
        if (Ex.p != E.p) HIPCHK(launch_cast(c, E, Ex, CAST_COPY));
        HIPCHK(launch_gemm(c, QCUR_OP_N, QCUR_OP_N, 1.0, Ex, Qr, 0.0, T, a.compute, gws, gw));
        if (Tx.p != T.p) HIPCHK(launch_cast(c, T, Tx, CAST_COPY));
        if (ident && st == a.refine - 1) {
          // the last step keeps its correction D apart: with ||E||^2 from the
          // residual's partials, ||A - Q_C (M + D) Q_R^H|| follows without
          // another m x n product when D is small next to E
          HIPCHK(launch_gemm(c, QCUR_OP_H, QCUR_OP_N, 1.0, Qc, Tx, 0.0, Dm, a.compute, gws, gw));
          HIPCHK(launch_core_correct(c, M, Dm, dpart));
          HIPCHK(launch_resid_identity(c, part, (int64_t)residual_tiles(m, n, a.compute), dpart,
                                       resid_identity_gate(a.compute), a.fro, rskip));
          skip_final = rskip;
        } else {
          HIPCHK(launch_gemm(c, QCUR_OP_H, QCUR_OP_N, 1.0, Qc, Tx, 1.0, M, a.compute, gws, gw));
        }
      }
      if (a.fro || a.hasB) CHK(left_factor(skip_final));
      if (a.fro) {
        // ||A - C U R||_F = ||A - Q_C M Q_R^H||_F (and C U R itself when asked, from the same tiles)
        HIPCHK(launch_residual_gemm(c, a.A, B1x, Qr, nullptr, 0, a.compute, part, nullptr, 0.0, QCUR_OP_H,
                                    a.hasB ? &a.B : nullptr, skip_final));
        HIPCHK(launch_sum_partials(c, part, (int64_t)residual_tiles(m, n, a.compute), a.fro, 1, skip_final));
      } else if (a.hasB) {
        HIPCHK(launch_gemm(c, QCUR_OP_N, QCUR_OP_H, 1.0, B1x, Qr, 0.0, a.B, a.compute, gws, gw));
      }
      // U = P_C^H (M P_R) in FP64
      if (M64.p != M.p) HIPCHK(launch_cast(c, M, M64, CAST_COPY));
      HIPCHK(launch_gemm(c, QCUR_OP_N, QCUR_OP_N, 1.0, M64, Pv[1], 0.0, W1, QCUR_F64, gws, gw));
      HIPCHK(launch_gemm(c, QCUR_OP_H, QCUR_OP_N, 1.0, Pv[0], W1, 0.0, U64, QCUR_F64, gws, gw));
      if (U64.p != a.U.p) HIPCHK(launch_cast(c, U64, a.U, CAST_COPY));
      return QCUR_OK;
    };
    // The factors' certificate needs one host synchronisation.  When the
    // products are cheap next to that round trip (A Q_R at most 4e10 flops,
    // about 0.4 ms), the products of the fast path are enqueued before it, so
    // the GPU stays busy while the host waits; if the certificate then
    // rejects the fast path (or asks for a second CholeskyQR pass), the
    // factors are recomputed without speculation and the products run again.
    // Larger problems wait first: a rejected guess would cost more than the
    // round trip saves.
    PinvSpec spec;
    const bool speculate = 32.0 * (double)m * (double)n * (double)r <= 4e10;
    CHK(pinv_group_qp(c, 2, xs, a.rtol, a.max_rank, ro, gw, jw, Qv, Pv, orth_tol, speculate ? &spec : nullptr));
    CHK(products());
    bool valid = true;
    CHK(pinv_spec_resolve(c, spec, &valid));
    if (!valid) {
      CHK(pinv_group_qp(c, 2, xs, a.rtol, a.max_rank, ro, gw, jw, Qv, Pv, orth_tol));
      CHK(products());
    }
    return QCUR_OK;
  }
  if (a.hasB) {
    // B = (C U) R for the intersection core
    QView Cx = as_dtype(c, a.C, idt, b, count_only, &err);
    QView Rx = as_dtype(c, a.R, idt, b, count_only, &err);
    QView Ux = as_dtype(c, a.U, idt, b, count_only, &err);
    if (err != hipSuccess) return fail(QCUR_ERR_DEVICE, "cast: %s", hipGetErrorString(err));
    QView B1 = b.mat(m, r, adt);
    QView B1x = (idt == adt) ? B1 : b.mat(m, r, idt);
    size_t gw = std::max(gemm_workspace(m, r, cc, a.compute), gemm_workspace(m, n, r, a.compute));
    void* gws = b.take(gw);
    if (!count_only) {
      HIPCHK(launch_gemm(c, QCUR_OP_N, QCUR_OP_N, 1.0, Cx, Ux, 0.0, B1, a.compute, gws, gw));
      if (B1x.p != B1.p) HIPCHK(launch_cast(c, B1, B1x, CAST_COPY));
      HIPCHK(launch_gemm(c, QCUR_OP_N, QCUR_OP_N, 1.0, B1x, Rx, 0.0, a.B, a.compute, gws, gw));
    }
  }
  return QCUR_OK;
}

// Shapes of U/B views used for sizing only.
ApproxArgs sizing_args(int64_t m, int64_t n, int64_t cc, int64_t r, int core, int compute) {
  ApproxArgs a{};
  const int adt = acc_dt(compute);
  a.A = QView{nullptr, m, n, n, m * n, compute == QCUR_F64 ? QCUR_F64 : QCUR_F32};
  a.C = QView{nullptr, m, cc, cc, m * cc, compute};
  a.R = QView{nullptr, r, n, n, r * n, compute};
  a.W = QView{nullptr, r, cc, cc, r * cc, compute};
  a.U = QView{nullptr, cc, r, r, cc * r, adt};
  a.B = QView{nullptr, m, n, n, m * n, adt};
  a.core = core;
  a.compute = compute;
  a.refine = 1;
  a.hasB = true;
  return a;
}

// ---- residual ---------------------------------------------------------------
qcur_status residual_run(const Ctx& c, QView A, QView C, QView U, QView R, const uint8_t* mask, int64_t mask_ld,
                         int compute, double* out, int take_sqrt, QView* E, double e_scale, Bump& b,
                         bool count_only) {
  hipError_t err = hipSuccess;
  const int idt = in_dt(compute), adt = acc_dt(compute);
  const int64_t m = A.rows, n = A.cols, r = R.rows;
  QView Cx = as_dtype(c, C, idt, b, count_only, &err);
  QView Ux = as_dtype(c, U, idt, b, count_only, &err);
  QView Rx = as_dtype(c, R, idt, b, count_only, &err);
  if (err != hipSuccess) return fail(QCUR_ERR_DEVICE, "cast: %s", hipGetErrorString(err));
  QView B1 = b.mat(m, r, adt);
  QView B1x = (idt == adt) ? B1 : b.mat(m, r, idt);
  size_t gw = gemm_workspace(m, r, C.cols, compute);
  void* gws = b.take(gw);
  double* part = (double*)b.take(std::max<size_t>(residual_tiles(m, n, compute), 1) * 8);
  if (count_only) return QCUR_OK;
  HIPCHK(launch_gemm(c, QCUR_OP_N, QCUR_OP_N, 1.0, Cx, Ux, 0.0, B1, compute, gws, gw));
  if (B1x.p != B1.p) HIPCHK(launch_cast(c, B1, B1x, CAST_COPY));
  HIPCHK(launch_residual_gemm(c, A, B1x, Rx, mask, mask_ld, compute, part, E, e_scale));
  HIPCHK(launch_sum_partials(c, part, (int64_t)residual_tiles(m, n, compute), out, take_sqrt));
  return QCUR_OK;
}

// ---- backward ---------------------------------------------------------------
struct BwdArgs {
  QView A, gB, dA;
  bool hasgB, hasdA;
  const int64_t* I;
  const int64_t* J;
  int64_t r, cc;
  const uint8_t* mask;
  int64_t mask_ld;
  double rtol;
  int64_t max_rank;
  int compute;
  double* loss;
};

qcur_status backward_run(const Ctx& c, const BwdArgs& a, Bump& b, bool count_only) {
  const int dt = a.compute;  // F64 or F32 for every large operand
  const int64_t m = a.A.rows, n = a.A.cols, r = a.r, cc = a.cc;
  QView C = b.mat(m, cc, dt), R = b.mat(r, n, dt), W = b.mat(r, cc, QCUR_F64);
  QView U64 = b.mat(cc, r, QCUR_F64);
  QView Ux = dt == QCUR_F64 ? U64 : b.mat(cc, r, dt);
  QView G = b.mat(m, n, dt);  // 2 P_Omega(A - CUR) in loss mode
  QView X1 = b.mat(m, r, dt), X2 = b.mat(cc, n, dt);
  QView gC = b.mat(m, cc, dt), gR = b.mat(r, n, dt), gU = b.mat(cc, r, dt);
  QView gU64 = dt == QCUR_F64 ? gU : b.mat(cc, r, QCUR_F64);
  // pinv adjoint temporaries (FP64)
  QView Q1 = b.mat(r, r, QCUR_F64), M2 = b.mat(r, r, QCUR_F64), Q3 = b.mat(r, cc, QCUR_F64);
  QView Q4 = b.mat(r, cc, QCUR_F64), M3 = b.mat(cc, cc, QCUR_F64), gW = b.mat(r, cc, QCUR_F64);
  QView Q2 = b.mat(r, r, QCUR_F64);
  int32_t* iinv = (int32_t*)b.take((size_t)std::max<int64_t>(m, 1) * 4);
  int32_t* jinv = (int32_t*)b.take((size_t)std::max<int64_t>(n, 1) * 4);
  const size_t gw = std::max({gemm_workspace(m, r, n, dt), gemm_workspace(m, cc, r, dt),
                              gemm_workspace(cc, n, m, dt), gemm_workspace(r, n, cc, dt),
                              gemm_workspace(cc, r, m, dt), gemm_workspace(r, r, cc, QCUR_F64),
                              gemm_workspace(r, cc, r, QCUR_F64), gemm_workspace(cc, cc, r, QCUR_F64),
                              gemm_workspace(r, cc, cc, QCUR_F64)});
  void* gws = b.take(gw);
  // the rest is shared: first the pinv of W, then the residual pass
  const Bump shared = b;
  Bump t1 = shared;
  PinvWs pw = pinv_carve(t1, r, cc);
  PinvPlan wpl = pinv_plan(r, cc);
  GroupWs pgw = group_carve(t1, 1, wpl.pp, wpl.qq);
  Bump t2 = shared;
  double* lossbuf = (double*)t2.take(8);
  CHK(residual_run(c, a.A, C, Ux, R, a.mask, a.mask_ld, dt, nullptr, 0, nullptr, 0.0, t2, true));
  b.used = std::max(t1.used, t2.used);
  if (count_only) return QCUR_OK;

  HIPCHK(launch_gather(c, a.A, a.I, r, a.J, cc, &C, &R, &W));
  HIPCHK(launch_inverse_map(c, a.I, r, m, iinv));
  HIPCHK(launch_inverse_map(c, a.J, cc, n, jinv));
  // U = W^+ recomputed (not stored by the forward pass)
  CHK(pinv_impl(c, W, a.rtol, a.max_rank, U64, nullptr, pw, pgw));
  if (Ux.p != U64.p) HIPCHK(launch_cast(c, U64, Ux, CAST_COPY));
  double sgn;
  QView Gb;
  if (a.hasgB) {
    Gb = a.gB;
    sgn = 1.0;
  } else {
    // G = 2 P_Omega(A - C U R), loss = ||P_Omega(A - CUR)||^2; the cotangent of B is -G
    Bump t = shared;
    t.take(8);
    double* lossp = a.loss ? a.loss : lossbuf;
    CHK(residual_run(c, a.A, C, Ux, R, a.mask, a.mask_ld, dt, lossp, 0, a.hasdA ? &G : nullptr, 2.0, t, false));
    if (!a.hasdA) return QCUR_OK;  // the loss alone
    Gb = G;
    sgn = -1.0;
  }
  // X1 = Gb R^H (m x r);  gC = sgn X1 U^H (m x c)
  HIPCHK(launch_gemm(c, QCUR_OP_N, QCUR_OP_H, 1.0, Gb, R, 0.0, X1, dt, gws, gw));
  HIPCHK(launch_gemm(c, QCUR_OP_N, QCUR_OP_H, sgn, X1, Ux, 0.0, gC, dt, gws, gw));
  // X2 = C^H Gb (c x n);  gR = sgn U^H X2 (r x n)
  HIPCHK(launch_gemm(c, QCUR_OP_H, QCUR_OP_N, 1.0, C, Gb, 0.0, X2, dt, gws, gw));
  HIPCHK(launch_gemm(c, QCUR_OP_H, QCUR_OP_N, sgn, Ux, X2, 0.0, gR, dt, gws, gw));
  // gU = sgn C^H X1 (c x r)
  HIPCHK(launch_gemm(c, QCUR_OP_H, QCUR_OP_N, sgn, C, X1, 0.0, gU, dt, gws, gw));
  if (gU64.p != gU.p) HIPCHK(launch_cast(c, gU, gU64, CAST_COPY));
  // gW = -U^H gU U^H + (I - W U) gU^H U U^H + U^H U gU^H (I - U W)   (FP64)
  HIPCHK(launch_gemm(c, QCUR_OP_H, QCUR_OP_N, 1.0, U64, gU64, 0.0, Q1, QCUR_F64, gws, gw));   // U^H gU
  HIPCHK(launch_gemm(c, QCUR_OP_N, QCUR_OP_H, -1.0, Q1, U64, 0.0, gW, QCUR_F64, gws, gw));    // t1
  HIPCHK(launch_gemm(c, QCUR_OP_N, QCUR_OP_N, 1.0, W, U64, 0.0, M2, QCUR_F64, gws, gw));      // W U
  HIPCHK(launch_identity_minus(c, M2));                                                     // I - W U
  HIPCHK(launch_gemm(c, QCUR_OP_H, QCUR_OP_N, 1.0, gU64, U64, 0.0, Q2, QCUR_F64, gws, gw));   // gU^H U
  HIPCHK(launch_gemm(c, QCUR_OP_N, QCUR_OP_H, 1.0, Q2, U64, 0.0, Q3, QCUR_F64, gws, gw));     // gU^H U U^H
  HIPCHK(launch_gemm(c, QCUR_OP_N, QCUR_OP_N, 1.0, M2, Q3, 1.0, gW, QCUR_F64, gws, gw));      // + t2
  HIPCHK(launch_gemm(c, QCUR_OP_H, QCUR_OP_N, 1.0, U64, U64, 0.0, Q1, QCUR_F64, gws, gw));    // U^H U
  HIPCHK(launch_gemm(c, QCUR_OP_N, QCUR_OP_H, 1.0, Q1, gU64, 0.0, Q4, QCUR_F64, gws, gw));    // U^H U gU^H
  HIPCHK(launch_gemm(c, QCUR_OP_N, QCUR_OP_N, 1.0, U64, W, 0.0, M3, QCUR_F64, gws, gw));      // U W
  HIPCHK(launch_identity_minus(c, M3));                                                     // I - U W
  HIPCHK(launch_gemm(c, QCUR_OP_N, QCUR_OP_N, 1.0, Q4, M3, 1.0, gW, QCUR_F64, gws, gw));      // + t3
  HIPCHK(launch_backward_assemble(c, a.dA, G, a.hasgB ? 0 : 1, gC, gR, gW, iinv, jinv));
  return QCUR_OK;
}

// ---- whole solve ------------------------------------------------------------
struct SolveArgs {
  QView A;
  int64_t c, r;
  int sampling, core, compute, with_replacement, refine;
  uint64_t seed;
  double rtol;
  int64_t max_rank;
  int64_t *I, *J;
  QView U;
  double* residual;
  int64_t* rank_out;
  double *p, *q;
  const QView *C, *R, *W;  // optional caller buffers for the gathers
  const QView* B;           // optional output C U R
};

// Algorithm 1 end to end: probabilities, the two draws in one launch, the
// gathers, the core and the residual, all on the handle's stream.
qcur_status solve_run(const Ctx& c, const SolveArgs& s, Bump& b, bool count_only) {
  const int64_t m = s.A.rows, n = s.A.cols;
  double* p = s.p ? s.p : (double*)b.take((size_t)n * 8);
  double* q = s.q ? s.q : (double*)b.take((size_t)m * 8);
  int rb, nrb, ncb;
  probs_grid(m, n, &rb, &nrb, &ncb);
  const bool pass = s.sampling == QCUR_LENGTH;
  double* colpart = (double*)b.take(pass ? (size_t)nrb * n * 8 : 8);
  double* rowpart = (double*)b.take(pass ? (size_t)ncb * m * 8 : 8);
  double* f2 = (double*)b.take(8);
  QView C = s.C ? *s.C : b.mat(m, s.c, s.A.dt);
  QView R = s.R ? *s.R : b.mat(s.r, n, s.A.dt);
  QView W = s.W ? *s.W : b.mat(s.r, s.c, s.A.dt);
  ApproxArgs a{};
  a.A = s.A;
  a.C = C;
  a.R = R;
  a.W = W;
  a.U = s.U;
  a.hasB = s.B != nullptr;
  if (s.B) a.B = *s.B;
  a.core = s.core;
  a.compute = s.compute;
  a.refine = s.core == QCUR_CORE_CAR ? s.refine : 0;
  a.rtol = s.rtol;
  a.max_rank = s.max_rank;
  int64_t* ranks = s.rank_out ? s.rank_out : (int64_t*)b.take(16);
  a.rank_out = ranks;
  // the least-squares core computes the residual itself (orthonormal form)
  const bool car = s.core == QCUR_CORE_CAR;
  a.fro = car ? s.residual : nullptr;
  const size_t base = b.used;
  Bump ta = b;
  CHK(approx_run(c, a, m, n, s.c, s.r, ta, true));
  Bump tr = b;
  if (!car) CHK(residual_run(c, s.A, C, s.U, R, nullptr, 0, s.compute, nullptr, 1, nullptr, 0.0, tr, true));
  b.used = std::max(ta.used, tr.used);
  if (count_only) return QCUR_OK;
  if (pass) {
    HIPCHK(launch_probs_partials(c, s.A, colpart, rowpart, rb, ncb));
    HIPCHK(launch_probs_finish(c, m, n, colpart, rowpart, nrb, ncb, s.sampling, p, q, f2, nullptr));
  } else {
    HIPCHK(launch_probs_finish(c, m, n, nullptr, nullptr, 0, 0, s.sampling, p, q, nullptr, nullptr));
  }
  HIPCHK(launch_draw_pair(c, p, n, s.c, 0, s.J, q, m, s.r, 1, s.I, s.seed, s.with_replacement));
  HIPCHK(launch_gather(c, s.A, s.I, s.r, s.J, s.c, &C, &R, s.core == QCUR_CORE_WPINV || s.W ? &W : nullptr));
  {
    Bump run(b.base);
    run.used = base;
    CHK(approx_run(c, a, m, n, s.c, s.r, run, false));
  }
  if (!car) {
    Bump run(b.base);
    run.used = base;
    CHK(residual_run(c, s.A, C, s.U, R, nullptr, 0, s.compute, s.residual, 1, nullptr, 0.0, run, false));
  }
  return QCUR_OK;
}


// ---- batched solve ----------------------------------------------------------
struct BatchShape {
  int count;
  const int32_t* dims;  // host [count][4]: m, n, c, r
  int64_t mx, nx, cx, rx;
  int a_dt, sampling, compute, refine;
  int autotune;
};

constexpr int TUNE_MAX_SPLITS = 4;

struct BatchWs {
  int *dm, *dn, *dc, *dr, *zp, *zq, *order, *forder;  // header (uploaded by qcur_batch_prepare)
  double *colpart, *rowpart, *p, *q;
  Slots Ax;
  double *Z, *G, *L, *P1, *P2, *P, *Sch, *Q1, *Q, *norms;
  int *fail, *ok, *zq2, *skip;
  double *Y, *V;
  Slots Qcx, Qrx, T, Tx, M, Mx, B1, B1x, E, Ex, M64, W1, U64;
  // the last refinement step's corrections D_b, their sums of squares and
  // the per-problem flags that skip the final residual products
  Slots Dm;
  double* dpart;
  int* rskip;
  double* part;
  int64_t tiles, tiles32;
  int64_t* ranks;
  void* gws;
  size_t gws_bytes;
  int64_t px, qx;
};

Slots slots_of(Bump& b, int count, int64_t rows, int64_t cols, int dt) {
  Slots s;
  s.ld = std::max<int64_t>(cols, 1);
  s.ps = std::max<int64_t>(rows, 1) * s.ld;
  s.slab = 4 * s.ps;
  s.dt = dt;
  s.p = b.take((size_t)count * s.slab * dtype_size(dt));
  return s;
}

QView slot_view(const Slots& s, int64_t rows, int64_t cols) { return QView{s.p, rows, cols, s.ld, s.ps, s.dt}; }

Slots sl(double* p, int64_t rows, int64_t /*cols*/, int64_t ld) {
  return Slots{p, ld, rows * ld, 4 * rows * ld, QCUR_F64};
}

// Workspace layout of a batch; the same code sizes (null base) and carves.
BatchWs batch_carve(Bump& b, const BatchShape& s) {
  BatchWs w{};
  const int n = s.count, n2 = 2 * s.count;
  const int idt = in_dt(s.compute), adt = acc_dt(s.compute);
  w.dm = (int*)b.take((size_t)n * 4);
  w.dn = (int*)b.take((size_t)n * 4);
  w.dc = (int*)b.take((size_t)n * 4);
  w.dr = (int*)b.take((size_t)n * 4);
  w.zp = (int*)b.take((size_t)n2 * 4);
  w.zq = (int*)b.take((size_t)n2 * 4);
  w.order = (int*)b.take((size_t)n * 4);
  w.forder = (int*)b.take((size_t)n2 * 4);
  const int64_t nrbx = (s.mx + BATCH_RB - 1) / BATCH_RB, ncbx = (s.nx + BATCH_CB - 1) / BATCH_CB;
  w.colpart = (double*)b.take((size_t)n * nrbx * s.nx * 8);
  w.rowpart = (double*)b.take((size_t)n * ncbx * s.mx * 8);
  w.p = (double*)b.take((size_t)n * s.nx * 8);
  w.q = (double*)b.take((size_t)n * s.mx * 8);
  w.Ax = s.a_dt != idt ? slots_of(b, n, s.mx, s.nx, idt) : Slots{};
  // FP64 factor slots: Z_t = C_b (t = b) or R_b^H (t = count + b), px x qx
  // with qx a multiple of 4 (rows of whole runs for the tall products)
  w.px = std::max(s.mx, s.nx);
  w.qx = (std::max(s.cx, s.rx) + 3) / 4 * 4;
  const size_t gsl = (size_t)n2 * 4 * w.qx * w.qx * 8, zsl = (size_t)n2 * 4 * w.px * w.qx * 8;
  w.Z = (double*)b.take(zsl);
  w.G = (double*)b.take(gsl);
  w.L = (double*)b.take(gsl);
  w.P1 = (double*)b.take(gsl);
  w.Sch = (double*)b.take((size_t)n2 * 4 * CHOL_BLOCK * w.qx * 8);
  w.Q = (double*)b.take(zsl);
  w.P2 = (double*)b.take(gsl);
  w.P = (double*)b.take(gsl);
  w.Q1 = (double*)b.take(zsl);
  w.norms = (double*)b.take((size_t)n2 * 4 * 8);
  w.fail = (int*)b.take((size_t)n2 * 4);
  w.ok = (int*)b.take((size_t)n2 * 4);
  w.zq2 = (int*)b.take((size_t)n2 * 4);
  w.skip = (int*)b.take((size_t)n2 * 4);
  w.Y = (double*)b.take(zsl);
  w.V = (double*)b.take(gsl);
  if (idt != QCUR_F64) {
    w.Qcx = slots_of(b, n, s.mx, s.cx, idt);
    w.Qrx = slots_of(b, n, s.nx, s.rx, idt);
  }
  w.T = slots_of(b, n, s.mx, s.rx, adt);
  w.Tx = idt != adt ? slots_of(b, n, s.mx, s.rx, idt) : w.T;
  w.M = slots_of(b, n, s.cx, s.rx, adt);
  w.Mx = idt != adt ? slots_of(b, n, s.cx, s.rx, idt) : w.M;
  w.B1 = slots_of(b, n, s.mx, s.rx, adt);
  w.B1x = idt != adt ? slots_of(b, n, s.mx, s.rx, idt) : w.B1;
  if (s.refine > 0) {
    w.E = slots_of(b, n, s.mx, s.nx, adt);
    w.Ex = idt != adt ? slots_of(b, n, s.mx, s.nx, idt) : w.E;
    if (adt == QCUR_F32 || adt == QCUR_F64) {
      w.Dm = slots_of(b, n, s.cx, s.rx, adt);
      w.dpart = (double*)b.take((size_t)n * CORE_PARTS * 8);
      w.rskip = (int*)b.take((size_t)n * 4);
    }
  }
  w.M64 = adt != QCUR_F64 ? slots_of(b, n, s.cx, s.rx, QCUR_F64) : w.M;
  w.W1 = slots_of(b, n, s.cx, s.rx, QCUR_F64);
  w.U64 = adt != QCUR_F64 ? slots_of(b, n, s.cx, s.rx, QCUR_F64) : Slots{};
  w.tiles = (int64_t)((s.mx + 63) / 64) * ((s.nx + 63) / 64);
  w.tiles32 = (int64_t)((s.mx + 31) / 32) * ((s.nx + 31) / 32);
  w.part = (double*)b.take((size_t)n * (s.autotune ? w.tiles32 : w.tiles) * 8);
  w.ranks = (int64_t*)b.take((size_t)n * 2 * 8);
  const int64_t px = w.px, qx = w.qx;
  const int cp = s.compute;
  w.gws_bytes = std::max({gemm_workspace(qx, qx, px, QCUR_F64, n), gemm_workspace(qx, qx, qx, QCUR_F64, n2),
                          gemm_workspace(px, qx, qx, QCUR_F64, n), gemm_workspace(px, qx, qx, QCUR_F64, n2),
                          gemm_workspace(qx, qx, px, QCUR_F64, n2), gemm_workspace(s.mx, s.rx, s.nx, cp, n),
                          gemm_workspace(s.cx, s.rx, s.mx, cp, n), gemm_workspace(s.mx, s.rx, s.cx, cp, n),
                          gemm_workspace(s.cx, s.rx, qx, QCUR_F64, n)});
  if (s.autotune) {
    // room for every candidate plan (up to TUNE_MAX_SPLITS slices of K)
    const int T = TUNE_MAX_SPLITS;
    w.gws_bytes = std::max({w.gws_bytes, gemm_workspace_splits(qx, qx, QCUR_F64, n2, T),
                            gemm_workspace_splits(px, qx, QCUR_F64, n2, T),
                            gemm_workspace_splits(s.mx, s.rx, cp, n, T), gemm_workspace_splits(s.cx, s.rx, cp, n, T),
                            gemm_workspace_splits(s.cx, s.rx, QCUR_F64, n, T)});
  }
  w.gws = b.take(w.gws_bytes);
  return w;
}

uint64_t batch_key(const BatchShape& s) {
  uint64_t h = 1469598103934665603ull;
  auto mix = [&](uint64_t v) {
    for (int k = 0; k < 8; ++k) {
      h ^= (v >> (8 * k)) & 0xff;
      h *= 1099511628211ull;
    }
  };
  mix((uint64_t)s.count);
  for (int64_t e = 0; e < 4 * (int64_t)s.count; ++e) mix((uint64_t)(uint32_t)s.dims[e]);
  mix((uint64_t)s.a_dt);
  mix((uint64_t)s.sampling);
  mix((uint64_t)s.compute);
  mix((uint64_t)(s.refine > 0));
  mix((uint64_t)s.autotune);
  return h;
}

constexpr int64_t BATCH_MAX_SIDE = 4096;

qcur_status check_batch_shape(int count, const int32_t* dims, int a_dt, int sampling, int compute, int refine,
                              int with_replacement, int autotune, BatchShape* out) {
  if (count < 1 || count > 16384) return fail(QCUR_ERR_ARG, "count must be in [1, 16384]");
  if (!dims) return fail(QCUR_ERR_ARG, "dims is NULL");
  if (!valid_dtype(a_dt)) return fail(QCUR_ERR_DTYPE, "unknown dtype of A");
  if (compute == QCUR_BF16X3) return fail(QCUR_ERR_UNSUPPORTED, "split BF16 is not offered for batches");
  if (!valid_dtype(compute)) return fail(QCUR_ERR_DTYPE, "unknown compute dtype");
  if (sampling != QCUR_LENGTH && sampling != QCUR_UNIFORM) return fail(QCUR_ERR_ARG, "unknown sampling %d", sampling);
  if (refine < 0) return fail(QCUR_ERR_ARG, "refine_steps must be >= 0");
  if (autotune != 0 && autotune != 1) return fail(QCUR_ERR_ARG, "autotune must be 0 or 1");
  BatchShape s{};
  s.count = count;
  s.autotune = autotune;
  s.dims = dims;
  for (int b = 0; b < count; ++b) {
    const int64_t m = dims[4 * b], n = dims[4 * b + 1], c = dims[4 * b + 2], r = dims[4 * b + 3];
    if (m < 1 || n < 1 || m > BATCH_MAX_SIDE || n > BATCH_MAX_SIDE)
      return fail(QCUR_ERR_SHAPE, "problem %d: m and n must be in [1, %lld]", b, (long long)BATCH_MAX_SIDE);
    if (c < 1 || r < 1 || c > JB_MAXQ || r > JB_MAXQ)
      return fail(QCUR_ERR_SHAPE, "problem %d: c and r must be in [1, %d]", b, JB_MAXQ);
    if (!with_replacement && (c > n || r > m))
      return fail(QCUR_ERR_SHAPE, "problem %d: c > n or r > m without replacement", b);
    s.mx = std::max(s.mx, m);
    s.nx = std::max(s.nx, n);
    s.cx = std::max(s.cx, c);
    s.rx = std::max(s.rx, r);
  }
  s.a_dt = a_dt;
  s.sampling = sampling;
  s.compute = compute;
  s.refine = refine;
  *out = s;
  return QCUR_OK;
}

// A slotted operand: rows x cols at least (mx, nx), slots bstride apart.
qcur_status check_slotted(const qcur_qmat* X, const char* name, int64_t rows, int64_t cols, int64_t bstride) {
  CHK(check_qmat(X, name));
  if (X->rows < rows || X->cols < cols)
    return fail(QCUR_ERR_SHAPE, "%s slots are %lldx%lld, need at least %lldx%lld", name, (long long)X->rows,
                (long long)X->cols, (long long)rows, (long long)cols);
  if (bstride < 3 * X->pstride + (X->rows - 1) * X->ld + X->cols)
    return fail(QCUR_ERR_SHAPE, "%s: slots overlap (bstride too small)", name);
  return QCUR_OK;
}

struct BatchArgs {
  Slots A;
  uint64_t seed;
  int repl;
  double rtol;
  int64_t max_rank;
  int64_t *I, *J;
  Slots U;
  double* residual;
  int64_t* rank_out;
  double *p, *q;
  Slots B;  // optional C_b U_b R_b (B.p == nullptr: not formed)
};

BatchSpec bspec(int count, const Slots& A, const Slots& B, const Slots& D, const int* M, const int* N,
                const int* K, int tri = 0) {
  BatchSpec bs;
  bs.tri = tri;
  bs.count = count;
  bs.sA = A.slab;
  bs.sB = B.slab;
  bs.sD = D.slab;
  bs.M = M;
  bs.N = N;
  bs.K = K;
  return bs;
}

// The batched pipeline: one pass of launches over all problems, no host
// synchronisation, so a caller may capture it in a graph.
//
// The least-squares core is evaluated in an orthonormal form.  Each tall
// Z = C_b or R_b^H is factored Z = Q T (CholeskyQR, or the Jacobi SVD where
// the certificate fails) with Z^+ = P^H Q^H, P = T^{-H}.  Then
//   U = C^+ A R^+ = P_C^H M P_R,   M = Q_C^H A Q_R,   C U R = Q_C M Q_R^H,
// so the products that touch A run on the orthonormal Q's in the product
// dtype (rounding errors stay near u ||A||, whatever the conditioning of C
// and R), and only the small triangular factors P meet M, in FP64.
qcur_status batch_run(const Ctx& c, const BatchShape& s, const BatchArgs& a, BatchWs& w, BatchTuning* tu) {
  const int n = s.count, n2 = 2 * n;
  const int idt = in_dt(s.compute), adt = acc_dt(s.compute);
  const int64_t mx = s.mx, nx = s.nx, cx = s.cx, rx = s.rx, px = w.px, qx = w.qx;
  const bool cast_A = s.a_dt != idt;
  Slots resid_R{};
  int64_t resid_tiles = w.tiles;
  int resid_tile_of = 64;

  // One GEMM stage: with the autotuner measuring, every candidate plan (tile
  // 32 or 64, 1..TUNE_MAX_SPLITS slices of K) is timed on the real operands
  // and the fastest kept; stages that accumulate into D (beta != 0) reuse the
  // plan of their beta = 0 twin.  The last launch uses the kept plan.
  auto timed = [&](auto&& launch, float* ms) -> qcur_status {
    HIPCHK(launch());
    HIPCHK(hipEventRecord(tu->e0, c.stream));
    HIPCHK(launch());
    HIPCHK(launch());
    HIPCHK(hipEventRecord(tu->e1, c.stream));
    HIPCHK(hipEventSynchronize(tu->e1));
    HIPCHK(hipEventElapsedTime(ms, tu->e0, tu->e1));
    return QCUR_OK;
  };
  auto stage = [&](int id, int opA, int opB, double alpha, QView A, QView B, double beta, QView D, int compute,
                   BatchSpec bs) -> qcur_status {
    if (tu && tu->measure && beta == 0.0 && tu->plan[id].tile == 0) {
      float best = INFINITY;
      StagePlan bp{};
      for (int tile : {32, 64})
        for (int sp = 1; sp <= TUNE_MAX_SPLITS; sp *= 2) {
          BatchSpec t = bs;
          t.tile = tile;
          t.splits = sp;
          float ms = 0.f;
          CHK(timed([&] { return launch_gemm_batched(c, opA, opB, alpha, A, B, beta, D, compute, w.gws, w.gws_bytes, t); },
                    &ms));
          if (ms < best) {
            best = ms;
            bp = StagePlan{tile, sp};
          }
        }
      tu->plan[id] = bp;
    }
    if (tu) {
      bs.tile = tu->plan[id].tile;
      bs.splits = tu->plan[id].splits;
    }
    if (bs.count == n) bs.order = w.order;  // (an order of the problems, not of the 2 count factors)
    HIPCHK(launch_gemm_batched(c, opA, opB, alpha, A, B, beta, D, compute, w.gws, w.gws_bytes, bs));
    return QCUR_OK;
  };
  auto resid = [&](const Slots* E, const Slots* Bout, const int* skip) -> qcur_status {
    auto run = [&](int tile) {
      return launch_residual_gemm_batched(c, s.count, a.A, w.B1x, resid_R, QCUR_OP_H, s.mx, s.nx, s.rx, w.dm, w.dn,
                                          w.dr, s.compute, w.part, E, 1.0, tile, Bout, w.order, skip);
    };
    if (tu && tu->measure && tu->plan[BS_RESID].tile == 0) {
      float t64 = 0.f, t32 = 0.f;
      CHK(timed([&] { return run(64); }, &t64));
      CHK(timed([&] { return run(32); }, &t32));
      tu->plan[BS_RESID].tile = t32 < t64 ? 32 : 64;
    }
    const int tile = (s.autotune && tu && tu->plan[BS_RESID].tile) ? tu->plan[BS_RESID].tile : 64;
    HIPCHK(run(tile));
    resid_tiles = tile == 32 ? w.tiles32 : w.tiles;
    resid_tile_of = tile;
    return QCUR_OK;
  };
  // probabilities and draws
  double* p = a.p ? a.p : w.p;
  double* q = a.q ? a.q : w.q;
  if (s.sampling == QCUR_LENGTH || cast_A)
    HIPCHK(launch_norms_batch(c, n, a.A, w.dm, w.dn, mx, nx, w.colpart, w.rowpart, cast_A ? &w.Ax : nullptr));
  DrawBatch d{};
  d.dm = w.dm; d.dn = w.dn; d.dc = w.dc; d.dr = w.dr;
  d.colpart = w.colpart; d.rowpart = w.rowpart;
  d.mx = mx; d.nx = nx; d.cx = cx; d.rx = rx;
  d.p = p; d.q = q; d.I = a.I; d.J = a.J;
  d.seed = a.seed; d.sampling = s.sampling; d.repl = a.repl;
  HIPCHK(launch_draw_batch(c, n, d));
  // factors of C_b and R_b^H in FP64
  const Slots G = sl(w.G, qx, qx, qx), P1 = sl(w.P1, qx, qx, qx), Q = sl(w.Q, px, qx, qx);
  const Slots Zs = sl(w.Z, px, qx, qx);
  auto half = [&](const Slots& x) {  // the R_b half of a 2*count array
    Slots y = x;
    y.p = (char*)x.p + (size_t)n * x.slab * dtype_size(x.dt);
    return y;
  };
  // gathers straight into the factor slots: Z_b = C_b = A_b(:, J_b) and
  // Z_{count+b} = R_b^H with R_b = A_b(I_b, :)
  HIPCHK(launch_gather_batch(c, n, a.A, w.dm, w.dn, nullptr, 0, a.J, cx, w.dm, w.dc, mx, cx, Zs, nullptr, 0));
  HIPCHK(launch_gather_batch(c, n, a.A, w.dm, w.dn, a.I, rx, nullptr, 0, w.dr, w.dn, rx, nx, half(Zs), nullptr, 1));
  // Gram matrices and Z P^H products of all 2 count factors run in the
  // fragment-streaming kernels with per-problem sizes (launch plans fixed:
  // reported as 16-blocks, not tuned)
  const QView Zv{w.Z, px, qx, qx, px * qx, QCUR_F64}, Q1v{w.Q1, px, qx, qx, px * qx, QCUR_F64};
  const QView Qv{w.Q, px, qx, qx, px * qx, QCUR_F64}, Gv{w.G, qx, qx, qx, qx * qx, QCUR_F64};
  const QView P1v{w.P1, qx, qx, qx, qx * qx, QCUR_F64}, P2v{w.P2, qx, qx, qx, qx * qx, QCUR_F64};
  const int64_t zslab = 4 * px * qx, gslab = 4 * qx * qx;
  auto fixed_stage = [&](int id) {
    if (tu && tu->measure && tu->plan[id].tile == 0) tu->plan[id] = StagePlan{16, 1};
  };
  auto gram = [&](const QView& X, int id) -> qcur_status {  // G_t = X_t^H X_t, lower
    fixed_stage(id);
    HIPCHK(launch_thin_hn(c, QCUR_F64, 1.0, X, X, 0.0, Gv, px, n2, zslab, zslab, gslab, true, nullptr, 0, w.zq,
                          w.zq, w.zp));
    return QCUR_OK;
  };
  // D_t = X_t P_t^H over the leading q_t columns (qd: per-factor orders),
  // and/or its copy in the product dtype into the C and R factor slots
  auto product_copy = [&]() {  // the C and R factor slots in the product dtype
    TallCopy cp{};
    cp.p[0] = w.Qcx.p;
    cp.p[1] = w.Qrx.p;
    cp.ld[0] = w.Qcx.ld;
    cp.ld[1] = w.Qrx.ld;
    cp.ps[0] = w.Qcx.ps;
    cp.ps[1] = w.Qrx.ps;
    cp.slab[0] = w.Qcx.slab;
    cp.slab[1] = w.Qrx.slab;
    cp.dt = idt;
    cp.split = n;
    return cp;
  };
  auto zph = [&](const QView& X, const QView& Pv, const QView* D, const int* qd, bool to_product,
                 int id) -> qcur_status {
    fixed_stage(id);
    const TallCopy cp = to_product ? product_copy() : TallCopy{};
    const QView Dv = D ? *D : QView{nullptr, px, qx, qx, px * qx, QCUR_F64};
    HIPCHK(launch_tall_nh(c, 1.0, X, Pv, 0.0, Dv, qx, n2, zslab, gslab, zslab, true, w.zp, qd, qd,
                          to_product ? &cp : nullptr));
    return QCUR_OK;
  };
  GroupWs gw{};
  gw.nb = n2;
  gw.qq = qx;
  gw.G = w.G;
  gw.L = w.L;
  gw.S = w.Sch;
  gw.fail = w.fail;
  gw.gws = w.gws;
  gw.gws_bytes = w.gws_bytes;
  // Gram matrices that fit one diagonal block are factored over each
  // factor's own order; larger ones get an identity block outside it
  const bool padded = qx > CHOL_BLOCK;
  HIPCHK(launch_zero_i32(c, w.fail, n2));
  // CholeskyQR2: Q1^H Q1 = L2 L2^H, P = P2 P1, Q = Q1 P2^H.  FP64 products
  // always take the second pass; FP32 and BF16 products only for the
  // factors whose first-pass defect ||Q1^H Q1 - I||_F exceeds the bound of
  // the single solve (q2 = 0 and P = P1 for the others, which then skip
  // the second pass's factorisation and products)
  const bool f64 = idt == QCUR_F64;
  const double otol = orth_bound(s.compute, s.refine);
  const Slots P2 = sl(w.P2, qx, qx, qx), P = sl(w.P, qx, qx, qx);
  const int* q2 = w.zq;
  if (!padded) {
    // CholeskyQR2 of every factor (Gram matrices, factors and inverses, Q1
    // with its product-dtype copy, the defect and, where it is needed, the
    // second pass): one launch, one workgroup per factor
    for (int id : {BS_GRAM_C, BS_GRAM_R, BS_Q1_C, BS_Q1_R, BS_G2, BS_P, BS_Q}) fixed_stage(id);
    const TallCopy cp = product_copy();
    HIPCHK(launch_cholqr_batch(c, n2, w.Z, w.Q1, f64 ? w.Q : nullptr, qx, px * qx, zslab, w.P1, w.P, qx, qx * qx,
                               gslab, w.zp, w.zq, w.fail, w.norms, w.zq2, w.skip, otol * otol, f64 ? 0 : 1,
                               f64 ? nullptr : &cp, w.forder));
  } else {
    // G = Z^H Z:  C_b^H C_b  and  R_b R_b^H, one launch
    CHK(gram(Zv, BS_GRAM_C));
    fixed_stage(BS_GRAM_R);
    HIPCHK(launch_pad_gram_batch(c, n2, w.G, qx, G.slab, w.zq));
    gw.dims = w.zq;
    CHK(chol_inv(c, gw, w.P1));
    HIPCHK(launch_sumsq_ragged(c, n2, Zs, w.zp, w.zq, w.norms, 4));
    HIPCHK(launch_sumsq_ragged(c, n2, P1, w.zq, w.zq, w.norms + 1, 4));
    // Q1 = Z P1^H:  C_b P1^H  and  R_b^H P1^H, one launch (with its copy in the
    // product dtype: the orthonormal factors of the factors that keep one pass)
    CHK(zph(Zv, P1v, &Q1v, w.zq, !f64, BS_Q1_C));
    fixed_stage(BS_Q1_R);
    CHK(gram(Q1v, BS_G2));
    if (!f64) {
      HIPCHK(launch_defect_plan_batch(c, n2, w.G, qx, G.slab, w.zq, w.fail, otol * otol, w.P1, w.P, w.zq2, w.skip));
      q2 = w.zq2;
    }
    HIPCHK(launch_pad_gram_batch(c, n2, w.G, qx, G.slab, w.zq));
    gw.dims = q2;
    CHK(chol_inv(c, gw, w.P2));
    CHK(stage(BS_P, QCUR_OP_N, QCUR_OP_N, 1.0, slot_view(P2, qx, qx), slot_view(P1, qx, qx), 0.0,
              slot_view(P, qx, qx), QCUR_F64, bspec(n2, P2, P1, P, q2, q2, q2, TRI_A_LOWER | TRI_B_LOWER)));
    // FP64 products read Q; the others read the product-dtype copy (Q itself
    // is then only written by the Jacobi fallback below)
    CHK(zph(Q1v, P2v, f64 ? &Qv : nullptr, q2, !f64, BS_Q));
  }
  const Slots Pf = P;
  HIPCHK(launch_sumsq_ragged(c, n2, Pf, w.zq, w.zq, w.norms + 2, 4));
  int64_t* ranks = a.rank_out ? a.rank_out : w.ranks;
  HIPCHK(launch_decide_batch(c, n2, n, w.norms, w.fail, a.rtol, a.max_rank, w.zp, w.zq, ranks, w.ok));
  {
    // problems whose certificate failed: Jacobi SVD, same (Q, P) form
    JacobiBatch jb{};
    jb.ok = w.ok;
    jb.Cz = w.Z; jb.cld = qx; jb.cps = px * qx; jb.cslab = zslab;
    jb.Rz = nullptr;  // both halves are tall slots of Z
    jb.dm = w.dm; jb.dn = w.dn; jb.dc = w.dc; jb.dr = w.dr;
    jb.Y = w.Y; jb.V = w.V;
    jb.yslab = 4 * px * qx;
    jb.vslab = 4 * qx * qx;
    jb.Q = (double*)Q.p; jb.qld = Q.ld; jb.qps = Q.ps; jb.qslab = Q.slab;
    jb.P = (double*)Pf.p; jb.pld = Pf.ld; jb.pps = Pf.ps; jb.pslab = Pf.slab;
    jb.rank_out = ranks;
    jb.rtol = a.rtol;
    jb.max_rank = a.max_rank;
    jb.count = n;
    jb.max_sweeps = MAX_SWEEPS;
    HIPCHK(launch_jacobi_pinv_batch(c, jb, n2));
  }
  // orthonormal factors in the product dtype: those of the Jacobi fallback
  // still to be cast (the others were written by the products above)
  Slots Qc = Q, Qr = half(Q);
  if (!f64) {
    HIPCHK(launch_cast_batch(c, n, Q, w.Qcx, w.dm, w.dc, mx, cx, CAST_COPY, w.ok));
    HIPCHK(launch_cast_batch(c, n, half(Q), w.Qrx, w.dn, w.dr, nx, rx, CAST_COPY, w.ok + n));
    Qc = w.Qcx;
    Qr = w.Qrx;
  }
  // M = Q_C^H (A Q_R)
  const Slots Ain = cast_A ? w.Ax : a.A;
  CHK(stage(BS_T, QCUR_OP_N, QCUR_OP_N, 1.0, slot_view(Ain, mx, nx), slot_view(Qr, nx, rx), 0.0,
                             slot_view(w.T, mx, rx), s.compute, bspec(n, Ain, Qr, w.T, w.dm, w.dr, w.dn)));
  if (w.Tx.p != w.T.p) HIPCHK(launch_cast_batch(c, n, w.T, w.Tx, w.dm, w.dr, mx, rx, CAST_COPY));
  CHK(stage(BS_M, QCUR_OP_H, QCUR_OP_N, 1.0, slot_view(Qc, mx, cx), slot_view(w.Tx, mx, rx), 0.0,
                             slot_view(w.M, cx, rx), s.compute, bspec(n, Qc, w.Tx, w.M, w.dc, w.dr, w.dm)));
  // B1 = Q_C M in the product dtype (problem b not written when skip[b] is set)
  auto left_factor = [&](const int* skip) -> qcur_status {
    if (w.Mx.p != w.M.p) HIPCHK(launch_cast_batch(c, n, w.M, w.Mx, w.dc, w.dr, cx, rx, CAST_COPY));
    BatchSpec bs = bspec(n, Qc, w.Mx, w.B1, w.dm, w.dr, w.dc);
    bs.skip = skip;
    CHK(stage(BS_B1, QCUR_OP_N, QCUR_OP_N, 1.0, slot_view(Qc, mx, cx), slot_view(w.Mx, cx, rx), 0.0,
                               slot_view(w.B1, mx, rx), s.compute, bs));
    if (w.B1x.p != w.B1.p) HIPCHK(launch_cast_batch(c, n, w.B1, w.B1x, w.dm, w.dr, mx, rx, CAST_COPY));
    return QCUR_OK;
  };
  // with no C U R asked for, the last step's correction D_b stays apart and
  // the residual of the refined core follows from ||E_b||^2 - ||D_b||^2 where
  // D_b is small next to E_b (as in the single solve)
  const bool ident = s.refine > 0 && !a.B.p && w.Dm.p != nullptr;
  const int* skip_final = nullptr;
  for (int st = 0; st < s.refine; ++st) {
    // E = A - Q_C M Q_R^H;  M += Q_C^H (E Q_R)
    CHK(left_factor(nullptr));
    resid_R = Qr;
    CHK(resid(&w.E, nullptr, nullptr));
    if (w.Ex.p != w.E.p) HIPCHK(launch_cast_batch(c, n, w.E, w.Ex, w.dm, w.dn, mx, nx, CAST_COPY));
    CHK(stage(BS_T, QCUR_OP_N, QCUR_OP_N, 1.0, slot_view(w.Ex, mx, nx), slot_view(Qr, nx, rx), 0.0,
                               slot_view(w.T, mx, rx), s.compute, bspec(n, w.Ex, Qr, w.T, w.dm, w.dr, w.dn)));
    if (w.Tx.p != w.T.p) HIPCHK(launch_cast_batch(c, n, w.T, w.Tx, w.dm, w.dr, mx, rx, CAST_COPY));
    if (ident && st == s.refine - 1) {
      CHK(stage(BS_M, QCUR_OP_H, QCUR_OP_N, 1.0, slot_view(Qc, mx, cx), slot_view(w.Tx, mx, rx), 0.0,
                                 slot_view(w.Dm, cx, rx), s.compute, bspec(n, Qc, w.Tx, w.Dm, w.dc, w.dr, w.dm)));
      HIPCHK(launch_core_correct_batch(c, n, w.M, w.Dm, w.dc, w.dr, w.dpart));
      HIPCHK(launch_resid_identity_batch(c, n, w.part, resid_tiles, (s.nx + resid_tile_of - 1) / resid_tile_of,
                                         resid_tile_of, w.dm, w.dn, w.dpart, resid_identity_gate(s.compute),
                                         a.residual, w.rskip));
      skip_final = w.rskip;
    } else {
      CHK(stage(BS_M, QCUR_OP_H, QCUR_OP_N, 1.0, slot_view(Qc, mx, cx), slot_view(w.Tx, mx, rx), 1.0,
                                 slot_view(w.M, cx, rx), s.compute, bspec(n, Qc, w.Tx, w.M, w.dc, w.dr, w.dm)));
    }
  }
  // residual_b = ||A_b - Q_C M Q_R^H||_F = ||A_b - C_b U_b R_b||_F (and
  // B_b = C_b U_b R_b from the same tiles when asked)
  CHK(left_factor(skip_final));
  resid_R = Qr;
  CHK(resid(nullptr, a.B.p ? &a.B : nullptr, skip_final));
  HIPCHK(launch_resid_sum_batch(c, n, w.part, resid_tiles, (s.nx + resid_tile_of - 1) / resid_tile_of, resid_tile_of,
                                w.dm, w.dn, a.residual, skip_final));
  // U = P_C^H M P_R in FP64
  if (w.M64.p != w.M.p) HIPCHK(launch_cast_batch(c, n, w.M, w.M64, w.dc, w.dr, cx, rx, CAST_COPY));
  CHK(stage(BS_W1, QCUR_OP_N, QCUR_OP_N, 1.0, slot_view(w.M64, cx, rx), slot_view(half(Pf), rx, rx), 0.0,
                             slot_view(w.W1, cx, rx), QCUR_F64, bspec(n, w.M64, Pf, w.W1, w.dc, w.dr, w.dr)));
  const Slots U64 = adt == QCUR_F64 ? a.U : w.U64;
  CHK(stage(BS_U, QCUR_OP_H, QCUR_OP_N, 1.0, slot_view(Pf, cx, cx), slot_view(w.W1, cx, rx), 0.0,
                             slot_view(U64, cx, rx), QCUR_F64, bspec(n, Pf, w.W1, U64, w.dc, w.dr, w.dc)));
  if (U64.p != a.U.p) HIPCHK(launch_cast_batch(c, n, U64, a.U, w.dc, w.dr, cx, rx, CAST_COPY));
  (void)adt;
  return QCUR_OK;
}


// ---- completion (Algorithm 2) ------------------------------------------------
struct CompleteArgs {
  QView Y, X;
  const uint8_t* mask;
  int64_t mask_ld;
  const int64_t *I, *J;
  // index sets drawn again at every step (I, J then point to the caller's
  // output arrays)
  bool resample;
  int sampling;
  uint64_t seed;
  int64_t r, cc;
  int compute;
  double rtol;
  int64_t max_rank;
  int max_iter;
  double tol;
  int* iters;
  double* rel;
};

// X^0 = P_Omega(Y); then M^{t+1} = C U R of X^t (Algorithm 1 on the fixed
// index sets I, J, least-squares core in orthonormal form) and
// X^{t+1} = P_Omega(Y) + P_Omega^c(M^{t+1}) in one fused product, until
// ||X^{t+1} - X^t||_F / ||X^t||_F <= tol or max_iter steps.  The iterates
// alternate between the output X and one workspace copy (with fixed index
// sets and cheap steps they rotate through a ring of workspace copies, so
// that several steps run between host round trips); the last one is left
// in X.
qcur_status complete_run(const Ctx& c, const CompleteArgs& a, Bump& b, bool count_only) {
  const int64_t m = a.Y.rows, n = a.Y.cols, r = a.r, cc = a.cc;
  const int xdt = a.X.dt, idt = in_dt(a.compute), adt = acc_dt(a.compute);
  QView Xw = b.mat(m, n, xdt);
  QView C = b.mat(m, cc, xdt), R = b.mat(r, n, xdt);
  PinvPlan pc = pinv_plan(m, cc), pr = pinv_plan(r, n);
  const int64_t pp = std::max(pc.pp, pr.pp), qq = std::max(pc.qq, pr.qq);
  PinvWs jw = pinv_carve(b, pp, qq);
  GroupWs gw = group_carve(b, 2, pp, qq);
  QView Qc = b.mat(m, cc, idt), Qr = b.mat(n, r, idt);
  QView Xx = (idt == xdt) ? QView{} : b.mat(m, n, idt);
  QView T = b.mat(m, r, adt), Tx = (idt == adt) ? T : b.mat(m, r, idt);
  QView M = b.mat(cc, r, adt), Mx = (idt == adt) ? M : b.mat(cc, r, idt);
  QView B1 = b.mat(m, r, adt), B1x = (idt == adt) ? B1 : b.mat(m, r, idt);
  const int64_t tiles = (int64_t)std::max<size_t>(residual_tiles(m, n, a.compute), 1);
  double* pd = (double*)b.take((size_t)tiles * 8);
  double* po = (double*)b.take((size_t)tiles * 8);
  double* sums = (double*)b.take(16);
  int64_t* ranks = (int64_t*)b.take(16);
  const size_t gwb = std::max({gemm_workspace(m, r, n, a.compute), gemm_workspace(cc, r, m, a.compute),
                              gemm_workspace(m, r, cc, a.compute)});
  void* gws = b.take(gwb);
  // probabilities of the iterate (resampled variant)
  int rb = 0, nrb = 0, ncb = 0;
  probs_grid(m, n, &rb, &nrb, &ncb);
  const bool pass = a.resample && a.sampling == QCUR_LENGTH;
  double* pcol = a.resample ? (double*)b.take((size_t)n * 8) : nullptr;
  double* qrow = a.resample ? (double*)b.take((size_t)m * 8) : nullptr;
  double* colpart = pass ? (double*)b.take((size_t)nrb * n * 8) : nullptr;
  double* rowpart = pass ? (double*)b.take((size_t)ncb * m * 8) : nullptr;
  double* f2 = a.resample ? (double*)b.take(8) : nullptr;
  const bool speculate = 32.0 * (double)m * (double)n * (double)r <= 4e10;
  // Fixed index sets and cheap steps: up to CHUNK steps are enqueued between
  // host round trips.  Each step leaves its certificate verdict, stopping
  // sums and a copy of the status word in a device record; the iterates go to
  // a ring of chunk + 1 buffers (X itself, Xw and more), so that the host,
  // reading the chunk's records at once, can take the iterate of the first
  // step that meets the stopping rule, or go back to the step before a
  // rejected certificate and redo it without speculation.  Steps enqueued
  // past the one that stands are discarded, and so are the status bits they
  // raised.  The ring is held to about 512 MiB.
  constexpr int CHUNK = 8;
  struct StepRec {
    DevVerdict v;
    double sums[2];
    unsigned st;
  };
  const bool chunked = speculate && !a.resample;
  const size_t xbytes = (size_t)4 * m * n * dtype_size(xdt);
  const int chunk = chunked ? (int)std::clamp<size_t>(((size_t)512 << 20) / std::max<size_t>(xbytes, 1), 2, CHUNK) : 0;
  QView ring[CHUNK + 1];
  StepRec* recs = nullptr;
  if (chunked) {
    ring[0] = a.X;
    ring[1] = Xw;
    for (int k = 2; k <= chunk; ++k) ring[k] = b.mat(m, n, xdt);
    recs = (StepRec*)b.take(sizeof(StepRec) * (CHUNK + 1));
  }
  if (count_only) return QCUR_OK;
  HIPCHK(launch_mask_init(c, a.Y, a.mask, a.mask_ld, a.X));
  // the iterate of step t lives in cur; the next goes to nxt
  QView cur = a.X, nxt = Xw;
  const double orth_tol = orth_bound(a.compute, 0);
  int t = 0;
  double rel = INFINITY;
  // one step X^t (cur) -> X^{t+1} (nxt); with spec, the certificate's verdict
  // is left pending (in the device record spec->dev_dst when that is set)
  auto step = [&](QView from, QView to, double* sums_to, PinvSpec* spec) -> qcur_status {
    HIPCHK(launch_gather(c, from, a.I, r, a.J, cc, &C, &R, nullptr));
    QView Qv[2], Pv[2];
    QView xs[2] = {C, R};
    int64_t* ro[2] = {ranks, ranks + 1};
    CHK(pinv_group_qp(c, 2, xs, a.rtol, a.max_rank, ro, gw, jw, Qv, Pv, orth_tol, spec));
    const QView cs[3] = {Qv[0], Qv[1], from}, cd[3] = {Qc, Qr, Xx};
    const int cm[3] = {CAST_COPY, CAST_COPY, CAST_COPY};
    HIPCHK(launch_cast_set(c, Xx.p ? 3 : 2, cs, cd, cm));
    const QView Xin = Xx.p ? Xx : from;
    HIPCHK(launch_gemm(c, QCUR_OP_N, QCUR_OP_N, 1.0, Xin, Qr, 0.0, T, a.compute, gws, gwb));
    if (Tx.p != T.p) HIPCHK(launch_cast(c, T, Tx, CAST_COPY));
    HIPCHK(launch_gemm(c, QCUR_OP_H, QCUR_OP_N, 1.0, Qc, Tx, 0.0, M, a.compute, gws, gwb));
    if (Mx.p != M.p) HIPCHK(launch_cast(c, M, Mx, CAST_COPY));
    HIPCHK(launch_gemm(c, QCUR_OP_N, QCUR_OP_N, 1.0, Qc, Mx, 0.0, B1, a.compute, gws, gwb));
    if (B1x.p != B1.p) HIPCHK(launch_cast(c, B1, B1x, CAST_COPY));
    HIPCHK(launch_merge_gemm(c, a.Y, a.mask, a.mask_ld, from, B1x, Qr, QCUR_OP_H, a.compute, to, pd, po));
    HIPCHK(launch_sum_partials(c, pd, tiles, sums_to, 0));
    HIPCHK(launch_sum_partials(c, po, tiles, sums_to + 1, 0));
    return QCUR_OK;
  };
  auto rel_of = [](const double* h2) {
    return h2[1] > 0.0 ? std::sqrt(h2[0] / h2[1]) : (h2[0] > 0.0 ? INFINITY : 0.0);
  };
  if (chunked) {
    const int ring_n = chunk + 1;
    StepRec* const base = recs + CHUNK;  // status word before the chunk
    int slot = 0;                         // ring slot of X^t
    int hold = 0;   // steps still to run one at a time after a rejection
    int fails = 0;  // chunks rejected in a row
    bool stop = false;
    while (t < a.max_iter && !stop) {
      if (hold > 0) {
        // one step with the host waiting for the certificate's verdict
        // (Jacobi when it fails): after a rejection the next ones are
        // likely rejected too, and a rejected chunk costs up to a chunk of
        // steps; the hold doubles with every chunk rejected in a row
        StepRec h1;
        CHK(step(ring[slot], ring[(slot + 1) % ring_n], recs[0].sums, nullptr));
        HIPCHK(hipMemcpyAsync(h1.sums, recs[0].sums, sizeof(h1.sums), hipMemcpyDeviceToHost, c.stream));
        HIPCHK(hipStreamSynchronize(c.stream));
        rel = rel_of(h1.sums);
        ++t;
        --hold;
        slot = (slot + 1) % ring_n;
        stop = rel <= a.tol;
        continue;
      }
      const int kc = std::min(chunk, a.max_iter - t);
      bool pending[CHUNK];
      PinvSpec specs[CHUNK];
      HIPCHK(hipMemcpyAsync(&base->st, c.status, sizeof(unsigned), hipMemcpyDeviceToDevice, c.stream));
      for (int s = 0; s < kc; ++s) {
        specs[s].dev_dst = &recs[s].v;
        CHK(step(ring[(slot + s) % ring_n], ring[(slot + s + 1) % ring_n], recs[s].sums, &specs[s]));
        HIPCHK(hipMemcpyAsync(&recs[s].st, c.status, sizeof(unsigned), hipMemcpyDeviceToDevice, c.stream));
        pending[s] = specs[s].pending;
      }
      StepRec host[CHUNK];
      HIPCHK(hipMemcpyAsync(host, recs, sizeof(StepRec) * kc, hipMemcpyDeviceToHost, c.stream));
      HIPCHK(hipStreamSynchronize(c.stream));
      int done = kc;  // steps of the chunk that stand
      for (int s = 0; s < kc; ++s) {
        if (pending[s] && !verdict_valid(specs[s], host[s].v.ok, host[s].v.nrm)) {
          done = s;
          hold = chunk << std::min(fails++, 5);
          break;
        }
        rel = rel_of(host[s].sums);
        if (rel <= a.tol) {
          done = s + 1;
          stop = true;
          break;
        }
      }
      if (hold == 0) fails = 0;
      // the status word as the last standing step left it
      if (done < kc) {
        const unsigned* keep = done == 0 ? &base->st : &recs[done - 1].st;
        HIPCHK(hipMemcpyAsync(c.status, keep, sizeof(unsigned), hipMemcpyDeviceToDevice, c.stream));
      }
      t += done;
      slot = (slot + done) % ring_n;
    }
    if (slot != 0) HIPCHK(launch_cast(c, ring[slot], a.X, CAST_COPY));
    if (a.iters) *a.iters = t;
    if (a.rel) *a.rel = rel;
    return QCUR_OK;
  }
  while (t < a.max_iter) {
    if (a.resample) {
      // step t draws J (set 0) and I (set 1) from the probabilities of X^t
      // with seed + t
      if (pass) {
        HIPCHK(launch_probs_partials(c, cur, colpart, rowpart, rb, ncb));
        HIPCHK(launch_probs_finish(c, m, n, colpart, rowpart, nrb, ncb, a.sampling, pcol, qrow, f2, nullptr));
      } else {
        HIPCHK(launch_probs_finish(c, m, n, nullptr, nullptr, 0, 0, a.sampling, pcol, qrow, nullptr, nullptr));
      }
      HIPCHK(launch_draw_pair(c, pcol, n, cc, 0, (int64_t*)a.J, qrow, m, r, 1, (int64_t*)a.I, a.seed + (uint64_t)t, 0));
    }
    HIPCHK(launch_gather(c, cur, a.I, r, a.J, cc, &C, &R, nullptr));
    QView Qv[2], Pv[2];
    QView xs[2] = {C, R};
    int64_t* ro[2] = {ranks, ranks + 1};
    auto products = [&]() -> qcur_status {
      // the factors and, when needed, the iterate in the product dtype:
      // one launch when the dtypes agree
      const QView cs[3] = {Qv[0], Qv[1], cur}, cd[3] = {Qc, Qr, Xx};
      const int cm[3] = {CAST_COPY, CAST_COPY, CAST_COPY};
      HIPCHK(launch_cast_set(c, Xx.p ? 3 : 2, cs, cd, cm));
      QView Xin = cur;
      if (Xx.p) Xin = Xx;
      // M = Q_C^H (X^t Q_R);  B1 = Q_C M;  X^{t+1} = P_Omega(Y) + P_Omega^c(B1 Q_R^H)
      HIPCHK(launch_gemm(c, QCUR_OP_N, QCUR_OP_N, 1.0, Xin, Qr, 0.0, T, a.compute, gws, gwb));
      if (Tx.p != T.p) HIPCHK(launch_cast(c, T, Tx, CAST_COPY));
      HIPCHK(launch_gemm(c, QCUR_OP_H, QCUR_OP_N, 1.0, Qc, Tx, 0.0, M, a.compute, gws, gwb));
      if (Mx.p != M.p) HIPCHK(launch_cast(c, M, Mx, CAST_COPY));
      HIPCHK(launch_gemm(c, QCUR_OP_N, QCUR_OP_N, 1.0, Qc, Mx, 0.0, B1, a.compute, gws, gwb));
      if (B1x.p != B1.p) HIPCHK(launch_cast(c, B1, B1x, CAST_COPY));
      HIPCHK(launch_merge_gemm(c, a.Y, a.mask, a.mask_ld, cur, B1x, Qr, QCUR_OP_H, a.compute, nxt, pd, po));
      HIPCHK(launch_sum_partials(c, pd, tiles, sums, 0));
      HIPCHK(launch_sum_partials(c, po, tiles, sums + 1, 0));
      return QCUR_OK;
    };
    // as in the solve: the step's products are enqueued before the factors'
    // certificate is read when they are cheap, and redone if it rejects them
    PinvSpec spec;
    CHK(pinv_group_qp(c, 2, xs, a.rtol, a.max_rank, ro, gw, jw, Qv, Pv, orth_tol, speculate ? &spec : nullptr));
    CHK(products());
    bool valid = true;
    CHK(pinv_spec_resolve(c, spec, &valid));
    if (!valid) {
      CHK(pinv_group_qp(c, 2, xs, a.rtol, a.max_rank, ro, gw, jw, Qv, Pv, orth_tol));
      CHK(products());
    }
    double* h2 = ((HostVerdict*)c.pinned)->aux;
    HIPCHK(hipMemcpyAsync(h2, sums, 16, hipMemcpyDeviceToHost, c.stream));
    HIPCHK(hipStreamSynchronize(c.stream));
    rel = h2[1] > 0.0 ? std::sqrt(h2[0] / h2[1]) : (h2[0] > 0.0 ? INFINITY : 0.0);
    std::swap(cur, nxt);
    ++t;
    if (rel <= a.tol) break;
  }
  if (cur.p != a.X.p) HIPCHK(launch_cast(c, cur, a.X, CAST_COPY));
  if (a.iters) *a.iters = t;
  if (a.rel) *a.rel = rel;
  return QCUR_OK;
}

// Validation and dispatch shared by qcur_complete and qcur_complete_resampled.
qcur_status complete_entry(qcur_handle h, const qcur_qmat* Y, const uint8_t* mask, int64_t mask_ld,
                           const int64_t* I, int64_t r, const int64_t* J, int64_t c, int compute, double rtol,
                           int64_t max_rank, int max_iter, double tol, qcur_qmat* X, int* iters, double* rel,
                           void* ws, size_t ws_bytes, bool resample, int sampling, uint64_t seed);

}  // namespace

// ============================================================================
extern "C" {

int qcur_version(void) { return 100; }

const char* qcur_status_string(qcur_status s) {
  switch (s) {
    case QCUR_OK: return "QCUR_OK";
    case QCUR_ERR_ARG: return "QCUR_ERR_ARG";
    case QCUR_ERR_SHAPE: return "QCUR_ERR_SHAPE";
    case QCUR_ERR_DTYPE: return "QCUR_ERR_DTYPE";
    case QCUR_ERR_WORKSPACE: return "QCUR_ERR_WORKSPACE";
    case QCUR_ERR_SAMPLE: return "QCUR_ERR_SAMPLE";
    case QCUR_ERR_NUMERIC: return "QCUR_ERR_NUMERIC";
    case QCUR_ERR_DEVICE: return "QCUR_ERR_DEVICE";
    case QCUR_ERR_UNSUPPORTED: return "QCUR_ERR_UNSUPPORTED";
  }
  return "unknown qcur_status";
}

const char* qcur_last_error(void) { return g_last_error.c_str(); }

qcur_status qcur_create(qcur_handle* handle, int device) {
  if (!handle) return fail(QCUR_ERR_ARG, "handle output pointer is NULL");
  *handle = nullptr;
  int count = 0;
  HIPCHK(hipGetDeviceCount(&count));
  if (device < 0 || device >= count) return fail(QCUR_ERR_ARG, "device %d out of range (%d devices)", device, count);
  int old = 0;
  HIPCHK(hipGetDevice(&old));
  HIPCHK(hipSetDevice(device));
  unsigned* st = nullptr;
  void* pinned = nullptr;
  hipEvent_t done = nullptr;
  hipError_t e = hipMalloc(&st, 256);
  if (e == hipSuccess) e = hipMemset(st, 0, 256);
  if (e == hipSuccess) e = hipHostMalloc(&pinned, sizeof(HostVerdict), hipHostMallocDefault);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&done, hipEventDisableTiming);
  void* scr = nullptr;
  if (e == hipSuccess) e = scratch_address(device, &scr);
  (void)hipSetDevice(old);
  if (e != hipSuccess) {
    if (st) (void)hipFree(st);
    if (pinned) (void)hipHostFree(pinned);
    return fail(QCUR_ERR_DEVICE, "handle resources: %s", hipGetErrorString(e));
  }
  qcur_ctx* h = new qcur_ctx;
  h->c.device = device;
  h->c.stream = nullptr;
  h->c.status = st;
  h->c.pinned = pinned;
  h->c.done = done;
  h->c.scratch = scr;
  *handle = h;
  return QCUR_OK;
}

qcur_status qcur_destroy(qcur_handle h) {
  if (!h) return QCUR_OK;
  for (auto& rec : h->batches) {
    if (rec.tun.e0) (void)hipEventDestroy(rec.tun.e0);
    if (rec.tun.e1) (void)hipEventDestroy(rec.tun.e1);
  }
  (void)hipFree(h->c.status);
  (void)hipHostFree(h->c.pinned);
  (void)hipEventDestroy(h->c.done);
  delete h;
  return QCUR_OK;
}

qcur_status qcur_set_stream(qcur_handle h, void* stream) {
  CHK(check_handle(h));
  h->c.stream = (hipStream_t)stream;
  return QCUR_OK;
}

qcur_status qcur_sync_status(qcur_handle h) {
  CHK(check_handle(h));
  unsigned bits = 0;
  HIPCHK(hipStreamSynchronize(h->c.stream));
  HIPCHK(hipMemcpy(&bits, h->c.status, sizeof(unsigned), hipMemcpyDeviceToHost));
  HIPCHK(hipMemset(h->c.status, 0, sizeof(unsigned)));
  if (bits & ST_ARG) return fail(QCUR_ERR_ARG, "a kernel reported an invalid index");
  if (bits & ST_SAMPLE) return fail(QCUR_ERR_SAMPLE, "a kernel reported invalid sampling weights");
  if (bits & ST_NUMERIC) return fail(QCUR_ERR_NUMERIC, "a kernel reported a zero or non-finite value");
  return QCUR_OK;
}

size_t qcur_probs_workspace(int64_t m, int64_t n) {
  if (m <= 0 || n <= 0) return 0;
  int rb, nrb, ncb;
  probs_grid(m, n, &rb, &nrb, &ncb);
  Bump b(nullptr);
  b.take((size_t)nrb * n * 8);
  b.take((size_t)ncb * m * 8);
  b.take((size_t)(m + n) * 8);
  return b.used + 256;
}

size_t qcur_pinv_workspace(int64_t p, int64_t q) {
  if (p < 0 || q < 0) return 0;
  return pinv_ws_size(p, q);
}

size_t qcur_svd_workspace(int64_t p, int64_t q) {
  if (p < 1 || q < 1) return 0;
  Bump b(nullptr);
  pinv_carve(b, p, q);
  b.take((size_t)std::min(p, q) * 4);
  return b.used + 256;
}

size_t qcur_gemm_workspace(int64_t M, int64_t N, int64_t K, int compute) {
  if (M <= 0 || N <= 0 || K <= 0 || !valid_compute(compute)) return 0;
  return gemm_workspace(M, N, K, compute);
}

size_t qcur_approx_workspace(int64_t m, int64_t n, int64_t c, int64_t r, int core, int compute) {
  if (m < 0 || n < 0 || c < 0 || r < 0 || !valid_compute(compute)) return 0;
  Ctx dummy{};
  ApproxArgs a = sizing_args(m, n, c, r, core, compute);
  Bump b(nullptr);
  // operands may arrive in any dtype: size for the worst case (all converted)
  a.A.dt = a.C.dt = a.R.dt = a.W.dt = (compute == QCUR_F64) ? QCUR_F32 : QCUR_F64;
  a.U.dt = (compute == QCUR_F64) ? QCUR_F32 : QCUR_F32;
  approx_run(dummy, a, m, n, c, r, b, true);
  return b.used + 256;
}

size_t qcur_residual_workspace(int64_t m, int64_t n, int64_t c, int64_t r, int compute) {
  if (m < 0 || n < 0 || c < 0 || r < 0 || !valid_compute(compute)) return 0;
  Ctx dummy{};
  const int other = compute == QCUR_F64 ? QCUR_F32 : QCUR_F64;
  QView A{nullptr, m, n, n, m * n, other}, C{nullptr, m, c, c, m * c, other};
  QView U{nullptr, c, r, r, c * r, other}, R{nullptr, r, n, n, r * n, other};
  Bump b(nullptr);
  residual_run(dummy, A, C, U, R, nullptr, 0, compute, nullptr, 1, nullptr, 0.0, b, true);
  return b.used + 256;
}

size_t qcur_backward_workspace(int64_t m, int64_t n, int64_t c, int64_t r, int compute) {
  if (m < 0 || n < 0 || c < 0 || r < 0 || (compute != QCUR_F64 && compute != QCUR_F32)) return 0;
  Ctx dummy{};
  BwdArgs a{};
  a.A = QView{nullptr, m, n, n, m * n, compute};
  a.r = r;
  a.cc = c;
  a.compute = compute;
  Bump b(nullptr);
  backward_run(dummy, a, b, true);
  return b.used + 256 + 64;
}

// ---- probs
qcur_status qcur_probs(qcur_handle h, const qcur_qmat* A, int sampling, double* p_col, double* q_row, double* fro2,
                       void* ws, size_t ws_bytes) {
  CHK(check_qmat(A, "A"));
  if (A->rows < 1 || A->cols < 1) return fail(QCUR_ERR_SHAPE, "A must have at least one row and column");
  if (sampling != QCUR_LENGTH && sampling != QCUR_UNIFORM) return fail(QCUR_ERR_ARG, "unknown sampling %d", sampling);
  if (!p_col || !q_row) return fail(QCUR_ERR_ARG, "p_col and q_row must not be NULL");
  const bool need_pass = sampling == QCUR_LENGTH || fro2 != nullptr;
  const size_t need = need_pass ? qcur_probs_workspace(A->rows, A->cols) : 0;
  if (need_pass && (!ws || ws_bytes < need))
    return fail(QCUR_ERR_WORKSPACE, "probs needs %zu workspace bytes", need);
  CHK(check_handle(h));
  const Ctx& c = h->c;
  QView Av = view_of(*A);
  const int64_t m = Av.rows, n = Av.cols;
  if (!need_pass) {
    HIPCHK(launch_probs_finish(c, m, n, nullptr, nullptr, 0, 0, sampling, p_col, q_row, nullptr, nullptr));
    return QCUR_OK;
  }
  int rb, nrb, ncb;
  probs_grid(m, n, &rb, &nrb, &ncb);
  Bump b(ws);
  double* colpart = (double*)b.take((size_t)nrb * n * 8);
  double* rowpart = (double*)b.take((size_t)ncb * m * 8);
  double* scratch = (double*)b.take((size_t)(m + n) * 8);
  HIPCHK(launch_probs_partials(c, Av, colpart, rowpart, rb, ncb));
  HIPCHK(launch_probs_finish(c, m, n, colpart, rowpart, nrb, ncb, sampling, p_col, q_row, fro2, scratch));
  return QCUR_OK;
}

// The same computation with the static scratch as workspace: no allocation,
// no caller workspace.
qcur_status qcur_probs_noalloc(qcur_handle h, const qcur_qmat* A, int sampling, double* p_col, double* q_row,
                               double* fro2) {
  static_assert(QCUR_SCRATCH_BYTES == SCRATCH_BYTES, "the header states the scratch size");
  CHK(check_qmat(A, "A"));
  if (A->rows < 1 || A->cols < 1) return fail(QCUR_ERR_SHAPE, "A must have at least one row and column");
  const size_t need = qcur_probs_workspace(A->rows, A->cols);
  if (need > SCRATCH_BYTES)
    return fail(QCUR_ERR_UNSUPPORTED, "a %lld x %lld matrix needs %zu bytes of scratch; the static scratch holds %zu",
                (long long)A->rows, (long long)A->cols, need, SCRATCH_BYTES);
  CHK(check_handle(h));
  if (!h->c.scratch) return fail(QCUR_ERR_DEVICE, "the handle has no static scratch address");
  return qcur_probs(h, A, sampling, p_col, q_row, fro2, h->c.scratch, SCRATCH_BYTES);
}

// ---- draw
qcur_status qcur_draw(qcur_handle h, const double* probs, int64_t n, int64_t count, uint64_t seed, uint64_t set_id,
                      int with_replacement, int64_t* idx) {
  if (n < 1) return fail(QCUR_ERR_ARG, "n must be >= 1");
  if (count < 0 || count >= ((int64_t)1 << 31)) return fail(QCUR_ERR_ARG, "count out of range");
  if (with_replacement != 0 && with_replacement != 1) return fail(QCUR_ERR_ARG, "with_replacement must be 0 or 1");
  if (!with_replacement && count > n) return fail(QCUR_ERR_ARG, "count > n without replacement");
  if (n > (with_replacement ? 8192 : 16384))
    return fail(QCUR_ERR_UNSUPPORTED, "n = %lld exceeds the sampler's LDS limit", (long long)n);
  if (count > 0 && (!probs || !idx)) return fail(QCUR_ERR_ARG, "probs and idx must not be NULL");
  CHK(check_handle(h));
  if (count == 0) return QCUR_OK;
  HIPCHK(launch_draw(h->c, probs, n, count, seed, set_id, with_replacement, idx));
  return QCUR_OK;
}

// ---- gather
qcur_status qcur_gather(qcur_handle h, const qcur_qmat* A, const int64_t* I, int64_t r, const int64_t* J, int64_t c,
                        qcur_qmat* C, qcur_qmat* R, qcur_qmat* W) {
  CHK(check_qmat(A, "A"));
  if (r < 0 || c < 0) return fail(QCUR_ERR_ARG, "negative index count");
  if (C) {
    CHK(check_qmat(C, "C"));
    CHK(check_dims(C, "C", A->rows, c));
    if (c > 0 && !J) return fail(QCUR_ERR_ARG, "J is NULL");
  }
  if (R) {
    CHK(check_qmat(R, "R"));
    CHK(check_dims(R, "R", r, A->cols));
    if (r > 0 && !I) return fail(QCUR_ERR_ARG, "I is NULL");
  }
  if (W) {
    CHK(check_qmat(W, "W"));
    CHK(check_dims(W, "W", r, c));
    if ((r > 0 && !I) || (c > 0 && !J)) return fail(QCUR_ERR_ARG, "I or J is NULL");
  }
  CHK(check_handle(h));
  QView Av = view_of(*A);
  QView Cv, Rv, Wv;
  if (C) Cv = view_of(*C);
  if (R) Rv = view_of(*R);
  if (W) Wv = view_of(*W);
  HIPCHK(launch_gather(h->c, Av, I, r, J, c, C ? &Cv : nullptr, R ? &Rv : nullptr, W ? &Wv : nullptr));
  return QCUR_OK;
}

// ---- pinv
qcur_status qcur_pinv(qcur_handle h, const qcur_qmat* X, double rtol, int64_t max_rank, qcur_qmat* Xp,
                      int64_t* rank_out, void* ws, size_t ws_bytes) {
  CHK(check_qmat(X, "X"));
  CHK(check_qmat(Xp, "Xp"));
  if (X->dtype != QCUR_F64 || Xp->dtype != QCUR_F64) return fail(QCUR_ERR_DTYPE, "pinv works in FP64");
  CHK(check_dims(Xp, "Xp", X->cols, X->rows));
  if (!std::isfinite(rtol)) return fail(QCUR_ERR_ARG, "rtol must be finite");
  if (max_rank < 0) return fail(QCUR_ERR_ARG, "max_rank must be >= 0");
  const size_t need = qcur_pinv_workspace(X->rows, X->cols);
  if (!ws || ws_bytes < need) return fail(QCUR_ERR_WORKSPACE, "pinv needs %zu workspace bytes", need);
  CHK(check_handle(h));
  Bump b(ws);
  PinvWs w = pinv_carve(b, X->rows, X->cols);
  PinvPlan pl = pinv_plan(X->rows, X->cols);
  GroupWs gw = group_carve(b, 1, pl.pp, pl.qq);
  return pinv_impl(h->c, view_of(*X), rtol, max_rank, view_of(*Xp), rank_out, w, gw);
}

// ---- thin QSVD
qcur_status qcur_svd(qcur_handle h, const qcur_qmat* X, double* s, qcur_qmat* U, qcur_qmat* V, void* ws,
                     size_t ws_bytes) {
  CHK(check_qmat(X, "X"));
  if (X->rows < 1 || X->cols < 1) return fail(QCUR_ERR_SHAPE, "X must have at least one row and column");
  if (!s) return fail(QCUR_ERR_ARG, "s is NULL");
  const int64_t p = X->rows, q = X->cols, k = std::min(p, q);
  if (U) {
    CHK(check_qmat(U, "U"));
    CHK(check_dims(U, "U", p, k));
    if (U->dtype != QCUR_F64) return fail(QCUR_ERR_DTYPE, "U must be FP64");
  }
  if (V) {
    CHK(check_qmat(V, "V"));
    CHK(check_dims(V, "V", q, k));
    if (V->dtype != QCUR_F64) return fail(QCUR_ERR_DTYPE, "V must be FP64");
  }
  const size_t need = qcur_svd_workspace(p, q);
  if (!ws || ws_bytes < need) return fail(QCUR_ERR_WORKSPACE, "svd needs %zu workspace bytes", need);
  CHK(check_handle(h));
  const Ctx& c = h->c;
  Bump b(ws);
  PinvWs w = pinv_carve(b, p, q);
  int32_t* rank = (int32_t*)b.take((size_t)k * 4);
  PinvPlan pl = pinv_plan(p, q);
  const int64_t pp = pl.pp, qq = pl.qq;
  const QView Xv = view_of(*X);
  HIPCHK(launch_check_finite(c, Xv));
  QView Yv{w.Y, qq, pp, pp, qq * pp, QCUR_F64};
  HIPCHK(launch_cast(c, Xv, Yv, pl.tall ? CAST_T : CAST_CONJ));
  HIPCHK(launch_fill_identity(c, w.V, qq));
  const double tol = std::sqrt((double)pp) * std::ldexp(1.0, -53);
  if (jacobi_small_fits(pp, qq)) {
    HIPCHK(launch_jacobi_small(c, w.Y, pp, qq, w.V, tol, MAX_SWEEPS, w.flag));
  } else {
    CHK(jacobi_sweeps(c, w, pp, qq, tol, 0.0));  // rtol 0: every column is kept
  }
  HIPCHK(launch_svd_out(c, w.Y, pp, qq, w.V, w.sig, rank, s, pl.tall, U ? (double*)U->p : nullptr,
                        U ? U->ld : 0, U ? U->pstride : 0, V ? (double*)V->p : nullptr, V ? V->ld : 0,
                        V ? V->pstride : 0));
  return QCUR_OK;
}

// ---- gemm
qcur_status qcur_gemm(qcur_handle h, int opA, int opB, double alpha, const qcur_qmat* A, const qcur_qmat* B,
                      double beta, qcur_qmat* D, int compute, void* ws, size_t ws_bytes) {
  CHK(check_qmat(A, "A"));
  CHK(check_qmat(B, "B"));
  CHK(check_qmat(D, "D"));
  if ((opA != QCUR_OP_N && opA != QCUR_OP_H) || (opB != QCUR_OP_N && opB != QCUR_OP_H))
    return fail(QCUR_ERR_ARG, "op must be QCUR_OP_N or QCUR_OP_H");
  if (!valid_compute(compute)) return fail(QCUR_ERR_DTYPE, "unknown compute dtype");
  if (A->dtype != in_dt(compute) || B->dtype != in_dt(compute) || D->dtype != acc_dt(compute))
    return fail(QCUR_ERR_DTYPE, "operands must be in the compute dtype (BF16: D FP32; split BF16: all FP32)");
  const int64_t M = opA == QCUR_OP_N ? A->rows : A->cols;
  const int64_t K = opA == QCUR_OP_N ? A->cols : A->rows;
  const int64_t K2 = opB == QCUR_OP_N ? B->rows : B->cols;
  const int64_t N = opB == QCUR_OP_N ? B->cols : B->rows;
  if (K != K2) return fail(QCUR_ERR_SHAPE, "inner sizes differ (%lld vs %lld)", (long long)K, (long long)K2);
  CHK(check_dims(D, "D", M, N));
  if (!std::isfinite(alpha) || !std::isfinite(beta)) return fail(QCUR_ERR_ARG, "alpha/beta must be finite");
  CHK(check_handle(h));
  HIPCHK(launch_gemm(h->c, opA, opB, alpha, view_of(*A), view_of(*B), beta, view_of(*D), compute, ws, ws_bytes));
  return QCUR_OK;
}

// ---- approx
qcur_status qcur_approx(qcur_handle h, const qcur_qmat* A, const qcur_qmat* C, const qcur_qmat* R,
                        const qcur_qmat* W, int core, int compute, int refine_steps, double rtol, int64_t max_rank,
                        qcur_qmat* U, qcur_qmat* B, int64_t* rank_out, void* ws, size_t ws_bytes) {
  if (core != QCUR_CORE_WPINV && core != QCUR_CORE_CAR) return fail(QCUR_ERR_ARG, "unknown core %d", core);
  if (!valid_compute(compute)) return fail(QCUR_ERR_DTYPE, "unknown compute dtype");
  if (refine_steps < 0) return fail(QCUR_ERR_ARG, "refine_steps must be >= 0");
  if (!std::isfinite(rtol)) return fail(QCUR_ERR_ARG, "rtol must be finite");
  if (max_rank < 0) return fail(QCUR_ERR_ARG, "max_rank must be >= 0");
  CHK(check_qmat(U, "U"));
  if (U->dtype != acc_dt(compute)) return fail(QCUR_ERR_DTYPE, "U must be FP64 (F64 compute) or FP32");
  int64_t m = 0, n = 0, cc = U->rows, r = U->cols;
  ApproxArgs a{};
  if (core == QCUR_CORE_WPINV) {
    CHK(check_qmat(W, "W"));
    CHK(check_dims(W, "W", r, cc));
    a.W = view_of(*W);
  } else {
    CHK(check_qmat(A, "A"));
    CHK(check_qmat(C, "C"));
    CHK(check_qmat(R, "R"));
    m = A->rows;
    n = A->cols;
    CHK(check_dims(C, "C", m, cc));
    CHK(check_dims(R, "R", r, n));
    a.A = view_of(*A);
    a.C = view_of(*C);
    a.R = view_of(*R);
  }
  if (B) {
    CHK(check_qmat(B, "B"));
    if (B->dtype != acc_dt(compute)) return fail(QCUR_ERR_DTYPE, "B must be FP64 (F64 compute) or FP32");
    if (core == QCUR_CORE_WPINV) {
      CHK(check_qmat(C, "C"));
      CHK(check_qmat(R, "R"));
      m = C->rows;
      n = R->cols;
      CHK(check_dims(C, "C", m, cc));
      CHK(check_dims(R, "R", r, n));
      a.C = view_of(*C);
      a.R = view_of(*R);
    }
    CHK(check_dims(B, "B", m, n));
    a.B = view_of(*B);
  }
  a.U = view_of(*U);
  a.hasB = B != nullptr;
  a.core = core;
  a.compute = compute;
  a.refine = core == QCUR_CORE_CAR ? refine_steps : 0;
  a.rtol = rtol;
  a.max_rank = max_rank;
  a.rank_out = rank_out;
  {
    Bump sz(nullptr);
    Ctx dummy{};
    approx_run(dummy, a, m, n, cc, r, sz, true);
    const size_t need = sz.used + 256;
    if (!ws || ws_bytes < need) return fail(QCUR_ERR_WORKSPACE, "approx needs %zu workspace bytes", need);
  }
  CHK(check_handle(h));
  Bump b(ws);
  return approx_run(h->c, a, m, n, cc, r, b, false);
}

// ---- residual
qcur_status qcur_residual(qcur_handle h, const qcur_qmat* A, const qcur_qmat* C, const qcur_qmat* U,
                          const qcur_qmat* R, const uint8_t* mask, int64_t mask_ld, int compute, double* fro,
                          qcur_qmat* E, double e_scale, void* ws, size_t ws_bytes) {
  CHK(check_qmat(A, "A"));
  CHK(check_qmat(C, "C"));
  CHK(check_qmat(U, "U"));
  CHK(check_qmat(R, "R"));
  if (!valid_compute(compute)) return fail(QCUR_ERR_DTYPE, "unknown compute dtype");
  const int64_t m = A->rows, n = A->cols, cc = C->cols, r = R->rows;
  CHK(check_dims(C, "C", m, cc));
  CHK(check_dims(U, "U", cc, r));
  CHK(check_dims(R, "R", r, n));
  if (mask && mask_ld < n) return fail(QCUR_ERR_SHAPE, "mask_ld < n");
  if (!fro) return fail(QCUR_ERR_ARG, "fro must not be NULL");
  if (E) {
    CHK(check_qmat(E, "E"));
    CHK(check_dims(E, "E", m, n));
    if (E->dtype != acc_dt(compute)) return fail(QCUR_ERR_DTYPE, "E must be FP64 (F64 compute) or FP32");
  }
  if (!std::isfinite(e_scale)) return fail(QCUR_ERR_ARG, "e_scale must be finite");
  QView Av = view_of(*A), Cv = view_of(*C), Uv = view_of(*U), Rv = view_of(*R);
  {
    Bump sz(nullptr);
    Ctx dummy{};
    residual_run(dummy, Av, Cv, Uv, Rv, mask, mask_ld, compute, nullptr, 1, nullptr, 0.0, sz, true);
    const size_t need = sz.used + 256;
    if (!ws || ws_bytes < need) return fail(QCUR_ERR_WORKSPACE, "residual needs %zu workspace bytes", need);
  }
  CHK(check_handle(h));
  Bump b(ws);
  QView Ev;
  if (E) Ev = view_of(*E);
  return residual_run(h->c, Av, Cv, Uv, Rv, mask, mask_ld, compute, fro, 1, E ? &Ev : nullptr, e_scale, b, false);
}

// ---- backward
qcur_status qcur_backward(qcur_handle h, const qcur_qmat* A, const int64_t* I, int64_t r, const int64_t* J, int64_t c,
                          const qcur_qmat* gB, const uint8_t* mask, int64_t mask_ld, double rtol, int64_t max_rank,
                          int compute, qcur_qmat* dA, double* loss, void* ws, size_t ws_bytes) {
  CHK(check_qmat(A, "A"));
  if (!dA && (gB || !loss)) return fail(QCUR_ERR_ARG, "dA may be NULL only for the loss alone (gB NULL, loss given)");
  if (dA) CHK(check_qmat(dA, "dA"));
  if (compute != QCUR_F64 && compute != QCUR_F32) return fail(QCUR_ERR_DTYPE, "backward computes in FP64 or FP32");
  if (A->dtype != compute || (dA && dA->dtype != compute))
    return fail(QCUR_ERR_DTYPE, "A and dA must be in the compute dtype");
  const int64_t m = A->rows, n = A->cols;
  if (dA) CHK(check_dims(dA, "dA", m, n));
  if (r < 1 || c < 1 || r > m || c > n) return fail(QCUR_ERR_ARG, "index counts out of range");
  if (!I || !J) return fail(QCUR_ERR_ARG, "I and J must not be NULL");
  if (gB) {
    CHK(check_qmat(gB, "gB"));
    CHK(check_dims(gB, "gB", m, n));
    if (gB->dtype != compute) return fail(QCUR_ERR_DTYPE, "gB must be in the compute dtype");
  }
  if (mask && mask_ld < n) return fail(QCUR_ERR_SHAPE, "mask_ld < n");
  if (!std::isfinite(rtol)) return fail(QCUR_ERR_ARG, "rtol must be finite");
  if (max_rank < 0) return fail(QCUR_ERR_ARG, "max_rank must be >= 0");
  const size_t need = qcur_backward_workspace(m, n, c, r, compute);
  if (!ws || ws_bytes < need) return fail(QCUR_ERR_WORKSPACE, "backward needs %zu workspace bytes", need);
  CHK(check_handle(h));
  BwdArgs a{};
  a.A = view_of(*A);
  if (dA) a.dA = view_of(*dA);
  a.hasdA = dA != nullptr;
  a.hasgB = gB != nullptr;
  if (gB) a.gB = view_of(*gB);
  a.I = I;
  a.J = J;
  a.r = r;
  a.cc = c;
  a.mask = mask;
  a.mask_ld = mask_ld;
  a.rtol = rtol;
  a.max_rank = max_rank;
  a.compute = compute;
  a.loss = loss;
  Bump b(ws);
  return backward_run(h->c, a, b, false);
}

static qcur_status check_solve(const qcur_qmat* A, int64_t c, int64_t r, int sampling, int core, int compute,
                               int with_replacement, int refine_steps, double rtol, int64_t max_rank) {
  CHK(check_qmat(A, "A"));
  if (A->rows < 1 || A->cols < 1) return fail(QCUR_ERR_SHAPE, "A must have at least one row and column");
  if (sampling != QCUR_LENGTH && sampling != QCUR_UNIFORM) return fail(QCUR_ERR_ARG, "unknown sampling %d", sampling);
  if (core != QCUR_CORE_WPINV && core != QCUR_CORE_CAR) return fail(QCUR_ERR_ARG, "unknown core %d", core);
  if (!valid_compute(compute)) return fail(QCUR_ERR_DTYPE, "unknown compute dtype");
  if (with_replacement != 0 && with_replacement != 1) return fail(QCUR_ERR_ARG, "with_replacement must be 0 or 1");
  if (c < 1 || r < 1) return fail(QCUR_ERR_ARG, "c and r must be >= 1");
  if (!with_replacement && (c > A->cols || r > A->rows)) return fail(QCUR_ERR_ARG, "c > n or r > m without replacement");
  const int64_t lim = with_replacement ? 8192 : 16384;
  if (A->cols > lim || A->rows > lim) return fail(QCUR_ERR_UNSUPPORTED, "matrix side exceeds the sampler's LDS limit");
  if (refine_steps < 0) return fail(QCUR_ERR_ARG, "refine_steps must be >= 0");
  if (!std::isfinite(rtol)) return fail(QCUR_ERR_ARG, "rtol must be finite");
  if (max_rank < 0) return fail(QCUR_ERR_ARG, "max_rank must be >= 0");
  return QCUR_OK;
}

size_t qcur_solve_workspace(int64_t m, int64_t n, int64_t c, int64_t r, int core, int compute) {
  if (m < 1 || n < 1 || c < 1 || r < 1 || !valid_compute(compute)) return 0;
  // the input may come in any dtype: size for the largest element
  SolveArgs s{};
  s.A = QView{nullptr, m, n, n, m * n, QCUR_F64};
  s.c = c;
  s.r = r;
  s.sampling = QCUR_LENGTH;
  s.core = core;
  s.compute = compute;
  s.refine = 1;
  s.U = QView{nullptr, c, r, r, c * r, acc_dt(compute)};
  const QView Bs{nullptr, m, n, n, m * n, acc_dt(compute)};
  s.B = &Bs;
  Ctx dummy{};
  size_t worst = 0;
  for (int dt : {QCUR_F64, QCUR_F32, QCUR_BF16}) {
    s.A.dt = dt;
    Bump b(nullptr);
    solve_run(dummy, s, b, true);
    worst = std::max(worst, b.used);
  }
  return worst + 256;
}

qcur_status qcur_solve(qcur_handle h, const qcur_qmat* A, int64_t c, int64_t r, int sampling, int core, int compute,
                       uint64_t seed, int with_replacement, int refine_steps, double rtol, int64_t max_rank,
                       int64_t* I, int64_t* J, qcur_qmat* U, double* residual, int64_t* rank_out, double* p_col,
                       double* q_row, qcur_qmat* C, qcur_qmat* R, qcur_qmat* W, qcur_qmat* B, void* ws,
                       size_t ws_bytes) {
  CHK(check_solve(A, c, r, sampling, core, compute, with_replacement, refine_steps, rtol, max_rank));
  if (!I || !J || !residual) return fail(QCUR_ERR_ARG, "I, J and residual must not be NULL");
  CHK(check_qmat(U, "U"));
  CHK(check_dims(U, "U", c, r));
  if (U->dtype != acc_dt(compute)) return fail(QCUR_ERR_DTYPE, "U must be FP64 (F64 compute) or FP32");
  const qcur_qmat* outs[3] = {C, R, W};
  const char* names[3] = {"C", "R", "W"};
  const int64_t rows[3] = {A->rows, r, r}, cols[3] = {c, A->cols, c};
  for (int k = 0; k < 3; ++k) {
    if (!outs[k]) continue;
    CHK(check_qmat(outs[k], names[k]));
    CHK(check_dims(outs[k], names[k], rows[k], cols[k]));
    if (outs[k]->dtype != A->dtype) return fail(QCUR_ERR_DTYPE, "%s must have A's dtype", names[k]);
  }
  SolveArgs s{};
  s.A = view_of(*A);
  s.c = c;
  s.r = r;
  s.sampling = sampling;
  s.core = core;
  s.compute = compute;
  s.with_replacement = with_replacement;
  s.refine = refine_steps;
  s.seed = seed;
  s.rtol = rtol;
  s.max_rank = max_rank;
  s.I = I;
  s.J = J;
  s.U = view_of(*U);
  s.residual = residual;
  s.rank_out = rank_out;
  s.p = p_col;
  s.q = q_row;
  QView Cv, Rv, Wv;
  if (C) { Cv = view_of(*C); s.C = &Cv; }
  if (R) { Rv = view_of(*R); s.R = &Rv; }
  if (W) { Wv = view_of(*W); s.W = &Wv; }
  QView Bv;
  if (B) {
    CHK(check_qmat(B, "B"));
    CHK(check_dims(B, "B", A->rows, A->cols));
    if (B->dtype != acc_dt(compute)) return fail(QCUR_ERR_DTYPE, "B must be FP64 (F64 compute) or FP32");
    Bv = view_of(*B);
    s.B = &Bv;
  }
  {
    Bump sz(nullptr);
    Ctx dummy{};
    solve_run(dummy, s, sz, true);
    const size_t need = sz.used + 256;
    if (!ws || ws_bytes < need) return fail(QCUR_ERR_WORKSPACE, "solve needs %zu workspace bytes", need);
  }
  CHK(check_handle(h));
  Bump b(ws);
  return solve_run(h->c, s, b, false);
}

// ---- batched solve ------------------------------------------------------------
size_t qcur_batch_workspace(int32_t count, const int32_t* dims, int a_dtype, int sampling, int compute,
                            int refine_steps, int autotune) {
  BatchShape s{};
  if (check_batch_shape(count, dims, a_dtype, sampling, compute, refine_steps, 1, autotune, &s) != QCUR_OK) return 0;
  Bump b(nullptr);
  batch_carve(b, s);
  return b.used + 256;
}

qcur_status qcur_batch_prepare(qcur_handle h, int32_t count, const int32_t* dims, int a_dtype, int sampling,
                               int compute, int refine_steps, int autotune, void* ws, size_t ws_bytes) {
  BatchShape s{};
  CHK(check_batch_shape(count, dims, a_dtype, sampling, compute, refine_steps, 1, autotune, &s));
  {
    Bump sz(nullptr);
    batch_carve(sz, s);
    if (!ws || ws_bytes < sz.used + 256) return fail(QCUR_ERR_WORKSPACE, "batch needs %zu workspace bytes", sz.used + 256);
  }
  CHK(check_handle(h));
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  HIPCHK(hipStreamIsCapturing(h->c.stream, &cap));
  if (cap != hipStreamCaptureStatusNone) return fail(QCUR_ERR_ARG, "qcur_batch_prepare cannot run under stream capture");
  Bump b(ws);
  BatchWs w = batch_carve(b, s);
  // dm, dn, dc, dr (count each), then zp, zq (2 * count each)
  std::vector<int> hdr((size_t)8 * count);
  int* hm = hdr.data();
  int *hn = hm + count, *hc = hn + count, *hr = hc + count, *hp = hr + count, *hq = hp + 2 * count;
  for (int i = 0; i < count; ++i) {
    hm[i] = dims[4 * i];
    hn[i] = dims[4 * i + 1];
    hc[i] = dims[4 * i + 2];
    hr[i] = dims[4 * i + 3];
    hp[i] = hm[i];
    hq[i] = hc[i];
    hp[count + i] = hn[i];
    hq[count + i] = hr[i];
  }
  // the order in which persistent launches hand out the problems' tiles:
  // largest m n (c + r) first (the products' work), ties by index
  std::vector<int> order(count);
  for (int i = 0; i < count; ++i) order[i] = i;
  auto work = [&](int i) { return (double)hm[i] * (double)hn[i] * (double)(hc[i] + hr[i]); };
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return work(x) > work(y); });
  // the order of the factors' CholeskyQR workgroups, longest first: the
  // passes over Z and Q_1 cost p per 16 x 16 block of the lower triangle
  // (three of them, five when the second pass runs, which on measured
  // workloads it mostly does for more than 48 columns), the factorisations
  // a pivot chain per 16 columns
  std::vector<int> forder(2 * count);
  for (int i = 0; i < 2 * count; ++i) forder[i] = i;
  auto fwork = [&](int t) {
    const double nb = (double)((hq[t] + 15) / 16), blk = nb * (nb + 1) / 2;
    return (double)hp[t] * blk * (hq[t] > 48 ? 5.0 : 3.0) + 2500.0 * nb;
  };
  std::stable_sort(forder.begin(), forder.end(), [&](int x, int y) { return fwork(x) > fwork(y); });
  const int* srcs[8] = {hm, hn, hc, hr, hp, hq, order.data(), forder.data()};
  int* dsts[8] = {w.dm, w.dn, w.dc, w.dr, w.zp, w.zq, w.order, w.forder};
  const size_t lens[8] = {(size_t)count, (size_t)count, (size_t)count, (size_t)count, (size_t)2 * count,
                          (size_t)2 * count, (size_t)count, (size_t)2 * count};
  for (int k = 0; k < 8; ++k)
    HIPCHK(hipMemcpyAsync(dsts[k], srcs[k], lens[k] * sizeof(int), hipMemcpyHostToDevice, h->c.stream));
  HIPCHK(hipStreamSynchronize(h->c.stream));
  int slot = -1;
  for (int k = 0; k < 8; ++k)
    if (h->batches[k].ws == ws) slot = k;
  if (slot < 0) {
    slot = h->next_batch;
    h->next_batch = (h->next_batch + 1) % 8;
  }
  BatchRecord& rec = h->batches[slot];
  if (rec.tun.e0) (void)hipEventDestroy(rec.tun.e0);
  if (rec.tun.e1) (void)hipEventDestroy(rec.tun.e1);
  rec = BatchRecord{};
  rec.ws = ws;
  rec.key = batch_key(s);
  rec.autotune = autotune;
  if (autotune) {
    HIPCHK(hipEventCreate(&rec.tun.e0));
    HIPCHK(hipEventCreate(&rec.tun.e1));
  }
  return QCUR_OK;
}

int qcur_batch_plans(qcur_handle h, const void* ws, int* tiles, int* splits, int n) {
  if (!h) return 0;
  for (int k = 0; k < 8; ++k) {
    const BatchRecord& rec = h->batches[k];
    if (rec.ws != ws || !rec.ws) continue;
    const int cnt = std::min<int>(n, BS_COUNT);
    for (int i = 0; i < cnt; ++i) {
      if (tiles) tiles[i] = rec.tun.plan[i].tile;
      if (splits) splits[i] = rec.tun.plan[i].splits;
    }
    return rec.tuned ? BS_COUNT : 0;
  }
  return 0;
}

qcur_status qcur_solve_batched(qcur_handle h, int32_t count, const int32_t* dims, const qcur_qmat* A,
                               int64_t a_bstride, int sampling, int compute, uint64_t seed, int with_replacement,
                               int refine_steps, double rtol, int64_t max_rank, int64_t* I, int64_t* J,
                               qcur_qmat* U, int64_t u_bstride, double* residual, int64_t* rank_out, double* p_col,
                               double* q_row, qcur_qmat* B, int64_t b_bstride, void* ws, size_t ws_bytes) {
  if (with_replacement != 0 && with_replacement != 1) return fail(QCUR_ERR_ARG, "with_replacement must be 0 or 1");
  if (!A) return fail(QCUR_ERR_ARG, "A is NULL");
  BatchShape s{};
  CHK(check_batch_shape(count, dims, (int)A->dtype, sampling, compute, refine_steps, with_replacement, 0, &s));
  CHK(check_slotted(A, "A", s.mx, s.nx, a_bstride));
  CHK(check_slotted(U, "U", s.cx, s.rx, u_bstride));
  if (U->dtype != acc_dt(compute)) return fail(QCUR_ERR_DTYPE, "U must be FP64 (F64 compute) or FP32");
  if (B) {
    CHK(check_slotted(B, "B", s.mx, s.nx, b_bstride));
    if (B->dtype != acc_dt(compute)) return fail(QCUR_ERR_DTYPE, "B must be FP64 (F64 compute) or FP32");
  }
  if (!I || !J || !residual) return fail(QCUR_ERR_ARG, "I, J and residual must not be NULL");
  if (!std::isfinite(rtol)) return fail(QCUR_ERR_ARG, "rtol must be finite");
  if (max_rank < 0) return fail(QCUR_ERR_ARG, "max_rank must be >= 0");
  {
    Bump sz(nullptr);
    batch_carve(sz, s);  // the smaller layout (no autotuning)
    if (!ws || ws_bytes < sz.used + 256) return fail(QCUR_ERR_WORKSPACE, "batch needs %zu workspace bytes", sz.used + 256);
  }
  CHK(check_handle(h));
  // the record of this workspace fixes the layout (with or without autotuning)
  BatchRecord* rec = nullptr;
  for (int k = 0; k < 8; ++k) {
    if (h->batches[k].ws != ws || !ws) continue;
    s.autotune = h->batches[k].autotune;
    if (h->batches[k].key == batch_key(s)) rec = &h->batches[k];
  }
  if (!rec) return fail(QCUR_ERR_ARG, "the workspace was not prepared for this batch (qcur_batch_prepare)");
  {
    Bump sz(nullptr);
    batch_carve(sz, s);
    if (ws_bytes < sz.used + 256) return fail(QCUR_ERR_WORKSPACE, "batch needs %zu workspace bytes", sz.used + 256);
  }
  Bump b(ws);
  BatchWs w = batch_carve(b, s);
  BatchArgs a{};
  a.A = Slots{A->p, A->ld, A->pstride, a_bstride, (int)A->dtype};
  a.seed = seed;
  a.repl = with_replacement;
  a.rtol = rtol;
  a.max_rank = max_rank;
  a.I = I;
  a.J = J;
  a.U = Slots{U->p, U->ld, U->pstride, u_bstride, (int)U->dtype};
  a.residual = residual;
  a.rank_out = rank_out;
  a.p = p_col;
  a.q = q_row;
  if (B) a.B = Slots{B->p, B->ld, B->pstride, b_bstride, (int)B->dtype};
  BatchTuning* tu = nullptr;
  if (rec->autotune) {
    tu = &rec->tun;
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    HIPCHK(hipStreamIsCapturing(h->c.stream, &cap));
    // measure on the first call that is not being captured
    tu->measure = !rec->tuned && cap == hipStreamCaptureStatusNone;
  }
  const qcur_status st = batch_run(h->c, s, a, w, tu);
  if (tu && tu->measure && st == QCUR_OK) rec->tuned = true;
  if (tu) tu->measure = false;
  return st;
}

// ---- completion -----------------------------------------------------------------
size_t qcur_complete_workspace(int64_t m, int64_t n, int64_t c, int64_t r, int compute) {
  if (m < 1 || n < 1 || c < 1 || r < 1 || !valid_compute(compute))
    return 0;
  CompleteArgs a{};
  a.Y = QView{nullptr, m, n, n, m * n, QCUR_F64};
  a.X = QView{nullptr, m, n, n, m * n, acc_dt(compute)};
  a.r = r;
  a.cc = c;
  a.compute = compute;
  Bump b(nullptr);
  Ctx dummy{};
  complete_run(dummy, a, b, true);
  return b.used + 256;
}

size_t qcur_complete_resampled_workspace(int64_t m, int64_t n, int64_t c, int64_t r, int sampling, int compute) {
  if (m < 1 || n < 1 || c < 1 || r < 1) return 0;
  CompleteArgs a{};
  a.Y = QView{nullptr, m, n, n, m * n, QCUR_F64};
  a.X = QView{nullptr, m, n, n, m * n, acc_dt(compute)};
  a.r = r;
  a.cc = c;
  a.compute = compute;
  a.resample = true;
  a.sampling = sampling;
  Bump b(nullptr);
  Ctx dummy{};
  complete_run(dummy, a, b, true);
  return b.used + 256;
}

int64_t qcur_sample_size(int64_t k, int64_t limit) {
  if (k < 1 || limit < 1) return 0;
  const int64_t s = k > 1 ? (int64_t)std::ceil((double)k * std::log((double)k)) : 1;
  return std::min(limit, std::max(k, s));
}

qcur_status qcur_complete_resampled(qcur_handle h, const qcur_qmat* Y, const uint8_t* mask, int64_t mask_ld,
                                    int64_t r, int64_t c, int sampling, uint64_t seed, int compute, double rtol,
                                    int64_t max_rank, int max_iter, double tol, qcur_qmat* X, int64_t* I, int64_t* J,
                                    int* iters, double* rel, void* ws, size_t ws_bytes) {
  if (sampling != QCUR_LENGTH && sampling != QCUR_UNIFORM) return fail(QCUR_ERR_ARG, "unknown sampling mode");
  if (Y && (r > Y->rows || c > Y->cols)) return fail(QCUR_ERR_ARG, "r and c must not exceed m and n");
  return complete_entry(h, Y, mask, mask_ld, I, r, J, c, compute, rtol, max_rank, max_iter, tol, X, iters, rel, ws,
                        ws_bytes, true, sampling, seed);
}

qcur_status qcur_complete(qcur_handle h, const qcur_qmat* Y, const uint8_t* mask, int64_t mask_ld, const int64_t* I,
                          int64_t r, const int64_t* J, int64_t c, int compute, double rtol, int64_t max_rank,
                          int max_iter, double tol, qcur_qmat* X, int* iters, double* rel, void* ws,
                          size_t ws_bytes) {
  return complete_entry(h, Y, mask, mask_ld, I, r, J, c, compute, rtol, max_rank, max_iter, tol, X, iters, rel, ws,
                        ws_bytes, false, 0, 0);
}

}  // extern "C"

namespace {
qcur_status complete_entry(qcur_handle h, const qcur_qmat* Y, const uint8_t* mask, int64_t mask_ld,
                           const int64_t* I, int64_t r, const int64_t* J, int64_t c, int compute, double rtol,
                           int64_t max_rank, int max_iter, double tol, qcur_qmat* X, int* iters, double* rel,
                           void* ws, size_t ws_bytes, bool resample, int sampling, uint64_t seed) {
  CHK(check_qmat(Y, "Y"));
  CHK(check_qmat(X, "X"));
  if (Y->rows < 1 || Y->cols < 1) return fail(QCUR_ERR_SHAPE, "Y must have at least one row and column");
  CHK(check_dims(X, "X", Y->rows, Y->cols));
  if (!valid_compute(compute)) return fail(QCUR_ERR_DTYPE, "unknown compute dtype");
  if (X->dtype != acc_dt(compute)) return fail(QCUR_ERR_DTYPE, "X must be FP64 (F64 compute) or FP32");
  if (!mask || mask_ld < Y->cols) return fail(QCUR_ERR_ARG, "mask is NULL or mask_ld < n");
  if (!I || !J || r < 1 || c < 1 || r > Y->rows || c > Y->cols) return fail(QCUR_ERR_ARG, "bad index sets");
  if (max_iter < 0) return fail(QCUR_ERR_ARG, "max_iter must be >= 0");
  if (!std::isfinite(rtol) || !(tol >= 0.0)) return fail(QCUR_ERR_ARG, "rtol must be finite and tol >= 0");
  if (max_rank < 0) return fail(QCUR_ERR_ARG, "max_rank must be >= 0");
  if (resample && (Y->rows > 16384 || Y->cols > 16384))
    return fail(QCUR_ERR_UNSUPPORTED, "matrix side exceeds the sampler's LDS limit");
  CompleteArgs a{};
  a.Y = view_of(*Y);
  a.X = view_of(*X);
  a.mask = mask;
  a.mask_ld = mask_ld;
  a.I = I;
  a.J = J;
  a.r = r;
  a.cc = c;
  a.compute = compute;
  a.rtol = rtol;
  a.max_rank = max_rank;
  a.max_iter = max_iter;
  a.tol = tol;
  a.iters = iters;
  a.rel = rel;
  a.resample = resample;
  a.sampling = sampling;
  a.seed = seed;
  {
    Bump sz(nullptr);
    Ctx dummy{};
    complete_run(dummy, a, sz, true);
    if (!ws || ws_bytes < sz.used + 256) return fail(QCUR_ERR_WORKSPACE, "completion needs %zu workspace bytes", sz.used + 256);
  }
  CHK(check_handle(h));
  Bump b(ws);
  return complete_run(h->c, a, b, false);
}
}  // namespace

extern "C" {

qcur_status qcur_cast(qcur_handle h, const qcur_qmat* X, qcur_qmat* Y) {
  CHK(check_qmat(X, "X"));
  CHK(check_qmat(Y, "Y"));
  CHK(check_dims(Y, "Y", X->rows, X->cols));
  CHK(check_handle(h));
  HIPCHK(launch_cast(h->c, view_of(*X), view_of(*Y), CAST_COPY));
  return QCUR_OK;
}

}  // extern "C"
