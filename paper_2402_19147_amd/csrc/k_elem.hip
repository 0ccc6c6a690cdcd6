// Bandwidth-bound kernels of the QMCUR path: length probabilities (Section
// 3.1), gathers of C = A(:,J), R = A(I,:), W = A(I,J) (Algorithm 1 steps 1-2),
// dtype casts and small helpers.  All reductions run in FP64 in a fixed
// order so results do not depend on scheduling.
#include <algorithm>

#include "qcur_internal.hpp"

namespace qcur {

template <typename T> __device__ inline double to_d(T v);
template <> __device__ inline double to_d<double>(double v) { return v; }
template <> __device__ inline double to_d<float>(float v) { return (double)v; }
template <> __device__ inline double to_d<uint16_t>(uint16_t v) { return (double)bf16_to_f32(v); }

template <typename T> __device__ inline T from_d(double v);
template <> __device__ inline double from_d<double>(double v) { return v; }
template <> __device__ inline float from_d<float>(double v) { return (float)v; }
template <> __device__ inline uint16_t from_d<uint16_t>(double v) { return f32_to_bf16((float)v); }

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// ---------------------------------------------------------------------------
// probs, pass 1: tile (rb rows) x (256 columns).  Thread t owns column
// j = 256*bx + t and sums |a_ij|^2 over the tile's rows into colpart[by][j];
// each row of the tile is reduced across the 256 columns (wave sums, then the
// four wave results in order) into rowpart[bx][i].
template <typename T>
__global__ __launch_bounds__(256) void k_probs_partials(const T* __restrict__ A, int64_t m, int64_t n,
                                                        int64_t ld, int64_t ps, int rb,
                                                        double* __restrict__ colpart,
                                                        double* __restrict__ rowpart) {
  __shared__ double wsum[4][64];
  const int t = threadIdx.x;
  const int64_t j = (int64_t)blockIdx.x * 256 + t;
  const int64_t i0 = (int64_t)blockIdx.y * rb;
  const int64_t i1 = min(m, i0 + rb);
  double cacc = 0.0;
  for (int64_t i = i0; i < i1; ++i) {
    double s = 0.0;
    if (j < n) {
      const int64_t off = i * ld + j;
      double a0 = to_d<T>(A[off]), a1 = to_d<T>(A[off + ps]);
      double a2 = to_d<T>(A[off + 2 * ps]), a3 = to_d<T>(A[off + 3 * ps]);
      s = a0 * a0 + a1 * a1 + a2 * a2 + a3 * a3;
    }
    cacc += s;
    double w = wave_sum(s);
    if ((t & 63) == 0) wsum[t >> 6][(i - i0) & 63] = w;
    if (((i - i0) & 63) == 63 || i == i1 - 1) {
      __syncthreads();
      const int64_t base = i - ((i - i0) & 63);
      for (int64_t k = t; k <= (i - base); k += 256) {
        double r = ((wsum[0][k] + wsum[1][k]) + wsum[2][k]) + wsum[3][k];
        rowpart[(int64_t)blockIdx.x * m + base + k] = r;
      }
      __syncthreads();
    }
  }
  if (j < n) colpart[(int64_t)blockIdx.y * n + j] = cacc;
}

// Row tiles of rb rows: at most 64 row tiles per column (one wave folds them),
// and enough tiles to cover the chip when the matrix is large.
void probs_grid(int64_t m, int64_t n, int* rb, int* nrb, int* ncb) {
  int64_t cb = (n + 255) / 256;
  int64_t r = std::max<int64_t>(4, (m + 63) / 64);
  while (r > 4 && ((m + r - 1) / r) * cb < 1024 && (m + r / 2 - 1) / (r / 2) <= 64) r >>= 1;
  *rb = (int)r;
  *nrb = (int)((m + r - 1) / r);
  *ncb = (int)cb;
}

hipError_t launch_probs_partials(const Ctx& c, QView A, double* colpart, double* rowpart, int rb, int ncb) {
  int nrb = (int)((A.rows + rb - 1) / rb);
  dim3 grid(ncb, nrb);
  switch (A.dt) {
    case QCUR_F64:
      hipLaunchKernelGGL(k_probs_partials<double>, grid, dim3(256), 0, c.stream, (const double*)A.p,
                         A.rows, A.cols, A.ld, A.ps, rb, colpart, rowpart);
      break;
    case QCUR_F32:
      hipLaunchKernelGGL(k_probs_partials<float>, grid, dim3(256), 0, c.stream, (const float*)A.p,
                         A.rows, A.cols, A.ld, A.ps, rb, colpart, rowpart);
      break;
    default:
      hipLaunchKernelGGL(k_probs_partials<uint16_t>, grid, dim3(256), 0, c.stream,
                         (const uint16_t*)A.p, A.rows, A.cols, A.ld, A.ps, rb, colpart, rowpart);
  }
  return hipGetLastError();
}

// probs, pass 2: col2[j] = sum over row tiles, row2[i] = sum over column
// tiles, one wave per output (lane-strided partial sums, then a fixed
// xor-tree), written into p and q.
__global__ __launch_bounds__(256) void k_probs_fold(int64_t m, int64_t n, const double* __restrict__ colpart,
                                                    const double* __restrict__ rowpart, int nrb, int ncb,
                                                    double* p, double* q) {
  const int64_t t = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (t >= n + m) return;
  double s = 0.0;
  if (t < n) {
    for (int r = lane; r < nrb; r += 64) s += colpart[(int64_t)r * n + t];
  } else {
    for (int b = lane; b < ncb; b += 64) s += rowpart[(int64_t)b * m + (t - n)];
  }
  s = wave_sum(s);
  if (lane == 0) {
    if (t < n) p[t] = s; else q[t - n] = s;
  }
}

// probs, pass 3 (one workgroup): fro2 = sum of row sums by a fixed tree, then
// normalise (length) or fill 1/n, 1/m (uniform).
__global__ __launch_bounds__(1024) void k_probs_norm(int64_t m, int64_t n, int sampling, int have_sums,
                                                     double* p, double* q, double* fro2,
                                                     unsigned* status) {
  __shared__ double red[1024];
  __shared__ double total;
  const int t = threadIdx.x;
  if (have_sums) {
    double s = 0.0;
    for (int64_t i = t; i < m; i += 1024) s += q[i];
    red[t] = s;
    __syncthreads();
    for (int w = 512; w >= 1; w >>= 1) {
      if (t < w) red[t] += red[t + w];
      __syncthreads();
    }
    if (t == 0) {
      total = red[0];
      if (fro2) fro2[0] = red[0];
      if (sampling == QCUR_LENGTH && status && !(red[0] > 0.0 && red[0] < INFINITY)) atomicOr(status, ST_NUMERIC);
    }
    __syncthreads();
  }
  if (sampling == QCUR_LENGTH) {
    const double f = total;
    for (int64_t j = t; j < n; j += 1024) p[j] = p[j] / f;
    for (int64_t i = t; i < m; i += 1024) q[i] = q[i] / f;
  } else {
    const double pn = 1.0 / (double)n, qm = 1.0 / (double)m;
    for (int64_t j = t; j < n; j += 1024) p[j] = pn;
    for (int64_t i = t; i < m; i += 1024) q[i] = qm;
  }
}

hipError_t launch_probs_finish(const Ctx& c, int64_t m, int64_t n, const double* colpart,
                               const double* rowpart, int nrb, int ncb, int sampling, double* p,
                               double* q, double* fro2, double* scratch) {
  const int have = colpart != nullptr;
  double* pp = p;
  double* qq = q;
  if (have && sampling == QCUR_UNIFORM) {  // sums only feed fro2
    pp = scratch;
    qq = scratch + n;
  }
  if (have) {
    int64_t tot = m + n;
    hipLaunchKernelGGL(k_probs_fold, dim3((unsigned)((tot + 3) / 4)), dim3(256), 0, c.stream, m, n,
                       colpart, rowpart, nrb, ncb, pp, qq);
    if (sampling == QCUR_UNIFORM) {
      hipLaunchKernelGGL(k_probs_norm, dim3(1), dim3(1024), 0, c.stream, m, n, (int)QCUR_LENGTH, 1, pp,
                         qq, fro2, (unsigned*)nullptr);
    }
  }
  if (sampling == QCUR_LENGTH) {
    hipLaunchKernelGGL(k_probs_norm, dim3(1), dim3(1024), 0, c.stream, m, n, sampling, 1, p, q, fro2,
                       c.status);
  } else {
    hipLaunchKernelGGL(k_probs_norm, dim3(1), dim3(1024), 0, c.stream, m, n, sampling, 0, p, q,
                       (double*)nullptr, c.status);
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Gather out[c][s][t] = A[c][rows(s)][cols(t)] where rows/cols are the index
// lists or the identity.  One thread per output element and plane group.
template <typename TI, typename TO>
__global__ __launch_bounds__(256) void k_gather(const TI* __restrict__ A, int64_t am, int64_t an, int64_t ald,
                                                int64_t aps, const int64_t* __restrict__ ridx,
                                                const int64_t* __restrict__ cidx, TO* __restrict__ O,
                                                int64_t om, int64_t on, int64_t old, int64_t ops,
                                                unsigned* status) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  for (int64_t s = blockIdx.y; s < om; s += gridDim.y) {
  if (t >= on || s >= om) continue;
  int64_t i = ridx ? ridx[s] : s;
  int64_t j = cidx ? cidx[t] : t;
  const bool ok = i >= 0 && i < am && j >= 0 && j < an;
  if (!ok) atomicOr(status, ST_ARG);
  const int64_t src = i * ald + j;
  const int64_t dst = s * old + t;
#pragma unroll
  for (int c = 0; c < 4; ++c) O[dst + c * ops] = ok ? from_d<TO>(to_d<TI>(A[src + c * aps])) : from_d<TO>(0.0);
  }
}

template <typename TI>
static void gather_dispatch_out(const Ctx& c, QView A, const int64_t* ri, const int64_t* ci, QView O) {
  dim3 grid((unsigned)((O.cols + 255) / 256), (unsigned)std::min<int64_t>(O.rows, 65535));
  switch (O.dt) {
    case QCUR_F64:
      hipLaunchKernelGGL((k_gather<TI, double>), grid, dim3(256), 0, c.stream, (const TI*)A.p, A.rows,
                         A.cols, A.ld, A.ps, ri, ci, (double*)O.p, O.rows, O.cols, O.ld, O.ps, c.status);
      break;
    case QCUR_F32:
      hipLaunchKernelGGL((k_gather<TI, float>), grid, dim3(256), 0, c.stream, (const TI*)A.p, A.rows,
                         A.cols, A.ld, A.ps, ri, ci, (float*)O.p, O.rows, O.cols, O.ld, O.ps, c.status);
      break;
    default:
      hipLaunchKernelGGL((k_gather<TI, uint16_t>), grid, dim3(256), 0, c.stream, (const TI*)A.p, A.rows,
                         A.cols, A.ld, A.ps, ri, ci, (uint16_t*)O.p, O.rows, O.cols, O.ld, O.ps,
                         c.status);
  }
}

static void gather_one(const Ctx& c, QView A, const int64_t* ri, const int64_t* ci, QView O) {
  if (O.rows == 0 || O.cols == 0) return;
  switch (A.dt) {
    case QCUR_F64: gather_dispatch_out<double>(c, A, ri, ci, O); break;
    case QCUR_F32: gather_dispatch_out<float>(c, A, ri, ci, O); break;
    default: gather_dispatch_out<uint16_t>(c, A, ri, ci, O);
  }
}

// Up to three gathers from one A into outputs of one dtype in a single
// launch: a flat grid over the output elements of all of them (output v
// starts at element first[v]), each element as in k_gather.
struct GatherSet {
  const int64_t* ridx[3];
  const int64_t* cidx[3];
  void* O[3];
  int64_t om[3], on[3], old[3], ops[3], first[4];
  int n;
};

template <typename TI, typename TO>
__global__ __launch_bounds__(256) void k_gather_set(const TI* __restrict__ A, int64_t am, int64_t an, int64_t ald,
                                                    int64_t aps, GatherSet g, unsigned* status) {
  const int64_t total = g.first[g.n];
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
    int v = 0;
    while (v + 1 < g.n && e >= g.first[v + 1]) ++v;
    const int64_t l = e - g.first[v], s = l / g.on[v], t = l % g.on[v];
    const int64_t i = g.ridx[v] ? g.ridx[v][s] : s;
    const int64_t j = g.cidx[v] ? g.cidx[v][t] : t;
    const bool ok = i >= 0 && i < am && j >= 0 && j < an;
    if (!ok) atomicOr(status, ST_ARG);
    const int64_t src = i * ald + j;
    TO* __restrict__ O = (TO*)g.O[v] + s * g.old[v] + t;
#pragma unroll
    for (int c = 0; c < 4; ++c) O[c * g.ops[v]] = ok ? from_d<TO>(to_d<TI>(A[src + c * aps])) : from_d<TO>(0.0);
  }
}

template <typename TI, typename TO>
static void gather_set_out(const Ctx& c, QView A, const GatherSet& g) {
  const int64_t blocks = std::min<int64_t>((g.first[g.n] + 255) / 256, 65536);
  hipLaunchKernelGGL((k_gather_set<TI, TO>), dim3((unsigned)blocks), dim3(256), 0, c.stream, (const TI*)A.p, A.rows,
                     A.cols, A.ld, A.ps, g, c.status);
}

template <typename TI>
static void gather_set_in(const Ctx& c, QView A, const GatherSet& g, int odt) {
  switch (odt) {
    case QCUR_F64: gather_set_out<TI, double>(c, A, g); break;
    case QCUR_F32: gather_set_out<TI, float>(c, A, g); break;
    default: gather_set_out<TI, uint16_t>(c, A, g);
  }
}

hipError_t launch_gather(const Ctx& c, QView A, const int64_t* I, int64_t /*r*/, const int64_t* J, int64_t /*cc*/,
                         const QView* C, const QView* R, const QView* W) {
  const QView* outs[3] = {C, R, W};
  const int64_t* ri[3] = {nullptr, I, I};
  const int64_t* ci[3] = {J, nullptr, J};
  GatherSet g = {};
  int odt = -1;
  bool same = true;
  for (int k = 0; k < 3; ++k) {
    const QView* o = outs[k];
    if (!o || o->rows == 0 || o->cols == 0) continue;
    if (odt >= 0 && o->dt != odt) same = false;
    odt = o->dt;
    g.ridx[g.n] = ri[k];
    g.cidx[g.n] = ci[k];
    g.O[g.n] = o->p;
    g.om[g.n] = o->rows;
    g.on[g.n] = o->cols;
    g.old[g.n] = o->ld;
    g.ops[g.n] = o->ps;
    g.first[g.n + 1] = g.first[g.n] + o->rows * o->cols;
    ++g.n;
  }
  if (g.n == 0) return hipSuccess;
  if (!same) {  // outputs of different dtypes: one launch each
    if (C) gather_one(c, A, nullptr, J, *C);
    if (R) gather_one(c, A, I, nullptr, *R);
    if (W) gather_one(c, A, I, J, *W);
    return hipGetLastError();
  }
  switch (A.dt) {
    case QCUR_F64: gather_set_in<double>(c, A, g, odt); break;
    case QCUR_F32: gather_set_in<float>(c, A, g, odt); break;
    default: gather_set_in<uint16_t>(c, A, g, odt);
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Cast Y = X with optional transpose (mode bit 1) and entrywise quaternion
// conjugation (mode bit 2): Y[c][j][i] (transposed) or Y[c][i][j] receives
// sign_c X[c][i][j] with sign_c = -1 for c > 0 when conjugating.  Mode bit 4
// also checks every element read and raises ST_NUMERIC for one that is not
// finite (the check a separate pass would make).
template <typename TI, typename TO>
__global__ __launch_bounds__(256) void k_cast(const TI* __restrict__ X, int64_t rows, int64_t cols, int64_t xld,
                                              int64_t xps, TO* __restrict__ Y, int64_t yld, int64_t yps,
                                              int mode, unsigned* status) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  bool bad = false;
  for (int64_t i = blockIdx.y; i < rows; i += gridDim.y) {
  if (j >= cols) continue;
  const int64_t src = i * xld + j;
  const int64_t dst = (mode & 1) ? (j * yld + i) : (i * yld + j);
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    double v = to_d<TI>(X[src + c * xps]);
    bad |= !(v - v == 0.0);
    if ((mode & 2) && c > 0) v = -v;
    Y[dst + c * yps] = from_d<TO>(v);
  }
  }
  if ((mode & 4) && bad) atomicOr(status, ST_NUMERIC);
}

template <typename TI>
static void cast_out(const Ctx& c, QView X, QView Y, int mode) {
  dim3 grid((unsigned)((X.cols + 255) / 256), (unsigned)std::min<int64_t>(X.rows, 65535));
  switch (Y.dt) {
    case QCUR_F64:
      hipLaunchKernelGGL((k_cast<TI, double>), grid, dim3(256), 0, c.stream, (const TI*)X.p, X.rows, X.cols,
                         X.ld, X.ps, (double*)Y.p, Y.ld, Y.ps, mode, c.status);
      break;
    case QCUR_F32:
      hipLaunchKernelGGL((k_cast<TI, float>), grid, dim3(256), 0, c.stream, (const TI*)X.p, X.rows, X.cols,
                         X.ld, X.ps, (float*)Y.p, Y.ld, Y.ps, mode, c.status);
      break;
    default:
      hipLaunchKernelGGL((k_cast<TI, uint16_t>), grid, dim3(256), 0, c.stream, (const TI*)X.p, X.rows,
                         X.cols, X.ld, X.ps, (uint16_t*)Y.p, Y.ld, Y.ps, mode, c.status);
  }
}

// Up to MAXB casts with one input and one output dtype in one launch: a
// flat grid over the elements of all inputs (view v starts at element
// first[v]), each element as in k_cast above.
struct CastSet {
  const void* X[MAXB];
  void* Y[MAXB];
  int64_t cols[MAXB], xld[MAXB], xps[MAXB], yld[MAXB], yps[MAXB], first[MAXB + 1];
  int mode[MAXB];
  int n;
};

template <typename TI, typename TO>
__global__ __launch_bounds__(256) void k_cast_set(CastSet s, unsigned* status) {
  const int64_t total = s.first[s.n];
  bool bad = false;  // a non-finite element of a view that asks for the check
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
    int v = 0;
    while (v + 1 < s.n && e >= s.first[v + 1]) ++v;
    const int64_t l = e - s.first[v], i = l / s.cols[v], j = l % s.cols[v];
    const int mode = s.mode[v];
    const TI* __restrict__ X = (const TI*)s.X[v] + i * s.xld[v] + j;
    TO* __restrict__ Y = (TO*)s.Y[v] + ((mode & 1) ? (j * s.yld[v] + i) : (i * s.yld[v] + j));
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      double x = to_d<TI>(X[c * s.xps[v]]);
      bad |= (mode & 4) && !(x - x == 0.0);
      if ((mode & 2) && c > 0) x = -x;
      Y[c * s.yps[v]] = from_d<TO>(x);
    }
  }
  if (bad) atomicOr(status, ST_NUMERIC);
}

template <typename TI, typename TO>
static void cast_set_out(const Ctx& c, const CastSet& s) {
  const int64_t blocks = std::min<int64_t>((s.first[s.n] + 255) / 256, 65536);
  hipLaunchKernelGGL((k_cast_set<TI, TO>), dim3((unsigned)blocks), dim3(256), 0, c.stream, s, c.status);
}

template <typename TI>
static void cast_set_in(const Ctx& c, const CastSet& s, int odt) {
  switch (odt) {
    case QCUR_F64: cast_set_out<TI, double>(c, s); break;
    case QCUR_F32: cast_set_out<TI, float>(c, s); break;
    default: cast_set_out<TI, uint16_t>(c, s);
  }
}

hipError_t launch_cast_set(const Ctx& c, int n, const QView* X, const QView* Y, const int* modes) {
  bool same = n >= 1 && n <= MAXB;
  for (int v = 1; v < n && same; ++v) same = X[v].dt == X[0].dt && Y[v].dt == Y[0].dt;
  if (!same) {  // one launch per view
    for (int v = 0; v < n; ++v) {
      const hipError_t e = launch_cast(c, X[v], Y[v], modes[v]);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }
  CastSet s = {};
  for (int v = 0; v < n; ++v) {
    if (X[v].rows == 0 || X[v].cols == 0) continue;  // nothing to cast
    const int k = s.n++;
    s.X[k] = X[v].p;
    s.Y[k] = Y[v].p;
    s.cols[k] = X[v].cols;
    s.xld[k] = X[v].ld;
    s.xps[k] = X[v].ps;
    s.yld[k] = Y[v].ld;
    s.yps[k] = Y[v].ps;
    s.mode[k] = modes[v];
    s.first[k + 1] = s.first[k] + X[v].rows * X[v].cols;
  }
  if (s.n == 0) return hipSuccess;
  switch (X[0].dt) {
    case QCUR_F64: cast_set_in<double>(c, s, Y[0].dt); break;
    case QCUR_F32: cast_set_in<float>(c, s, Y[0].dt); break;
    default: cast_set_in<uint16_t>(c, s, Y[0].dt);
  }
  return hipGetLastError();
}

hipError_t launch_cast(const Ctx& c, QView X, QView Y, int mode) {
  if (X.rows == 0 || X.cols == 0) return hipSuccess;
  switch (X.dt) {
    case QCUR_F64: cast_out<double>(c, X, Y, mode); break;
    case QCUR_F32: cast_out<float>(c, X, Y, mode); break;
    default: cast_out<uint16_t>(c, X, Y, mode);
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
__global__ void k_check_finite(const void* X, int dt, int64_t rows, int64_t cols, int64_t ld, int64_t ps,
                               unsigned* status) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  for (int64_t i = blockIdx.y; i < rows; i += gridDim.y) {
  if (j >= cols) continue;
  bool bad = false;
  for (int c = 0; c < 4; ++c) {
    double v = load_as_double(X, dt, i * ld + j + c * ps);
    bad |= !(v - v == 0.0);
  }
  if (bad) atomicOr(status, ST_NUMERIC);
  }
}

hipError_t launch_check_finite(const Ctx& c, QView X) {
  if (X.rows == 0 || X.cols == 0) return hipSuccess;
  hipLaunchKernelGGL(k_check_finite, dim3((unsigned)((X.cols + 255) / 256), (unsigned)std::min<int64_t>(X.rows, 65535)), dim3(256), 0,
                     c.stream, (const void*)X.p, X.dt, X.rows, X.cols, X.ld, X.ps, c.status);
  return hipGetLastError();
}

__global__ void k_fill_identity(double* V, int64_t q) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t tot = q * q;
  if (t >= tot) return;
  const int64_t i = t / q, j = t % q;
  V[t] = (i == j) ? 1.0 : 0.0;
  V[t + tot] = 0.0;
  V[t + 2 * tot] = 0.0;
  V[t + 3 * tot] = 0.0;
}

hipError_t launch_fill_identity(const Ctx& c, double* V, int64_t q) {
  if (q == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_identity, dim3((unsigned)((q * q + 255) / 256)), dim3(256), 0, c.stream, V, q);
  return hipGetLastError();
}

// Entry t of the flat four-plane array: the SplitMix64 output function of
// seed + (t + 1) * 0x9E3779B97F4A7C15, its top 53 bits scaled to [-1, 1).
__global__ void k_sketch(double* S, int64_t total, uint64_t seed) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= total) return;
  uint64_t z = seed + 0x9E3779B97F4A7C15ull * (uint64_t)(t + 1);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  S[t] = (double)(z >> 11) * 0x1p-52 - 1.0;
}

hipError_t launch_sketch(const Ctx& c, QView S, uint64_t seed) {
  if (S.dt != QCUR_F64 || S.ld != S.cols || S.ps != S.rows * S.cols) return hipErrorInvalidValue;
  const int64_t total = 4 * S.rows * S.cols;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_sketch, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, c.stream, (double*)S.p, total,
                     seed);
  return hipGetLastError();
}

// Y = alpha X + beta Y, elementwise over four planes (any dtypes).
__global__ void k_axpby(double alpha, const void* X, int xdt, int64_t xld, int64_t xps, double beta, void* Y,
                        int ydt, int64_t yld, int64_t yps, int64_t rows, int64_t cols) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  for (int64_t i = blockIdx.y; i < rows; i += gridDim.y) {
  if (j >= cols) continue;
  for (int c = 0; c < 4; ++c) {
    const int64_t yo = i * yld + j + c * yps;
    double y = beta == 0.0 ? 0.0 : beta * load_as_double(Y, ydt, yo);
    store_from_double(Y, ydt, yo, alpha * load_as_double(X, xdt, i * xld + j + c * xps) + y);
  }
  }
}

hipError_t launch_axpby(const Ctx& c, double alpha, QView X, double beta, QView Y) {
  if (Y.rows == 0 || Y.cols == 0) return hipSuccess;
  hipLaunchKernelGGL(k_axpby, dim3((unsigned)((Y.cols + 255) / 256), (unsigned)std::min<int64_t>(Y.rows, 65535)), dim3(256), 0, c.stream,
                     alpha, (const void*)X.p, X.dt, X.ld, X.ps, beta, Y.p, Y.dt, Y.ld, Y.ps, Y.rows, Y.cols);
  return hipGetLastError();
}

// X = I - X for a square matrix.
__global__ void k_identity_minus(void* X, int dt, int64_t n, int64_t ld, int64_t ps) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  for (int64_t i = blockIdx.y; i < n; i += gridDim.y) {
  if (j >= n) continue;
  for (int c = 0; c < 4; ++c) {
    const int64_t o = i * ld + j + c * ps;
    double v = -load_as_double(X, dt, o);
    if (c == 0 && i == j) v += 1.0;
    store_from_double(X, dt, o, v);
  }
  }
}

hipError_t launch_identity_minus(const Ctx& c, QView X) {
  if (X.rows == 0) return hipSuccess;
  hipLaunchKernelGGL(k_identity_minus, dim3((unsigned)((X.cols + 255) / 256), (unsigned)std::min<int64_t>(X.rows, 65535)), dim3(256), 0,
                     c.stream, X.p, X.dt, X.rows, X.ld, X.ps);
  return hipGetLastError();
}

// Fixed-order sum of `count` doubles by one workgroup.
__global__ __launch_bounds__(1024) void k_sum_partials(const double* __restrict__ part, int64_t count,
                                                       double* out, int take_sqrt, const int* skip) {
  __shared__ double red[1024];
  if (skip && *skip) return;  // the result is already in out
  const int t = threadIdx.x;
  double s = 0.0;
  for (int64_t i = t; i < count; i += 1024) s += part[i];
  red[t] = s;
  __syncthreads();
  for (int w = 512; w >= 1; w >>= 1) {
    if (t < w) red[t] += red[t + w];
    __syncthreads();
  }
  if (t == 0) out[0] = take_sqrt ? sqrt(red[0]) : red[0];
}

hipError_t launch_sum_partials(const Ctx& c, const double* partials, int64_t count, double* out, int take_sqrt,
                               const int* skip) {
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(1024), 0, c.stream, partials, count, out, take_sqrt, skip);
  return hipGetLastError();
}

// M += D elementwise over the four planes; workgroup w writes the FP64 sum of
// squares of the D elements it visited (fixed element order) to dpart[w].
template <typename T>
__global__ __launch_bounds__(256) void k_core_correct(T* M, int64_t ldm, int64_t psm, const T* D, int64_t ldd,
                                                      int64_t psd, int64_t rows, int64_t cols, double* dpart) {
  __shared__ double red[256];
  const int64_t n = rows * cols;
  double s = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) {
    const int64_t i = e / cols, j = e % cols;
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      const T d = D[i * ldd + j + p * psd];
      M[i * ldm + j + p * psm] += d;
      s += (double)d * (double)d;
    }
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) dpart[blockIdx.x] = red[0];
}

hipError_t launch_core_correct(const Ctx& c, QView M, QView D, double* dpart) {
  if (M.dt != D.dt || M.rows != D.rows || M.cols != D.cols) return hipErrorInvalidValue;
  if (M.dt == QCUR_F64)
    hipLaunchKernelGGL(k_core_correct<double>, dim3(CORE_PARTS), dim3(256), 0, c.stream, (double*)M.p, M.ld, M.ps,
                       (const double*)D.p, D.ld, D.ps, M.rows, M.cols, dpart);
  else if (M.dt == QCUR_F32)
    hipLaunchKernelGGL(k_core_correct<float>, dim3(CORE_PARTS), dim3(256), 0, c.stream, (float*)M.p, M.ld, M.ps,
                       (const float*)D.p, D.ld, D.ps, M.rows, M.cols, dpart);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_resid_identity(const double* epart, int64_t ecount, const double* dpart,
                                                        double gate, double* out, int* skip) {
  __shared__ double red[2][256];
  double se = 0.0, sd = 0.0;
  for (int64_t i = threadIdx.x; i < ecount; i += 256) se += epart[i];
  for (int i = threadIdx.x; i < CORE_PARTS; i += 256) sd += dpart[i];
  red[0][threadIdx.x] = se;
  red[1][threadIdx.x] = sd;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w) {
      red[0][threadIdx.x] += red[0][threadIdx.x + w];
      red[1][threadIdx.x] += red[1][threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double e2 = red[0][0], d2 = red[1][0];
    const bool take = isfinite(e2) && isfinite(d2) && d2 <= gate * e2;
    if (take) out[0] = sqrt(fmax(e2 - d2, 0.0));
    skip[0] = take ? 1 : 0;
  }
}

hipError_t launch_resid_identity(const Ctx& c, const double* epart, int64_t ecount, const double* dpart, double gate,
                                 double* out, int* skip) {
  hipLaunchKernelGGL(k_resid_identity, dim3(1), dim3(256), 0, c.stream, epart, ecount, dpart, gate, out, skip);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Inverse index map: inv[idx[s]] = s, -1 elsewhere; repeated or out-of-range
// indices raise ST_ARG.
__global__ void k_fill_i32(int32_t* p, int64_t n, int32_t v) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t < n) p[t] = v;
}
__global__ void k_inverse_map(const int64_t* idx, int64_t cnt, int64_t n, int32_t* inv, unsigned* status) {
  const int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (s >= cnt) return;
  const int64_t i = idx[s];
  if (i < 0 || i >= n) {
    atomicOr(status, ST_ARG);
    return;
  }
  if (atomicCAS(&inv[i], -1, (int32_t)s) != -1) atomicOr(status, ST_ARG);
}

hipError_t launch_inverse_map(const Ctx& c, const int64_t* idx, int64_t cnt, int64_t n, int32_t* inv) {
  if (n > 0)
    hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c.stream, inv, n, -1);
  if (cnt > 0)
    hipLaunchKernelGGL(k_inverse_map, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, c.stream, idx, cnt, n,
                       inv, c.status);
  return hipGetLastError();
}

// dA[i][j] = G[i][j] + gC[i][jinv[j]] + gR[iinv[i]][j] + gW[iinv[i]][jinv[j]]
// (terms present only where the row/column was sampled).  No atomics.
template <typename TO>
__global__ __launch_bounds__(256) void k_backward_assemble(TO* __restrict__ dA, int64_t m, int64_t n, int64_t ld,
                                                           int64_t ps, const void* G, int gdt, int64_t gld,
                                                           int64_t gps, int has_G, const void* gC, int cdt,
                                                           int64_t cld, int64_t cps, const void* gR, int rdt,
                                                           int64_t rld, int64_t rps, const void* gW, int wdt,
                                                           int64_t wld, int64_t wps,
                                                           const int32_t* __restrict__ iinv,
                                                           const int32_t* __restrict__ jinv) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  for (int64_t i = blockIdx.y; i < m; i += gridDim.y) {
  if (j >= n) continue;
  const int32_t s = iinv[i];
  const int32_t t = jinv[j];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    double v = has_G ? load_as_double(G, gdt, i * gld + j + c * gps) : 0.0;
    if (t >= 0) v += load_as_double(gC, cdt, i * cld + t + c * cps);
    if (s >= 0) v += load_as_double(gR, rdt, (int64_t)s * rld + j + c * rps);
    if (s >= 0 && t >= 0) v += load_as_double(gW, wdt, (int64_t)s * wld + t + c * wps);
    dA[i * ld + j + c * ps] = from_d<TO>(v);
  }
  }
}

hipError_t launch_backward_assemble(const Ctx& c, QView dA, QView G, int has_G, QView gC, QView gR, QView gW,
                                    const int32_t* iinv, const int32_t* jinv) {
  if (dA.rows == 0 || dA.cols == 0) return hipSuccess;
  dim3 grid((unsigned)((dA.cols + 255) / 256), (unsigned)std::min<int64_t>(dA.rows, 65535));
  if (dA.dt == QCUR_F64) {
    hipLaunchKernelGGL(k_backward_assemble<double>, grid, dim3(256), 0, c.stream, (double*)dA.p, dA.rows, dA.cols,
                       dA.ld, dA.ps, (const void*)G.p, G.dt, G.ld, G.ps, has_G, (const void*)gC.p, gC.dt, gC.ld,
                       gC.ps, (const void*)gR.p, gR.dt, gR.ld, gR.ps, (const void*)gW.p, gW.dt, gW.ld, gW.ps,
                       iinv, jinv);
  } else {
    hipLaunchKernelGGL(k_backward_assemble<float>, grid, dim3(256), 0, c.stream, (float*)dA.p, dA.rows, dA.cols,
                       dA.ld, dA.ps, (const void*)G.p, G.dt, G.ld, G.ps, has_G, (const void*)gC.p, gC.dt, gC.ld,
                       gC.ps, (const void*)gR.p, gR.dt, gR.ld, gR.ps, (const void*)gW.p, gW.dt, gW.ld, gW.ps,
                       iinv, jinv);
  }
  return hipGetLastError();
}

// X = P_Omega(Y): observed entries copied (converted to X's dtype), the
// others set to zero (the starting point of Algorithm 2).
__global__ __launch_bounds__(256) void k_mask_init(const void* Y, int ydt, int64_t rows, int64_t cols, int64_t yld,
                                                   int64_t yps, const uint8_t* __restrict__ mask, int64_t mask_ld,
                                                   void* X, int xdt, int64_t xld, int64_t xps) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j >= cols) return;
  for (int64_t i = blockIdx.y; i < rows; i += gridDim.y) {
    const bool obs = mask[i * mask_ld + j] != 0;
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      const double v = obs ? load_as_double(Y, ydt, i * yld + j + p * yps) : 0.0;
      store_from_double(X, xdt, i * xld + j + p * xps, v);
    }
  }
}

hipError_t launch_mask_init(const Ctx& c, QView Y, const uint8_t* mask, int64_t mask_ld, QView X) {
  if (Y.rows == 0 || Y.cols == 0) return hipSuccess;
  dim3 grid((unsigned)((Y.cols + 255) / 256), (unsigned)std::min<int64_t>(Y.rows, 65535));
  hipLaunchKernelGGL(k_mask_init, grid, dim3(256), 0, c.stream, Y.p, Y.dt, Y.rows, Y.cols, Y.ld, Y.ps, mask,
                     mask_ld, X.p, X.dt, X.ld, X.ps);
  return hipGetLastError();
}

}  // namespace qcur
