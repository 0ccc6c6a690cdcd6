// Pieces of the fast pseudoinverse path for numerically full-rank tall
// matrices (CholeskyQR2 with explicit inverse factors):
//   G = Z^H Z = L L^H,  P = L^{-1}  (Z = Q L^H with Q = Z P^H orthonormal)
// Cholesky is blocked: a single-workgroup kernel factors and inverts each
// diagonal block of at most 64 x 64 quaternions in LDS, the panels and the
// trailing updates are quaternion GEMMs.  Quaternion Hermitian positive
// definite matrices have real positive pivots, so the scalar recurrences are
// the usual ones with the Hamilton product and quaternion conjugation.
#include <algorithm>

#include "qcur_internal.hpp"

namespace qcur {

constexpr int CB = 64;  // diagonal block size

struct Qd {
  double w, x, y, z;
};
// a * conj(b)
__device__ inline Qd qmul_conj(Qd a, Qd b) {
  const double b0 = b.w, b1 = -b.x, b2 = -b.y, b3 = -b.z;
  return Qd{a.w * b0 - a.x * b1 - a.y * b2 - a.z * b3, a.w * b1 + a.x * b0 + a.y * b3 - a.z * b2,
            a.w * b2 - a.x * b3 + a.y * b0 + a.z * b1, a.w * b3 + a.x * b2 - a.y * b1 + a.z * b0};
}
__device__ inline Qd qmul(Qd a, Qd b) {
  return Qd{a.w * b.w - a.x * b.x - a.y * b.y - a.z * b.z, a.w * b.x + a.x * b.w + a.y * b.z - a.z * b.y,
            a.w * b.y - a.x * b.z + a.y * b.w + a.z * b.x, a.w * b.z + a.x * b.y - a.y * b.x + a.z * b.w};
}

// In-place factorisation of one w x w Hermitian diagonal block (w <= 64)
// with one barrier per step and every operand of a step loaded before any
// store.  Cholesky (right-looking): at step j every
// thread subtracts a[i][j] conj(a[k][j]) / d_j from its trailing elements
// (j < k <= i), while the scaled column L[i][j] = a[i][j] / sqrt(d_j) is
// stored conjugated in the unused upper triangle (a[j][i] = conj(L[i][j]),
// i.e. L^H).  Then the triangular inverse P = L^{-1} overwrites the stale
// lower triangle, column by column from the last one:
//   P[i][j] = -(sum_{k=j+1..i} P[i][k] L[k][j]) / L[j][j]   (i > j).
// Only P is written back (lower triangle; the upper one is zeroed).  A pivot
// that is not finite and positive sets *fail.
constexpr int CHOL_THREADS = 512;

// 1/sqrt(d) from the hardware estimate refined by two Newton steps (the
// pivot feeds only products, so correct rounding is not needed).
__device__ inline double rsqrt_nr(double d) {
  double r = __builtin_amdgcn_rsq(d);
  r = r * (1.5 - 0.5 * d * r * r);
  r = r * (1.5 - 0.5 * d * r * r);
  return r;
}

__global__ __launch_bounds__(CHOL_THREADS) void k_chol_block(const double* __restrict__ G0, double* __restrict__ P0,
                                                             int w, int64_t ld, int64_t ps, int64_t sbatch,
                                                             int* fail0) {
  const double* __restrict__ G = G0 + (int64_t)blockIdx.x * sbatch;
  double* __restrict__ Pg = P0 + (int64_t)blockIdx.x * sbatch;
  int* fail = fail0 + blockIdx.x;
  __shared__ double a[4][CB][CB + 1];
  __shared__ double rdg[CB];  // 1 / L[j][j]
  __shared__ int bad;
  const int tid = threadIdx.x;
  if (tid == 0) bad = 0;
  for (int e = tid; e < w * w; e += CHOL_THREADS) {
    const int i = e / w, j = e % w;
    if (j <= i) {
      const int64_t o = (int64_t)i * ld + j;
#pragma unroll
      for (int c = 0; c < 4; ++c) a[c][i][j] = G[o + c * ps];
    }
  }
  __syncthreads();
  // Cholesky: the t(t+1)/2 trailing entries of step j are spread over the
  // threads (entry e is row r, column q of the trailing triangle with
  // e = r(r+1)/2 + q), so the work per step shrinks with the triangle.
  for (int j = 0; j < w; ++j) {
    const double d = a[0][j][j];
    const bool ok = d > 0.0 && d < INFINITY;
    const double rs = rsqrt_nr(ok ? d : 1.0);
    const double rd = rs * rs;
    const int t = w - j - 1;
    const int cnt = t * (t + 1) / 2;
    if (tid == 0) {
      rdg[j] = rs;
      if (!ok) bad = 1;
    }
    if (tid < t) {  // L^H row j into the upper triangle (never read in this step)
      const int k = j + 1 + tid;
      a[0][j][k] = a[0][k][j] * rs;
      a[1][j][k] = -a[1][k][j] * rs;
      a[2][j][k] = -a[2][k][j] * rs;
      a[3][j][k] = -a[3][k][j] * rs;
    }
    for (int e = tid; e < cnt; e += CHOL_THREADS) {
      const int r = (int)((sqrtf((float)(8 * e + 1)) - 1.0f) * 0.5f);
      const int i = j + 1 + r, k = j + 1 + (e - r * (r + 1) / 2);
      const Qd q = qmul_conj(Qd{a[0][i][j], a[1][i][j], a[2][i][j], a[3][i][j]},
                             Qd{a[0][k][j], a[1][k][j], a[2][k][j], a[3][k][j]});
      a[0][i][k] -= q.w * rd;
      a[1][i][k] -= q.x * rd;
      a[2][i][k] -= q.y * rd;
      a[3][i][k] -= q.z * rd;
    }
    __syncthreads();
  }
  // P's diagonal (1 / L[i][i]) replaces the stale lower diagonal
  for (int i = tid; i < w; i += CHOL_THREADS) {
    a[0][i][i] = rdg[i];
    a[1][i][i] = a[2][i][i] = a[3][i][i] = 0.0;
  }
  __syncthreads();
  // inverse: 8 threads per row; waves whose rows are all done only wait
  const int sub = tid & 7, row = tid >> 3;
  const int wave_row0 = (tid >> 6) * 8;
  for (int j = w - 2; j >= 0; --j) {
    const int t = w - j - 1;
    if (wave_row0 < t) {
      const int i = j + 1 + row;
      Qd s{0, 0, 0, 0};
      if (row < t) {
        for (int k = j + 1 + sub; k <= i; k += 8) {
          // P[i][k] L[k][j] with L[k][j] = conj(a[j][k])
          const Qd u = qmul_conj(Qd{a[0][i][k], a[1][i][k], a[2][i][k], a[3][i][k]},
                                 Qd{a[0][j][k], a[1][j][k], a[2][j][k], a[3][j][k]});
          s.w += u.w;
          s.x += u.x;
          s.y += u.y;
          s.z += u.z;
        }
      }
#pragma unroll
      for (int o = 4; o >= 1; o >>= 1) {
        s.w += __shfl_xor(s.w, o, 8);
        s.x += __shfl_xor(s.x, o, 8);
        s.y += __shfl_xor(s.y, o, 8);
        s.z += __shfl_xor(s.z, o, 8);
      }
      if (row < t && sub == 0) {
        const double f = -rdg[j];
        a[0][i][j] = f * s.w;
        a[1][i][j] = f * s.x;
        a[2][i][j] = f * s.y;
        a[3][i][j] = f * s.z;
      }
    }
    __syncthreads();
  }
  for (int e = tid; e < w * w; e += CHOL_THREADS) {
    const int i = e / w, j = e % w;
    const int64_t o = (int64_t)i * ld + j;
#pragma unroll
    for (int c = 0; c < 4; ++c) Pg[o + c * ps] = (j <= i) ? a[c][i][j] : 0.0;
  }
  if (tid == 0 && bad) atomicOr(fail, 1);
}

hipError_t launch_chol_block(const Ctx& c, const double* G, double* P, int w, int64_t ld, int64_t ps, int* fail,
                             int batch, int64_t sbatch) {
  hipLaunchKernelGGL(k_chol_block, dim3(batch), dim3(CHOL_THREADS), 0, c.stream, G, P, w, ld, ps, sbatch, fail);
  return hipGetLastError();
}

// Sum of squares of a quaternion view, one FP64 partial per workgroup.
__global__ __launch_bounds__(256) void k_sumsq(const void* X, int dt, int64_t rows, int64_t cols, int64_t ld,
                                               int64_t ps, double* partials) {
  __shared__ double red[4];
  const int tid = threadIdx.x;
  double s = 0.0;
  const int64_t total = rows * cols;
  for (int64_t e = (int64_t)blockIdx.x * 256 + tid; e < total; e += (int64_t)gridDim.x * 256) {
    const int64_t i = e / cols, j = e % cols;
    const int64_t o = i * ld + j;
    for (int c = 0; c < 4; ++c) {
      const double v = load_as_double(X, dt, o + c * ps);
      s += v * v;
    }
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o, 64);
  if ((tid & 63) == 0) red[tid >> 6] = s;
  __syncthreads();
  if (tid == 0) partials[blockIdx.x] = ((red[0] + red[1]) + red[2]) + red[3];
}

constexpr int SUMSQ_BLOCKS = 256;

hipError_t launch_sumsq(const Ctx& c, QView X, double* partials, double* out) {
  hipLaunchKernelGGL(k_sumsq, dim3(SUMSQ_BLOCKS), dim3(256), 0, c.stream, (const void*)X.p, X.dt, X.rows, X.cols,
                     X.ld, X.ps, partials);
  return launch_sum_partials(c, partials, SUMSQ_BLOCKS, out, 0);
}

// Sums of squares of up to MAXB views in one launch (grid y = view); the
// fixed-order fold writes out[b * ostride].
struct SumsqBatch {
  const double* p[MAXB];
  int64_t rows[MAXB], cols[MAXB], ld[MAXB], ps[MAXB];
};

__global__ __launch_bounds__(256) void k_sumsq_batch(SumsqBatch v, double* partials) {
  __shared__ double red[4];
  const int tid = threadIdx.x, b = blockIdx.y;
  const int64_t rows = v.rows[b], cols = v.cols[b], ld = v.ld[b], ps = v.ps[b];
  const double* X = v.p[b];
  double s = 0.0;
  const int64_t total = rows * cols;
  for (int64_t e = (int64_t)blockIdx.x * 256 + tid; e < total; e += (int64_t)gridDim.x * 256) {
    const int64_t i = e / cols, j = e % cols;
    const int64_t o = i * ld + j;
#pragma unroll
    for (int c = 0; c < 4; ++c) s += X[o + c * ps] * X[o + c * ps];
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o, 64);
  if ((tid & 63) == 0) red[tid >> 6] = s;
  __syncthreads();
  if (tid == 0) partials[(int64_t)b * gridDim.x + blockIdx.x] = ((red[0] + red[1]) + red[2]) + red[3];
}

__global__ __launch_bounds__(256) void k_fold_batch(const double* partials, int n, double* out, int ostride) {
  __shared__ double red[256];
  const int tid = threadIdx.x, b = blockIdx.x;
  double s = 0.0;
  for (int i = tid; i < n; i += 256) s += partials[(int64_t)b * n + i];
  red[tid] = s;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if (tid < w) red[tid] += red[tid + w];
    __syncthreads();
  }
  if (tid == 0) out[(int64_t)b * ostride] = red[0];
}

hipError_t launch_sumsq_batch(const Ctx& c, int nb, const QView* X, double* partials, double* out, int ostride) {
  SumsqBatch v{};
  for (int b = 0; b < nb; ++b) {
    v.p[b] = (const double*)X[b].p;
    v.rows[b] = X[b].rows;
    v.cols[b] = X[b].cols;
    v.ld[b] = X[b].ld;
    v.ps[b] = X[b].ps;
  }
  hipLaunchKernelGGL(k_sumsq_batch, dim3(SUMSQ_BLOCKS, nb), dim3(256), 0, c.stream, v, partials);
  hipLaunchKernelGGL(k_fold_batch, dim3(nb), dim3(256), 0, c.stream, (const double*)partials, SUMSQ_BLOCKS, out,
                     ostride);
  return hipGetLastError();
}

// G_b[i][i] += 1 for q_b <= i < n (padding of a smaller Gram to n x n).
struct PadBatch {
  int q[MAXB];
};
__global__ void k_pad_identity(double* G, int64_t n, int64_t sbatch, PadBatch pb) {
  const int b = blockIdx.y;
  const int64_t i = pb.q[b] + (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) G[(int64_t)b * sbatch + i * n + i] += 1.0;
}

hipError_t launch_pad_identity(const Ctx& c, double* G, int64_t n, int64_t sbatch, int nb, const int64_t* q) {
  PadBatch pb{};
  int64_t most = 0;
  for (int b = 0; b < nb; ++b) {
    pb.q[b] = (int)q[b];
    most = std::max<int64_t>(most, n - q[b]);
  }
  if (most <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_pad_identity, dim3((unsigned)((most + 255) / 256), nb), dim3(256), 0, c.stream, G, n, sbatch,
                     pb);
  return hipGetLastError();
}

// Fast-path certificate.  kappa_F = ||Z||_F ||P||_F bounds the 2-norm
// condition number from above; the fast path is taken when both Cholesky
// factorisations succeeded, the first pass was well enough conditioned for
// CholeskyQR2 (kappa_F1 < 1e7), no singular value can fall below
// rtol * sigma_max (kappa_F * rtol < 1e-2) and no rank cap applies.
struct DecideBatch {
  int64_t q[MAXB];
  int64_t* rank_out[MAXB];
};
__global__ void k_pinv_decide(const double* norms0, const int* fail0, double rtol, int64_t max_rank, DecideBatch db,
                              int nb, int* ok0) {
  const int b = threadIdx.x;
  if (b >= nb) return;
  const double* norms = norms0 + 4 * b;
  const int* fail = fail0 + b;
  int* ok = ok0 + b;
  const int64_t q = db.q[b];
  int64_t* rank_out = db.rank_out[b];
  const double z2 = norms[0], p1 = norms[1], p2 = norms[2];
  const double k1 = sqrt(z2) * sqrt(p1);
  const double k = sqrt(z2) * sqrt(p2);
  const bool good = fail[0] == 0 && z2 > 0.0 && k1 < 1e7 && k * rtol < 1e-2 && k < INFINITY &&
                    (max_rank <= 0 || max_rank >= q);
  ok[0] = good ? 1 : 0;
  if (good && rank_out) rank_out[0] = q;
}

hipError_t launch_pinv_decide(const Ctx& c, const double* norms, const int* fail, double rtol, int64_t max_rank,
                              int nb, const int64_t* q, int64_t* const* rank_out, int* ok) {
  DecideBatch db{};
  for (int b = 0; b < nb; ++b) {
    db.q[b] = q[b];
    db.rank_out[b] = rank_out[b];
  }
  hipLaunchKernelGGL(k_pinv_decide, dim3(1), dim3(64), 0, c.stream, norms, fail, rtol, max_rank, db, nb, ok);
  return hipGetLastError();
}

__global__ void k_zero(double* p, int64_t n) {
  for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < n; t += (int64_t)gridDim.x * 256) p[t] = 0.0;
}
__global__ void k_zero_i32(int* p, int64_t n) {
  for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < n; t += (int64_t)gridDim.x * 256) p[t] = 0;
}

hipError_t launch_zero(const Ctx& c, double* p, int64_t n) {
  if (n <= 0) return hipSuccess;
  const int64_t b = std::min<int64_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_zero, dim3((unsigned)b), dim3(256), 0, c.stream, p, n);
  return hipGetLastError();
}
hipError_t launch_zero_i32(const Ctx& c, int* p, int64_t n) {
  if (n <= 0) return hipSuccess;
  const int64_t b = std::min<int64_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_zero_i32, dim3((unsigned)b), dim3(256), 0, c.stream, p, n);
  return hipGetLastError();
}

}  // namespace qcur
