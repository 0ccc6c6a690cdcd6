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

template <int CTRL, int ROWS>
__device__ inline double dpp_f64(double v) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)u, CTRL, ROWS, 0xf, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(u >> 32), CTRL, ROWS, 0xf, true);
  return __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

// Sum over the 8 lanes 8g..8g+7; the total is valid in lane 8g+4.
__device__ inline double sum8_dpp(double v) {
  v += dpp_f64<0xB1, 0xf>(v);   // quad_perm [1,0,3,2]: pairs
  v += dpp_f64<0x4E, 0xf>(v);   // quad_perm [2,3,0,1]: quads
  v += dpp_f64<0x114, 0xf>(v);  // row_shr:4: lane 8g+4 adds the quad below it
  return v;
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
  // e = r(r+1)/2 + q; a thread's (r, q) pairs do not depend on j), so the work
  // per step shrinks with the triangle.  Each step issues all its loads
  // before the pivot's reciprocal square root is needed.
  constexpr int SLOTS = (CB * (CB - 1) / 2 + CHOL_THREADS - 1) / CHOL_THREADS;
  int tr[SLOTS], tq[SLOTS];
#pragma unroll
  for (int m = 0; m < SLOTS; ++m) {
    const int e = tid + m * CHOL_THREADS;
    const int r = (int)((sqrtf((float)(8 * e + 1)) - 1.0f) * 0.5f);
    tr[m] = r;
    tq[m] = e - r * (r + 1) / 2;
  }
  const int wave_e0 = (tid >> 6) * 64;
  for (int j = 0; j < w; ++j) {
    const int t = w - j - 1;
    const int cnt = t * (t + 1) / 2;
    const double d = a[0][j][j];
    Qd li[SLOTS], lk[SLOTS], x[SLOTS];
#pragma unroll
    for (int m = 0; m < SLOTS; ++m) {
      if (wave_e0 + m * CHOL_THREADS < cnt) {  // uniform over the wave
        const int e = tid + m * CHOL_THREADS;
        const int i = j + 1 + tr[m], k = j + 1 + tq[m];
        if (e < cnt) {
          li[m] = Qd{a[0][i][j], a[1][i][j], a[2][i][j], a[3][i][j]};
          lk[m] = Qd{a[0][k][j], a[1][k][j], a[2][k][j], a[3][k][j]};
          x[m] = Qd{a[0][i][k], a[1][i][k], a[2][i][k], a[3][i][k]};
        }
      }
    }
    Qd lh{0, 0, 0, 0};
    if (tid < t) lh = Qd{a[0][j + 1 + tid][j], a[1][j + 1 + tid][j], a[2][j + 1 + tid][j], a[3][j + 1 + tid][j]};
    const bool ok = d > 0.0 && d < INFINITY;
    const double rs = rsqrt_nr(ok ? d : 1.0);
    const double rd = rs * rs;
    if (tid == 0) {
      rdg[j] = rs;
      if (!ok) bad = 1;
    }
    if (tid < t) {  // L^H row j into the upper triangle (never read in this step)
      const int k = j + 1 + tid;
      a[0][j][k] = lh.w * rs;
      a[1][j][k] = -lh.x * rs;
      a[2][j][k] = -lh.y * rs;
      a[3][j][k] = -lh.z * rs;
    }
#pragma unroll
    for (int m = 0; m < SLOTS; ++m) {
      if (wave_e0 + m * CHOL_THREADS < cnt) {
        const int e = tid + m * CHOL_THREADS;
        const int i = j + 1 + tr[m], k = j + 1 + tq[m];
        if (e < cnt) {
          const Qd q = qmul_conj(li[m], lk[m]);
          a[0][i][k] = x[m].w - q.w * rd;
          a[1][i][k] = x[m].x - q.x * rd;
          a[2][i][k] = x[m].y - q.y * rd;
          a[3][i][k] = x[m].z - q.z * rd;
        }
      }
    }
    __syncthreads();
  }
  // P's diagonal (1 / L[i][i]) replaces the stale lower diagonal
  for (int i = tid; i < w; i += CHOL_THREADS) {
    a[0][i][i] = rdg[i];
    a[1][i][i] = a[2][i][i] = a[3][i][i] = 0.0;
  }
  __syncthreads();
  // inverse: 8 threads per row (lanes 8g..8g+7 of a wave), reduced in
  // registers with DPP (pairs, quads, then the quad 4 lanes below); the row
  // total lands in lane 8g+4.  Waves whose rows are all done only wait.
  const int sub = tid & 7, row = tid >> 3;
  const int wave_row0 = (tid >> 6) * 8;
  for (int j = w - 2; j >= 0; --j) {
    const int t = w - j - 1;
    if (wave_row0 < t) {
      const int i = j + 1 + row;
      const double f = -rdg[j];
      Qd pk[8], lj[8];
#pragma unroll
      for (int m = 0; m < 8; ++m) {
        const int k = j + 1 + sub + 8 * m;
        if (row < t && k <= i) {
          pk[m] = Qd{a[0][i][k], a[1][i][k], a[2][i][k], a[3][i][k]};
          lj[m] = Qd{a[0][j][k], a[1][j][k], a[2][j][k], a[3][j][k]};  // conj(L[k][j])
        } else {
          pk[m] = Qd{0, 0, 0, 0};
          lj[m] = Qd{0, 0, 0, 0};
        }
      }
      Qd s{0, 0, 0, 0};
#pragma unroll
      for (int m = 0; m < 8; ++m) {
        const Qd u = qmul_conj(pk[m], lj[m]);  // P[i][k] L[k][j]
        s.w += u.w;
        s.x += u.x;
        s.y += u.y;
        s.z += u.z;
      }
      s.w = sum8_dpp(s.w);
      s.x = sum8_dpp(s.x);
      s.y = sum8_dpp(s.y);
      s.z = sum8_dpp(s.z);
      if (row < t && sub == 4) {
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

// ||G_b - I||_F^2 over the leading q_b x q_b block of up to MAXB Gram
// matrices (n x n, sbatch apart), one workgroup each, fixed-order sums:
// the orthogonality defect of Q after a CholeskyQR pass (G = Q^H Q).
struct DefectBatch {
  int q[MAXB];
};
__global__ __launch_bounds__(256) void k_defect(const double* __restrict__ G, int64_t n, int64_t sbatch,
                                                DefectBatch db, double* out, int ostride) {
  __shared__ double red[256];
  const int b = blockIdx.x, tid = threadIdx.x;
  const int64_t q = db.q[b], nn = n * n;
  const double* g = G + (int64_t)b * sbatch;
  double s = 0.0;
  for (int64_t e = tid; e < q * q; e += 256) {
    const int64_t i = e / q, j = e % q;
    const int64_t o = i * n + j;
    const double d0 = g[o] - (i == j ? 1.0 : 0.0);
    s += d0 * d0 + g[o + nn] * g[o + nn] + g[o + 2 * nn] * g[o + 2 * nn] + g[o + 3 * nn] * g[o + 3 * nn];
  }
  red[tid] = s;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if (tid < w) red[tid] += red[tid + w];
    __syncthreads();
  }
  if (tid == 0) out[(int64_t)b * ostride] = red[0];
}

hipError_t launch_defect_batch(const Ctx& c, int nb, const double* G, int64_t n, int64_t sbatch, const int64_t* q,
                               double* out, int ostride) {
  DefectBatch db{};
  for (int b = 0; b < nb; ++b) db.q[b] = (int)q[b];
  hipLaunchKernelGGL(k_defect, dim3(nb), dim3(256), 0, c.stream, G, n, sbatch, db, out, ostride);
  return hipGetLastError();
}

}  // namespace qcur
