// Element-wise and reduction kernels of the batched QMCUR path: many
// independent problems of uneven sizes, each in its own slot of the batched
// arrays.  The grid spans the largest problem; the z (or x) index selects the
// problem, and a workgroup whose tile lies outside its problem returns at
// once.  Every reduction runs in a fixed order, so results do not depend on
// scheduling.
#include <algorithm>
#include <type_traits>

#include "qcur_internal.hpp"

namespace qcur {

namespace {

template <typename T> __device__ inline double ld_d(const T* p, int64_t o);
template <> __device__ inline double ld_d<double>(const double* p, int64_t o) { return p[o]; }
template <> __device__ inline double ld_d<float>(const float* p, int64_t o) { return (double)p[o]; }
template <> __device__ inline double ld_d<uint16_t>(const uint16_t* p, int64_t o) {
  return (double)bf16_to_f32(p[o]);
}
template <typename T> __device__ inline void st_d(T* p, int64_t o, double v);
template <> __device__ inline void st_d<double>(double* p, int64_t o, double v) { p[o] = v; }
template <> __device__ inline void st_d<float>(float* p, int64_t o, double v) { p[o] = (float)v; }
template <> __device__ inline void st_d<uint16_t>(uint16_t* p, int64_t o, double v) {
  p[o] = f32_to_bf16((float)v);
}

__device__ inline double wave_sum_d(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Fixed-order sum of one value per thread of a 256-thread workgroup.
__device__ inline double block_sum_256(double v, double* red) {
  const int tid = threadIdx.x;
  red[tid] = v;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if (tid < w) red[tid] += red[tid + w];
    __syncthreads();
  }
  return red[0];
}

// Dispatch on the run-time dtype of a slot array.
template <typename F>
hipError_t by_dtype(int dt, F&& f) {
  switch (dt) {
    case QCUR_F64: f((double*)nullptr); break;
    case QCUR_F32: f((float*)nullptr); break;
    default: f((uint16_t*)nullptr);
  }
  return hipGetLastError();
}

}  // namespace

// ---- norm pass (length probabilities, Section 3.1) ------------------------
// Workgroup (x, y, b) covers rows [32y, 32y+32) and columns [256x, 256x+256)
// of A_b: colpart[b][y][j] = sum over its rows of |a_ij|^2 and
// rowpart[b][x][i] = sum over its columns.  With Ax, the tile is also copied
// into the product dtype (fusing the cast into the one pass over A).
template <typename TI, typename TX>
__global__ __launch_bounds__(256) void kb_norms(const TI* __restrict__ A, int64_t lda, int64_t psa, int64_t sa,
                                                const int* __restrict__ dm, const int* __restrict__ dn,
                                                int64_t mx, int64_t nx, double* __restrict__ colpart,
                                                double* __restrict__ rowpart, TX* __restrict__ Ax, int64_t ldx,
                                                int64_t psx, int64_t sx) {
  // BATCH_RB rows x BATCH_CB (one wave) columns per workgroup: wave w takes
  // rows i0 + 8w .. i0 + 8w + 7, all of whose loads are issued before any
  // sum (addresses clamped into the problem, values past it zeroed)
  static_assert(BATCH_RB == 32 && BATCH_CB == 64, "four waves of eight rows, one column per lane");
  __shared__ double ws[BATCH_RB];
  __shared__ double cs[4][BATCH_CB];
  const int b = blockIdx.z, t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int64_t m = dm[b], n = dn[b];
  const int64_t i0 = (int64_t)blockIdx.y * BATCH_RB, j0 = (int64_t)blockIdx.x * BATCH_CB;
  if (i0 >= m || j0 >= n) return;  // uniform over the workgroup
  const int64_t nrbx = (mx + BATCH_RB - 1) / BATCH_RB, ncbx = (nx + BATCH_CB - 1) / BATCH_CB;
  const int64_t j = j0 + lane, i1 = min(m, i0 + BATCH_RB);
  const bool jok = j < n;
  const int64_t jc = jok ? j : n - 1;
  const TI* Ab = A + (int64_t)b * sa;
  double v[8][4];
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    const int64_t ic = min(i0 + 8 * wv + r, m - 1);
    const int64_t o = ic * lda + jc;
#pragma unroll
    for (int q = 0; q < 4; ++q) v[r][q] = ld_d(Ab, o + q * psa);
  }
  double cacc = 0.0;
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    const int64_t i = i0 + 8 * wv + r;
    const bool ok = jok && i < i1;
    const double sq = ok ? v[r][0] * v[r][0] + v[r][1] * v[r][1] + v[r][2] * v[r][2] + v[r][3] * v[r][3] : 0.0;
    if (ok && Ax) {
      TX* X = Ax + (int64_t)b * sx + i * ldx + j;
#pragma unroll
      for (int q = 0; q < 4; ++q) st_d(X, q * psx, v[r][q]);
    }
    cacc += sq;
    const double w = wave_sum_d(sq);
    if (lane == 0) ws[8 * wv + r] = w;
  }
  cs[wv][lane] = cacc;
  __syncthreads();
  for (int64_t k = t; k < i1 - i0; k += 256) rowpart[((int64_t)b * ncbx + blockIdx.x) * mx + i0 + k] = ws[k];
  if (t < BATCH_CB && jok)
    colpart[((int64_t)b * nrbx + blockIdx.y) * nx + j] = ((cs[0][t] + cs[1][t]) + cs[2][t]) + cs[3][t];
}

hipError_t launch_norms_batch(const Ctx& c, int count, Slots A, const int* dm, const int* dn, int64_t mx,
                              int64_t nx, double* colpart, double* rowpart, const Slots* Ax) {
  if (count <= 0) return hipSuccess;
  const dim3 grid((unsigned)((nx + BATCH_CB - 1) / BATCH_CB), (unsigned)((mx + BATCH_RB - 1) / BATCH_RB),
                  (unsigned)count);
  return by_dtype(A.dt, [&](auto* ti) {
    typedef std::remove_pointer_t<decltype(ti)> TI;
    const int xdt = Ax ? Ax->dt : QCUR_F32;
    by_dtype(xdt, [&](auto* tx) {
      typedef std::remove_pointer_t<decltype(tx)> TX;
      hipLaunchKernelGGL((kb_norms<TI, TX>), grid, dim3(256), 0, c.stream, (const TI*)A.p, A.ld, A.ps, A.slab, dm,
                         dn, mx, nx, colpart, rowpart, Ax ? (TX*)Ax->p : (TX*)nullptr, Ax ? Ax->ld : 0,
                         Ax ? Ax->ps : 0, Ax ? Ax->slab : 0);
    });
  });
}

// ---- gathers (Algorithm 1, steps 1-2) ----------------------------------------
// O_b[s][t] = A_b[rows(s)][cols(t)] for s < orows[b], t < ocols[b], where the
// index lists (slots of stride ris/cis) or the identity give rows and
// columns.  An index outside A_b writes zeros and raises ST_ARG; a
// non-finite gathered value raises ST_NUMERIC.  One workgroup per 32 x 32
// tile of O_b (grid x: tiles of the largest extents, z: problems); the
// reads run along t and so do the writes, the conjugate transpose's through
// an LDS tile so that it writes along s.
constexpr int GT = 32;
template <typename TI, typename TX>
__global__ __launch_bounds__(256) void kb_gather(const TI* __restrict__ A, int64_t lda, int64_t psa, int64_t sa,
                                                 const int* __restrict__ dm, const int* __restrict__ dn,
                                                 const int64_t* __restrict__ ridx, int64_t ris,
                                                 const int64_t* __restrict__ cidx, int64_t cis,
                                                 const int* __restrict__ orows, const int* __restrict__ ocols,
                                                 double* __restrict__ O, int64_t ldo, int64_t pso, int64_t so,
                                                 TX* __restrict__ Ox, int64_t ldx, int64_t psx, int64_t sx,
                                                 int tconj, int tiles_t, unsigned* status) {
  // the transpose tile holds the input's values exactly: FP32 for FP32 and
  // BF16 inputs (half the LDS of FP64, twice the resident workgroups)
  typedef typename std::conditional<sizeof(TI) <= 4, float, double>::type TL;
  __shared__ TL tile[4][GT][GT + 1];
  const int b = blockIdx.z;
  const int64_t rows = orows[b], cols = ocols[b];
  const int64_t s0 = (int64_t)(blockIdx.x / tiles_t) * GT, t0 = (int64_t)(blockIdx.x % tiles_t) * GT;
  if (s0 >= rows || t0 >= cols) return;  // uniform over the workgroup
  const int64_t m = dm[b], n = dn[b];
  const TI* Ab = A + (int64_t)b * sa;
  const int tx = threadIdx.x % GT, ty = threadIdx.x / GT;  // 8 rows of 32 per pass
  const int64_t t = t0 + tx;
  const int64_t j = t < cols ? (cidx ? cidx[(int64_t)b * cis + t] : t) : 0;
  bool bad = false, finite = true;
#pragma unroll
  for (int r = 0; r < GT / 8; ++r) {
    const int64_t s = s0 + ty + 8 * r;
    if (s < rows && t < cols) {
      const int64_t i = ridx ? ridx[(int64_t)b * ris + s] : s;
      const bool ok = i >= 0 && i < m && j >= 0 && j < n;
      bad |= !ok;
      const int64_t src = i * lda + j;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const double v = ok ? ld_d(Ab, src + k * psa) : 0.0;
        finite &= isfinite(v);
        if (tconj) tile[k][ty + 8 * r][tx] = (TL)v;
        else O[(int64_t)b * so + s * ldo + t + k * pso] = v;
        if (Ox) st_d(Ox + (int64_t)b * sx, s * ldx + t + k * psx, v);
      }
    }
  }
  if (bad) atomicOr(status, ST_ARG);
  if (!finite) atomicOr(status, ST_NUMERIC);
  if (!tconj) return;
  double* Ob = O + (int64_t)b * so;
  // conjugate transpose: O receives element (t, s), planes 1..3 negated;
  // thread (ty, tx) now writes row t0 + ty + 8r, column s0 + tx
  __syncthreads();
#pragma unroll
  for (int r = 0; r < GT / 8; ++r) {
    const int64_t tt = t0 + ty + 8 * r, ss = s0 + tx;
    if (tt < cols && ss < rows)
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const double v = (double)tile[k][tx][ty + 8 * r];
        Ob[tt * ldo + ss + k * pso] = k > 0 ? -v : v;
      }
  }
}

hipError_t launch_gather_batch(const Ctx& c, int count, Slots A, const int* dm, const int* dn,
                               const int64_t* ridx, int64_t ris, const int64_t* cidx, int64_t cis,
                               const int* orows, const int* ocols, int64_t rowsx, int64_t colsx, Slots O,
                               const Slots* Ox, int tconj) {
  if (count <= 0 || rowsx <= 0 || colsx <= 0) return hipSuccess;
  const int64_t ts = (rowsx + GT - 1) / GT, tt = (colsx + GT - 1) / GT;
  if (ts * tt > 0x7fffffff) return hipErrorInvalidValue;
  const dim3 grid((unsigned)(ts * tt), 1, (unsigned)count);
  return by_dtype(A.dt, [&](auto* ti) {
    typedef std::remove_pointer_t<decltype(ti)> TI;
    const int xdt = Ox ? Ox->dt : QCUR_F32;
    by_dtype(xdt, [&](auto* tx) {
      typedef std::remove_pointer_t<decltype(tx)> TX;
      hipLaunchKernelGGL((kb_gather<TI, TX>), grid, dim3(256), 0, c.stream, (const TI*)A.p, A.ld, A.ps, A.slab,
                         dm, dn, ridx, ris, cidx, cis, orows, ocols, (double*)O.p, O.ld, O.ps, O.slab,
                         Ox ? (TX*)Ox->p : (TX*)nullptr, Ox ? Ox->ld : 0, Ox ? Ox->ps : 0, Ox ? Ox->slab : 0,
                         tconj, (int)tt, c.status);
    });
  });
}

// ---- casts --------------------------------------------------------------------
// Y_b = X_b (rows[b] x cols[b]) with optional transpose (mode bit 1) and
// quaternion conjugation (mode bit 2).
template <typename TI, typename TO>
__global__ __launch_bounds__(256) void kb_cast(const TI* __restrict__ X, int64_t ldx, int64_t psx, int64_t sx,
                                               TO* __restrict__ Y, int64_t ldy, int64_t psy, int64_t sy,
                                               const int* __restrict__ rows, const int* __restrict__ cols,
                                               int mode, const int* __restrict__ skip_if) {
  const int b = blockIdx.z;
  if (skip_if && skip_if[b]) return;
  const int64_t R = rows[b], C = cols[b];
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j >= C) return;
  const TI* Xb = X + (int64_t)b * sx;
  TO* Yb = Y + (int64_t)b * sy;
  for (int64_t i = blockIdx.y; i < R; i += gridDim.y) {
    const int64_t src = i * ldx + j;
    const int64_t dst = (mode & 1) ? (j * ldy + i) : (i * ldy + j);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      double v = ld_d(Xb, src + k * psx);
      if ((mode & 2) && k > 0) v = -v;
      st_d(Yb, dst + k * psy, v);
    }
  }
}

hipError_t launch_cast_batch(const Ctx& c, int count, Slots X, Slots Y, const int* rows, const int* cols,
                             int64_t rowsx, int64_t colsx, int mode, const int* skip_if) {
  if (count <= 0 || rowsx <= 0 || colsx <= 0) return hipSuccess;
  // rows strided over at most 64 workgroups per column stripe: problems
  // skipped, or smaller than the extents, then cost few idle workgroups
  const dim3 grid((unsigned)((colsx + 255) / 256), (unsigned)std::min<int64_t>(rowsx, 64), (unsigned)count);
  return by_dtype(X.dt, [&](auto* ti) {
    typedef std::remove_pointer_t<decltype(ti)> TI;
    by_dtype(Y.dt, [&](auto* to) {
      typedef std::remove_pointer_t<decltype(to)> TO;
      hipLaunchKernelGGL((kb_cast<TI, TO>), grid, dim3(256), 0, c.stream, (const TI*)X.p, X.ld, X.ps, X.slab,
                         (TO*)Y.p, Y.ld, Y.ps, Y.slab, rows, cols, mode, skip_if);
    });
  });
}

// ---- pseudoinverse helpers ---------------------------------------------------
// The Gram matrices of the problems share n x n slots; outside problem t's
// q_t x q_t block the slot is set to the identity, which leaves the Cholesky
// factor and its inverse of the real block unchanged.
__global__ __launch_bounds__(256) void kb_pad_gram(double* G, int64_t n, int64_t slab, const int* __restrict__ zq) {
  const int t = blockIdx.y;
  const int64_t q = zq[t];
  const int64_t nn = n * n;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < nn; e += (int64_t)gridDim.x * 256) {
    const int64_t i = e / n, j = e % n;
    if (i < q && j < q) continue;
    double* g = G + (int64_t)t * slab + e;
    g[0] = (i == j) ? 1.0 : 0.0;
    g[nn] = 0.0;
    g[2 * nn] = 0.0;
    g[3 * nn] = 0.0;
  }
}

hipError_t launch_pad_gram_batch(const Ctx& c, int count, double* G, int64_t n, int64_t slab, const int* zq) {
  if (count <= 0 || n <= 0) return hipSuccess;
  const int64_t blocks = std::min<int64_t>((n * n + 255) / 256, 64);
  hipLaunchKernelGGL(kb_pad_gram, dim3((unsigned)blocks, (unsigned)count), dim3(256), 0, c.stream, G, n, slab, zq);
  return hipGetLastError();
}

// out[b * ostride] = ||X_b||_F^2 over its rows[b] x cols[b] block.
__global__ __launch_bounds__(256) void kb_sumsq(const double* __restrict__ X, int64_t ld, int64_t ps, int64_t slab,
                                                const int* __restrict__ rows, const int* __restrict__ cols,
                                                double* out, int ostride) {
  __shared__ double red[256];
  const int b = blockIdx.x;
  const int64_t R = rows[b], C = cols[b];
  const double* Xb = X + (int64_t)b * slab;
  double s = 0.0;
  for (int64_t e = threadIdx.x; e < R * C; e += 256) {
    const int64_t o = (e / C) * ld + (e % C);
#pragma unroll
    for (int k = 0; k < 4; ++k) s += Xb[o + k * ps] * Xb[o + k * ps];
  }
  s = block_sum_256(s, red);
  if (threadIdx.x == 0) out[(int64_t)b * ostride] = s;
}

hipError_t launch_sumsq_ragged(const Ctx& c, int count, Slots X, const int* rows, const int* cols, double* out,
                               int ostride) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(kb_sumsq, dim3((unsigned)count), dim3(256), 0, c.stream, (const double*)X.p, X.ld, X.ps,
                     X.slab, rows, cols, out, ostride);
  return hipGetLastError();
}

// CholeskyQR certificate per problem (the rule of the single-matrix path):
// kappa_F = ||Z||_F ||P||_F bounds the condition number; the fast result is
// kept when Cholesky succeeded, kappa_F1 < 1e7, kappa_F * rtol < 1e-2 and no
// rank cap below q applies.  rtol < 0 means max(p, q) * 2^-52.
__global__ __launch_bounds__(256) void kb_decide(const double* __restrict__ norms, const int* __restrict__ fail,
                                                 double rtol, int64_t max_rank, const int* __restrict__ zp,
                                                 const int* __restrict__ zq, int count2, int count,
                                                 int64_t* rank_out, int* ok) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t >= count2) return;
  const int64_t p = zp[t], q = zq[t];
  const double rt = rtol < 0.0 ? (double)(p > q ? p : q) * 0x1p-52 : rtol;
  const double z2 = norms[4 * t], p1 = norms[4 * t + 1], p2 = norms[4 * t + 2];
  const double k1 = sqrt(z2) * sqrt(p1);
  const double k = sqrt(z2) * sqrt(p2);
  const bool good = fail[t] == 0 && z2 > 0.0 && k1 < 1e7 && k * rt < 1e-2 && k < INFINITY &&
                    (max_rank <= 0 || max_rank >= q);
  ok[t] = good ? 1 : 0;
  if (good && rank_out) rank_out[t < count ? 2 * t : 2 * (t - count) + 1] = q;
}

hipError_t launch_decide_batch(const Ctx& c, int count2, int count, const double* norms, const int* fail,
                               double rtol, int64_t max_rank, const int* zp, const int* zq, int64_t* rank_out,
                               int* ok) {
  if (count2 <= 0) return hipSuccess;
  hipLaunchKernelGGL(kb_decide, dim3((unsigned)((count2 + 255) / 256)), dim3(256), 0, c.stream, norms, fail, rtol,
                     max_rank, zp, zq, count2, count, rank_out, ok);
  return hipGetLastError();
}

// One workgroup per factor t: the defect sum over the leading q x q block in
// a fixed order (each thread a fixed set of entries, then the fixed-order
// workgroup sum), the plan, and the copy of P1 for a factor that keeps its
// first pass.
__global__ __launch_bounds__(256) void kb_defect_plan(const double* __restrict__ G, int64_t n, int64_t slab,
                                                      const int* __restrict__ zq, const int* __restrict__ fail,
                                                      double tol2, const double* __restrict__ P1,
                                                      double* __restrict__ P, int* q2, int* skip) {
  __shared__ double red[256];
  __shared__ int keep;
  const int t = blockIdx.x, tid = threadIdx.x;
  const int64_t q = zq[t], nn = n * n;
  const double* Gt = G + (int64_t)t * slab;
  double s = 0.0;
  for (int64_t e = tid; e < q * q; e += 256) {
    const int64_t i = e / q, j = e % q;
    if (j > i) continue;
    const double w = i == j ? 1.0 : 2.0;  // the strict lower part stands for both triangles
    const double d0 = Gt[i * n + j] - (i == j ? 1.0 : 0.0);
    const double d1 = Gt[i * n + j + nn], d2 = Gt[i * n + j + 2 * nn], d3 = Gt[i * n + j + 3 * nn];
    s += w * (d0 * d0 + d1 * d1 + d2 * d2 + d3 * d3);
  }
  s = block_sum_256(s, red);
  if (tid == 0) {
    keep = (fail[t] == 0 && s <= tol2) ? 1 : 0;
    q2[t] = keep ? 0 : (int)q;
    skip[t] = keep;
  }
  __syncthreads();
  if (!keep) return;
  const double* src = P1 + (int64_t)t * slab;
  double* dst = P + (int64_t)t * slab;
  for (int64_t e = tid; e < q * q; e += 256) {
    const int64_t o = (e / q) * n + e % q;
#pragma unroll
    for (int c = 0; c < 4; ++c) dst[o + c * nn] = src[o + c * nn];
  }
}

hipError_t launch_defect_plan_batch(const Ctx& c, int count, const double* G, int64_t n, int64_t slab, const int* zq,
                                    const int* fail, double tol2, const double* P1, double* P, int* q2, int* skip) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(kb_defect_plan, dim3((unsigned)count), dim3(256), 0, c.stream, G, n, slab, zq, fail, tol2, P1, P,
                     q2, skip);
  return hipGetLastError();
}

// residual_b = sqrt(sum of problem b's tile partials), in tile order over
// the problem's own tiles (the others are never written).
__global__ __launch_bounds__(256) void kb_resid_sum(const double* __restrict__ part, int64_t tiles, int64_t gx,
                                                   int tile, const int* __restrict__ dm,
                                                   const int* __restrict__ dn, double* out, const int* skip) {
  __shared__ double red[256];
  const int b = blockIdx.x;
  if (skip && skip[b]) return;  // out[b] already holds the residual
  const int64_t ty = (dm[b] + tile - 1) / tile, tx = (dn[b] + tile - 1) / tile;
  double s = 0.0;
  for (int64_t k = threadIdx.x; k < tiles; k += 256)
    if (k / gx < ty && k % gx < tx) s += part[(int64_t)b * tiles + k];
  s = block_sum_256(s, red);
  if (threadIdx.x == 0) out[b] = sqrt(s);
}

hipError_t launch_resid_sum_batch(const Ctx& c, int count, const double* part, int64_t tiles, int64_t gx, int tile,
                                  const int* dm, const int* dn, double* out, const int* skip) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(kb_resid_sum, dim3((unsigned)count), dim3(256), 0, c.stream, part, tiles, gx, tile, dm, dn,
                     out, skip);
  return hipGetLastError();
}

// M_b += D_b over problem b's rows x cols (blockIdx.y = b), FP64 sums of
// squares of D_b per workgroup into dpart[b * CORE_PARTS + blockIdx.x].
template <typename T>
__global__ __launch_bounds__(256) void kb_core_correct(T* M, int64_t ldm, int64_t psm, int64_t sm, const T* D,
                                                       int64_t ldd, int64_t psd, int64_t sd,
                                                       const int* __restrict__ rows, const int* __restrict__ cols,
                                                       double* dpart) {
  __shared__ double red[256];
  const int b = blockIdx.y;
  const int64_t nc = cols[b], n = (int64_t)rows[b] * nc;
  T* Mb = M + (int64_t)b * sm;
  const T* Db = D + (int64_t)b * sd;
  double s = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) {
    const int64_t i = e / nc, j = e % nc;
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      const T d = Db[i * ldd + j + p * psd];
      Mb[i * ldm + j + p * psm] += d;
      s += (double)d * (double)d;
    }
  }
  s = block_sum_256(s, red);
  if (threadIdx.x == 0) dpart[(int64_t)b * CORE_PARTS + blockIdx.x] = s;
}

hipError_t launch_core_correct_batch(const Ctx& c, int count, Slots M, Slots D, const int* rows, const int* cols,
                                     double* dpart) {
  if (count <= 0) return hipSuccess;
  if (M.dt != D.dt) return hipErrorInvalidValue;
  const dim3 grid(CORE_PARTS, (unsigned)count);
  if (M.dt == QCUR_F64)
    hipLaunchKernelGGL(kb_core_correct<double>, grid, dim3(256), 0, c.stream, (double*)M.p, M.ld, M.ps, M.slab,
                       (const double*)D.p, D.ld, D.ps, D.slab, rows, cols, dpart);
  else if (M.dt == QCUR_F32)
    hipLaunchKernelGGL(kb_core_correct<float>, grid, dim3(256), 0, c.stream, (float*)M.p, M.ld, M.ps, M.slab,
                       (const float*)D.p, D.ld, D.ps, D.slab, rows, cols, dpart);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

// Per problem (blockIdx.x = b): ||E_b||^2 from its own residual tile
// partials (as kb_resid_sum reads them) and ||D_b||^2 from dpart; the same
// decision as the single solve's.
__global__ __launch_bounds__(256) void kb_resid_identity(const double* __restrict__ part, int64_t tiles, int64_t gx,
                                                         int tile, const int* __restrict__ dm,
                                                         const int* __restrict__ dn, const double* dpart,
                                                         double gate, double* out, int* skip) {
  __shared__ double red[2][256];  // one array per sum: red[0][0] is read after the first one returns
  const int b = blockIdx.x;
  const int64_t ty = (dm[b] + tile - 1) / tile, tx = (dn[b] + tile - 1) / tile;
  double se = 0.0;
  for (int64_t k = threadIdx.x; k < tiles; k += 256)
    if (k / gx < ty && k % gx < tx) se += part[(int64_t)b * tiles + k];
  se = block_sum_256(se, red[0]);
  double sd = (int)threadIdx.x < CORE_PARTS ? dpart[(int64_t)b * CORE_PARTS + threadIdx.x] : 0.0;
  sd = block_sum_256(sd, red[1]);
  if (threadIdx.x == 0) {
    const bool take = isfinite(se) && isfinite(sd) && sd <= gate * se;
    if (take) out[b] = sqrt(fmax(se - sd, 0.0));
    skip[b] = take ? 1 : 0;
  }
}

hipError_t launch_resid_identity_batch(const Ctx& c, int count, const double* part, int64_t tiles, int64_t gx,
                                       int tile, const int* dm, const int* dn, const double* dpart, double gate,
                                       double* out, int* skip) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(kb_resid_identity, dim3((unsigned)count), dim3(256), 0, c.stream, part, tiles, gx, tile, dm, dn,
                     dpart, gate, out, skip);
  return hipGetLastError();
}

}  // namespace qcur
