// Moore-Penrose inverse of a quaternion matrix in FP64 (the (.)^+ of
// Section 2.1, used for W^+, C^+ and R^+ in Algorithm 1 step 3).
//
// Method: one-sided (Hestenes) Jacobi on quaternion columns.  For a tall Z
// (p x q, p >= q) columns are orthogonalised pairwise by right unitary
// transformations accumulated in V, so that Y = Z V has orthogonal columns
// and sigma_i = ||Y_i||.  For a column pair (a, b) with alpha = a^H a,
// beta = b^H b and the quaternion gamma = a^H b, the column b is first
// multiplied on the right by conj(mu), mu = gamma / |gamma|, which makes the
// pair's inner product the real number |gamma|; an ordinary real Jacobi
// rotation then zeroes it.  Pairs are visited in round-robin (circle
// method) order: each round holds q/2 disjoint pairs that run in parallel.
// Then Z^+ = sum over kept i of V_i Y_i^H / sigma_i^2.
//
// Storage: columns are stored contiguously ("column rows"): Yc[a][k] is
// element k of column a, Vc[a][k] element k of column a of V.
#include <algorithm>

#include "qcur_internal.hpp"

namespace qcur {

__device__ inline void pair_of(int round, int k, int qpad, int& a, int& b) {
  const int m = qpad - 1;
  if (k == 0) {
    a = m;
    b = round;
  } else {
    a = (round + k) % m;
    b = (round - k + m) % m;
  }
}

struct Rot {
  bool rotate;
  double c, s;
  double w0, w1, w2, w3;  // conj(mu)
};

__device__ inline Rot make_rot(double alpha, double beta, double g0, double g1, double g2, double g3, double tol) {
  Rot r;
  const double gn = sqrt(g0 * g0 + g1 * g1 + g2 * g2 + g3 * g3);
  r.rotate = (alpha > 0.0 && beta > 0.0 && gn > tol * sqrt(alpha) * sqrt(beta));
  r.c = 1.0;
  r.s = 0.0;
  r.w0 = 1.0;
  r.w1 = r.w2 = r.w3 = 0.0;
  if (!r.rotate) return r;
  r.w0 = g0 / gn;
  r.w1 = -g1 / gn;
  r.w2 = -g2 / gn;
  r.w3 = -g3 / gn;
  const double zeta = (beta - alpha) / (2.0 * gn);
  double t;
  if (fabs(zeta) > 1e150) {
    t = 0.5 / zeta;
  } else {
    t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
  }
  r.c = 1.0 / sqrt(1.0 + t * t);
  r.s = r.c * t;
  return r;
}

// New (a, b) = (c a - s b w, s a + c b w) elementwise, w = conj(mu).
__device__ inline void apply_rot(const Rot& r, double* pa, double* pb, int64_t ps, int64_t k) {
  const double a0 = pa[k], a1 = pa[k + ps], a2 = pa[k + 2 * ps], a3 = pa[k + 3 * ps];
  const double x0 = pb[k], x1 = pb[k + ps], x2 = pb[k + 2 * ps], x3 = pb[k + 3 * ps];
  // b w (Hamilton product, quaternion on the right)
  const double b0 = x0 * r.w0 - x1 * r.w1 - x2 * r.w2 - x3 * r.w3;
  const double b1 = x0 * r.w1 + x1 * r.w0 + x2 * r.w3 - x3 * r.w2;
  const double b2 = x0 * r.w2 - x1 * r.w3 + x2 * r.w0 + x3 * r.w1;
  const double b3 = x0 * r.w3 + x1 * r.w2 - x2 * r.w1 + x3 * r.w0;
  pa[k] = r.c * a0 - r.s * b0;
  pa[k + ps] = r.c * a1 - r.s * b1;
  pa[k + 2 * ps] = r.c * a2 - r.s * b2;
  pa[k + 3 * ps] = r.c * a3 - r.s * b3;
  pb[k] = r.s * a0 + r.c * b0;
  pb[k + ps] = r.s * a1 + r.c * b1;
  pb[k + 2 * ps] = r.s * a2 + r.c * b2;
  pb[k + 3 * ps] = r.s * a3 + r.c * b3;
}

// Partial dot products over elements k of columns a and b:
// alpha += |a|^2, beta += |b|^2, gamma += conj(a) b.
__device__ inline void acc_dots(const double* pa, const double* pb, int64_t ps, int64_t k, double* d) {
  const double a0 = pa[k], a1 = pa[k + ps], a2 = pa[k + 2 * ps], a3 = pa[k + 3 * ps];
  const double b0 = pb[k], b1 = pb[k + ps], b2 = pb[k + 2 * ps], b3 = pb[k + 3 * ps];
  d[0] += a0 * a0 + a1 * a1 + a2 * a2 + a3 * a3;
  d[1] += b0 * b0 + b1 * b1 + b2 * b2 + b3 * b3;
  d[2] += a0 * b0 + a1 * b1 + a2 * b2 + a3 * b3;
  d[3] += a0 * b1 - a1 * b0 - a2 * b3 + a3 * b2;
  d[4] += a0 * b2 + a1 * b3 - a2 * b0 - a3 * b1;
  d[5] += a0 * b3 - a1 * b2 + a2 * b1 - a3 * b0;
}

// 64-bit DPP move (lanes outside the pattern read 0).
template <int CTRL, int ROWS>
__device__ inline double dpp_d(double v) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)u, CTRL, ROWS, 0xf, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(u >> 32), CTRL, ROWS, 0xf, true);
  return __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

// Sum over the 64 lanes of a wave (all lanes active), the same value in
// every lane: scans within rows of 16 by row shifts, row totals carried by
// the row broadcasts, the total read from lane 63.
__device__ inline double wsum(double v) {
  v += dpp_d<0x111, 0xf>(v);  // row_shr:1
  v += dpp_d<0x112, 0xf>(v);  // row_shr:2
  v += dpp_d<0x114, 0xf>(v);  // row_shr:4
  v += dpp_d<0x118, 0xf>(v);  // row_shr:8
  v += dpp_d<0x142, 0xa>(v);  // row_bcast:15
  v += dpp_d<0x143, 0xc>(v);  // row_bcast:31
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = __builtin_amdgcn_readlane((int)(uint32_t)u, 63);
  const uint32_t hi = __builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), 63);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// Pairs of negligible columns.  Any column of Y = Z V has norm at most
// sigma_max(Z), so the largest squared column norm seen so far bounds
// sigma_max^2 from below.  A pair whose squared norms are both at most
// drop2 * that bound is not rotated.  When the sweeps stop, those columns
// D hold a block Y_D orthogonal to all other columns; if ||Y_D||_F <=
// rtol sigma_max / 2 its singular values fall below the truncation
// threshold rtol sigma_max and the kept singular triplets are those of the
// full SVD.  The caller takes drop2 = rtol^2 / 4 and checks that sum over D
// afterwards (k_deflation_check), else sweeps again with drop2 =
// rtol^2 / (4 q), for which the bound holds whatever D is.  Such pairs only
// slow convergence (columns of rounding noise of a rank-deficient Z).
//
// The bound is a running maximum kept in two slots that alternate by
// round: round t reads slot t % 2, which no workgroup of that launch
// writes, so every decision of the round uses the same value whatever the
// order in which its workgroups run (run-to-run identical results), and
// raises slot (t + 1) % 2 to the largest norm it sees (t counts the round
// launches of the whole factorisation, across sweeps) (atomicMax on the bit
// pattern: positive doubles order like their bits), workgroup 0 also
// carrying the value it read, so that slot holds the running maximum for
// round t + 1.
__device__ inline bool negligible_pair(double alpha, double beta, double drop2, const double* cmax_rd,
                                       double* cmax_wr, bool carry) {
  const double seen = *cmax_rd;
  const double m = alpha > beta ? alpha : beta;
  const double up = carry && seen > m ? seen : m;
  atomicMax((unsigned long long*)cmax_wr, (unsigned long long)__double_as_longlong(up));
  const double t = drop2 * (m > seen ? m : seen);
  return alpha <= t && beta <= t;
}

// One round of the circle schedule: workgroup k rotates pair k.
__global__ __launch_bounds__(256) void k_jacobi_round(double* __restrict__ Y, int64_t p, int64_t q,
                                                      double* __restrict__ V, int qpad, int round, double tol,
                                                      unsigned* rotated, double drop2, double* cmax, int slot) {
  __shared__ double red[4][6];
  __shared__ Rot rot;
  int a, b;
  pair_of(round, blockIdx.x, qpad, a, b);
  if (a >= q || b >= q) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t psy = q * p, psv = q * q;
  double* ya = Y + (int64_t)a * p;
  double* yb = Y + (int64_t)b * p;
  double d[6] = {0, 0, 0, 0, 0, 0};
  for (int64_t k = tid; k < p; k += 256) acc_dots(ya, yb, psy, k, d);
#pragma unroll
  for (int x = 0; x < 6; ++x) d[x] = wsum(d[x]);
  if (lane == 0)
    for (int x = 0; x < 6; ++x) red[wave][x] = d[x];
  __syncthreads();
  if (tid == 0) {
    double s[6];
    for (int x = 0; x < 6; ++x) s[x] = ((red[0][x] + red[1][x]) + red[2][x]) + red[3][x];
    rot = make_rot(s[0], s[1], s[2], s[3], s[4], s[5], tol);
    if (negligible_pair(s[0], s[1], drop2, cmax + slot, cmax + (slot ^ 1), blockIdx.x == 0))
      rot.rotate = false;
    if (rot.rotate) atomicOr(rotated, 1u);
  }
  __syncthreads();
  const Rot r = rot;
  if (!r.rotate) return;
  for (int64_t k = tid; k < p; k += 256) apply_rot(r, ya, yb, psy, k);
  double* va = V + (int64_t)a * q;
  double* vb = V + (int64_t)b * q;
  for (int64_t k = tid; k < q; k += 256) apply_rot(r, va, vb, psv, k);
}

// After deflated sweeps: bad = 1 unless the columns with ||y||^2 <= drop2 *
// max ||y||^2 have sum ||y||^2 <= (rtol^2 / 4) max ||y||^2.
__global__ __launch_bounds__(1024) void k_deflation_check(const double* __restrict__ Y, int64_t p, int64_t q,
                                                          double drop2, double rtol2q, unsigned* bad) {
  __shared__ double part[2][16];
  __shared__ double mx;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t psy = q * p;
  for (int pass = 0; pass < 2; ++pass) {
    double acc = 0.0;
    for (int64_t k = wave; k < q; k += 16) {
      const double* y = Y + k * p;
      double s = 0.0;
      for (int64_t i = lane; i < p; i += 64) {
        const double a0 = y[i], a1 = y[i + psy], a2 = y[i + 2 * psy], a3 = y[i + 3 * psy];
        s += a0 * a0 + a1 * a1 + a2 * a2 + a3 * a3;
      }
      s = wsum(s);
      if (pass == 0) acc = fmax(acc, s);
      else if (s <= drop2 * mx) acc += s;
    }
    if (lane == 0) part[pass][wave] = acc;
    __syncthreads();
    if (tid == 0) {
      double r = 0.0;
      for (int w = 0; w < 16; ++w) r = pass == 0 ? fmax(r, part[0][w]) : r + part[1][w];
      if (pass == 0) mx = r;
      else *bad = (r <= rtol2q * mx) ? 0u : 1u;
    }
    __syncthreads();
  }
}

hipError_t launch_deflation_check(const Ctx& c, const double* Y, int64_t p, int64_t q, double drop2, double rtol2q,
                                  unsigned* bad) {
  hipLaunchKernelGGL(k_deflation_check, dim3(1), dim3(1024), 0, c.stream, Y, p, q, drop2, rtol2q, bad);
  return hipGetLastError();
}

hipError_t launch_jacobi_round(const Ctx& c, double* Y, int64_t p, int64_t q, double* V, int64_t qpad, int round,
                               double tol, unsigned* rotated, double drop2, double* cmax, int slot) {
  hipLaunchKernelGGL(k_jacobi_round, dim3((unsigned)(qpad / 2)), dim3(256), 0, c.stream, Y, p, q, V, (int)qpad,
                     round, tol, rotated, drop2, cmax, slot & 1);
  return hipGetLastError();
}

// dst[e] = src[e], e < n (global to LDS), eight loads in flight per thread.
__device__ inline void copy_in8(double* __restrict__ dst, const double* __restrict__ src, int64_t n, int tid,
                                int nthr) {
  for (int64_t e0 = tid; e0 < n; e0 += 8 * (int64_t)nthr) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int64_t e = e0 + (int64_t)u * nthr;
      v[u] = e < n ? src[e] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int64_t e = e0 + (int64_t)u * nthr;
      if (e < n) dst[e] = v[u];
    }
  }
}

// Whole Jacobi SVD in one workgroup (16 waves, one pair per wave at a time);
// Y and V are staged in LDS when they fit.
static constexpr size_t SMALL_LDS = 150 * 1024;

bool jacobi_small_fits(int64_t p, int64_t q) {
  return q <= 128 && (size_t)(q * p + q * q) * 4 * sizeof(double) <= SMALL_LDS;
}

__global__ __launch_bounds__(1024) void k_jacobi_small(double* __restrict__ Yg, int64_t p, int64_t q,
                                                       double* __restrict__ Vg, double tol, int max_sweeps,
                                                       unsigned* rotated) {
  extern __shared__ double lds[];
  __shared__ int any;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t psy = q * p, psv = q * q;
  double* Y = lds;
  double* V = lds + 4 * psy;
  copy_in8(Y, Yg, 4 * psy, tid, 1024);
  copy_in8(V, Vg, 4 * psv, tid, 1024);
  const int qpad = (int)((q + 1) / 2 * 2);
  int sweep = 0;
  for (; sweep < max_sweeps; ++sweep) {
    if (tid == 0) any = 0;
    __syncthreads();
    for (int round = 0; round < qpad - 1; ++round) {
      for (int k = wave; k < qpad / 2; k += 16) {
        int a, b;
        pair_of(round, k, qpad, a, b);
        if (a >= q || b >= q) continue;
        double* ya = Y + (int64_t)a * p;
        double* yb = Y + (int64_t)b * p;
        double d[6] = {0, 0, 0, 0, 0, 0};
        for (int64_t k2 = lane; k2 < p; k2 += 64) acc_dots(ya, yb, psy, k2, d);
#pragma unroll
        for (int x = 0; x < 6; ++x) d[x] = wsum(d[x]);
        const Rot r = make_rot(d[0], d[1], d[2], d[3], d[4], d[5], tol);
        if (!r.rotate) continue;
        if (lane == 0) any = 1;
        for (int64_t k2 = lane; k2 < p; k2 += 64) apply_rot(r, ya, yb, psy, k2);
        double* va = V + (int64_t)a * q;
        double* vb = V + (int64_t)b * q;
        for (int64_t k2 = lane; k2 < q; k2 += 64) apply_rot(r, va, vb, psv, k2);
      }
      __syncthreads();
    }
    const int again = any;
    __syncthreads();
    if (!again) break;
  }
  if (tid == 0) rotated[0] = (sweep >= max_sweeps) ? 1u : 0u;
  for (int64_t e = tid; e < 4 * psy; e += 1024) Yg[e] = Y[e];
  for (int64_t e = tid; e < 4 * psv; e += 1024) Vg[e] = V[e];
}

hipError_t launch_jacobi_small(const Ctx& c, double* Y, int64_t p, int64_t q, double* V, double tol, int max_sweeps,
                               unsigned* rotated) {
  const size_t lds = (size_t)(q * p + q * q) * 4 * sizeof(double);
  hipError_t e = hipFuncSetAttribute((const void*)k_jacobi_small, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)SMALL_LDS);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_jacobi_small, dim3(1), dim3(1024), lds, c.stream, Y, p, q, V, tol, max_sweeps, rotated);
  return hipGetLastError();
}

// sigma_i^2 = ||Yc row i||^2, one workgroup per row.
__global__ __launch_bounds__(256) void k_row_norm2(const double* __restrict__ Y, int64_t p, int64_t q,
                                                   double* __restrict__ sig2) {
  __shared__ double red[4];
  const int tid = threadIdx.x;
  const int64_t i = blockIdx.x;
  const int64_t ps = q * p;
  const double* y = Y + i * p;
  double s = 0.0;
  for (int64_t k = tid; k < p; k += 256) {
    const double a0 = y[k], a1 = y[k + ps], a2 = y[k + 2 * ps], a3 = y[k + 3 * ps];
    s += a0 * a0 + a1 * a1 + a2 * a2 + a3 * a3;
  }
  s = wsum(s);
  if ((tid & 63) == 0) red[tid >> 6] = s;
  __syncthreads();
  if (tid == 0) sig2[i] = ((red[0] + red[1]) + red[2]) + red[3];
}

// Keep sigma_i > rtol * sigma_max, at most max_rank of the largest (ties by
// index); d_i = 1 / sigma_i^2 for kept columns, 0 otherwise.
__global__ __launch_bounds__(1024) void k_pinv_select(const double* __restrict__ sig2, int64_t q, double rtol,
                                                      int64_t max_rank, double* __restrict__ dsc,
                                                      int64_t* rank_out) {
  __shared__ double red[1024];
  __shared__ int64_t cnt[1024];
  const int tid = threadIdx.x;
  double mx = 0.0;
  for (int64_t i = tid; i < q; i += 1024) mx = fmax(mx, sig2[i]);
  red[tid] = mx;
  __syncthreads();
  for (int w = 512; w >= 1; w >>= 1) {
    if (tid < w) red[tid] = fmax(red[tid], red[tid + w]);
    __syncthreads();
  }
  const double smax = sqrt(red[0]);
  const double thr = rtol * smax;
  int64_t kept = 0;
  for (int64_t i = tid; i < q; i += 1024) {
    const double si2 = sig2[i];
    const double si = sqrt(si2);
    bool keep = smax > 0.0 && si > thr;
    if (keep && max_rank > 0) {
      int64_t rk = 0;
      for (int64_t j = 0; j < q; ++j) {
        const double sj2 = sig2[j];
        rk += (sj2 > si2 || (sj2 == si2 && j < i)) ? 1 : 0;
      }
      keep = rk < max_rank;
    }
    dsc[i] = keep ? 1.0 / si2 : 0.0;
    kept += keep ? 1 : 0;
  }
  cnt[tid] = kept;
  __syncthreads();
  for (int w = 512; w >= 1; w >>= 1) {
    if (tid < w) cnt[tid] += cnt[tid + w];
    __syncthreads();
  }
  if (tid == 0 && rank_out) rank_out[0] = cnt[0];
}

// Yc[i][:] <- conj(d_i Yc[i][:]) and Vc <- conj(Vc), one workgroup per row.
__global__ __launch_bounds__(256) void k_pinv_apply(double* __restrict__ Y, int64_t p, int64_t q,
                                                    double* __restrict__ V, const double* __restrict__ dsc) {
  const int64_t i = blockIdx.x;
  const double d = dsc[i];
  const int64_t psy = q * p, psv = q * q;
  double* y = Y + i * p;
  for (int64_t k = threadIdx.x; k < p; k += 256) {
    y[k] = d * y[k];
    y[k + psy] = -d * y[k + psy];
    y[k + 2 * psy] = -d * y[k + 2 * psy];
    y[k + 3 * psy] = -d * y[k + 3 * psy];
  }
  double* v = V + i * q;
  for (int64_t k = threadIdx.x; k < q; k += 256) {
    v[k + psv] = -v[k + psv];
    v[k + 2 * psv] = -v[k + 2 * psv];
    v[k + 3 * psv] = -v[k + 3 * psv];
  }
}

hipError_t launch_pinv_scale(const Ctx& c, double* Y, int64_t p, int64_t q, double rtol, int64_t max_rank,
                             int64_t* rank_out, double* sig) {
  // sig holds 2q doubles: sigma^2 then the scale factors
  hipLaunchKernelGGL(k_row_norm2, dim3((unsigned)q), dim3(256), 0, c.stream, Y, p, q, sig);
  hipLaunchKernelGGL(k_pinv_select, dim3(1), dim3(1024), 0, c.stream, sig, q, rtol, max_rank, sig + q, rank_out);
  return hipGetLastError();
}

hipError_t launch_pinv_apply(const Ctx& c, double* Y, int64_t p, int64_t q, double* V, const double* dsc) {
  hipLaunchKernelGGL(k_pinv_apply, dim3((unsigned)q), dim3(256), 0, c.stream, Y, p, q, V, dsc);
  return hipGetLastError();
}

// ---- thin QSVD output ---------------------------------------------------
// After the sweeps the columns Y_i of Y = Z V are orthogonal with
// sigma_i = ||Y_i||.  Rank of column i in descending order (ties by index).
__global__ __launch_bounds__(1024) void k_svd_rank(const double* __restrict__ sig2, int64_t q,
                                                   int32_t* __restrict__ rank, double* __restrict__ s) {
  for (int64_t i = threadIdx.x; i < q; i += 1024) {
    const double v = sig2[i];
    int64_t r = 0;
    for (int64_t j = 0; j < q; ++j) {
      const double w = sig2[j];
      r += (w > v || (w == v && j < i)) ? 1 : 0;
    }
    rank[i] = (int32_t)r;
    s[r] = sqrt(v);
  }
}

// Column i goes to output column rank[i]: Y_i / sigma_i and V_i into the
// left / right factors (tall: U <- Y, Vout <- V; wide: U <- V, Vout <- Y).
// Columns with sigma_i = 0 give zero vectors.  One workgroup per column.
__global__ __launch_bounds__(256) void k_svd_vectors(const double* __restrict__ Y, int64_t pp, int64_t qq,
                                                     const double* __restrict__ V, const double* __restrict__ sig2,
                                                     const int32_t* __restrict__ rank, int tall, double* U,
                                                     int64_t uld, int64_t ups, double* Vo, int64_t vld,
                                                     int64_t vps) {
  const int64_t i = blockIdx.x;
  const int64_t r = rank[i];
  const double sg = sqrt(sig2[i]);
  const double inv = sg > 0.0 ? 1.0 / sg : 0.0;
  const int64_t psy = qq * pp, psv = qq * qq;
  double* Yo = tall ? U : Vo;  // destination of Y_i / sigma_i (pp rows)
  const int64_t yld = tall ? uld : vld, yps = tall ? ups : vps;
  double* Vd = tall ? Vo : U;  // destination of V_i (qq rows)
  const int64_t dld = tall ? vld : uld, dps = tall ? vps : ups;
  if (Yo) {
    for (int64_t k = threadIdx.x; k < pp; k += 256) {
#pragma unroll
      for (int c = 0; c < 4; ++c) Yo[k * yld + r + c * yps] = Y[c * psy + i * pp + k] * inv;
    }
  }
  if (Vd) {
    for (int64_t k = threadIdx.x; k < qq; k += 256) {
#pragma unroll
      for (int c = 0; c < 4; ++c) Vd[k * dld + r + c * dps] = V[c * psv + i * qq + k];
    }
  }
}

hipError_t launch_svd_out(const Ctx& c, const double* Y, int64_t pp, int64_t qq, const double* V, double* sig2,
                          int32_t* rank, double* s, bool tall, double* U, int64_t uld, int64_t ups, double* Vo,
                          int64_t vld, int64_t vps) {
  hipLaunchKernelGGL(k_row_norm2, dim3((unsigned)qq), dim3(256), 0, c.stream, Y, pp, qq, sig2);
  hipLaunchKernelGGL(k_svd_rank, dim3(1), dim3(1024), 0, c.stream, sig2, qq, rank, s);
  hipLaunchKernelGGL(k_svd_vectors, dim3((unsigned)qq), dim3(256), 0, c.stream, Y, pp, qq, V, sig2, rank,
                     tall ? 1 : 0, U, uld, ups, Vo, vld, vps);
  return hipGetLastError();
}

}  // namespace qcur

namespace qcur {

// ---------------------------------------------------------------------------
// Batched fallback.  For every problem t whose CholeskyQR certificate failed
// (ok[t] == 0), one workgroup runs the whole one-sided Jacobi SVD above on a
// working copy in global memory and writes the factors of the orthonormal
// form Z^+ = P^H Q^H used by the batched core: with s_k = 1/sigma_k for kept
// singular values and 0 otherwise, Q[:, k] = Y_k s_k (orthonormal or zero
// columns) and P[k][a] = conj(V_{a,k}) s_k, so that P^H Q^H = V D Y^H.
// Problem t < count is C_b (m_b x c_b, Z = C_b); t >= count is R_b
// (r_b x n_b), handled as Z = R_b^H.  With jb.Rz NULL both halves are read
// from the tall slots jb.Cz (slot t holds Z_t itself, R_b^H for t >= count).
__global__ __launch_bounds__(1024) void kb_jacobi_pinv(JacobiBatch jb) {
  const int t = blockIdx.x;
  if (jb.ok[t]) return;  // uniform over the workgroup
  __shared__ int any;
  __shared__ double sig2[JB_MAXQ];
  __shared__ double scl[JB_MAXQ];
  __shared__ double red[1024];
  __shared__ long long cnt[1024];
  const bool isC = t < jb.count;
  const int b = isC ? t : t - jb.count;
  const int64_t p = isC ? jb.dm[b] : jb.dn[b];
  const int64_t q = isC ? jb.dc[b] : jb.dr[b];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double* Y = jb.Y + (int64_t)t * jb.yslab;
  double* V = jb.V + (int64_t)t * jb.vslab;
  const int64_t psy = q * p, psv = q * q;
  // Y[a][i] = Z[i][a]
  for (int64_t e = tid; e < q * p; e += 1024) {
    const int64_t a = e / p, i = e % p;
    if (isC || !jb.Rz) {
      const double* src = jb.Cz + (int64_t)(jb.Rz ? b : t) * jb.cslab + i * jb.cld + a;
#pragma unroll
      for (int k = 0; k < 4; ++k) Y[e + k * psy] = src[k * jb.cps];
    } else {
      const double* src = jb.Rz + (int64_t)b * jb.rslab + a * jb.rld + i;
      Y[e] = src[0];
#pragma unroll
      for (int k = 1; k < 4; ++k) Y[e + k * psy] = -src[k * jb.rps];
    }
  }
  for (int64_t e = tid; e < q * q; e += 1024) {
    const int64_t a = e / q, k = e % q;
    V[e] = (a == k) ? 1.0 : 0.0;
    V[e + psv] = V[e + 2 * psv] = V[e + 3 * psv] = 0.0;
  }
  __syncthreads();
  const double tol = sqrt((double)p) * 0x1p-53;
  const int qpad = (int)((q + 1) / 2 * 2);
  for (int sweep = 0; sweep < jb.max_sweeps; ++sweep) {
    if (tid == 0) any = 0;
    __syncthreads();
    for (int round = 0; round < qpad - 1; ++round) {
      for (int k = wave; k < qpad / 2; k += 16) {
        int a, c;
        pair_of(round, k, qpad, a, c);
        if (a >= q || c >= q) continue;
        double* ya = Y + (int64_t)a * p;
        double* yb = Y + (int64_t)c * p;
        double d[6] = {0, 0, 0, 0, 0, 0};
        for (int64_t k2 = lane; k2 < p; k2 += 64) acc_dots(ya, yb, psy, k2, d);
#pragma unroll
        for (int x = 0; x < 6; ++x) d[x] = wsum(d[x]);
        const Rot r = make_rot(d[0], d[1], d[2], d[3], d[4], d[5], tol);
        if (!r.rotate) continue;
        if (lane == 0) any = 1;
        for (int64_t k2 = lane; k2 < p; k2 += 64) apply_rot(r, ya, yb, psy, k2);
        double* va = V + (int64_t)a * q;
        double* vb = V + (int64_t)c * q;
        for (int64_t k2 = lane; k2 < q; k2 += 64) apply_rot(r, va, vb, psv, k2);
      }
      __syncthreads();
    }
    const int again = any;
    __syncthreads();
    if (!again) break;
  }
  // sigma_k^2 = ||Y_k||^2, one wave per column
  for (int64_t k = wave; k < q; k += 16) {
    const double* y = Y + k * p;
    double s = 0.0;
    for (int64_t i = lane; i < p; i += 64) {
      const double a0 = y[i], a1 = y[i + psy], a2 = y[i + 2 * psy], a3 = y[i + 3 * psy];
      s += a0 * a0 + a1 * a1 + a2 * a2 + a3 * a3;
    }
    s = wsum(s);
    if (lane == 0) sig2[k] = s;
  }
  __syncthreads();
  // keep sigma_k > rtol * sigma_max, at most max_rank of the largest (ties by index)
  double mx = 0.0;
  for (int64_t k = tid; k < q; k += 1024) mx = fmax(mx, sig2[k]);
  red[tid] = mx;
  __syncthreads();
  for (int w = 512; w >= 1; w >>= 1) {
    if (tid < w) red[tid] = fmax(red[tid], red[tid + w]);
    __syncthreads();
  }
  const double smax = sqrt(red[0]);
  const double rt = jb.rtol < 0.0 ? (double)(p > q ? p : q) * 0x1p-52 : jb.rtol;
  long long kept = 0;
  for (int64_t k = tid; k < q; k += 1024) {
    const double s2 = sig2[k];
    bool keep = smax > 0.0 && sqrt(s2) > rt * smax;
    if (keep && jb.max_rank > 0) {
      int64_t rk = 0;
      for (int64_t j = 0; j < q; ++j) rk += (sig2[j] > s2 || (sig2[j] == s2 && j < k)) ? 1 : 0;
      keep = rk < jb.max_rank;
    }
    scl[k] = keep ? 1.0 / sqrt(s2) : 0.0;
    kept += keep ? 1 : 0;
  }
  cnt[tid] = kept;
  __syncthreads();
  for (int w = 512; w >= 1; w >>= 1) {
    if (tid < w) cnt[tid] += cnt[tid + w];
    __syncthreads();
  }
  if (tid == 0 && jb.rank_out) jb.rank_out[isC ? 2 * b : 2 * b + 1] = cnt[0];
  // Q[i][k] = Y_k[i] s_k
  double* Qo = jb.Q + (int64_t)t * jb.qslab;
  for (int64_t e = tid; e < q * p; e += 1024) {
    const int64_t k = e / p, i = e % p;
    const double s = scl[k];
#pragma unroll
    for (int c = 0; c < 4; ++c) Qo[i * jb.qld + k + c * jb.qps] = Y[e + c * psy] * s;
  }
  // P[k][a] = conj(V_{a,k}) s_k,  V_{a,k} = Vc[k][a]
  double* Po = jb.P + (int64_t)t * jb.pslab;
  for (int64_t e = tid; e < q * q; e += 1024) {
    const int64_t k = e / q, a = e % q;
    const double s = scl[k];
    Po[k * jb.pld + a] = V[e] * s;
#pragma unroll
    for (int c = 1; c < 4; ++c) Po[k * jb.pld + a + c * jb.pps] = -V[e + c * psv] * s;
  }
}

hipError_t launch_jacobi_pinv_batch(const Ctx& c, const JacobiBatch& jb, int count2) {
  if (count2 <= 0) return hipSuccess;
  hipLaunchKernelGGL(kb_jacobi_pinv, dim3((unsigned)count2), dim3(1024), 0, c.stream, jb);
  return hipGetLastError();
}

}  // namespace qcur

namespace qcur {

// Orthonormal form of a Jacobi pseudoinverse: with s_k = sqrt(dsc_k)
// (1/sigma_k for kept columns, else 0), Q[i][k] = Y_k[i] s_k and
// P[k][a] = conj(V_{a,k}) s_k = conj(Vc[k][a]) s_k, so Z^+ = P^H Q^H.
__global__ __launch_bounds__(256) void k_pinv_qp(const double* __restrict__ Y, int64_t p, int64_t q,
                                                 const double* __restrict__ V, const double* __restrict__ dsc,
                                                 double* __restrict__ Qo, int64_t qld, int64_t qps,
                                                 double* __restrict__ Po, int64_t pld, int64_t pps) {
  const int64_t psy = q * p, psv = q * q;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < psy + psv; e += (int64_t)gridDim.x * 256) {
    if (e < psy) {
      const int64_t k = e / p, i = e % p;
      const double s = sqrt(dsc[k]);
#pragma unroll
      for (int c = 0; c < 4; ++c) Qo[i * qld + k + c * qps] = Y[e + c * psy] * s;
    } else {
      const int64_t f = e - psy;
      const int64_t k = f / q, a = f % q;
      const double s = sqrt(dsc[k]);
      Po[k * pld + a] = V[f] * s;
#pragma unroll
      for (int c = 1; c < 4; ++c) Po[k * pld + a + c * pps] = -V[f + c * psv] * s;
    }
  }
}

hipError_t launch_pinv_qp(const Ctx& c, const double* Y, int64_t p, int64_t q, const double* V, const double* dsc,
                          QView Q, QView P) {
  const int64_t total = q * p + q * q;
  if (total <= 0) return hipSuccess;
  const int64_t blocks = std::min<int64_t>((total + 255) / 256, 4096);
  hipLaunchKernelGGL(k_pinv_qp, dim3((unsigned)blocks), dim3(256), 0, c.stream, Y, p, q, V, dsc, (double*)Q.p, Q.ld,
                     Q.ps, (double*)P.p, P.ld, P.ps);
  return hipGetLastError();
}

}  // namespace qcur
