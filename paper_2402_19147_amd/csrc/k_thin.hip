// Thin quaternion products in FP64 or FP32: D = alpha A^H B + beta D with
// both operands stored K-major (A: K x M, B: K x N, four planes each), a
// small output and a long K.  These are the Gram matrices of the tall
// factors in CholeskyQR (Section 2.1 notation: G = Z^H Z) and the core
// product Q_C^H T of the least-squares core.
//
// The tiled product stages 32 x 32 tiles through LDS with a barrier per K
// slice; on a 200 x 200 output that leaves one or two waves per SIMD, which
// cannot cover the store, barrier and fragment-read phases.  Here one wave
// owns a 16 x 16 block of D and a range of K and loads its MFMA fragments
// straight from global memory: at each k the sixteen lanes of a row group
// read sixteen consecutive columns of one row (one 128-byte segment per
// plane).  Two register groups of four k-steps alternate: the loads of one
// group are issued (and fenced, so that the scheduler cannot sink them to
// their use) before the MFMAs of the other, so a group's loads have the
// other group's 64 MFMAs to arrive.  The four waves of a workgroup take
// consecutive quarters of the workgroup's K range and are added through LDS
// in a fixed order; more than one split of K gives partials that a
// fixed-order reduction adds.  With the lower output only (square D) just
// the blocks on and below the diagonal are computed; partials of the blocks
// above it are written as zeros.
//
// conj(a) b in the Hamilton product (Section 2.2), with v = a and w = -a in
// planes 1..3:
//   plane 0: v0 b0 + v1 b1 + v2 b2 + v3 b3
//   plane 1: w1 b0 + v0 b1 + v3 b2 + w2 b3
//   plane 2: w2 b0 + w3 b1 + v0 b2 + v1 b3
//   plane 3: w3 b0 + v2 b1 + w1 b2 + v0 b3
#include <algorithm>

#include "qcur_internal.hpp"

namespace qcur {
namespace {

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int PF = 4;  // k-steps per register group

struct ThinArgs {
  const void* A;
  int64_t lda, psa, sA;
  const void* B;
  int64_t ldb, psb, sB;
  void* D;  // D itself, or the partial slabs when splits > 1
  int64_t ldd, psd, sD;
  int64_t M, N, K;  // grid extents (the largest problem of a batch)
  double alpha, beta;
  int splits;
  // batches of uneven problems: problem b's own M, N, K (NULL: the extents)
  const int *bM, *bN, *bK;
};

// per dtype: element, accumulator vector, MFMA 16x16x4 and the row of
// output element r of lane l (FP64 rows interleave, FP32 rows are blocked)
template <typename E> struct TT;
template <> struct TT<double> {
  typedef f64x4 V;
  static __device__ inline V mfma(double a, double b, V c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ inline int out_row(int lane, int r) { return (lane >> 4) + 4 * r; }
};
template <> struct TT<float> {
  typedef f32x4 V;
  static __device__ inline V mfma(float a, float b, V c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
  static __device__ inline int out_row(int lane, int r) { return (lane >> 4) * 4 + r; }
};

// Workgroups go to the eight XCDs round-robin by linear id and each XCD has
// its own L2.  The linear id is remapped so that every XCD takes one
// contiguous range of (split, problem, block) with blocks fastest: an XCD
// then works on one K range of one problem at a time, whose rows fit its L2,
// instead of on every K range at once.
constexpr int NXCD = 8;

template <typename E, bool TRI>
__global__ __launch_bounds__(256) void k_thin_hn(ThinArgs g, int nblocks, int batch, int nbj) {
  typedef TT<E> X;
  typedef typename X::V V;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t total = gridDim.x, id = blockIdx.x;
  const int64_t x = id % NXCD, per = total / NXCD, rem = total % NXCD;
  const int64_t logical = x * per + (x < rem ? x : rem) + id / NXCD;
  const int t = (int)(logical % nblocks);
  const int b = (int)((logical / nblocks) % batch), split = (int)(logical / ((int64_t)nblocks * batch));
  const int splits = g.splits;
  int bi, bj;
  if (TRI) {  // t = bi (bi + 1) / 2 + bj with bj <= bi
    bi = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
    while ((bi + 1) * (bi + 2) / 2 <= t) ++bi;
    while (bi * (bi + 1) / 2 > t) --bi;
    bj = t - bi * (bi + 1) / 2;
  } else {
    bi = t / nbj;
    bj = t % nbj;
  }
  const int64_t M = g.bM ? (int64_t)g.bM[b] : g.M, N = g.bN ? (int64_t)g.bN[b] : g.N;
  const int64_t K = g.bK ? (int64_t)g.bK[b] : g.K;
  const int64_t i0 = (int64_t)bi * 16, j0 = (int64_t)bj * 16;
  // a block outside its problem (uniform over the workgroup; only with
  // per-problem sizes, where the K split is not used) stores nothing
  if (i0 >= M || j0 >= N) return;
  // this wave's k-steps (four rows of K each): a quarter of the split's share
  const int64_t ksteps = (K + 3) / 4;
  const int64_t per_split = (ksteps + splits - 1) / splits;
  const int64_t per_wave = (per_split + 3) / 4;
  const int64_t s0 = split * per_split + wave * per_wave;
  const int64_t s1 = std::min(std::min(s0 + per_wave, (int64_t)(split + 1) * per_split), ksteps);
  const int64_t n = s1 > s0 ? s1 - s0 : 0;
  // lane l supplies A^H[i0 + l % 16][k] and B[k][j0 + l % 16] at k = 4 s + l / 16.
  // Columns past the matrix and rows past K are read clamped (in range):
  // the former only reach rows and columns of D that are not stored, the
  // latter are zeroed before use.
  const int kl = lane >> 4;
  const E* __restrict__ pa = (const E*)g.A + (int64_t)b * g.sA + std::min(i0 + (lane & 15), M - 1);
  const E* __restrict__ pb = (const E*)g.B + (int64_t)b * g.sB + std::min(j0 + (lane & 15), N - 1);
  E ra[2][PF][4], rb[2][PF][4];
  auto load_group = [&](int buf, int64_t sbase) {
#pragma unroll
    for (int p = 0; p < PF; ++p) {
      const int64_t k = std::min(4 * (sbase + p) + kl, K - 1);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        ra[buf][p][q] = pa[k * g.lda + q * g.psa];
        rb[buf][p][q] = pb[k * g.ldb + q * g.psb];
      }
    }
    asm volatile("" ::: "memory");
  };
  V acc[4];
#pragma unroll
  for (int p = 0; p < 4; ++p) acc[p] = (V){0, 0, 0, 0};
  auto compute_group = [&](int buf, int64_t base) {
#pragma unroll
    for (int p = 0; p < PF; ++p) {
      // steps past this wave's range and rows past K contribute zero
      const bool ok = base + p < n && 4 * (s0 + base + p) + kl < K;
      const E v0 = ok ? ra[buf][p][0] : (E)0, v1 = ok ? ra[buf][p][1] : (E)0;
      const E v2 = ok ? ra[buf][p][2] : (E)0, v3 = ok ? ra[buf][p][3] : (E)0;
      const E w1 = -v1, w2 = -v2, w3 = -v3;
      const E b0 = rb[buf][p][0], b1 = rb[buf][p][1], b2 = rb[buf][p][2], b3 = rb[buf][p][3];
      acc[0] = X::mfma(v0, b0, acc[0]);
      acc[1] = X::mfma(w1, b0, acc[1]);
      acc[2] = X::mfma(w2, b0, acc[2]);
      acc[3] = X::mfma(w3, b0, acc[3]);
      acc[0] = X::mfma(v1, b1, acc[0]);
      acc[1] = X::mfma(v0, b1, acc[1]);
      acc[2] = X::mfma(w3, b1, acc[2]);
      acc[3] = X::mfma(v2, b1, acc[3]);
      acc[0] = X::mfma(v2, b2, acc[0]);
      acc[1] = X::mfma(v3, b2, acc[1]);
      acc[2] = X::mfma(v0, b2, acc[2]);
      acc[3] = X::mfma(w1, b2, acc[3]);
      acc[0] = X::mfma(v3, b3, acc[0]);
      acc[1] = X::mfma(w2, b3, acc[1]);
      acc[2] = X::mfma(v1, b3, acc[2]);
      acc[3] = X::mfma(v0, b3, acc[3]);
    }
  };
  load_group(0, s0);
  for (int64_t base = 0; base < n; base += 2 * PF) {
    load_group(1, s0 + base + PF);
    compute_group(0, base);
    load_group(0, s0 + base + 2 * PF);
    compute_group(1, base + PF);
  }
  __shared__ V red[3][4][64];
  if (wave > 0) {
#pragma unroll
    for (int p = 0; p < 4; ++p) red[wave - 1][p][lane] = acc[p];
  }
  __syncthreads();
  if (wave != 0) return;
#pragma unroll
  for (int p = 0; p < 4; ++p) acc[p] = ((acc[p] + red[0][p][lane]) + red[1][p][lane]) + red[2][p][lane];
  // MFMA 16x16 output: lane l holds column l % 16 of four rows
  const int64_t j = j0 + (lane & 15);
  if (splits == 1) {
    E* D = (E*)g.D + (int64_t)b * g.sD;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t i = i0 + X::out_row(lane, r);
      if (i < M && j < N) {
#pragma unroll
        for (int p = 0; p < 4; ++p) {
          const int64_t o = i * g.ldd + j + p * g.psd;
          double v = g.alpha * (double)acc[p][r];
          if (g.beta != 0.0) v += g.beta * (double)D[o];
          D[o] = (E)v;
        }
      }
    }
  } else {
    const int64_t MN = M * N;
    E* P = (E*)g.D + ((int64_t)b * splits + split) * 4 * MN;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t i = i0 + X::out_row(lane, r);
      if (i < M && j < N) {
#pragma unroll
        for (int p = 0; p < 4; ++p) P[p * MN + i * N + j] = acc[p][r];
      }
      // the mirrored block above the diagonal (rows j0.., columns i0..): zeros
      const int64_t mi = j0 + X::out_row(lane, r), mj = i0 + (lane & 15);
      if (TRI && bj < bi && mi < M && mj < N) {
#pragma unroll
        for (int p = 0; p < 4; ++p) P[p * MN + mi * N + mj] = (E)0;
      }
    }
  }
}

// D = alpha * (sum over the splits, in order, in FP64) + beta * D
template <typename E>
__global__ __launch_bounds__(256) void k_thin_reduce(const E* __restrict__ Pall, int splits, int64_t M, int64_t N,
                                                     double alpha, double beta, E* Dall, int64_t ldd, int64_t psd,
                                                     int64_t sD) {
  const int b = blockIdx.z;
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j >= N) return;
  const int64_t MN = M * N;
  const E* P = Pall + (int64_t)b * splits * 4 * MN;
  E* D = Dall + (int64_t)b * sD;
  for (int64_t i = blockIdx.y; i < M; i += gridDim.y) {
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      double s = 0.0;
      for (int z = 0; z < splits; ++z) s += (double)P[(int64_t)z * 4 * MN + p * MN + i * N + j];
      const int64_t o = i * ldd + j + p * psd;
      double v = alpha * s;
      if (beta != 0.0) v += beta * (double)D[o];
      D[o] = (E)v;
    }
  }
}

// Tall products D = alpha A B^H + beta D in FP64 with both operands
// contiguous in k (A: M x K, B: N x K, row-major) and a short K: the
// orthonormal factors Q = Z P^H of CholeskyQR (P lower triangular, so
// op(B) = P^H is upper triangular and the K range of column block j stops
// at its last column).  One wave owns a 16 x 16 block of D over the whole
// K range; a workgroup holds four row blocks of one column block.  The MFMA
// contraction index is permuted the same way in both operands: in each
// chunk of 16 k, lane group g (lanes 16g .. 16g + 15) takes k = 4g + s at
// MFMA step s, so a lane's fragments for the four steps are four
// consecutive elements of one row of A and of B: one 32-byte run each.
// Two register chunks alternate, the loads of one fenced ahead of the
// MFMAs of the other.
//
// A conj(b) in the Hamilton product (Section 2.2), with n = -a:
//   plane 0: a0 p0 + a1 p1 + a2 p2 + a3 p3
//   plane 1: a1 p0 + n0 p1 + a3 p2 + n2 p3
//   plane 2: a2 p0 + n3 p1 + n0 p2 + a1 p3
//   plane 3: a3 p0 + a2 p1 + n1 p2 + n0 p3
struct TallArgs {
  const double* A;
  int64_t lda, psa, sA;
  const double* B;
  int64_t ldb, psb, sB;
  double* D;
  int64_t ldd, psd, sD;
  int64_t M, N, K;
  double alpha, beta;
  int b_upper;  // op(B) upper triangular: column j meets k <= j only
  // batches of uneven problems: problem b's own M, N, K (NULL: the extents);
  // then K need not be a multiple of 4 (elements at k >= K are zeroed)
  const int *bM, *bN, *bK;
  TallCopy copy;  // optional copy of D in a product dtype (copy.p[0] NULL: none)
};

typedef double f64x2 __attribute__((ext_vector_type(2)));

__global__ __launch_bounds__(256) void k_tall_nh(TallArgs g, int nbi, int nbj) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int t = blockIdx.x;  // (problem, column block, group of four row blocks)
  const int ngi = (nbi + 3) / 4;
  const int b = t / (nbj * ngi), rem = t % (nbj * ngi);
  const int bj = rem / ngi, bi = (rem % ngi) * 4 + wave;
  if (bi >= nbi) return;  // no barrier follows: the wave may leave
  const int64_t M = g.bM ? (int64_t)g.bM[b] : g.M, N = g.bN ? (int64_t)g.bN[b] : g.N;
  const int64_t K = g.bK ? (int64_t)g.bK[b] : g.K;
  const int64_t i0 = (int64_t)bi * 16, j0 = (int64_t)bj * 16;
  if (i0 >= M || j0 >= N || K <= 0) return;  // outside its problem
  const int64_t kend = g.b_upper ? std::min(K, j0 + 16) : K;
  const int64_t nch = (kend + 15) / 16;
  const int r = lane & 15, kg = 4 * (lane >> 4);
  const double* __restrict__ pa = g.A + (int64_t)b * g.sA + std::min(i0 + r, M - 1) * g.lda;
  const double* __restrict__ pb = g.B + (int64_t)b * g.sB + std::min(j0 + r, N - 1) * g.ldb;
  // K is a multiple of 4, so a run starting below K lies inside the row;
  // runs starting at or past K (or past kend) read the row's last run and
  // are zeroed in A
  double ra[2][4][4], rb[2][4][4];
  // runs of four k are read from in-range addresses: the last run of a row
  // of the extents' width (a multiple of 4), so with per-problem K the
  // elements at k >= K of a straddling run are read from the slot's padding
  // and zeroed below
  const int64_t Kx = g.K;
  auto load_chunk = [&](int buf, int64_t ch) {
    const int64_t k = std::min(16 * ch + kg, Kx - 4);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const f64x2 a01 = *(const f64x2*)(pa + q * g.psa + k), a23 = *(const f64x2*)(pa + q * g.psa + k + 2);
      const f64x2 b01 = *(const f64x2*)(pb + q * g.psb + k), b23 = *(const f64x2*)(pb + q * g.psb + k + 2);
      ra[buf][q][0] = a01[0];
      ra[buf][q][1] = a01[1];
      ra[buf][q][2] = a23[0];
      ra[buf][q][3] = a23[1];
      rb[buf][q][0] = b01[0];
      rb[buf][q][1] = b01[1];
      rb[buf][q][2] = b23[0];
      rb[buf][q][3] = b23[1];
    }
    asm volatile("" ::: "memory");
  };
  f64x4 acc[4];
#pragma unroll
  for (int p = 0; p < 4; ++p) acc[p] = (f64x4){0, 0, 0, 0};
  auto compute_chunk = [&](int buf, int64_t ch) {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      // both operands are zeroed past kend: with per-problem K the elements
      // of a row past its problem's K are not part of the operand
      const bool ok = ch < nch && 16 * ch + kg + s < kend;
      const double a0 = ok ? ra[buf][0][s] : 0.0, a1 = ok ? ra[buf][1][s] : 0.0;
      const double a2 = ok ? ra[buf][2][s] : 0.0, a3 = ok ? ra[buf][3][s] : 0.0;
      const double n0 = -a0, n1 = -a1, n2 = -a2, n3 = -a3;
      const double p0 = ok ? rb[buf][0][s] : 0.0, p1 = ok ? rb[buf][1][s] : 0.0;
      const double p2 = ok ? rb[buf][2][s] : 0.0, p3 = ok ? rb[buf][3][s] : 0.0;
      acc[0] = TT<double>::mfma(a0, p0, acc[0]);
      acc[1] = TT<double>::mfma(a1, p0, acc[1]);
      acc[2] = TT<double>::mfma(a2, p0, acc[2]);
      acc[3] = TT<double>::mfma(a3, p0, acc[3]);
      acc[0] = TT<double>::mfma(a1, p1, acc[0]);
      acc[1] = TT<double>::mfma(n0, p1, acc[1]);
      acc[2] = TT<double>::mfma(n3, p1, acc[2]);
      acc[3] = TT<double>::mfma(a2, p1, acc[3]);
      acc[0] = TT<double>::mfma(a2, p2, acc[0]);
      acc[1] = TT<double>::mfma(a3, p2, acc[1]);
      acc[2] = TT<double>::mfma(n0, p2, acc[2]);
      acc[3] = TT<double>::mfma(n1, p2, acc[3]);
      acc[0] = TT<double>::mfma(a3, p3, acc[0]);
      acc[1] = TT<double>::mfma(n2, p3, acc[1]);
      acc[2] = TT<double>::mfma(a1, p3, acc[2]);
      acc[3] = TT<double>::mfma(n0, p3, acc[3]);
    }
  };
  load_chunk(0, 0);
  for (int64_t ch = 0; ch < nch; ch += 2) {
    load_chunk(1, ch + 1);
    compute_chunk(0, ch);
    load_chunk(0, ch + 2);
    compute_chunk(1, ch + 1);
  }
  const int64_t j = j0 + r;
  double* D = g.D ? g.D + (int64_t)b * g.sD : nullptr;
  const int h = b < g.copy.split ? 0 : 1;
  void* D2 = g.copy.p[0] ? (char*)g.copy.p[h] +
                               (size_t)(b - h * g.copy.split) * g.copy.slab[h] * dtype_size(g.copy.dt)
                         : nullptr;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int64_t i = i0 + TT<double>::out_row(lane, q);
    if (i < M && j < N) {
#pragma unroll
      for (int p = 0; p < 4; ++p) {
        const int64_t o = i * g.ldd + j + p * g.psd;
        double v = g.alpha * acc[p][q];
        if (g.beta != 0.0) v += g.beta * D[o];
        if (D) D[o] = v;
        if (D2) store_from_double(D2, g.copy.dt, i * g.copy.ld[h] + j + p * g.copy.ps[h], v);
      }
    }
  }
}

}  // namespace

bool thin_hn_applies(int compute, int opA, int opB, int64_t M, int64_t N, int64_t K, int tri, bool per_problem_dims) {
  return (compute == QCUR_F64 || compute == QCUR_F32) && opA == QCUR_OP_H && opB == QCUR_OP_N && !per_problem_dims &&
         (tri & ~TRI_LOWER_OUT) == 0 && (!(tri & TRI_LOWER_OUT) || M == N) && M <= 512 && N <= 512 &&
         K >= 4 * std::max(M, N);
}

template <typename E>
static hipError_t launch_thin_dt(const Ctx& c, double alpha, QView A, QView B, double beta, QView D, int64_t K,
                                 int batch, int64_t sA, int64_t sB, int64_t sD, bool lower_only, void* ws,
                                 size_t ws_bytes, const int* bM, const int* bN, const int* bK) {
  const int64_t M = D.rows, N = D.cols;
  const int nbi = (int)((M + 15) / 16), nbj = (int)((N + 15) / 16);
  const int64_t blocks = lower_only ? (int64_t)nbi * (nbi + 1) / 2 : (int64_t)nbi * nbj;
  const int64_t ksteps = (K + 3) / 4;
  // about three waves per SIMD over the chip, at most 256 k-steps (1024
  // rows) per split (long K streams better with more waves in flight), at
  // least 32 k-steps per split
  int64_t splits = std::max<int64_t>(1, 3072 / (4 * blocks * std::max(batch, 1)));
  splits = std::max<int64_t>(splits, ksteps / 256);
  splits = std::min<int64_t>(splits, std::max<int64_t>(1, ksteps / 32));
  splits = std::min<int64_t>(splits, 32);
  const size_t need = (size_t)batch * splits * 4 * (size_t)M * (size_t)N * sizeof(E);
  if (splits > 1 && (ws == nullptr || ws_bytes < need)) splits = 1;
  if (bM || bN || bK) splits = 1;  // per-problem sizes: no K split
  ThinArgs g;
  g.bM = bM;
  g.bN = bN;
  g.bK = bK;
  g.A = A.p;
  g.lda = A.ld;
  g.psa = A.ps;
  g.sA = sA;
  g.B = B.p;
  g.ldb = B.ld;
  g.psb = B.ps;
  g.sB = sB;
  g.D = splits > 1 ? ws : D.p;
  g.ldd = D.ld;
  g.psd = D.ps;
  g.sD = sD;
  g.M = M;
  g.N = N;
  g.K = K;
  g.alpha = alpha;
  g.beta = beta;
  g.splits = (int)splits;
  const dim3 grid((unsigned)(blocks * batch * splits));
  if (lower_only) hipLaunchKernelGGL((k_thin_hn<E, true>), grid, dim3(256), 0, c.stream, g, (int)blocks, batch, nbj);
  else hipLaunchKernelGGL((k_thin_hn<E, false>), grid, dim3(256), 0, c.stream, g, (int)blocks, batch, nbj);
  if (splits > 1)
    hipLaunchKernelGGL(k_thin_reduce<E>, dim3((unsigned)((N + 255) / 256), (unsigned)std::min<int64_t>(M, 65535), batch),
                       dim3(256), 0, c.stream, (const E*)ws, (int)splits, M, N, alpha, beta, (E*)D.p, D.ld, D.ps, sD);
  return hipGetLastError();
}

hipError_t launch_thin_hn(const Ctx& c, int compute, double alpha, QView A, QView B, double beta, QView D, int64_t K,
                          int batch, int64_t sA, int64_t sB, int64_t sD, bool lower_only, void* ws, size_t ws_bytes,
                          const int* bM, const int* bN, const int* bK) {
  if (compute == QCUR_F32)
    return launch_thin_dt<float>(c, alpha, A, B, beta, D, K, batch, sA, sB, sD, lower_only, ws, ws_bytes, bM, bN, bK);
  return launch_thin_dt<double>(c, alpha, A, B, beta, D, K, batch, sA, sB, sD, lower_only, ws, ws_bytes, bM, bN, bK);
}

bool tall_nh_applies(int compute, int opA, int opB, QView A, QView B, int64_t M, int64_t N, int64_t K, int tri,
                     bool per_problem_dims, int64_t sA, int64_t sB) {
  auto even = [](int64_t x) { return (x & 1) == 0; };
  return compute == QCUR_F64 && opA == QCUR_OP_N && opB == QCUR_OP_H && !per_problem_dims &&
         (tri & ~TRI_B_UPPER) == 0 && M >= 512 && N <= 512 && K >= 4 && K <= 512 && K % 4 == 0 &&
         ((uintptr_t)A.p % 16) == 0 && ((uintptr_t)B.p % 16) == 0 && even(A.ld) && even(A.ps) && even(B.ld) &&
         even(B.ps) && even(sA) && even(sB);
}

hipError_t launch_tall_nh(const Ctx& c, double alpha, QView A, QView B, double beta, QView D, int64_t K, int batch,
                          int64_t sA, int64_t sB, int64_t sD, bool b_upper, const int* bM, const int* bN,
                          const int* bK, const TallCopy* copy) {
  if (!D.p && beta != 0.0) return hipErrorInvalidValue;
  const int64_t M = D.rows, N = D.cols;
  const int nbi = (int)((M + 15) / 16), nbj = (int)((N + 15) / 16);
  TallArgs g;
  g.bM = bM;
  g.bN = bN;
  g.bK = bK;
  g.A = (const double*)A.p;
  g.lda = A.ld;
  g.psa = A.ps;
  g.sA = sA;
  g.B = (const double*)B.p;
  g.ldb = B.ld;
  g.psb = B.ps;
  g.sB = sB;
  g.D = (double*)D.p;
  g.ldd = D.ld;
  g.psd = D.ps;
  g.sD = sD;
  g.M = M;
  g.N = N;
  g.K = K;
  g.alpha = alpha;
  g.beta = beta;
  g.b_upper = b_upper ? 1 : 0;
  g.copy = copy ? *copy : TallCopy{};
  const int64_t wgs = (int64_t)batch * nbj * ((nbi + 3) / 4);
  hipLaunchKernelGGL(k_tall_nh, dim3((unsigned)wgs), dim3(256), 0, c.stream, g, nbi, nbj);
  return hipGetLastError();
}

}  // namespace qcur
