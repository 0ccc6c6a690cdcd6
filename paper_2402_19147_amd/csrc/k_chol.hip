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
typedef double f64x4d __attribute__((ext_vector_type(4)));

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

// Factorisation G = L L^H and inverse P = L^{-1} of one w x w Hermitian
// positive definite diagonal block (w <= 64) in LDS, blocked by 16:
//  1. the 16 x 16 diagonal block is factored and inverted in one pass (below);
//     the inverse's strict lower part is kept transposed in the block's unused
//     upper triangle and 1/L[j][j] in rdg;
//  2. the panel below becomes L_ik = A_ik (L_kk^{-1})^H;
//  3. the trailing lower triangle loses L_ik L_jk^H;
// then block row by block row P_ij = -P_ii sum_{k=j}^{i-1} L_ik P_kj.
// Only P is written back (lower triangle; the upper one is zeroed).  A pivot
// that is not finite and positive sets *fail.
constexpr int CHOL_THREADS = 512;
constexpr int SB = 16;  // sub-block edge

// 1/sqrt(d) from the hardware estimate refined by two Newton steps (the
// pivot feeds only products, so correct rounding is not needed).
__device__ inline double rsqrt_nr(double d) {
  double r = __builtin_amdgcn_rsq(d);
  r = r * (1.5 - 0.5 * d * r * r);
  r = r * (1.5 - 0.5 * d * r * r);
  return r;
}

typedef double Tile[4][CB][CB + 1];

__device__ inline Qd ldq(const Tile& a, int i, int j) { return Qd{a[0][i][j], a[1][i][j], a[2][i][j], a[3][i][j]}; }
__device__ inline void stq(Tile& a, int i, int j, Qd v) {
  a[0][i][j] = v.w;
  a[1][i][j] = v.x;
  a[2][i][j] = v.y;
  a[3][i][j] = v.z;
}
// tiles of the tile-task factorisation below (32 x 32 quaternions)
constexpr int DTS = 32;  // tile edge
typedef double DTile[4][DTS][DTS + 1];
__device__ inline Qd ldq(const DTile& a, int i, int j) { return Qd{a[0][i][j], a[1][i][j], a[2][i][j], a[3][i][j]}; }
__device__ inline void stq(DTile& a, int i, int j, Qd v) {
  a[0][i][j] = v.w;
  a[1][i][j] = v.x;
  a[2][i][j] = v.y;
  a[3][i][j] = v.z;
}
__device__ inline void qacc(Qd& s, Qd u) {
  s.w += u.w;
  s.x += u.x;
  s.y += u.y;
  s.z += u.z;
}
// Element (r, c) (r >= c) of the inverse of diagonal block at kb: 1/L on the
// diagonal, else kept transposed in the block's upper triangle.
template <typename TileT>
__device__ inline Qd pdiag(const TileT& a, const double* rdg, int kb, int r, int c) {
  return r == c ? Qd{rdg[kb + r], 0.0, 0.0, 0.0} : ldq(a, kb + c, kb + r);
}

// Column j of the reduced block and row j of the unscaled inverse, published
// once per pivot (double-buffered by the pivot's parity).  The pivot's own
// slot carries (d, 1/sqrt(d), 1/d, failed) instead of (d, 0, 0, 0).
struct DiagBuf {
  double col[2][SB][4];
  double row[2][SB][4];
};

__device__ inline Qd ldq4(const double* p) {
  const double2 a = *reinterpret_cast<const double2*>(p), b = *reinterpret_cast<const double2*>(p + 2);
  return Qd{a.x, a.y, b.x, b.y};
}
__device__ inline void stq4(double* p, Qd v) {
  *reinterpret_cast<double2*>(p) = double2{v.w, v.x};
  *reinterpret_cast<double2*>(p + 2) = double2{v.y, v.z};
}

// Factorisation and inversion of the diagonal sub-block at kb (kw <= 16) by
// the workgroup's first 256 threads, thread (i, c) = (tid / 16, tid % 16)
// holding element (i, c) of the lower triangle in registers.  Pivot j is the
// elementary lower-triangular step E_j that clears column j below the
// diagonal; the same step applied to the identity accumulates E_j ... E_0 =
// L^{-1}.  Keeping the rows unscaled until the end, step j is
//   A_ic -= (A_ij / d_j) conj(A_cj)   for j < c <= i   (trailing update),
//   X_ij  = -A_ij / d_j                                  (column j retires),
//   X_ic -= (A_ij / d_j) X_jc          for c < j < i    (inverse rows),
// with d_j = A_jj, and finally P = diag(d_j^{-1/2}) (X + I).  Every element
// of the lower triangle is either still a reduced entry (c > j) or an entry
// of X (c <= j), so the thread keeps one value; column j and row j travel
// through LDS with one barrier per pivot, and every thread issues all of its
// reads right after the barrier.
template <typename TileT>
__device__ void chol_diag(TileT& a, double* rdg, DiagBuf& db, int kb, int kw, int tid, int* bad) {
  const int i = tid >> 4, c = tid & 15;
  const bool in = tid < SB * SB && i < kw && c <= i;
  Qd x = in ? ldq(a, kb + i, kb + c) : Qd{0, 0, 0, 0};
  // the exchange slots start at zero, so that every read below returns a
  // value of the matrix (finite for a finite matrix) and the factors that
  // switch a term off can be plain multiplications by zero
  for (int e = tid; e < (int)(sizeof(DiagBuf) / sizeof(double)); e += 256)
    if (tid < 256) reinterpret_cast<double*>(&db)[e] = 0.0;
  __syncthreads();
  double rsi = 1.0;
  bool failed = false;
  for (int j = 0; j < kw; ++j) {
    const int par = j & 1;
    if (in && c == j) {
      if (i == j) {
        const bool ok = x.w > 0.0 && x.w < INFINITY;
        const double rs = rsqrt_nr(ok ? x.w : 1.0);
        stq4(db.col[par][i], Qd{x.w, rs, rs * rs, ok ? 0.0 : 1.0});
      } else {
        stq4(db.col[par][i], x);
      }
    }
    if (in && i == j && c < j) stq4(db.row[par][c], x);
    __syncthreads();
    // all three reads are unconditional and issued together
    const Qd piv = ldq4(db.col[par][j]);
    const Qd ar = ldq4(db.col[par][i & (SB - 1)]);
    const Qd vr = ldq4(c > j ? db.col[par][c] : db.row[par][c]);
    const double rs = piv.x, rd = piv.y;
    const bool act = in && i > j, ret = c == j;
    // inactive rows take u = 0 and the retiring column v = 0; then one fused
    // form covers the three cases with the roundings of the plain formulas
    const double fu = act ? rd : 0.0;
    const Qd u = Qd{ar.w * fu, ar.x * fu, ar.y * fu, ar.z * fu};
    const double f0 = ret ? 0.0 : 1.0, f1 = ret ? 0.0 : (c > j ? -1.0 : 1.0);
    const Qd v = Qd{vr.w * f0, vr.x * f1, vr.y * f1, vr.z * f1};
    const Qd q = qmul(u, v);
    const double m = ret && act ? -rd : 1.0;
    x = Qd{__builtin_fma(x.w, m, -q.w), __builtin_fma(x.x, m, -q.x), __builtin_fma(x.y, m, -q.y),
           __builtin_fma(x.z, m, -q.z)};
    rsi = i == j ? rs : rsi;
    failed |= piv.z != 0.0;
  }
  if (tid == 0 && failed) *bad = 1;
  if (in) {
    if (c < i)
      stq(a, kb + c, kb + i, Qd{x.w * rsi, x.x * rsi, x.y * rsi, x.z * rsi});
    else
      rdg[kb + i] = rsi;
  }
}

// Factorisation and inverse of the leading w x w block (w <= 64) of the
// lower triangle held in a: on return a holds P = L^{-1} in the layout of
// chol_diag (diagonal sub-blocks' strict lower parts transposed into their
// upper triangles, 1 / L[j][j] in rdg; read back through pdiag), the rest of
// P's lower triangle in place.  All CHOL_THREADS threads take part.
__device__ __attribute__((always_inline)) void chol_block_lds(Tile& a, double (*sbuf)[4][SB][SB + 1], double* rdg, DiagBuf& db, int* bad, int w) {
  const int tid = threadIdx.x;
  for (int kb = 0; kb < w; kb += SB) {
    const int kw = min(SB, w - kb);
    chol_diag(a, rdg, db, kb, kw, tid, bad);
    __syncthreads();
    const int r0 = kb + kw, rows = w - r0;
    if (rows <= 0) break;
    // panel: L[i][kb + c] = sum_{t <= c} A[i][kb + t] conj(P_kk[c][t])
    Qd pv[2];
    int pi[2], pc[2];
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      const int e = tid + CHOL_THREADS * m;
      pi[m] = -1;
      if (e < rows * kw) {
        pi[m] = r0 + e / kw;
        pc[m] = e % kw;
        Qd s{0, 0, 0, 0};
        for (int t = 0; t <= pc[m]; ++t) qacc(s, qmul_conj(ldq(a, pi[m], kb + t), pdiag(a, rdg, kb, pc[m], t)));
        pv[m] = s;
      }
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < 2; ++m)
      if (pi[m] >= 0) stq(a, pi[m], kb + pc[m], pv[m]);
    __syncthreads();
    // trailing: A[i][j] -= sum_t L[i][kb + t] conj(L[j][kb + t]),  r0 <= j <= i < w
    const int tcnt = rows * (rows + 1) / 2;
    for (int e = tid; e < tcnt; e += CHOL_THREADS) {
      const int r = (int)((sqrtf((float)(8 * e + 1)) - 1.0f) * 0.5f);
      const int q = e - r * (r + 1) / 2;
      const int i = r0 + r, j = r0 + q;
      Qd s = ldq(a, i, j);
      for (int t = 0; t < kw; ++t) {
        const Qd u = qmul_conj(ldq(a, i, kb + t), ldq(a, j, kb + t));
        s.w -= u.w;
        s.x -= u.x;
        s.y -= u.y;
        s.z -= u.z;
      }
      stq(a, i, j, s);
    }
    __syncthreads();
  }
  // inverse, block row by block row: S_j = sum_{k=j}^{i-1} L_ik P_kj for all
  // j < i at once, then P_ij = -P_ii S_j overwrites L_ij
  const int nsb = (w + SB - 1) / SB;
  for (int bi = 1; bi < nsb; ++bi) {
    const int i0 = bi * SB, iw = min(SB, w - i0);
    for (int e = tid; e < bi * SB * SB; e += CHOL_THREADS) {
      const int bj = e / (SB * SB), r = (e / SB) % SB, c = e % SB;
      if (r >= iw) continue;
      const int j0 = bj * SB;
      Qd s{0, 0, 0, 0};
      for (int bk = bj; bk < bi; ++bk) {
        const int k0 = bk * SB;
        for (int t = 0; t < SB; ++t) {
          const Qd pkj = bk == bj ? (t >= c ? pdiag(a, rdg, k0, t, c) : Qd{0, 0, 0, 0}) : ldq(a, k0 + t, j0 + c);
          qacc(s, qmul(ldq(a, i0 + r, k0 + t), pkj));
        }
      }
      sbuf[bj][0][r][c] = s.w;
      sbuf[bj][1][r][c] = s.x;
      sbuf[bj][2][r][c] = s.y;
      sbuf[bj][3][r][c] = s.z;
    }
    __syncthreads();
    for (int e = tid; e < bi * SB * SB; e += CHOL_THREADS) {
      const int bj = e / (SB * SB), r = (e / SB) % SB, c = e % SB;
      if (r >= iw) continue;
      Qd s{0, 0, 0, 0};
      for (int t = 0; t <= r; ++t) {
        const Qd sv{sbuf[bj][0][t][c], sbuf[bj][1][t][c], sbuf[bj][2][t][c], sbuf[bj][3][t][c]};
        qacc(s, qmul(pdiag(a, rdg, i0, r, t), sv));
      }
      stq(a, i0 + r, bj * SB + c, Qd{-s.w, -s.x, -s.y, -s.z});
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(CHOL_THREADS) void k_chol_block(const double* __restrict__ G0, double* __restrict__ P0,
                                                             int wx, int64_t ld, int64_t ps, int64_t sbatch,
                                                             int* fail0, const int* __restrict__ dims) {
  // matrix b's own order (dims: per-matrix orders; 0 = nothing to do, P
  // left as it is; outside the leading w x w block nothing is written)
  const int w = dims ? min(dims[blockIdx.x], wx) : wx;
  if (w <= 0) return;
  const double* __restrict__ G = G0 + (int64_t)blockIdx.x * sbatch;
  double* __restrict__ Pg = P0 + (int64_t)blockIdx.x * sbatch;
  int* fail = fail0 + blockIdx.x;
  __shared__ Tile a;
  __shared__ double sbuf[3][4][SB][SB + 1];  // block-row sums of the inverse phase
  __shared__ double rdg[CB];                 // 1 / L[j][j]
  __shared__ __align__(16) DiagBuf db;
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
  chol_block_lds(a, sbuf, rdg, db, &bad, w);
  for (int e = tid; e < w * w; e += CHOL_THREADS) {
    const int i = e / w, j = e % w;
    const int64_t o = (int64_t)i * ld + j;
    Qd v{0, 0, 0, 0};
    if (j <= i) v = (i / SB == j / SB) ? pdiag(a, rdg, (i / SB) * SB, i % SB, j % SB) : ldq(a, i, j);
    Pg[o] = v.w;
    Pg[o + ps] = v.x;
    Pg[o + 2 * ps] = v.y;
    Pg[o + 3 * ps] = v.z;
  }
  if (tid == 0 && bad) atomicOr(fail, 1);
}

hipError_t launch_chol_block(const Ctx& c, const double* G, double* P, int w, int64_t ld, int64_t ps, int* fail,
                             int batch, int64_t sbatch, const int* dims) {
  hipLaunchKernelGGL(k_chol_block, dim3(batch), dim3(CHOL_THREADS), 0, c.stream, G, P, w, ld, ps, sbatch, fail,
                     dims);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// The first CholeskyQR pass of every factor of a batch in one launch, one
// workgroup per factor Z_t (p_t x q_t, q_t <= 64, FP64 slots):
//   1. G = Z^H Z (lower 16 x 16 blocks, FP64 matrix cores) into LDS, and
//      ||Z||_F^2 from the same loads;
//   2. G = L L^H and P1 = L^{-1} in LDS (chol_block_lds), P1 and ||P1||_F^2
//      written out;
//   3. Q1 = Z P1^H (FP64 and the product-dtype copy);
//   4. G2 = Q1^H Q1 from the Q1 just written and its defect ||G2 - I||_F^2:
//      with `adaptive` the factor keeps its first pass (q2 = 0, P = P1) when
//      its Cholesky succeeded and the defect is at most tol2;
//   5. otherwise (always without `adaptive`) the second pass in place:
//      G2 = L2 L2^H, P2 = L2^{-1}, Q = Q1 P2^H (FP64 and/or the product-dtype
//      copy), P = P2 P1, q2 = q_t.
// The separate launches this replaces spread each factor over many
// workgroups; here every compute unit works through whole factors and Z is
// read from HBM once per pass.  Every sum runs in a fixed order.
struct CholqrBatch {
  const double* Z;
  double *Q1, *Q;             // Q: the second pass's FP64 factor (NULL: only the product-dtype copy)
  int64_t zld, zps, zslab;  // Z, Q1 and Q slots: row stride, plane stride, slot stride
  double *P1, *P;
  int64_t gld, gps, gslab;  // q x q slots
  const int *zp, *zq;
  int* fail;
  double* norms;  // [4 t]: ||Z_t||_F^2, [4 t + 1]: ||P1_t||_F^2
  int *q2, *skip;
  double tol2;
  int adaptive;
  TallCopy copy;
  // workgroup k takes factor order[k] (NULL: k): largest first
  const int* order;
};

// Hermitian Gram blocks of X (rows < p, columns < q) into the lower 16 x 16
// blocks of a: tasks (block, row slice) spread over the eight waves, the
// slices' partial blocks added into a in slice order.  *sq gains the sum of
// squares of the entries the diagonal-block tasks load (each entry once).
__device__ __attribute__((always_inline)) void cholqr_gram(const double* __restrict__ X, int64_t ld, int64_t ps, int p, int q, Tile& a,
                            double* sq) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, g4 = lane >> 4, cl = lane & 15;
  // (at most two tasks per wave, whose accumulators stay in registers: the
  // task loops are unrolled so that every index is a constant).  Up to eight
  // blocks: every block in H equal row slices.  Ten blocks (49-64 columns):
  // the first six in two halves, the last four whole, listed whole blocks
  // first, so that waves w and w + 4 (one SIMD) always get five halves
  const int nb = (q + 15) >> 4, nblk = nb * (nb + 1) / 2;
  const bool mixed = nblk > 8;
  const int nsplit = mixed ? 16 - nblk : 0, whole = nblk - nsplit;
  const int H = mixed ? 2 : max(1, min(8, 16 / nblk));
  const int ntask = mixed ? 16 : nblk * H;
  f64x4d acc[2][4];
  int tb[2], th[2];
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int task = wave + 8 * u;
    tb[u] = -1;
    th[u] = 0;
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[u][c] = (f64x4d){0, 0, 0, 0};
    if (task >= ntask) continue;  // wave-uniform
    int blk, h, nsl;
    if (!mixed) {
      blk = task / H;
      h = task % H;
      nsl = H;
    } else if (task < whole) {
      blk = nsplit + task;
      h = 0;
      nsl = 1;
    } else {
      blk = (task - whole) >> 1;
      h = (task - whole) & 1;
      nsl = 2;
    }
    const int rows = (((p + nsl - 1) / nsl) + 15) & ~15;
    int bi = 0;
    while ((bi + 1) * (bi + 2) / 2 <= blk) ++bi;
    const int bj = blk - bi * (bi + 1) / 2;
    tb[u] = blk;
    th[u] = h;
    const int r0 = h * rows, r1 = min(p, r0 + rows);
    const int ca = 16 * bi + cl, cb = 16 * bj + cl;
    const bool oka = ca < q, okb = cb < q, diag = bi == bj;
    const double* pa = X + min(ca, q - 1);
    const double* pb = X + min(cb, q - 1);
    // chunks of 16 rows; MFMA step s takes row k0 + 4 s + g4 (the same in
    // both operands); rows are clamped into the matrix, so every load is
    // unconditional, and rows past the slice are zeroed
    double va[1][4][4], vb[1][4][4];
    auto load = [&](int buf, int k0) __attribute__((always_inline)) {
#pragma unroll
      for (int st = 0; st < 4; ++st) {
        const int64_t kc = min(k0 + 4 * st + g4, p - 1);
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          va[buf][st][c] = pa[kc * ld + c * ps];
          vb[buf][st][c] = pb[kc * ld + c * ps];
        }
      }
    };
    auto comp = [&](int buf, int k0) __attribute__((always_inline)) {
#pragma unroll
      for (int st = 0; st < 4; ++st) {
        const bool okr = k0 + 4 * st + g4 < r1;
        const double a0 = okr && oka ? va[buf][st][0] : 0.0, a1 = okr && oka ? va[buf][st][1] : 0.0;
        const double a2 = okr && oka ? va[buf][st][2] : 0.0, a3 = okr && oka ? va[buf][st][3] : 0.0;
        const double b0 = okr && okb ? vb[buf][st][0] : 0.0, b1 = okr && okb ? vb[buf][st][1] : 0.0;
        const double b2 = okr && okb ? vb[buf][st][2] : 0.0, b3 = okr && okb ? vb[buf][st][3] : 0.0;
        if (diag) *sq += a0 * a0 + a1 * a1 + a2 * a2 + a3 * a3;
        const double n1 = -a1, n2 = -a2, n3 = -a3;
        // conj(a) b:  w = a0 b0 + a1 b1 + a2 b2 + a3 b3,  x = a0 b1 - a1 b0 - a2 b3 + a3 b2,
        //             y = a0 b2 + a1 b3 - a2 b0 - a3 b1,  z = a0 b3 - a1 b2 + a2 b1 - a3 b0
        acc[u][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[u][0], 0, 0, 0);
        acc[u][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[u][1], 0, 0, 0);
        acc[u][2] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b2, acc[u][2], 0, 0, 0);
        acc[u][3] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b3, acc[u][3], 0, 0, 0);
        acc[u][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[u][0], 0, 0, 0);
        acc[u][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(n1, b0, acc[u][1], 0, 0, 0);
        acc[u][2] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b3, acc[u][2], 0, 0, 0);
        acc[u][3] = __builtin_amdgcn_mfma_f64_16x16x4f64(n1, b2, acc[u][3], 0, 0, 0);
        acc[u][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a2, b2, acc[u][0], 0, 0, 0);
        acc[u][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(n2, b3, acc[u][1], 0, 0, 0);
        acc[u][2] = __builtin_amdgcn_mfma_f64_16x16x4f64(n2, b0, acc[u][2], 0, 0, 0);
        acc[u][3] = __builtin_amdgcn_mfma_f64_16x16x4f64(a2, b1, acc[u][3], 0, 0, 0);
        acc[u][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a3, b3, acc[u][0], 0, 0, 0);
        acc[u][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a3, b2, acc[u][1], 0, 0, 0);
        acc[u][2] = __builtin_amdgcn_mfma_f64_16x16x4f64(n3, b1, acc[u][2], 0, 0, 0);
        acc[u][3] = __builtin_amdgcn_mfma_f64_16x16x4f64(n3, b0, acc[u][3], 0, 0, 0);
      }
    };
    for (int k0 = r0; k0 < r1; k0 += 16) {
      load(0, k0);
      comp(0, k0);
    }
  }
  // slice h's partial blocks go into a after those of slices < h
  for (int h = 0; h < H; ++h) {
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      if (tb[u] < 0 || th[u] != h) continue;
      int bi = 0;
      while ((bi + 1) * (bi + 2) / 2 <= tb[u]) ++bi;
      const int bj = tb[u] - bi * (bi + 1) / 2;
#pragma unroll
      for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = 16 * bi + g4 + 4 * r, j = 16 * bj + cl;
          a[c][i][j] = h == 0 ? acc[u][c][r] : a[c][i][j] + acc[u][c][r];
        }
    }
  }
  __syncthreads();
}

// fixed-order sum over the workgroup (CHOL_THREADS threads); every thread
// gets the total
__device__ double cholqr_sum(double v, double* red) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int w = 0; w < CHOL_THREADS / 64; ++w) s += red[w];
  return s;
}

// D = X P^H over rows < p and columns < q with P (lower triangular, plain
// layout) in a: tasks (16-row block, 16-column block) over the waves; lane
// group g4 takes k = k0 + 4 g4 + s at MFMA step s, a run of four consecutive
// k in both operands.  A conj(b) with n = -a:
//   w: a0 p0 + a1 p1 + a2 p2 + a3 p3    x: a1 p0 + n0 p1 + a3 p2 + n2 p3
//   y: a2 p0 + n3 p1 + n0 p2 + a1 p3    z: a3 p0 + a2 p1 + n1 p2 + n0 p3
// D (FP64, may be NULL) and D2 (dtype d2dt, may be NULL) receive the result.
__device__ __attribute__((always_inline)) void cholqr_zph(const double* __restrict__ X, int64_t ld, int64_t ps, int p, int q, const Tile& a,
                           double* __restrict__ D, void* D2, int d2dt, int64_t d2ld, int64_t d2ps) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, g4 = lane >> 4, cl = lane & 15;
  const int nbj = (q + 15) >> 4, nbi = (p + 15) >> 4;
  // row blocks fastest, so that every wave gets a share of each column
  // block (column block bj costs bj + 1 chunks of 16 k)
  for (int task = wave; task < nbi * nbj; task += CHOL_THREADS / 64) {
    const int bi = task % nbi, bj = task / nbi;
    const int ir = 16 * bi + cl, jc = 16 * bj + cl;
    const double* pa = X + (int64_t)min(ir, p - 1) * ld;
    const int kend = min(q, 16 * bj + 16);
    f64x4d acc[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[c] = (f64x4d){0, 0, 0, 0};
    for (int k0 = 0; k0 < kend; k0 += 16) {
      double va[4][4];
#pragma unroll
      for (int st = 0; st < 4; ++st) {
        const int k = min(k0 + 4 * g4 + st, q - 1);
#pragma unroll
        for (int c = 0; c < 4; ++c) va[st][c] = pa[k + c * ps];
      }
#pragma unroll
      for (int st = 0; st < 4; ++st) {
        const int k = k0 + 4 * g4 + st;
        const bool ok = ir < p && k < kend;
        const bool okp = jc < q && k <= jc && k < q;
        const int kc = min(k, CB - 1);
        const double a0 = ok ? va[st][0] : 0.0, a1 = ok ? va[st][1] : 0.0;
        const double a2 = ok ? va[st][2] : 0.0, a3 = ok ? va[st][3] : 0.0;
        const double p0 = okp ? a[0][jc][kc] : 0.0, p1 = okp ? a[1][jc][kc] : 0.0;
        const double p2 = okp ? a[2][jc][kc] : 0.0, p3 = okp ? a[3][jc][kc] : 0.0;
        const double n0 = -a0, n1 = -a1, n2 = -a2, n3 = -a3;
        acc[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, p0, acc[0], 0, 0, 0);
        acc[1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, p0, acc[1], 0, 0, 0);
        acc[2] = __builtin_amdgcn_mfma_f64_16x16x4f64(a2, p0, acc[2], 0, 0, 0);
        acc[3] = __builtin_amdgcn_mfma_f64_16x16x4f64(a3, p0, acc[3], 0, 0, 0);
        acc[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, p1, acc[0], 0, 0, 0);
        acc[1] = __builtin_amdgcn_mfma_f64_16x16x4f64(n0, p1, acc[1], 0, 0, 0);
        acc[2] = __builtin_amdgcn_mfma_f64_16x16x4f64(n3, p1, acc[2], 0, 0, 0);
        acc[3] = __builtin_amdgcn_mfma_f64_16x16x4f64(a2, p1, acc[3], 0, 0, 0);
        acc[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a2, p2, acc[0], 0, 0, 0);
        acc[1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a3, p2, acc[1], 0, 0, 0);
        acc[2] = __builtin_amdgcn_mfma_f64_16x16x4f64(n0, p2, acc[2], 0, 0, 0);
        acc[3] = __builtin_amdgcn_mfma_f64_16x16x4f64(n1, p2, acc[3], 0, 0, 0);
        acc[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a3, p3, acc[0], 0, 0, 0);
        acc[1] = __builtin_amdgcn_mfma_f64_16x16x4f64(n2, p3, acc[1], 0, 0, 0);
        acc[2] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, p3, acc[2], 0, 0, 0);
        acc[3] = __builtin_amdgcn_mfma_f64_16x16x4f64(n0, p3, acc[3], 0, 0, 0);
      }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = 16 * bi + g4 + 4 * r;
      if (i < p && jc < q) {
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          if (D) D[(int64_t)i * ld + jc + c * ps] = acc[c][r];
          if (D2) store_from_double(D2, d2dt, (int64_t)i * d2ld + jc + c * d2ps, acc[c][r]);
        }
      }
    }
  }
}

// After chol_block_lds on the leading q x q block of a: P = L^{-1} written
// to Pg (q x q, upper part zero; NULL: not written) and put back into a as
// a plain lower triangle (upper part zero) for cholqr_zph; returns
// ||P||_F^2 (every thread).
__device__ __attribute__((always_inline)) double cholqr_restage(Tile& a, const double* rdg, int q, double* __restrict__ Pg, int64_t gld,
                                 int64_t gps, double* red) {
  const int tid = threadIdx.x;
  constexpr int PE = CB * CB / CHOL_THREADS;
  Qd pv[PE];
  double ps2 = 0.0;
#pragma unroll
  for (int m = 0; m < PE; ++m) {
    const int e = tid + CHOL_THREADS * m;
    const int i = e / q, j = e % q;
    Qd v{0, 0, 0, 0};
    if (e < q * q && j <= i) v = (i / SB == j / SB) ? pdiag(a, rdg, (i / SB) * SB, i % SB, j % SB) : ldq(a, i, j);
    pv[m] = v;
    if (e < q * q) {
      if (Pg) {
        const int64_t o = (int64_t)i * gld + j;
        Pg[o] = v.w;
        Pg[o + gps] = v.x;
        Pg[o + 2 * gps] = v.y;
        Pg[o + 3 * gps] = v.z;
      }
      ps2 += v.w * v.w + v.x * v.x + v.y * v.y + v.z * v.z;
    }
  }
  ps2 = cholqr_sum(ps2, red);  // (its barriers also end the reads of a above)
#pragma unroll
  for (int m = 0; m < PE; ++m) {
    const int e = tid + CHOL_THREADS * m;
    if (e < q * q) stq(a, e / q, e % q, pv[m]);
  }
  __syncthreads();
  return ps2;
}

// release the workgroup's global writes to its other waves
__device__ inline void cholqr_sync_global() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __syncthreads();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

__global__ __launch_bounds__(CHOL_THREADS) void kb_cholqr(CholqrBatch g) {
  __shared__ Tile a;
  __shared__ double sbuf[3][4][SB][SB + 1];
  __shared__ double rdg[CB];
  __shared__ __align__(16) DiagBuf db;
  __shared__ double red[CHOL_THREADS / 64];
  __shared__ int bad;
  const int t = g.order ? g.order[blockIdx.x] : blockIdx.x, tid = threadIdx.x;
  const int p = g.zp[t], q = g.zq[t];
  if (p <= 0 || q <= 0) {
    if (tid == 0) {
      g.norms[4 * t] = 0.0;
      g.norms[4 * t + 1] = 0.0;
      g.q2[t] = 0;
      g.skip[t] = 1;
    }
    return;
  }
  const double* __restrict__ Z = g.Z + (int64_t)t * g.zslab;
  double* __restrict__ Q1 = g.Q1 + (int64_t)t * g.zslab;
  double* __restrict__ P1 = g.P1 + (int64_t)t * g.gslab;
  double* __restrict__ Pt = g.P + (int64_t)t * g.gslab;
  const int h = t < g.copy.split ? 0 : 1;
  void* D2 = g.copy.p[0] ? (char*)g.copy.p[h] + (size_t)(t - h * g.copy.split) * g.copy.slab[h] * dtype_size(g.copy.dt)
                         : nullptr;
  if (tid == 0) bad = 0;
  // 1. G = Z^H Z
  double sq = 0.0;
  cholqr_gram(Z, g.zld, g.zps, p, q, a, &sq);
  sq = cholqr_sum(sq, red);
  if (tid == 0) g.norms[4 * t] = sq;
  // 2. P1 = L^{-1}, written out and put back into a
  chol_block_lds(a, sbuf, rdg, db, &bad, q);
  const double p1n = cholqr_restage(a, rdg, q, P1, g.gld, g.gps, red);
  if (tid == 0) g.norms[4 * t + 1] = p1n;
  // 3. Q1 = Z P1^H (and its product-dtype copy)
  cholqr_zph(Z, g.zld, g.zps, p, q, a, Q1, D2, g.copy.dt, g.copy.ld[h], g.copy.ps[h]);
  // 4. G2 = Q1^H Q1 from the Q1 this workgroup wrote, its defect, the plan
  cholqr_sync_global();
  double unused = 0.0;
  cholqr_gram(Q1, g.zld, g.zps, p, q, a, &unused);
  double d2 = 0.0;
  for (int e = tid; e < q * q; e += CHOL_THREADS) {
    const int i = e / q, j = e % q;
    if (j > i) continue;
    const double wgt = i == j ? 1.0 : 2.0;  // the strict lower part stands for both triangles
    const double d0 = a[0][i][j] - (i == j ? 1.0 : 0.0);
    d2 += wgt * (d0 * d0 + a[1][i][j] * a[1][i][j] + a[2][i][j] * a[2][i][j] + a[3][i][j] * a[3][i][j]);
  }
  d2 = cholqr_sum(d2, red);
  const bool keep = g.adaptive && bad == 0 && d2 <= g.tol2;
  if (tid == 0) {
    g.q2[t] = keep ? 0 : q;
    g.skip[t] = keep ? 1 : 0;
  }
  if (keep) {
    for (int e = tid; e < q * q; e += CHOL_THREADS) {
      const int64_t o = (int64_t)(e / q) * g.gld + e % q;
#pragma unroll
      for (int c = 0; c < 4; ++c) Pt[o + c * g.gps] = P1[o + c * g.gps];
    }
    if (tid == 0 && bad) g.fail[t] = 1;
    return;
  }
  // 5. second pass: G2 = L2 L2^H, P2 = L2^{-1} (into a), Q = Q1 P2^H (FP64
  //    to the Q slot when given, and the product-dtype copy), P = P2 P1
  chol_block_lds(a, sbuf, rdg, db, &bad, q);
  cholqr_restage(a, rdg, q, nullptr, 0, 0, red);
  double* __restrict__ Q = g.Q ? g.Q + (int64_t)t * g.zslab : nullptr;
  cholqr_zph(Q1, g.zld, g.zps, p, q, a, Q, D2, g.copy.dt, g.copy.ld[h], g.copy.ps[h]);
  // P[i][j] = sum_{j <= k <= i} P2[i][k] P1[k][j], in order of k
  for (int e = tid; e < q * q; e += CHOL_THREADS) {
    const int i = e / q, j = e % q;
    Qd s{0, 0, 0, 0};
    for (int k = j; k <= i; ++k) {
      const int64_t o = (int64_t)k * g.gld + j;
      qacc(s, qmul(ldq(a, i, k), Qd{P1[o], P1[o + g.gps], P1[o + 2 * g.gps], P1[o + 3 * g.gps]}));
    }
    const int64_t o = (int64_t)i * g.gld + j;
#pragma unroll
    for (int c = 0; c < 4; ++c) Pt[o + c * g.gps] = c == 0 ? s.w : c == 1 ? s.x : c == 2 ? s.y : s.z;
  }
  __syncthreads();
  if (tid == 0 && bad) g.fail[t] = 1;
}

hipError_t launch_cholqr_batch(const Ctx& c, int count, const double* Z, double* Q1, double* Q, int64_t zld, int64_t zps,
                               int64_t zslab, double* P1, double* P, int64_t gld, int64_t gps,
                               int64_t gslab, const int* zp, const int* zq, int* fail, double* norms, int* q2,
                               int* skip, double tol2, int adaptive, const TallCopy* copy, const int* order) {
  if (count <= 0) return hipSuccess;
  CholqrBatch g;
  g.Z = Z;
  g.Q1 = Q1;
  g.Q = Q;
  g.zld = zld;
  g.zps = zps;
  g.zslab = zslab;
  g.P1 = P1;
  g.P = P;
  g.gld = gld;
  g.gps = gps;
  g.gslab = gslab;
  g.zp = zp;
  g.zq = zq;
  g.fail = fail;
  g.norms = norms;
  g.q2 = q2;
  g.skip = skip;
  g.tol2 = tol2;
  g.adaptive = adaptive;
  g.copy = copy ? *copy : TallCopy{};
  g.order = order;
  hipLaunchKernelGGL(kb_cholqr, dim3((unsigned)count), dim3(CHOL_THREADS), 0, c.stream, g);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Factorisation G = L L^H and inverse P = L^{-1} of nb Hermitian positive
// definite n x n quaternion matrices in one launch, as a graph of 32 x 32
// tile tasks whose dependencies are met through ready flags in global memory
// (the blocked right-looking schedule above needs a launch per block step and
// waits for every tile of a step before the next one starts; here a tile
// starts as soon as the tiles it reads are ready).  Tasks, one per
// workgroup:
//   factor (i, j), j <= i:  S = G_ij - sum_{k<j} L_ik L_jk^H (k in order);
//       i == j: P_jj = (the factor of S)^{-1} by the elementary steps of
//       chol_diag;  i > j: L_ij = S P_jj^H;
//   inverse (i, j), i > j:  P_ij = -P_ii sum_{l=j}^{i-1} L_il P_lj (l in order).
// The 32 x 32 tile products run on the FP64 matrix cores (dag_mfma).  Only P
// and the off-diagonal L tiles are stored.  Every workgroup takes its
// task from a ticket counter, in an order in which each task depends only on
// tasks with smaller tickets, and a ticket is only held by a workgroup that
// is running, so every wait is on a task that is running or done, whatever
// the number of workgroups the device holds at once.  Waits are bounded:
// past the spin limit the task goes on, marks its matrix as failed (the
// caller then takes the Jacobi path) and raises ST_NUMERIC.  Sums run in a
// fixed order, so results do not depend on scheduling.
constexpr int DAG_THREADS = 256;
constexpr long DAG_SPIN_LIMIT = 1L << 22;

struct DagArgs {
  const double* G;  // lower triangles; matrix b at G + b * slab, row stride n, plane stride n * n
  double* L;        // off-diagonal tiles of L
  double* P;        // L^{-1}, lower (upper part zeroed)
  int64_t n, slab;
  int nb, nt;
  int64_t nfact;    // factor tasks: nb * nt (nt + 1) / 2
  int* flags;       // [nb][3][nt][nt]: 0 = L tile (and P_jj for a diagonal tile), 1 = P tile,
                    // 2 = S_{j+1,j} (the factor task's tile before its multiply by P_jj^H)
  int* ticket;
  int* fail;        // [nb]
  unsigned* status;
};

__device__ inline int* dag_flag(const DagArgs& g, int b, int kind, int i, int j) {
  return g.flags + (((int64_t)b * 3 + kind) * g.nt + i) * g.nt + j;
}

// Thread 0 waits for a flag (bounded); then every thread fences (acquire).
__device__ inline void dag_wait(const DagArgs& g, const int* f, int b, int* timed_out) {
  if (threadIdx.x == 0 && !*timed_out) {
    long it = 0;
    while (__hip_atomic_load(f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) {
      __builtin_amdgcn_s_sleep(2);
      if (++it > DAG_SPIN_LIMIT) {
        *timed_out = 1;
        break;
      }
    }
  }
  __syncthreads();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
}

// Every thread's stores are made visible, then thread 0 sets the flag.
__device__ inline void dag_publish(int* f) {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  __syncthreads();
  if (threadIdx.x == 0) __hip_atomic_store(f, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// tile (ti, tj) of one matrix (row stride n, plane stride n * n) into LDS;
// entries past n read as zero
__device__ inline void dag_load(DTile& t, const double* __restrict__ M, int64_t n, int ti, int tj) {
  const int64_t ps = n * n;
  for (int e = threadIdx.x; e < DTS * DTS; e += DAG_THREADS) {
    const int r = e / DTS, c = e % DTS;
    const int64_t gi = (int64_t)ti * DTS + r, gj = (int64_t)tj * DTS + c;
    const bool ok = gi < n && gj < n;
    const int64_t o = gi * n + gj;
#pragma unroll
    for (int q = 0; q < 4; ++q) t[q][r][c] = ok ? M[o + q * ps] : 0.0;
  }
}

// a tile from LDS to the matrix (row stride n, plane stride n * n); entries
// past n are not stored
__device__ inline void dag_store_tile(double* __restrict__ M, int64_t n, int ti, int tj, const DTile& t) {
  const int64_t ps = n * n;
  for (int e = threadIdx.x; e < DTS * DTS; e += DAG_THREADS) {
    const int r = e / DTS, c = e % DTS;
    const int64_t gi = (int64_t)ti * DTS + r, gj = (int64_t)tj * DTS + c;
    if (gi < n && gj < n) {
      const int64_t o = gi * n + gj;
#pragma unroll
      for (int q = 0; q < 4; ++q) M[o + q * ps] = t[q][r][c];
    }
  }
}
__device__ inline void dag_store_zero(double* __restrict__ M, int64_t n, int ti, int tj) {
  const int64_t ps = n * n;
  for (int e = threadIdx.x; e < DTS * DTS; e += DAG_THREADS) {
    const int r = e / DTS, c = e % DTS;
    const int64_t gi = (int64_t)ti * DTS + r, gj = (int64_t)tj * DTS + c;
    if (gi < n && gj < n) {
      const int64_t o = gi * n + gj;
#pragma unroll
      for (int q = 0; q < 4; ++q) M[o + q * ps] = 0.0;
    }
  }
}

// The tile S_{i,j} (j < i) kept in the unused upper slot (j, i) of L,
// transposed (its element (r, c) at row 32 j + c, column 32 i + r), so that
// the rows of S past n, the ones a partial last tile row i pads with, are the
// ones not stored
__device__ inline void dag_store_tile_t(double* __restrict__ M, int64_t n, int tj, int ti, const DTile& t) {
  const int64_t ps = n * n;
  for (int e = threadIdx.x; e < DTS * DTS; e += DAG_THREADS) {
    const int c = e / DTS, r = e % DTS;
    const int64_t gi = (int64_t)tj * DTS + c, gj = (int64_t)ti * DTS + r;
    if (gi < n && gj < n) {
      const int64_t o = gi * n + gj;
#pragma unroll
      for (int q = 0; q < 4; ++q) M[o + q * ps] = t[q][r][c];
    }
  }
}
__device__ inline void dag_load_t(DTile& t, const double* __restrict__ M, int64_t n, int tj, int ti) {
  const int64_t ps = n * n;
  for (int e = threadIdx.x; e < DTS * DTS; e += DAG_THREADS) {
    const int c = e / DTS, r = e % DTS;
    const int64_t gi = (int64_t)tj * DTS + c, gj = (int64_t)ti * DTS + r;
    const bool ok = gi < n && gj < n;
    const int64_t o = gi * n + gj;
#pragma unroll
    for (int q = 0; q < 4; ++q) t[q][r][c] = ok ? M[o + q * ps] : 0.0;
  }
}

__device__ inline Qd dldq(const DTile& t, int r, int c) { return Qd{t[0][r][c], t[1][r][c], t[2][r][c], t[3][r][c]}; }
__device__ inline void dstq(DTile& t, int r, int c, Qd v) {
  t[0][r][c] = v.w;
  t[1][r][c] = v.x;
  t[2][r][c] = v.y;
  t[3][r][c] = v.z;
}

// Tile products on the FP64 matrix cores.  Wave w owns the 16 x 16 quadrant
// (16 (w / 2), 16 (w % 2)) of a 32 x 32 product; its accumulators hold, per
// plane, the MFMA 16x16x4 output layout: lane l has column l % 16 and rows
// l / 16 + 4 r.  Each step of four k loads one fragment per plane of each
// operand and issues the sixteen real products of the Hamilton product.
struct DAcc {
  f64x4d p[4];
};
__device__ inline int dq_row(int r) { return 16 * ((threadIdx.x >> 6) >> 1) + ((threadIdx.x & 63) >> 4) + 4 * r; }
__device__ inline int dq_col() { return 16 * ((threadIdx.x >> 6) & 1) + (threadIdx.x & 15); }
__device__ inline void acc_zero(DAcc& a) {
#pragma unroll
  for (int q = 0; q < 4; ++q) a.p[q] = (f64x4d){0, 0, 0, 0};
}
__device__ inline void acc_from_tile(DAcc& a, const DTile& t) {
  const int c = dq_col();
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int r = 0; r < 4; ++r) a.p[q][r] = t[q][dq_row(r)][c];
}
__device__ inline void acc_to_tile(DTile& t, const DAcc& a) {
  const int c = dq_col();
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int r = 0; r < 4; ++r) t[q][dq_row(r)][c] = a.p[q][r];
}
// acc += sgn * X op(Y), op(Y) = Y^H when herm (entries conj(Y[c][k])), else Y
__device__ inline void dag_mfma(DAcc& acc, const DTile& X, const DTile& Y, bool herm, double sgn) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int ar = 16 * (wave >> 1) + (lane & 15), bc = 16 * (wave & 1) + (lane & 15), kl = lane >> 4;
  const double hs = herm ? -1.0 : 1.0;
#pragma unroll 2
  for (int k0 = 0; k0 < DTS; k0 += 4) {
    const int k = k0 + kl;
    // A fragments carry sgn; B fragments the conjugation's signs
    const double a0 = sgn * X[0][ar][k], a1 = sgn * X[1][ar][k], a2 = sgn * X[2][ar][k], a3 = sgn * X[3][ar][k];
    const double b0 = herm ? Y[0][bc][k] : Y[0][k][bc];
    const double b1 = hs * (herm ? Y[1][bc][k] : Y[1][k][bc]);
    const double b2 = hs * (herm ? Y[2][bc][k] : Y[2][k][bc]);
    const double b3 = hs * (herm ? Y[3][bc][k] : Y[3][k][bc]);
    const double n1 = -a1, n2 = -a2, n3 = -a3;
    // plane 0: a0 b0 - a1 b1 - a2 b2 - a3 b3
    acc.p[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc.p[0], 0, 0, 0);
    acc.p[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(n1, b1, acc.p[0], 0, 0, 0);
    acc.p[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(n2, b2, acc.p[0], 0, 0, 0);
    acc.p[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(n3, b3, acc.p[0], 0, 0, 0);
    // plane 1: a1 b0 + a0 b1 - a3 b2 + a2 b3
    acc.p[1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc.p[1], 0, 0, 0);
    acc.p[1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc.p[1], 0, 0, 0);
    acc.p[1] = __builtin_amdgcn_mfma_f64_16x16x4f64(n3, b2, acc.p[1], 0, 0, 0);
    acc.p[1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a2, b3, acc.p[1], 0, 0, 0);
    // plane 2: a2 b0 + a3 b1 + a0 b2 - a1 b3
    acc.p[2] = __builtin_amdgcn_mfma_f64_16x16x4f64(a2, b0, acc.p[2], 0, 0, 0);
    acc.p[2] = __builtin_amdgcn_mfma_f64_16x16x4f64(a3, b1, acc.p[2], 0, 0, 0);
    acc.p[2] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b2, acc.p[2], 0, 0, 0);
    acc.p[2] = __builtin_amdgcn_mfma_f64_16x16x4f64(n1, b3, acc.p[2], 0, 0, 0);
    // plane 3: a3 b0 - a2 b1 + a1 b2 + a0 b3
    acc.p[3] = __builtin_amdgcn_mfma_f64_16x16x4f64(a3, b0, acc.p[3], 0, 0, 0);
    acc.p[3] = __builtin_amdgcn_mfma_f64_16x16x4f64(n2, b1, acc.p[3], 0, 0, 0);
    acc.p[3] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b2, acc.p[3], 0, 0, 0);
    acc.p[3] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b3, acc.p[3], 0, 0, 0);
  }
}

// Factor and invert the 32 x 32 diagonal tile held in T (lower triangle;
// entries past the matrix edge, rows >= w, are made the identity), blocked
// by 16: T = [A 0; B D] = L L^H with
//   A = L_A L_A^H (chol_diag: P_A = L_A^{-1}),  L_B = B P_A^H,
//   D - L_B L_B^H = L_D L_D^H (chol_diag: P_D),
//   P = L^{-1} = [P_A 0; -P_D L_B P_A  P_D],
// the 16 x 16 products one element per thread.  On return T holds P (lower,
// upper part zero).  A pivot that is not finite and positive sets *bad.
struct DagDiag {
  DiagBuf d;
  double rdg[DTS];
};
__device__ void dag_potri(DTile& T, DagDiag& db, int w, int* bad) {
  const int tid = threadIdx.x;
  if (tid >= w && tid < DTS) T[0][tid][tid] = 1.0;  // identity past the edge (the rest there is zero)
  __syncthreads();
  chol_diag(T, db.rdg, db.d, 0, SB, tid, bad);
  __syncthreads();
  const int bi = SB + (tid >> 4), bc = tid & 15;  // this thread's element of the lower-left block
  // L_B[i][c] = sum_{t <= c} B[i][t] conj(P_A[c][t])
  Qd s{0, 0, 0, 0};
  for (int t = 0; t <= bc; ++t) qacc(s, qmul_conj(ldq(T, bi, t), pdiag(T, db.rdg, 0, bc, t)));
  __syncthreads();
  stq(T, bi, bc, s);
  __syncthreads();
  // D[i][c] -= sum_t L_B[i][t] conj(L_B[c][t]) on the lower triangle of D
  {
    const int di = SB + (tid >> 4), dc = SB + (tid & 15);
    if (dc <= di) {
      Qd u = ldq(T, di, dc);
      for (int t = 0; t < SB; ++t) {
        const Qd v = qmul_conj(ldq(T, di, t), ldq(T, dc, t));
        u = Qd{u.w - v.w, u.x - v.x, u.y - v.y, u.z - v.z};
      }
      stq(T, di, dc, u);
    }
  }
  __syncthreads();
  chol_diag(T, db.rdg, db.d, SB, SB, tid, bad);
  __syncthreads();
  // W = L_B P_A (P_A lower: t >= c), then Y = -P_D W (P_D lower: t <= i)
  s = Qd{0, 0, 0, 0};
  for (int t = bc; t < SB; ++t) qacc(s, qmul(ldq(T, bi, t), pdiag(T, db.rdg, 0, t, bc)));
  __syncthreads();
  stq(T, bi, bc, s);
  __syncthreads();
  s = Qd{0, 0, 0, 0};
  for (int t = SB; t <= bi; ++t) qacc(s, qmul(pdiag(T, db.rdg, SB, bi - SB, t - SB), ldq(T, t, bc)));
  __syncthreads();
  stq(T, bi, bc, Qd{-s.w, -s.x, -s.y, -s.z});
  __syncthreads();
  // P into the lower triangle, zeros above
  Qd v[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int e = tid + DAG_THREADS * k, r = e / DTS, c = e % DTS;
    v[k] = Qd{0, 0, 0, 0};
    if (c <= r) {
      if (r < SB) v[k] = pdiag(T, db.rdg, 0, r, c);
      else if (c >= SB) v[k] = pdiag(T, db.rdg, SB, r - SB, c - SB);
      else v[k] = ldq(T, r, c);
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int e = tid + DAG_THREADS * k;
    stq(T, e / DTS, e % DTS, v[k]);
  }
  __syncthreads();
}

__global__ __launch_bounds__(DAG_THREADS) void k_chol_dag(DagArgs g) {
  __shared__ DTile ta, tb;
  __shared__ __align__(16) DagDiag db;
  __shared__ int task_s, bad, timed_out;
  const int tid = threadIdx.x;
  if (tid == 0) {
    task_s = atomicAdd(g.ticket, 1);
    bad = 0;
    timed_out = 0;
  }
  __syncthreads();
  const int64_t t = task_s;
  const int nt = g.nt;
  const bool fact = t < g.nfact;
  const int64_t u0 = fact ? t : t - g.nfact;
  const int b = (int)(u0 % g.nb);
  int64_t u = u0 / g.nb;
  // column-major position of the tile among the lower (factor) or strictly
  // lower (inverse) tiles
  int j = 0;
  while (u >= (fact ? nt - j : nt - 1 - j)) {
    u -= fact ? nt - j : nt - 1 - j;
    ++j;
  }
  const int i = j + (int)u + (fact ? 0 : 1);
  const double* G = g.G + (int64_t)b * g.slab;
  double* L = g.L + (int64_t)b * g.slab;
  double* P = g.P + (int64_t)b * g.slab;
  const int64_t n = g.n;
  DAcc acc;
  if (fact) {
    // S = G_ij - sum_k L_ik L_jk^H, in k order
    dag_load(ta, G, n, i, j);
    __syncthreads();
    acc_from_tile(acc, ta);
    __syncthreads();
    for (int k = 0; k < j; ++k) {
      if (i == j && k == j - 1) {
        // the last tile of the row, L_{j,j-1} = S_{j,j-1} P_{j-1,j-1}^H, is
        // formed here from the factor task's S (the same operands and the
        // same products, so bit for bit its tile) instead of waiting for
        // that task to publish it: one dependency hop less per diagonal step
        dag_wait(g, dag_flag(g, b, 2, j, k), b, &timed_out);
        dag_wait(g, dag_flag(g, b, 0, k, k), b, &timed_out);
        dag_load_t(tb, L, n, k, j);
        dag_load(ta, P, n, k, k);
        __syncthreads();
        DAcc lt;
        acc_zero(lt);
        dag_mfma(lt, tb, ta, true, 1.0);
        __syncthreads();
        acc_to_tile(ta, lt);
        __syncthreads();
        dag_mfma(acc, ta, ta, true, -1.0);
        __syncthreads();
        continue;
      }
      dag_wait(g, dag_flag(g, b, 0, i, k), b, &timed_out);
      if (i != j) dag_wait(g, dag_flag(g, b, 0, j, k), b, &timed_out);
      dag_load(ta, L, n, i, k);
      if (i != j) dag_load(tb, L, n, j, k);
      __syncthreads();
      dag_mfma(acc, ta, i != j ? tb : ta, true, -1.0);
      __syncthreads();
    }
    acc_to_tile(ta, acc);
    __syncthreads();
    if (i == j + 1) {
      // S_{j+1,j} for the next diagonal task
      dag_store_tile_t(L, n, j, i, ta);
      dag_publish(dag_flag(g, b, 2, i, j));
    }
    if (i == j) {
      const int w = (int)std::min<int64_t>(DTS, n - (int64_t)j * DTS);
      dag_potri(ta, db, w, &bad);
      dag_store_tile(P, n, j, j, ta);
      // the tiles of P right of the diagonal are zero
      for (int tj = j + 1; tj < nt; ++tj) dag_store_zero(P, n, j, tj);
    } else {
      // L_ij = S P_jj^H (P_jj lower triangular)
      dag_wait(g, dag_flag(g, b, 0, j, j), b, &timed_out);
      dag_load(tb, P, n, j, j);
      __syncthreads();
      acc_zero(acc);
      dag_mfma(acc, ta, tb, true, 1.0);
      __syncthreads();
      acc_to_tile(ta, acc);
      __syncthreads();
      dag_store_tile(L, n, i, j, ta);
    }
    if (tid == 0 && (bad || timed_out)) atomicOr(g.fail + b, 1);
    if (tid == 0 && timed_out) atomicOr(g.status, ST_NUMERIC);
    dag_publish(dag_flag(g, b, 0, i, j));
  } else {
    // P_ij = -P_ii sum_{l=j}^{i-1} L_il P_lj, in l order
    acc_zero(acc);
    for (int l = j; l < i; ++l) {
      dag_wait(g, dag_flag(g, b, 0, i, l), b, &timed_out);
      dag_wait(g, l == j ? dag_flag(g, b, 0, j, j) : dag_flag(g, b, 1, l, j), b, &timed_out);
      dag_load(ta, L, n, i, l);
      dag_load(tb, P, n, l, j);
      __syncthreads();
      dag_mfma(acc, ta, tb, false, 1.0);
      __syncthreads();
    }
    acc_to_tile(tb, acc);
    dag_wait(g, dag_flag(g, b, 0, i, i), b, &timed_out);
    dag_load(ta, P, n, i, i);
    __syncthreads();
    acc_zero(acc);
    dag_mfma(acc, ta, tb, false, -1.0);
    __syncthreads();
    acc_to_tile(ta, acc);
    __syncthreads();
    dag_store_tile(P, n, i, j, ta);
    if (tid == 0 && timed_out) {
      atomicOr(g.fail + b, 1);
      atomicOr(g.status, ST_NUMERIC);
    }
    dag_publish(dag_flag(g, b, 1, i, j));
  }
}

size_t chol_dag_flag_ints(int nb, int64_t n) {
  const int64_t nt = (n + DTS - 1) / DTS;
  return (size_t)nb * 3 * nt * nt + 1;
}

hipError_t launch_chol_dag(const Ctx& c, const double* G, double* L, double* P, int64_t n, int64_t slab, int nb,
                           int* flags, int* fail) {
  const int nt = (int)((n + DTS - 1) / DTS);
  DagArgs g;
  g.G = G;
  g.L = L;
  g.P = P;
  g.n = n;
  g.slab = slab;
  g.nb = nb;
  g.nt = nt;
  g.nfact = (int64_t)nb * nt * (nt + 1) / 2;
  g.flags = flags;
  g.ticket = flags + (chol_dag_flag_ints(nb, n) - 1);
  g.fail = fail;
  g.status = c.status;
  hipError_t e = launch_zero_i32(c, flags, (int64_t)chol_dag_flag_ints(nb, n));
  if (e != hipSuccess) return e;
  const int64_t tasks = (int64_t)nb * nt * nt;
  hipLaunchKernelGGL(k_chol_dag, dim3((unsigned)tasks), dim3(DAG_THREADS), 0, c.stream, g);
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
// matrices (n x n, sbatch apart, lower triangle valid): the orthogonality
// defect of Q after a CholeskyQR pass (G = Q^H Q).  Grid (SUMSQ_BLOCKS, nb) of partial sums,
// then the fixed-order fold of the sums of squares.
struct DefectBatch {
  int q[MAXB];
};
__global__ __launch_bounds__(256) void k_defect(const double* __restrict__ G, int64_t n, int64_t sbatch,
                                                DefectBatch db, double* partials) {
  __shared__ double red[4];
  const int b = blockIdx.y, tid = threadIdx.x;
  const int64_t q = db.q[b], nn = n * n;
  const double* g = G + (int64_t)b * sbatch;
  double s = 0.0;
  // G is Hermitian and only its lower triangle is formed: off-diagonal
  // entries count twice
  for (int64_t e = (int64_t)blockIdx.x * 256 + tid; e < q * q; e += (int64_t)gridDim.x * 256) {
    const int64_t i = e / q, j = e % q;
    if (j > i) continue;
    const int64_t o = i * n + j;
    const double d0 = g[o] - (i == j ? 1.0 : 0.0);
    const double v = d0 * d0 + g[o + nn] * g[o + nn] + g[o + 2 * nn] * g[o + 2 * nn] + g[o + 3 * nn] * g[o + 3 * nn];
    s += (i == j) ? v : 2.0 * v;
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o, 64);
  if ((tid & 63) == 0) red[tid >> 6] = s;
  __syncthreads();
  if (tid == 0) partials[(int64_t)b * gridDim.x + blockIdx.x] = ((red[0] + red[1]) + red[2]) + red[3];
}

hipError_t launch_defect_batch(const Ctx& c, int nb, const double* G, int64_t n, int64_t sbatch, const int64_t* q,
                               double* partials, double* out, int ostride) {
  DefectBatch db{};
  for (int b = 0; b < nb; ++b) db.q[b] = (int)q[b];
  hipLaunchKernelGGL(k_defect, dim3(SUMSQ_BLOCKS, nb), dim3(256), 0, c.stream, G, n, sbatch, db, partials);
  hipLaunchKernelGGL(k_fold_batch, dim3(nb), dim3(256), 0, c.stream, (const double*)partials, SUMSQ_BLOCKS, out,
                     ostride);
  return hipGetLastError();
}

}  // namespace qcur
