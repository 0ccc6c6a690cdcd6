// Quaternion matrix product on gfx950 matrix cores.
//
// D = alpha * op(A) op(B) + beta * D with op(X) = X or X^H.  A quaternion
// product expands into sixteen real products (Section 2.2 multiplication
// laws):
//   D0 = A0B0 - A1B1 - A2B2 - A3B3      D1 = A1B0 + A0B1 - A3B2 + A2B3
//   D2 = A2B0 + A3B1 + A0B2 - A1B3      D3 = A3B0 - A2B1 + A1B2 + A0B3
// i.e. stack(D) = L(A) stack(B) with the 4x4 signed block matrix L(A).  The
// kernel never materialises L(A): each wave loads the four planes of its A
// and B fragments once per k-step, forms -A1, -A2, -A3 in registers, and
// issues the sixteen MFMAs, so one quaternion multiply-accumulate costs
// exactly sixteen real ones.
//
// Tiles: a 256-thread workgroup owns a 64 x 64 quaternion output tile (four
// real 64 x 64 planes); each of its four waves owns 32 x 32 (2 x 2 MFMA
// 16x16 blocks per plane).  MFMA shapes: f64 16x16x4, f32 16x16x4,
// bf16 16x16x32 (FP32 accumulation).  K is staged through two LDS buffers
// in slices of 16 (f32/f64) or 32 (bf16): the MFMAs of one slice overlap the
// store of the next and the global loads of the one after.
//
// Epilogues: (a) store alpha*acc + beta*D, or a split-K partial;
// (b) residual: subtract the tile of A, apply the mask, square and reduce
// in FP64 to one partial per workgroup, optionally writing e_scale*(A-CUR).
#include <algorithm>

#include "qcur_internal.hpp"

namespace qcur {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

constexpr int NT = 256;

template <int DT> struct MT;
template <> struct MT<QCUR_F64> {
  typedef double In;
  typedef double Acc;
  typedef f64x4 AccV;
  typedef double Frag;
  static constexpr int BK = 16, KM = 4, PAD = 1;
  // output element r of lane l sits at row (l/16) + 4r (rows interleaved)
  static __device__ inline int out_row(int lane, int r) { return (lane >> 4) + 4 * r; }
  static __device__ inline AccV mfma(Frag a, Frag b, AccV c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ inline Frag neg(Frag a) { return -a; }
};
template <> struct MT<QCUR_F32> {
  typedef float In;
  typedef float Acc;
  typedef f32x4 AccV;
  typedef float Frag;
  static constexpr int BK = 16, KM = 4, PAD = 1;
  // output element r of lane l sits at row 4(l/16) + r
  static __device__ inline int out_row(int lane, int r) { return (lane >> 4) * 4 + r; }
  static __device__ inline AccV mfma(Frag a, Frag b, AccV c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ inline Frag neg(Frag a) { return -a; }
};
template <> struct MT<QCUR_BF16> {
  typedef uint16_t In;
  typedef float Acc;
  typedef f32x4 AccV;
  typedef bf16x8 Frag;
  static constexpr int BK = 32, KM = 32, PAD = 0;
  static __device__ inline int out_row(int lane, int r) { return (lane >> 4) * 4 + r; }
  static __device__ inline AccV mfma(Frag a, Frag b, AccV c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
  static __device__ inline Frag neg(Frag a) {
    u32x4 u = __builtin_bit_cast(u32x4, a);
    u ^= (u32x4){0x80008000u, 0x80008000u, 0x80008000u, 0x80008000u};
    return __builtin_bit_cast(Frag, u);
  }
};

// Split BF16: FP32 operands, each element x staged as hi = bf16(x) and
// lo = bf16(x - hi); a product is hi.hi + hi.lo + lo.hi on BF16 MFMAs with
// FP32 accumulation (the lo.lo term is below FP32 rounding of the sum).
template <> struct MT<QCUR_BF16X3> {
  typedef float In;
  typedef float Acc;
  typedef f32x4 AccV;
  typedef bf16x8 Frag;
  static constexpr int BK = 32, KM = 32, PAD = 8;
  static __device__ inline int out_row(int lane, int r) { return (lane >> 4) * 4 + r; }
  static __device__ inline AccV mfma(Frag a, Frag b, AccV c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
  static __device__ inline Frag neg(Frag a) { return MT<QCUR_BF16>::neg(a); }
};

template <typename T> __device__ inline T negv(T v);
template <> __device__ inline double negv<double>(double v) { return -v; }
template <> __device__ inline float negv<float>(float v) { return -v; }
template <> __device__ inline uint16_t negv<uint16_t>(uint16_t v) { return (uint16_t)(v ^ 0x8000u); }

struct GemmArgs {
  const void* A;
  int64_t lda, psa;
  const void* B;
  int64_t ldb, psb;
  void* D;
  int64_t ldd, psd;
  int64_t M, N, K;  // grid extents (the largest problem of a batch)
  int opA, opB;
  double alpha, beta;
  int ktiles_per_split;
  int splits;
  // batches: problem b uses pointers offset by b * stride and, when the dims
  // arrays are given, its own (M, N, K) <= the grid extents
  int batch;
  int64_t sA, sB, sD, sR0, sE, sMask;
  const int* bM;
  const int* bN;
  const int* bK;
  // residual epilogue
  const void* R0;  // the matrix subtracted from (A of the residual)
  int r0dt;
  int64_t r0ld, r0ps;
  const uint8_t* mask;
  int64_t mask_ld;
  double* partials;
  void* E;
  int edt;
  int64_t eld, eps;
  double e_scale;
  // optional copy of the product tile itself (C U R) next to E
  void* Bo;
  int bodt;
  int64_t bold, bops, sBo;
  // BF16: operands are 16-byte aligned with row, plane and batch strides that
  // are multiples of 8, so eight consecutive elements load as one vector
  int vec;
  // launch plan overrides (0: automatic)
  int force_tile, force_splits;
  // per-problem device flags: problem b is not computed when skip[b] != 0
  // (its result was not needed after all; tiles and partials of it are left
  // unwritten)
  const int* skip;
  // triangular structure of op(A), op(B) and of the wanted output (TRI_*)
  int tri;
  // batches with per-problem sizes: the problems in the order their tiles
  // are handed out (largest first; NULL: the grid mapping)
  const int* order;
  // merge epilogue (completion step): X0 = current iterate, partials2
  const void* X0;
  int x0dt;
  int64_t x0ld, x0ps;
  double* partials2;
};

enum { EPI_STORE = 0, EPI_PARTIAL = 1, EPI_RESID = 2, EPI_MERGE = 3 };

// LDS layouts: [i][k] (A) and [j][k] (B), rows of BK + PAD elements.
// f32/f64 (PAD 1, an odd row length in elements): the 16 lanes of an MFMA
// operand read 16 different rows at the same k and the staging stores of
// consecutive threads hit consecutive or odd-strided addresses, so neither
// conflicts on the LDS banks.  bf16: each lane reads its 8 consecutive k
// values (one 16-byte chunk) at once; rows are 64 bytes without padding and
// the four chunks of row r are stored in the order chunk ^ ((r >> 2) & 3),
// so that the eight rows read in one LDS cycle fall on distinct banks.  The
// unpadded stages (64 KiB for 64 x 64 tiles) let two workgroups share a
// compute unit.
template <int DT, int BM, int BN> struct alignas(16) Smem {
  typedef typename MT<DT>::In In;
  static constexpr int BK = MT<DT>::BK, PAD = MT<DT>::PAD;
  static constexpr bool KMAJ = false;
  static constexpr int AR = KMAJ ? BK : BM, AC = KMAJ ? BM + PAD : BK + PAD;
  static constexpr int BR = KMAJ ? BK : BN, BC = KMAJ ? BN + PAD : BK + PAD;
  In a[2][4][AR][AC];  // two stages: one is read by the MFMAs while the
  In b[2][4][BR][BC];  // next K slice is stored into the other
};

// Split BF16: both halves of each staged FP32 element, [stage][hi, lo][plane][row][k]
template <int BM, int BN> struct alignas(16) Smem<QCUR_BF16X3, BM, BN> {
  static constexpr int BK = 32, PAD = 8;
  static constexpr bool KMAJ = false;
  uint16_t a[2][2][4][BM][BK + PAD];
  uint16_t b[2][2][4][BN][BK + PAD];
};

// element offset of k-chunk c (8 bf16) in row r of a BF16 stage
__device__ inline int bf16_chunk(int r, int c) { return (c ^ ((r >> 2) & 3)) * 8; }

template <int DT, int EPI, int BM, int BN>
__device__ __forceinline__ void gemm_tile(const GemmArgs& g, int b, int64_t tile_m, int64_t tile_n, int split,
                                          int64_t part_index, Smem<DT, BM, BN>& sm) {
  typedef MT<DT> T;
  typedef typename T::In In;
  typedef typename T::AccV AccV;
  typedef typename T::Frag Frag;
  constexpr int BK = T::BK;
  constexpr bool KMAJ = Smem<DT, BM, BN>::KMAJ;
  constexpr int EA = BM * BK / NT;  // elements per thread per plane
  constexpr int EB = BK * BN / NT;
  // waves: 2 x 2 on square tiles (each 32 x 32 or 16 x 16), 4 x 1 on the
  // 64 x 80 tile (each 16 x 80); XB x YB MFMA 16x16 blocks per wave
  constexpr int WM = BM == BN ? 2 : 4, WN = 4 / WM;
  constexpr int XB = BM / (16 * WM), YB = BN / (16 * WN);
  static_assert(XB >= 1 && YB >= 1 && XB * 16 * WM == BM && YB * 16 * WN == BN, "tile shape");
  static_assert(BM * BK % NT == 0 && BN * BK % NT == 0, "whole elements per thread");

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = (wave / WN) * (BM / WM), wn = (wave % WN) * (BN / WN);
  const int64_t bm = tile_m * BM, bn = tile_n * BN;
  const int64_t M = g.bM ? (int64_t)g.bM[b] : g.M;
  const int64_t N = g.bN ? (int64_t)g.bN[b] : g.N;
  const int64_t K = g.bK ? (int64_t)g.bK[b] : g.K;
  if (bm >= M || bn >= N) {  // uniform over the workgroup
    if ((EPI == EPI_RESID || EPI == EPI_MERGE) && threadIdx.x == 0) g.partials[part_index] = 0.0;
    if (EPI == EPI_MERGE && threadIdx.x == 0) g.partials2[part_index] = 0.0;
    return;
  }
  const In* __restrict__ Ag = (const In*)g.A + (int64_t)b * g.sA;
  const In* __restrict__ Bg = (const In*)g.B + (int64_t)b * g.sB;

  const int64_t ktiles = (K + BK - 1) / BK;
  int64_t kt0 = (int64_t)split * g.ktiles_per_split;
  int64_t kt1 = min(ktiles, kt0 + g.ktiles_per_split);
  if (g.tri) {
    // triangular operands: only the K steps that can meet nonzeros (an
    // empty range leaves an exact zero tile)
    if (g.tri & TRI_A_LOWER) kt1 = min(kt1, (bm + BM + BK - 1) / BK);
    if (g.tri & TRI_A_UPPER) kt0 = max(kt0, bm / BK);
    if (g.tri & TRI_B_UPPER) kt1 = min(kt1, (bn + BN + BK - 1) / BK);
    if (g.tri & TRI_B_LOWER) kt0 = max(kt0, bn / BK);
    // lower triangle wanted only: tiles wholly above the diagonal are left
    // alone (split-K partials still write their zero tile)
    if ((g.tri & TRI_LOWER_OUT) && bm + BM <= bn) {
      if (EPI != EPI_PARTIAL) return;
      kt1 = kt0;
    }
  }

  In ra[4][EA], rb[4][EB];

  auto load_tiles = [&](int64_t kt) {
    const int64_t k0 = kt * BK;
#pragma unroll
    for (int r = 0; r < EA; ++r) {
      const int e = tid + NT * r;
      int i, k;
      if (g.opA == QCUR_OP_N) { i = e / BK; k = e % BK; } else { i = e % BM; k = e / BM; }
      const int64_t gi = bm + i, gk = k0 + k;
      const bool ok = gi < M && gk < K;
      const int64_t off = (g.opA == QCUR_OP_N) ? gi * g.lda + gk : gk * g.lda + gi;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        ra[q][r] = ok ? Ag[off + q * g.psa] : (In)0;
      }
    }
#pragma unroll
    for (int r = 0; r < EB; ++r) {
      const int e = tid + NT * r;
      int k, j;
      if (g.opB == QCUR_OP_N) { k = e / BN; j = e % BN; } else { k = e % BK; j = e / BK; }
      const int64_t gk = k0 + k, gj = bn + j;
      const bool ok = gk < K && gj < N;
      const int64_t off = (g.opB == QCUR_OP_N) ? gk * g.ldb + gj : gj * g.ldb + gk;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        rb[q][r] = ok ? Bg[off + q * g.psb] : (In)0;
      }
    }
  };
  auto store_tiles = [&](int st) {
#pragma unroll
    for (int r = 0; r < EA; ++r) {
      const int e = tid + NT * r;
      int i, k;
      if (g.opA == QCUR_OP_N) { i = e / BK; k = e % BK; } else { i = e % BM; k = e / BM; }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        // conjugation (op H) is applied here, not at the load, so that the
        // loads stay in flight through the MFMAs of the current slice
        const In v = (g.opA == QCUR_OP_H && q > 0) ? negv<In>(ra[q][r]) : ra[q][r];
        if constexpr (DT == QCUR_BF16X3) {
          const uint16_t hi = f32_to_bf16(v);
          sm.a[st][0][q][i][k] = hi;
          sm.a[st][1][q][i][k] = f32_to_bf16(v - bf16_to_f32(hi));
        } else {
          if (KMAJ) sm.a[st][q][k][i] = v; else sm.a[st][q][i][k] = v;
        }
      }
    }
#pragma unroll
    for (int r = 0; r < EB; ++r) {
      const int e = tid + NT * r;
      int k, j;
      if (g.opB == QCUR_OP_N) { k = e / BN; j = e % BN; } else { k = e % BK; j = e / BK; }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const In v = (g.opB == QCUR_OP_H && q > 0) ? negv<In>(rb[q][r]) : rb[q][r];
        if constexpr (DT == QCUR_BF16X3) {
          const uint16_t hi = f32_to_bf16(v);
          sm.b[st][0][q][j][k] = hi;
          sm.b[st][1][q][j][k] = f32_to_bf16(v - bf16_to_f32(hi));
        } else {
          if (KMAJ) sm.b[st][q][k][j] = v; else sm.b[st][q][j][k] = v;
        }
      }
    }
  };

  AccV acc[4][XB][YB];
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int x = 0; x < XB; ++x)
#pragma unroll
      for (int y = 0; y < YB; ++y) acc[p][x][y] = (AccV){0, 0, 0, 0};

  // BF16 operands.  One stored contiguous in k (A op N, B op H) moves as
  // whole 8-element vectors, one 16-byte load per plane and thread, stored
  // unchanged.  An operand stored contiguous in i or j (A op
  // H, B op N) is moved in 4 (k) x 8 (i or j) blocks, one plane per wave:
  // a lane loads four 16-byte rows, transposes them in registers and writes
  // eight 8-byte k-runs into the [i][k] / [j][k] layout.  Vectors or blocks
  // that cross a matrix edge, or operands without that alignment, fall back
  // to element loads.
  // NV: 16-byte vectors per plane and thread (k-contiguous) = 4 x 8 blocks
  // per lane (x-contiguous)
  static_assert(BM == BN || (DT != QCUR_BF16 && DT != QCUR_BF16X3), "square BF16 tiles");
  static_assert(DT != QCUR_BF16 || BK == T::KM, "one BF16 MFMA k-step per staged slice");
  constexpr int NV = (DT == QCUR_BF16) ? (BM * BK / 8 + NT - 1) / NT : 1;
  u32x4 va[4 * NV], vb[4 * NV];
  constexpr uint32_t SIGN2 = 0x80008000u;
  const bool aligned = g.vec != 0;
  // k-contiguous operand: vector v of plane q holds X[x][k..k+7]
  auto kvec_load = [&](const uint16_t* __restrict__ Xg, int64_t ld, int64_t ps, int64_t x0, int64_t X, int BX,
                       int64_t kbase, int64_t K, u32x4* out) {
#pragma unroll
    for (int r = 0; r < NV; ++r) {
      const int v = tid + NT * r;
      if (v >= BX * BK / 8) break;
      const int x = v / (BK / 8), k = (v % (BK / 8)) * 8;
      const int64_t gx = x0 + x, gk = kbase + k;
      const int64_t off = gx * ld + gk;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        u32x4 w = (u32x4){0, 0, 0, 0};
        if (aligned && gx < X && gk + 7 < K) {
          w = *(const u32x4*)(Xg + off + q * ps);
        } else if (gx < X) {
          uint16_t e[8];
#pragma unroll
          for (int t = 0; t < 8; ++t) e[t] = (gk + t < K) ? Xg[off + t + q * ps] : (uint16_t)0;
          w = __builtin_bit_cast(u32x4, e);
        }
        out[4 * r + q] = w;
      }
    }
  };
  // okbits: bit r clear zeroes vector r (a clamped load past K)
  auto kvec_store = [&](In (*dst)[BK + T::PAD], int BX, const u32x4* in, bool conj, int plane_stride_rows,
                        uint32_t okbits) {
#pragma unroll
    for (int r = 0; r < NV; ++r) {
      const int v = tid + NT * r;
      if (v >= BX * BK / 8) break;
      const int x = v / (BK / 8), k = (v % (BK / 8)) * 8;
      const bool ok = (okbits >> r) & 1u;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        u32x4 w = ok ? in[4 * r + q] : (u32x4){0, 0, 0, 0};
        if (conj && q > 0) w ^= (u32x4){SIGN2, SIGN2, SIGN2, SIGN2};
        const int row = q * plane_stride_rows + x;
        *(u32x4*)&dst[row][bf16_chunk(row, k / 8)] = w;
      }
    }
  };
  // x-contiguous operand: lane l of wave q takes rows k0..k0+3 of X[k][x0..x0+7].
  // Consecutive lanes take consecutive k blocks of one x block: a load
  // instruction covers the same eight whole 128-byte rows of X as with the x
  // blocks fastest, while the eight lanes sharing an x block write one
  // contiguous 64-byte run of an LDS row, so the 16 lanes of an LDS write
  // cycle hit distinct banks (x blocks fastest put rows 8 apart, 32 banks
  // apart at this row length, into the same cycle).
  auto xblk_load = [&](const uint16_t* __restrict__ Xg, int64_t ld, int64_t ps, int64_t xbase, int64_t X, int BX,
                       int64_t kbase, int64_t K, u32x4* out) {
    const int xbl = BX / 8;
    const uint16_t* base = Xg + wave * ps;
#pragma unroll
    for (int n = 0; n < NV; ++n) {
      const int blk = lane + 64 * n;
      if (blk >= (BK / 4) * xbl) break;
      const int k0 = (blk % (BK / 4)) * 4, x0 = (blk / (BK / 4)) * 8;
      const int64_t gx = xbase + x0;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t gk = kbase + k0 + r;
        const int64_t off = gk * ld + gx;
        u32x4 w = (u32x4){0, 0, 0, 0};
        if (aligned && gk < K && gx + 7 < X) {
          w = *(const u32x4*)(base + off);
        } else if (gk < K) {
          uint16_t e[8];
#pragma unroll
          for (int t = 0; t < 8; ++t) e[t] = (gx + t < X) ? base[off + t] : (uint16_t)0;
          w = __builtin_bit_cast(u32x4, e);
        }
        out[4 * n + r] = w;
      }
    }
  };
  // okbits: bit 4n + r clear zeroes row r of block n (a clamped load past K)
  auto xblk_store = [&](In (*dst)[BK + T::PAD], int BX, const u32x4* in, bool conj, int plane_stride_rows,
                        uint32_t okbits) {
    const int xbl = BX / 8;
    const uint32_t flip = (conj && wave > 0) ? SIGN2 : 0u;
#pragma unroll
    for (int n = 0; n < NV; ++n) {
    const int blk = lane + 64 * n;
    if (blk >= (BK / 4) * xbl) break;
    const int k0 = (blk % (BK / 4)) * 4, x0 = (blk / (BK / 4)) * 8;
#pragma unroll
    for (int d = 0; d < 4; ++d) {
      const uint32_t r0 = ((okbits >> (4 * n)) & 1u) ? in[4 * n][d] : 0u;
      const uint32_t r1 = ((okbits >> (4 * n + 1)) & 1u) ? in[4 * n + 1][d] : 0u;
      const uint32_t r2 = ((okbits >> (4 * n + 2)) & 1u) ? in[4 * n + 2][d] : 0u;
      const uint32_t r3 = ((okbits >> (4 * n + 3)) & 1u) ? in[4 * n + 3][d] : 0u;
      // element 2d (low halves) and 2d+1 (high halves) of the four k rows
      const uint32_t lo0 = ((r0 & 0xFFFFu) | (r1 << 16)) ^ flip, hi0 = ((r2 & 0xFFFFu) | (r3 << 16)) ^ flip;
      const uint32_t lo1 = ((r0 >> 16) | (r1 & 0xFFFF0000u)) ^ flip, hi1 = ((r2 >> 16) | (r3 & 0xFFFF0000u)) ^ flip;
      typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
      // rows 2d and 2d + 1 of the x block; lanes of odd x blocks write the
      // odd row first, so that the two x blocks of one LDS write cycle
      // (64-byte rows: banks repeat every four rows) never share banks
      const bool odd = (x0 >> 3) & 1;
      const int ra = wave * plane_stride_rows + x0 + 2 * d + (odd ? 1 : 0);
      const int rb2 = wave * plane_stride_rows + x0 + 2 * d + (odd ? 0 : 1);
      const int kc = k0 / 8, ko = k0 & 7;
      *(u32x2*)&dst[ra][bf16_chunk(ra, kc) + ko] = odd ? (u32x2){lo1, hi1} : (u32x2){lo0, hi0};
      *(u32x2*)&dst[rb2][bf16_chunk(rb2, kc) + ko] = odd ? (u32x2){lo0, hi0} : (u32x2){lo1, hi1};
    }
    }
  };
  auto vec_load = [&](int64_t kt) {
    if constexpr (DT == QCUR_BF16) {
      const int64_t k0 = kt * BK;
      if (g.opA == QCUR_OP_N) kvec_load(Ag, g.lda, g.psa, bm, M, BM, k0, K, va);
      else xblk_load(Ag, g.lda, g.psa, bm, M, BM, k0, K, va);
      if (g.opB == QCUR_OP_H) kvec_load(Bg, g.ldb, g.psb, bn, N, BN, k0, K, vb);
      else xblk_load(Bg, g.ldb, g.psb, bn, N, BN, k0, K, vb);
    }
  };
  // Interior tiles of aligned operands (with K a multiple of 8 when an
  // operand is contiguous in k): every vector load is unconditional, from a
  // clamped in-range address when its k lies past K, and such data is
  // zeroed at the LDS store.  With no branch around a load its value stays
  // in the register it was loaded into, so the wait for it falls at the LDS
  // store one K step later instead of right after the load (a load path
  // that merges with the element path needs a register copy, hence an
  // immediate wait that exposes the whole load latency every step).
  uint32_t oka = ~0u, okb = ~0u;
  auto kvec_load_fast = [&](const uint16_t* __restrict__ Xg, int64_t ld, int64_t ps, int64_t x0, int BX,
                            int64_t kbase, int64_t K, u32x4* out, uint32_t& okbits) {
    const int nvec = BX * BK / 8;
    okbits = 0;
#pragma unroll
    for (int r = 0; r < NV; ++r) {
      const int v = (tid + NT * r) % nvec;  // lanes past nvec repeat a load and store nothing
      const int x = v / (BK / 8), k = (v % (BK / 8)) * 8;
      const int64_t gk = kbase + k;
      const bool ok = gk < K;
      const int64_t off = (x0 + x) * ld + (ok ? gk : 0);
#pragma unroll
      for (int q = 0; q < 4; ++q) out[4 * r + q] = *(const u32x4*)(Xg + off + q * ps);
      okbits |= (ok ? 1u : 0u) << r;
    }
  };
  auto xblk_load_fast = [&](const uint16_t* __restrict__ Xg, int64_t ld, int64_t ps, int64_t xbase, int BX,
                            int64_t kbase, int64_t K, u32x4* out, uint32_t& okbits) {
    const int nblk = (BK / 4) * (BX / 8);
    const uint16_t* base = Xg + wave * ps;
    okbits = 0;
#pragma unroll
    for (int n = 0; n < NV; ++n) {
      const int blk = (lane + 64 * n) % nblk;  // lanes past nblk repeat a load and store nothing
      const int k0 = (blk % (BK / 4)) * 4, x0 = (blk / (BK / 4)) * 8;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t gk = kbase + k0 + r;
        const bool ok = gk < K;
        out[4 * n + r] = *(const u32x4*)(base + (ok ? gk : 0) * ld + xbase + x0);
        okbits |= (ok ? 1u : 0u) << (4 * n + r);
      }
    }
  };
  auto fast_load = [&](int64_t kt) {
    if constexpr (DT == QCUR_BF16) {
      const int64_t k0 = kt * BK;
      if (g.opA == QCUR_OP_N) kvec_load_fast(Ag, g.lda, g.psa, bm, BM, k0, K, va, oka);
      else xblk_load_fast(Ag, g.lda, g.psa, bm, BM, k0, K, va, oka);
      if (g.opB == QCUR_OP_H) kvec_load_fast(Bg, g.ldb, g.psb, bn, BN, k0, K, vb, okb);
      else xblk_load_fast(Bg, g.ldb, g.psb, bn, BN, k0, K, vb, okb);
    }
  };
  auto vec_store = [&](int st) {
    if constexpr (DT == QCUR_BF16) {
      if (g.opA == QCUR_OP_N) kvec_store(sm.a[st][0], BM, va, false, BM, oka);
      else xblk_store(sm.a[st][0], BM, va, true, BM, oka);
      if (g.opB == QCUR_OP_H) kvec_store(sm.b[st][0], BN, vb, true, BN, okb);
      else xblk_store(sm.b[st][0], BN, vb, false, BN, okb);
    }
  };

  // Pipeline: while the MFMAs read stage st, the slice kt+1 (in registers
  // since the previous step) goes to stage st^1 and slice kt+2 is fetched;
  // one barrier per K step.
  auto run = [&](auto&& load, auto&& store) {
    if (kt0 < kt1) {
      load(kt0);
      store(0);
      if (kt0 + 1 < kt1) load(kt0 + 1);
    }
    __syncthreads();
    for (int64_t kt = kt0; kt < kt1; ++kt) {
      const int st = (int)((kt - kt0) & 1);
      if (kt + 1 < kt1) {
        store(st ^ 1);
        if (kt + 2 < kt1) load(kt + 2);
      }
#pragma unroll
      for (int kk = 0; kk < BK / T::KM; ++kk) {
        // one quaternion multiply-accumulate of the fragments: sixteen MFMAs
        auto qmac = [&](const Frag (&a)[4][XB], const Frag (&na)[4][XB], const Frag (&b)[4][YB]) {
#pragma unroll
          for (int x = 0; x < XB; ++x)
#pragma unroll
            for (int y = 0; y < YB; ++y) {
              // plane 0: A0B0 - A1B1 - A2B2 - A3B3
              acc[0][x][y] = T::mfma(a[0][x], b[0][y], acc[0][x][y]);
              acc[0][x][y] = T::mfma(na[1][x], b[1][y], acc[0][x][y]);
              acc[0][x][y] = T::mfma(na[2][x], b[2][y], acc[0][x][y]);
              acc[0][x][y] = T::mfma(na[3][x], b[3][y], acc[0][x][y]);
              // plane 1: A1B0 + A0B1 - A3B2 + A2B3
              acc[1][x][y] = T::mfma(a[1][x], b[0][y], acc[1][x][y]);
              acc[1][x][y] = T::mfma(a[0][x], b[1][y], acc[1][x][y]);
              acc[1][x][y] = T::mfma(na[3][x], b[2][y], acc[1][x][y]);
              acc[1][x][y] = T::mfma(a[2][x], b[3][y], acc[1][x][y]);
              // plane 2: A2B0 + A3B1 + A0B2 - A1B3
              acc[2][x][y] = T::mfma(a[2][x], b[0][y], acc[2][x][y]);
              acc[2][x][y] = T::mfma(a[3][x], b[1][y], acc[2][x][y]);
              acc[2][x][y] = T::mfma(a[0][x], b[2][y], acc[2][x][y]);
              acc[2][x][y] = T::mfma(na[1][x], b[3][y], acc[2][x][y]);
              // plane 3: A3B0 - A2B1 + A1B2 + A0B3
              acc[3][x][y] = T::mfma(a[3][x], b[0][y], acc[3][x][y]);
              acc[3][x][y] = T::mfma(na[2][x], b[1][y], acc[3][x][y]);
              acc[3][x][y] = T::mfma(a[1][x], b[2][y], acc[3][x][y]);
              acc[3][x][y] = T::mfma(a[0][x], b[3][y], acc[3][x][y]);
            }
        };
        if constexpr (DT == QCUR_BF16X3) {
          // hi.hi + hi.lo + lo.hi, the small terms first
          Frag ah[4][XB], nah[4][XB], al[4][XB], nal[4][XB], bh[4][YB], bl[4][YB];
#pragma unroll
          for (int x = 0; x < XB; ++x) {
            const int ii = wm + x * 16 + (lane & 15);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              ah[q][x] = *(const Frag*)&sm.a[st][0][q][ii][(lane >> 4) * 8];
              al[q][x] = *(const Frag*)&sm.a[st][1][q][ii][(lane >> 4) * 8];
            }
#pragma unroll
            for (int q = 1; q < 4; ++q) {
              nah[q][x] = T::neg(ah[q][x]);
              nal[q][x] = T::neg(al[q][x]);
            }
          }
#pragma unroll
          for (int y = 0; y < YB; ++y) {
            const int jj = wn + y * 16 + (lane & 15);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              bh[q][y] = *(const Frag*)&sm.b[st][0][q][jj][(lane >> 4) * 8];
              bl[q][y] = *(const Frag*)&sm.b[st][1][q][jj][(lane >> 4) * 8];
            }
          }
          qmac(al, nal, bh);
          qmac(ah, nah, bl);
          qmac(ah, nah, bh);
        } else {
          Frag a[4][XB], na[4][XB], b[4][YB];
#pragma unroll
          for (int x = 0; x < XB; ++x) {
            const int ii = wm + x * 16 + (lane & 15);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              if constexpr (DT == QCUR_BF16) a[q][x] = *(const Frag*)&sm.a[st][q][ii][bf16_chunk(ii, lane >> 4)];
              else a[q][x] = sm.a[st][q][ii][kk * 4 + (lane >> 4)];
            }
#pragma unroll
            for (int q = 1; q < 4; ++q) na[q][x] = T::neg(a[q][x]);
          }
#pragma unroll
          for (int y = 0; y < YB; ++y) {
            const int jj = wn + y * 16 + (lane & 15);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              if constexpr (DT == QCUR_BF16) b[q][y] = *(const Frag*)&sm.b[st][q][jj][bf16_chunk(jj, lane >> 4)];
              else b[q][y] = sm.b[st][q][jj][kk * 4 + (lane >> 4)];
            }
          }
          qmac(a, na, b);
        }
      }
    __syncthreads();
    }
  };
  // Small tiles of the fused epilogues (one 16 x 16 block per wave) with FP32
  // operands fetch the tile of the matrix they subtract from (and the merge's
  // previous iterate) before the K loop, so that the reads are in flight
  // during the MFMAs instead of starting after them: a short K loop (the
  // batch's residual has K = r <= 64) left them exposed.  Addresses are
  // clamped into the matrix so that every load is unconditional.
  constexpr bool PREF = (EPI == EPI_RESID || EPI == EPI_MERGE) && XB == 1 && YB == 1;
  const bool pref_r0 = PREF && g.r0dt == QCUR_F32;
  const bool pref_x0 = PREF && EPI == EPI_MERGE && g.x0dt == QCUR_F32;
  float r0f[PREF ? 16 : 1], x0f[PREF ? 16 : 1];
  if constexpr (PREF) {
    const int64_t jc = min(bn + wn + (lane & 15), N - 1);
    if (pref_r0) {
      const float* R0 = (const float*)g.R0 + (EPI == EPI_RESID ? b * g.sR0 : 0);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t ic = min(bm + wm + T::out_row(lane, r), M - 1);
#pragma unroll
        for (int p = 0; p < 4; ++p) r0f[4 * r + p] = R0[ic * g.r0ld + jc + p * g.r0ps];
      }
    }
    if (pref_x0) {
      const float* X0 = (const float*)g.X0;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t ic = min(bm + wm + T::out_row(lane, r), M - 1);
#pragma unroll
        for (int p = 0; p < 4; ++p) x0f[4 * r + p] = X0[ic * g.x0ld + jc + p * g.x0ps];
      }
    }
  }
  if constexpr (DT == QCUR_BF16) {
    const bool kvec_op = g.opA == QCUR_OP_N || g.opB == QCUR_OP_H;
    const bool fast = aligned && bm + BM <= M && bn + BN <= N && (!kvec_op || (K & 7) == 0);
    if (fast) run(fast_load, vec_store);
    else run(vec_load, vec_store);
  } else {
    run(load_tiles, store_tiles);
  }

  // Epilogue.  MFMA 16x16 output: lane holds column lane%16 and four rows
  // given by out_row (f32/bf16: 4(lane/16)+r; f64: lane/16 + 4r).
  if constexpr (EPI == EPI_RESID) {
    double sq = 0.0;
#pragma unroll
    for (int x = 0; x < XB; ++x)
#pragma unroll
      for (int y = 0; y < YB; ++y)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t i = bm + wm + x * 16 + T::out_row(lane, r);
          const int64_t j = bn + wn + y * 16 + (lane & 15);
          if (i < M && j < N) {
            const bool keep = g.mask ? (g.mask[b * g.sMask + i * g.mask_ld + j] != 0) : true;
#pragma unroll
            for (int p = 0; p < 4; ++p) {
              const double a0 = pref_r0 ? (double)r0f[PREF ? 4 * r + p : 0]
                                        : load_as_double(g.R0, g.r0dt, b * g.sR0 + i * g.r0ld + j + p * g.r0ps);
              double d = a0 - (double)acc[p][x][y][r];
              if (!keep) d = 0.0;
              sq += d * d;
              if (g.E) store_from_double(g.E, g.edt, b * g.sE + i * g.eld + j + p * g.eps, g.e_scale * d);
              if (g.Bo)
                store_from_double(g.Bo, g.bodt, b * g.sBo + i * g.bold + j + p * g.bops, (double)acc[p][x][y][r]);
            }
          }
        }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) sq += __shfl_xor(sq, o, 64);
    __shared__ double wpart[4];
    if (lane == 0) wpart[wave] = sq;
    __syncthreads();
    if (tid == 0) g.partials[part_index] = ((wpart[0] + wpart[1]) + wpart[2]) + wpart[3];
  } else if constexpr (EPI == EPI_MERGE) {
    // X1 = P_Omega(Y) + P_Omega^c(B) with B the product tile, written in the
    // dtype of X1; per tile, sum |X1 - X0|^2 and |X0|^2 (FP64)
    double sd = 0.0, so = 0.0;
#pragma unroll
    for (int x = 0; x < XB; ++x)
#pragma unroll
      for (int y = 0; y < YB; ++y)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t i = bm + wm + x * 16 + T::out_row(lane, r);
          const int64_t j = bn + wn + y * 16 + (lane & 15);
          if (i < M && j < N) {
            const bool obs = g.mask[i * g.mask_ld + j] != 0;
#pragma unroll
            for (int p = 0; p < 4; ++p) {
              const double xo = pref_x0 ? (double)x0f[PREF ? 4 * r + p : 0]
                                        : load_as_double(g.X0, g.x0dt, i * g.x0ld + j + p * g.x0ps);
              const double yo = pref_r0 ? (double)r0f[PREF ? 4 * r + p : 0]
                                        : load_as_double(g.R0, g.r0dt, i * g.r0ld + j + p * g.r0ps);
              const double xn = obs ? yo : (double)acc[p][x][y][r];
              store_from_double(g.E, g.edt, i * g.eld + j + p * g.eps, xn);
              const double xs = load_as_double(g.E, g.edt, i * g.eld + j + p * g.eps);  // as stored
              sd += (xs - xo) * (xs - xo);
              so += xo * xo;
            }
          }
        }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
      sd += __shfl_xor(sd, o, 64);
      so += __shfl_xor(so, o, 64);
    }
    __shared__ double wpart[2][4];
    if (lane == 0) {
      wpart[0][wave] = sd;
      wpart[1][wave] = so;
    }
    __syncthreads();
    if (tid == 0) {
      g.partials[part_index] = ((wpart[0][0] + wpart[0][1]) + wpart[0][2]) + wpart[0][3];
      g.partials2[part_index] = ((wpart[1][0] + wpart[1][1]) + wpart[1][2]) + wpart[1][3];
    }
  } else {
    typedef typename T::Acc Acc;
    Acc* Dg = (Acc*)g.D;
    int64_t ps = g.psd, ld = g.ldd;
    if (EPI == EPI_PARTIAL) Dg += ((int64_t)b * g.splits + split) * 4 * ps;
    else Dg += (int64_t)b * g.sD;
#pragma unroll
    for (int x = 0; x < XB; ++x)
#pragma unroll
      for (int y = 0; y < YB; ++y)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t i = bm + wm + x * 16 + T::out_row(lane, r);
          const int64_t j = bn + wn + y * 16 + (lane & 15);
          if (i < M && j < N) {
#pragma unroll
            for (int p = 0; p < 4; ++p) {
              const int64_t o = i * ld + j + p * ps;
              if (EPI == EPI_PARTIAL) {
                Dg[o] = acc[p][x][y][r];
              } else {
                double v = g.alpha * (double)acc[p][x][y][r];
                if (g.beta != 0.0) v += g.beta * (double)Dg[o];
                Dg[o] = (Acc)v;
              }
            }
          }
        }
  }
}

// XCD-aware order of the tiles.  Workgroups are handed to the eight XCDs
// round-robin by linear id, and each XCD has its own L2; the logical tile
// index gives every XCD one contiguous range of tiles (column tiles fastest),
// so the tiles that share a row block of A, and the same B, run behind the
// same L2 instead of being spread over all eight.
constexpr int NXCD = 8;
__device__ inline int64_t xcd_tile(int64_t id, int64_t total) {
  const int64_t x = id % NXCD, s = id / NXCD;
  const int64_t per = total / NXCD, rem = total % NXCD;
  return x * per + (x < rem ? x : rem) + s;
}

// grid: x = column tiles, y = row tiles, z = batch * splits (tile order
// remapped per XCD as above)
template <int DT, int EPI, int BM, int BN>
__global__ __launch_bounds__(NT) void k_qgemm(GemmArgs g) {
  __shared__ Smem<DT, BM, BN> sm;
  const int64_t gx = gridDim.x, gy = gridDim.y;
  const int64_t total = gx * gy * gridDim.z;
  const int64_t id = blockIdx.x + gx * (blockIdx.y + gy * (int64_t)blockIdx.z);
  const int64_t L = xcd_tile(id, total);
  const int64_t tx = L % gx, ty = (L / gx) % gy, tz = L / (gx * gy);
  const int b = (int)(tz / g.splits), split = (int)(tz % g.splits);
  if (g.skip && g.skip[b]) return;  // uniform over the workgroup
  const int64_t tiles = gx * gy;
  gemm_tile<DT, EPI, BM, BN>(g, b, ty, tx, split, (int64_t)b * tiles + ty * gx + tx, sm);
}

// Persistent form for batches of uneven problems: a grid of about one
// resident wave of workgroups takes the tiles of all problems as one list,
// problem after problem in the given order (largest first: a longest-
// processing-time order, so that the last tiles to start are short), the
// tiles of one problem in (K slice, row, column) order.  Every workgroup
// builds the prefix sums of the per-problem tile counts in LDS, then takes
// list entries x, x + grid, ... with x its XCD-remapped id, so that each
// XCD works through contiguous runs of the list (the tiles that share rows
// of A and the same B behind one L2).  No tile outside a problem is
// visited.
constexpr int LIST_MAX = 2048;  // problems a list launch takes
template <int DT, int EPI, int BM, int BN>
__global__ __launch_bounds__(NT) void k_qgemm_list(GemmArgs g) {
  __shared__ Smem<DT, BM, BN> sm;
  __shared__ int off[LIST_MAX + 1];
  __shared__ int wsum[NT / 64];
  const int tid = threadIdx.x, count = g.batch;
  const int64_t gx = (g.N + BN - 1) / BN, gy = (g.M + BM - 1) / BM;
  // tiles of the problem at list position k
  auto tiles_of = [&](int k) -> int {
    const int b = g.order[k];
    if (g.skip && g.skip[b]) return 0;  // a skipped problem has no tiles
    const int64_t M = g.bM ? (int64_t)g.bM[b] : g.M, N = g.bN ? (int64_t)g.bN[b] : g.N;
    return (int)(((M + BM - 1) / BM) * ((N + BN - 1) / BN) * g.splits);
  };
  // exclusive prefix sums: thread tid sums its contiguous run of positions,
  // the runs are scanned across the workgroup, then the run is written out
  const int per = (count + NT - 1) / NT, k0 = tid * per, k1 = min(count, k0 + per);
  int run = 0;
  for (int k = k0; k < k1; ++k) run += tiles_of(k);
  int incl = run;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int v = __shfl_up(incl, o, 64);
    if ((tid & 63) >= o) incl += v;
  }
  if ((tid & 63) == 63) wsum[tid >> 6] = incl;
  __syncthreads();
  int base = incl - run;
  for (int w = 0; w < (tid >> 6); ++w) base += wsum[w];
  for (int k = k0; k < k1; ++k) {
    off[k] = base;
    base += tiles_of(k);
  }
  if (tid == NT - 1) off[count] = base;
  __syncthreads();
  const int total = off[count];
  for (int64_t t = xcd_tile(blockIdx.x, gridDim.x); t < total; t += gridDim.x) {
    // the list position holding entry t: the last k with off[k] <= t
    int lo = 0, hi = count - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (off[mid] <= t) lo = mid;
      else hi = mid - 1;
    }
    const int b = g.order[lo];
    const int64_t M = g.bM ? (int64_t)g.bM[b] : g.M, N = g.bN ? (int64_t)g.bN[b] : g.N;
    const int64_t tn = (N + BN - 1) / BN, tm = (M + BM - 1) / BM;
    const int64_t local = t - off[lo];
    const int split = (int)(local / (tm * tn));
    const int64_t rem = local % (tm * tn), ty = rem / tn, tx = rem % tn;
    gemm_tile<DT, EPI, BM, BN>(g, b, ty, tx, split, (int64_t)b * gx * gy + ty * gx + tx, sm);
  }
}

// Launch of the tile kernel: the persistent list form for batches with
// per-problem sizes and an order, else one workgroup per tile of the grid.
int list_workers(const void* kernel, int device) {
  static int cus[64] = {0};
  const int d = device < 0 || device >= 64 ? 0 : device;
  if (cus[d] == 0) {
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, d) != hipSuccess || n <= 0) n = 256;
    cus[d] = n;
  }
  int per = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, NT, 0) != hipSuccess || per <= 0) per = 1;
  return per * cus[d];
}

template <int DT, int EPI, int BM, int BN>
static void launch_tiles(const Ctx& c, const GemmArgs& g, dim3 grid) {
  if constexpr (BM == BN) {  // batches take square tiles only
    if (g.order && g.batch > 1 && g.batch <= LIST_MAX && (g.bM || g.bN)) {
      static int workers = 0;  // per instantiation (the same on every MI355X)
      if (workers == 0) workers = list_workers((const void*)k_qgemm_list<DT, EPI, BM, BN>, c.device);
      const int64_t upper = (int64_t)grid.x * grid.y * grid.z;
      hipLaunchKernelGGL((k_qgemm_list<DT, EPI, BM, BN>), dim3((unsigned)std::min<int64_t>(upper, workers)),
                         dim3(NT), 0, c.stream, g);
      return;
    }
  }
  hipLaunchKernelGGL((k_qgemm<DT, EPI, BM, BN>), grid, dim3(NT), 0, c.stream, g);
}

// Split-K reduction: D = alpha * sum_z P[z] + beta * D, z in fixed order.
template <typename Acc>
__global__ void k_splitk_reduce(const Acc* __restrict__ Pall, int splits, int64_t Mx, int64_t Nx, double alpha,
                                double beta, Acc* Dall, int64_t ldd, int64_t psd, int64_t sD, const int* bM,
                                const int* bN, const int* skip) {
  const int b = blockIdx.z;
  if (skip && skip[b]) return;
  const int64_t M = bM ? bM[b] : Mx, N = bN ? bN[b] : Nx;
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j >= N) return;
  const int64_t MN = Mx * Nx;
  const Acc* P = Pall + (int64_t)b * splits * 4 * MN;
  Acc* D = Dall + (int64_t)b * sD;
  for (int64_t i = blockIdx.y; i < M; i += gridDim.y) {
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      double s = 0.0;
      for (int z = 0; z < splits; ++z) s += (double)P[(int64_t)z * 4 * MN + p * MN + i * Nx + j];
      const int64_t o = i * ldd + j + p * psd;
      double v = alpha * s;
      if (beta != 0.0) v += beta * (double)D[o];
      D[o] = (Acc)v;
    }
  }
}

// Launch plan: 64 x 64 quaternion tiles, or 32 x 32 when 64-tiles would
// leave most of the 256 compute units idle (measured faster on the thin
// products of the solve than 64-tiles split further along K); then K is
// split until the grid covers the chip twice over, keeping at least two
// K-steps per split.
struct Plan {
  int tile, splits;
};
static Plan plan_of(int64_t M, int64_t N, int64_t K, int bk, int batch, int force_tile = 0) {
  const int64_t t64 = ((M + 63) / 64) * ((N + 63) / 64);
  const int tile = force_tile ? force_tile : (t64 >= 192 ? 64 : 32);
  const int64_t tiles = ((M + tile - 1) / tile) * ((N + tile - 1) / tile) * std::max(batch, 1);
  const int64_t kt = (K + bk - 1) / bk;
  int s = 1;
  while (s < 32 && tiles * s < 512 && kt / (s * 2) >= 2) s *= 2;
  return Plan{tile, s};
}

static int bk_of(int compute) { return compute == QCUR_BF16 || compute == QCUR_BF16X3 ? 32 : 16; }

// Single (not batched) FP32 / FP64 products with a tall output (M >= 2048,
// K >= 256: A Q_R, E Q_R and Q_C M of the large solves):
// 64 x 64 tiles, or for FP32 64 x 80 (which covers N = 400 without a padded
// column tile), and 1..8 slices of K, chosen by a cost model: workgroups
// run in rounds of `slots` (two per compute unit when the kernel's LDS and
// registers allow it: FP32 64 x 64, and 64 x 80 writing split-K partials;
// one otherwise), a workgroup costs its K steps plus two of pipeline fill
// times its tile width, and each extra slice adds the partials' write and
// read (about 22 s / K of the product's time).
struct WidePlan {
  int tn, splits;  // tn = 0: not applicable
};
static WidePlan wide_plan(int64_t M, int64_t N, int64_t K, int compute, int batch, bool per_problem) {
  if ((compute != QCUR_F32 && compute != QCUR_F64) || batch != 1 || per_problem || M < 2048 || K < 256 || N < 64)
    return WidePlan{0, 0};
  const int64_t kt = (K + 15) / 16;
  double best = 1e300;
  WidePlan bp{64, 1};
  for (int tn : {64, 80}) {
    if (tn == 80 && compute != QCUR_F32) continue;
    const int64_t tiles = ((M + 63) / 64) * ((N + tn - 1) / tn);
    for (int sp : {1, 2, 3, 4, 6, 8}) {
      if (sp > 1 && kt / sp < 4) break;
      const int64_t slots = compute == QCUR_F32 && (tn == 64 || sp > 1) ? 512 : 256;
      const int64_t per = (kt + sp - 1) / sp;
      const int64_t rounds = (tiles * sp + slots - 1) / slots;
      const double cost = (double)rounds * (double)(per + 2) * tn * (1.0 + (sp > 1 ? 22.0 * sp / (double)K : 0.0));
      if (cost < best * 0.999) {
        best = cost;
        bp = WidePlan{tn, sp};
      }
    }
  }
  return bp;
}
// split BF16 stages two BF16 halves per operand: 32-tiles only
static int tile_of(int compute) { return compute == QCUR_BF16X3 ? 32 : 0; }
static size_t acc_size(int compute) { return compute == QCUR_F64 ? 8 : 4; }

size_t gemm_workspace_splits(int64_t M, int64_t N, int compute, int batch, int max_splits) {
  if (max_splits <= 1) return 0;
  return (size_t)batch * max_splits * 4 * (size_t)M * (size_t)N * acc_size(compute);
}

size_t gemm_workspace(int64_t M, int64_t N, int64_t K, int compute, int batch) {
  // room for either plan (triangular products keep the square-tile plan)
  const WidePlan wp = wide_plan(M, N, K, compute, batch, false);
  const int s = std::max(wp.tn ? wp.splits : 1, plan_of(M, N, K, bk_of(compute), batch, tile_of(compute)).splits);
  if (s <= 1) return 0;
  return (size_t)batch * s * 4 * (size_t)M * (size_t)N * acc_size(compute);
}

template <int DT, int TILE, int TN = TILE>
static hipError_t gemm_dt_tile(const Ctx& c, GemmArgs g, void* ws, size_t ws_bytes, int plan_splits = 0) {
  constexpr int BK = MT<DT>::BK;
  const int64_t kt = (g.K + BK - 1) / BK;
  int splits = g.force_splits > 0 ? g.force_splits
                                  : plan_splits > 0 ? plan_splits : plan_of(g.M, g.N, g.K, BK, g.batch, TILE).splits;
  const size_t need = (size_t)g.batch * splits * 4 * (size_t)g.M * (size_t)g.N * acc_size(DT);
  if (splits > 1 && (ws == nullptr || ws_bytes < need)) splits = 1;
  dim3 grid((unsigned)((g.N + TN - 1) / TN), (unsigned)((g.M + TILE - 1) / TILE), 1);
  if (splits == 1) {
    g.ktiles_per_split = (int)kt;
    g.splits = 1;
    grid.z = g.batch;
    launch_tiles<DT, EPI_STORE, TILE, TN>(c, g, grid);
    return hipGetLastError();
  }
  const int per = (int)((kt + splits - 1) / splits);
  splits = (int)((kt + per - 1) / per);
  grid.z = g.batch * splits;
  g.ktiles_per_split = per;
  g.splits = splits;
  typedef typename MT<DT>::Acc Acc;
  GemmArgs gp = g;
  gp.D = ws;
  gp.ldd = g.N;
  gp.psd = g.M * g.N;
  launch_tiles<DT, EPI_PARTIAL, TILE, TN>(c, gp, grid);
  hipLaunchKernelGGL(k_splitk_reduce<Acc>,
                     dim3((unsigned)((g.N + 255) / 256), (unsigned)std::min<int64_t>(g.M, 65535), (unsigned)g.batch),
                     dim3(256), 0, c.stream, (const Acc*)ws, splits, g.M, g.N, g.alpha, g.beta, (Acc*)g.D, g.ldd,
                     g.psd, g.sD, g.bM, g.bN, g.skip);
  return hipGetLastError();
}

template <int DT>
static hipError_t gemm_dt(const Ctx& c, GemmArgs g, void* ws, size_t ws_bytes) {
  if constexpr (DT == QCUR_F32 || DT == QCUR_F64) {
    if (!g.force_tile && !g.force_splits && !g.tri) {
      const WidePlan wp = wide_plan(g.M, g.N, g.K, DT, g.batch, g.bM || g.bN || g.bK);
      if (wp.tn == 80) return gemm_dt_tile<DT, 64, 80>(c, g, ws, ws_bytes, wp.splits);
      if (wp.tn == 64) return gemm_dt_tile<DT, 64, 64>(c, g, ws, ws_bytes, wp.splits);
    }
  }
  const int tile = g.force_tile ? g.force_tile : plan_of(g.M, g.N, g.K, MT<DT>::BK, g.batch).tile;
  if (tile == 64) return gemm_dt_tile<DT, 64>(c, g, ws, ws_bytes);
  return gemm_dt_tile<DT, 32>(c, g, ws, ws_bytes);
}

static bool vec_ok(const QView& X, int64_t sbatch) {
  return X.dt == QCUR_BF16 && ((uintptr_t)X.p % 16) == 0 && X.ld % 8 == 0 && X.ps % 8 == 0 && sbatch % 8 == 0;
}

hipError_t launch_gemm_batched(const Ctx& c, int opA, int opB, double alpha, QView A, QView B, double beta,
                               QView D, int compute, void* ws, size_t ws_bytes, const BatchSpec& bs) {
  GemmArgs g = {};
  g.batch = bs.count;
  g.sA = bs.sA;
  g.sB = bs.sB;
  g.sD = bs.sD;
  g.bM = bs.M;
  g.bN = bs.N;
  g.bK = bs.K;
  g.force_tile = bs.tile;
  g.tri = bs.tri;
  g.force_splits = bs.splits;
  g.order = bs.order;
  g.skip = bs.skip;
  g.A = A.p; g.lda = A.ld; g.psa = A.ps;
  g.B = B.p; g.ldb = B.ld; g.psb = B.ps;
  g.D = D.p; g.ldd = D.ld; g.psd = D.ps;
  g.M = D.rows; g.N = D.cols;
  g.K = (opA == QCUR_OP_N) ? A.cols : A.rows;
  g.opA = opA; g.opB = opB; g.alpha = alpha; g.beta = beta;
  g.vec = compute == QCUR_BF16 && vec_ok(A, bs.sA) && vec_ok(B, bs.sB);
  if (g.M == 0 || g.N == 0) return hipSuccess;
  if (g.K == 0) {  // D = beta * D
    return launch_axpby(c, 0.0, D, beta, D);
  }
  // tall FP64 products Z P^H with a short K: the run-streaming kernel
  if (bs.tile == 0 && bs.splits == 0 &&
      tall_nh_applies(compute, opA, opB, A, B, g.M, g.N, g.K, g.tri, bs.M || bs.N || bs.K, bs.sA, bs.sB))
    return launch_tall_nh(c, alpha, A, B, beta, D, g.K, g.batch, bs.sA, bs.sB, bs.sD, (g.tri & TRI_B_UPPER) != 0);
  // thin FP64 / FP32 products with a long K (Gram matrices, cores): the
  // fragment-streaming kernel
  if (bs.tile == 0 && bs.splits == 0 && thin_hn_applies(compute, opA, opB, g.M, g.N, g.K, g.tri, bs.M || bs.N || bs.K))
    return launch_thin_hn(c, compute, alpha, A, B, beta, D, g.K, g.batch, bs.sA, bs.sB, bs.sD,
                          (g.tri & TRI_LOWER_OUT) != 0, ws, ws_bytes);
  switch (compute) {
    case QCUR_F64: return gemm_dt<QCUR_F64>(c, g, ws, ws_bytes);
    case QCUR_F32: return gemm_dt<QCUR_F32>(c, g, ws, ws_bytes);
    case QCUR_BF16X3: return gemm_dt_tile<QCUR_BF16X3, 32>(c, g, ws, ws_bytes);
    default: return gemm_dt<QCUR_BF16>(c, g, ws, ws_bytes);
  }
}

hipError_t launch_gemm(const Ctx& c, int opA, int opB, double alpha, QView A, QView B, double beta, QView D,
                       int compute, void* ws, size_t ws_bytes) {
  return launch_gemm_batched(c, opA, opB, alpha, A, B, beta, D, compute, ws, ws_bytes, BatchSpec{});
}

// Tile edge of the fused residual and merge products (no K split: their
// epilogues reduce): 32 when 64-tiles would give fewer than two workgroups
// per compute unit, and always for split BF16.
static int resid_tile(int64_t m, int64_t n, int compute) {
  if (compute == QCUR_BF16X3) return 32;
  return ((m + 63) / 64) * ((n + 63) / 64) < 512 ? 32 : 64;
}

size_t residual_tiles(int64_t m, int64_t n, int compute) {
  const int64_t t = resid_tile(m, n, compute);
  return (size_t)((m + t - 1) / t) * (size_t)((n + t - 1) / t);
}

// One launch of the fused epilogue product on tiles of edge t.
template <int EPI>
static void launch_fused(const Ctx& c, GemmArgs& g, int compute, int t) {
  const dim3 grid((unsigned)((g.N + t - 1) / t), (unsigned)((g.M + t - 1) / t), 1);
  switch (compute) {
    case QCUR_F64:
      g.ktiles_per_split = (int)((g.K + 15) / 16);
      if (t == 64) hipLaunchKernelGGL((k_qgemm<QCUR_F64, EPI, 64, 64>), grid, dim3(NT), 0, c.stream, g);
      else hipLaunchKernelGGL((k_qgemm<QCUR_F64, EPI, 32, 32>), grid, dim3(NT), 0, c.stream, g);
      break;
    case QCUR_F32:
      g.ktiles_per_split = (int)((g.K + 15) / 16);
      if (t == 64) hipLaunchKernelGGL((k_qgemm<QCUR_F32, EPI, 64, 64>), grid, dim3(NT), 0, c.stream, g);
      else hipLaunchKernelGGL((k_qgemm<QCUR_F32, EPI, 32, 32>), grid, dim3(NT), 0, c.stream, g);
      break;
    case QCUR_BF16X3:
      g.ktiles_per_split = (int)((g.K + 31) / 32);
      hipLaunchKernelGGL((k_qgemm<QCUR_BF16X3, EPI, 32, 32>), grid, dim3(NT), 0, c.stream, g);
      break;
    default:
      g.ktiles_per_split = (int)((g.K + 31) / 32);
      if (t == 64) hipLaunchKernelGGL((k_qgemm<QCUR_BF16, EPI, 64, 64>), grid, dim3(NT), 0, c.stream, g);
      else hipLaunchKernelGGL((k_qgemm<QCUR_BF16, EPI, 32, 32>), grid, dim3(NT), 0, c.stream, g);
  }
}

hipError_t launch_residual_gemm(const Ctx& c, QView A, QView B1, QView R, const uint8_t* mask, int64_t mask_ld,
                                int compute, double* partials, QView* E, double e_scale, int opR, const QView* Bout,
                                const int* skip) {
  GemmArgs g = {};
  g.skip = skip;
  g.A = B1.p; g.lda = B1.ld; g.psa = B1.ps;
  g.B = R.p; g.ldb = R.ld; g.psb = R.ps;
  g.M = A.rows; g.N = A.cols; g.K = B1.cols;
  g.opA = QCUR_OP_N; g.opB = opR;
  g.alpha = 1.0; g.beta = 0.0;
  g.R0 = A.p; g.r0dt = A.dt; g.r0ld = A.ld; g.r0ps = A.ps;
  g.mask = mask; g.mask_ld = mask_ld;
  g.partials = partials;
  g.batch = 1;
  g.splits = 1;
  g.vec = compute == QCUR_BF16 && vec_ok(B1, 0) && vec_ok(R, 0);
  if (E) { g.E = E->p; g.edt = E->dt; g.eld = E->ld; g.eps = E->ps; g.e_scale = e_scale; }
  if (Bout) { g.Bo = Bout->p; g.bodt = Bout->dt; g.bold = Bout->ld; g.bops = Bout->ps; }
  if (g.M == 0 || g.N == 0) return hipSuccess;
  g.splits = 1;
  launch_fused<EPI_RESID>(c, g, compute, resid_tile(g.M, g.N, compute));
  return hipGetLastError();
}

// Batched residual: problem b's tiles write partials[b * tiles + tile]
// (zero for tiles outside the problem); E_b = e_scale (A_b - B1_b op(R_b))
// when E is given.
hipError_t launch_residual_gemm_batched(const Ctx& c, int count, Slots A, Slots B1, Slots R, int opR, int64_t mx,
                                        int64_t nx, int64_t kx, const int* bM, const int* bN, const int* bK,
                                        int compute, double* partials, const Slots* E, double e_scale, int tile,
                                        const Slots* Bout, const int* order, const int* skip) {
  if (count <= 0 || mx <= 0 || nx <= 0) return hipSuccess;
  GemmArgs g = {};
  g.order = order;
  g.skip = skip;
  g.A = B1.p; g.lda = B1.ld; g.psa = B1.ps; g.sA = B1.slab;
  g.B = R.p; g.ldb = R.ld; g.psb = R.ps; g.sB = R.slab;
  g.M = mx; g.N = nx; g.K = kx;
  g.bM = bM; g.bN = bN; g.bK = bK;
  g.opA = QCUR_OP_N; g.opB = opR;
  g.alpha = 1.0; g.beta = 0.0;
  g.R0 = A.p; g.r0dt = A.dt; g.r0ld = A.ld; g.r0ps = A.ps; g.sR0 = A.slab;
  g.partials = partials;
  g.batch = count;
  g.splits = 1;
  g.vec = compute == QCUR_BF16 && vec_ok(QView{B1.p, 1, 1, B1.ld, B1.ps, B1.dt}, B1.slab) &&
          vec_ok(QView{R.p, 1, 1, R.ld, R.ps, R.dt}, R.slab);
  if (E) { g.E = E->p; g.edt = E->dt; g.eld = E->ld; g.eps = E->ps; g.sE = E->slab; g.e_scale = e_scale; }
  if (Bout) { g.Bo = Bout->p; g.bodt = Bout->dt; g.bold = Bout->ld; g.bops = Bout->ps; g.sBo = Bout->slab; }
  if (compute == QCUR_BF16X3) return hipErrorInvalidValue;  // not offered for batches
  const int t = tile == 32 ? 32 : 64;
  const dim3 grid((unsigned)((nx + t - 1) / t), (unsigned)((mx + t - 1) / t), (unsigned)count);
  switch (compute) {
    case QCUR_F64:
      g.ktiles_per_split = (int)((kx + 15) / 16);
      if (t == 64) launch_tiles<QCUR_F64, EPI_RESID, 64, 64>(c, g, grid);
      else launch_tiles<QCUR_F64, EPI_RESID, 32, 32>(c, g, grid);
      break;
    case QCUR_F32:
      g.ktiles_per_split = (int)((kx + 15) / 16);
      if (t == 64) launch_tiles<QCUR_F32, EPI_RESID, 64, 64>(c, g, grid);
      else launch_tiles<QCUR_F32, EPI_RESID, 32, 32>(c, g, grid);
      break;
    default:
      g.ktiles_per_split = (int)((kx + 31) / 32);
      if (t == 64) launch_tiles<QCUR_BF16, EPI_RESID, 64, 64>(c, g, grid);
      else launch_tiles<QCUR_BF16, EPI_RESID, 32, 32>(c, g, grid);
  }
  return hipGetLastError();
}

// Completion step: X1 = P_Omega(Y) + P_Omega^c(B1 op(R)), tile partials of
// |X1 - X0|^2 into partials and of |X0|^2 into partials2 (64 x 64 tiles).
hipError_t launch_merge_gemm(const Ctx& c, QView Y, const uint8_t* mask, int64_t mask_ld, QView X0, QView B1,
                             QView R, int opR, int compute, QView X1, double* partials, double* partials2) {
  GemmArgs g = {};
  g.A = B1.p; g.lda = B1.ld; g.psa = B1.ps;
  g.B = R.p; g.ldb = R.ld; g.psb = R.ps;
  g.M = Y.rows; g.N = Y.cols; g.K = B1.cols;
  g.opA = QCUR_OP_N; g.opB = opR;
  g.alpha = 1.0; g.beta = 0.0;
  g.R0 = Y.p; g.r0dt = Y.dt; g.r0ld = Y.ld; g.r0ps = Y.ps;
  g.X0 = X0.p; g.x0dt = X0.dt; g.x0ld = X0.ld; g.x0ps = X0.ps;
  g.E = X1.p; g.edt = X1.dt; g.eld = X1.ld; g.eps = X1.ps;
  g.mask = mask; g.mask_ld = mask_ld;
  g.partials = partials;
  g.partials2 = partials2;
  g.batch = 1;
  g.splits = 1;
  g.vec = compute == QCUR_BF16 && vec_ok(B1, 0) && vec_ok(R, 0);
  if (g.M == 0 || g.N == 0) return hipSuccess;
  launch_fused<EPI_MERGE>(c, g, compute, resid_tile(g.M, g.N, compute));
  return hipGetLastError();
}

}  // namespace qcur
