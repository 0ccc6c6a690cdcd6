// Index sampler for Algorithm 1, steps 1-2 (drawing J from {p_j} and I from
// {q_i}).  The paper does not say how indices are drawn; this library uses an
// integer-CDF sampler so that draws are exact and reproducible:
//   w_j = floor(p_j * 2^60)                    (exact in FP64 for p_j in [0,1])
//   u_t = SplitMix64 output number set_id*2^32 + t, state started at `seed`
//   tau = floor(u_t * T / 2^64), T = current weight total
//   j   = smallest index whose inclusive prefix sum exceeds tau
//   without replacement, w_j is then removed from T.
// One workgroup per draw.  The search descends a 64-ary tree (superblocks
// of 4096, blocks of 64 elements) of inclusive prefix sums, updated in place
// when a weight is removed: a draw costs one ballot per level.
#include <algorithm>

#include "qcur_internal.hpp"

namespace qcur {

static constexpr int DRAW_THREADS = 256;
static constexpr int64_t DRAW_MAX_N_NOREPL = 16384;
static constexpr int64_t DRAW_MAX_N_REPL = 8192;

__device__ inline uint64_t splitmix64_nth(uint64_t seed, uint64_t n) {
  // state after n+1 steps of adding the golden gamma, then the output mix
  uint64_t z = seed + (n + 1ull) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Wave-wide sum of nonnegative 64-bit integers with overflow detection.
__device__ inline uint64_t wave_sum_u64(uint64_t v, bool& ovf) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    uint64_t w = __shfl_xor(v, o, 64);
    uint64_t s = v + w;
    ovf |= (s < v);
    v = s;
  }
  return v;
}

// 64-bit DPP move of lane data (lanes outside the pattern read 0).
template <int CTRL, int ROWS>
__device__ inline uint64_t dpp_u64(uint64_t v) {
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)v, CTRL, ROWS, 0xf, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(v >> 32), CTRL, ROWS, 0xf, true);
  return ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
}

// Inclusive wave-wide prefix sum of 64-bit integers: shifts by 1, 2, 4, 8
// within rows of 16 lanes, then the row totals broadcast into rows 1, 3
// (lane 15) and rows 2, 3 (lane 31).
__device__ inline uint64_t wave_incl_scan_u64(uint64_t x) {
  x += dpp_u64<0x111, 0xf>(x);  // row_shr:1
  x += dpp_u64<0x112, 0xf>(x);  // row_shr:2
  x += dpp_u64<0x114, 0xf>(x);  // row_shr:4
  x += dpp_u64<0x118, 0xf>(x);  // row_shr:8
  x += dpp_u64<0x142, 0xa>(x);  // row_bcast:15
  x += dpp_u64<0x143, 0xc>(x);  // row_bcast:31
  return x;
}

__device__ inline uint64_t readlane_u64(uint64_t v, int k) {
  const uint32_t lo = __builtin_amdgcn_readlane((int)(uint32_t)v, k);
  const uint32_t hi = __builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), k);
  return ((uint64_t)hi << 32) | lo;
}

struct DrawJob {
  const double* probs;
  int64_t n, count;
  uint64_t seed, set_id;
  int64_t* idx;
};
struct DrawJobs {
  DrawJob j[2];
};

// One draw job run by the whole workgroup (DRAW_THREADS threads); lds holds
// draw_lds(n, repl) bytes.
__device__ void draw_body(const double* __restrict__ probs, int64_t n, int64_t count, uint64_t seed,
                          uint64_t set_id, int repl, int64_t* __restrict__ idx, unsigned* status, uint64_t* lds) {
  const int64_t npad = (n + 63) / 64 * 64;
  const int64_t nb = npad / 64;
  const int64_t nsb = (nb + 63) / 64;
  constexpr int NB1 = (int)(DRAW_MAX_N_NOREPL / 64 / 64);  // superblocks the draw loop keeps in registers
  if (nsb > NB1) {  // beyond the sampler's size limit: refuse rather than index past the registers
    for (int64_t t = threadIdx.x; t < count; t += DRAW_THREADS) idx[t] = -1;
    if (threadIdx.x == 0) atomicOr(status, ST_SAMPLE);
    return;
  }
  uint64_t* wl = lds;              // npad weights, then in-block inclusive prefix sums
  uint64_t* L1 = wl + npad;        // nb block sums
  uint64_t* L2 = L1 + nb;          // nsb superblock sums
  uint32_t* cnt = (uint32_t*)(L2 + 64);  // npad pick counts (with replacement)
  uint8_t* taken = (uint8_t*)(L2 + 64);  // npad taken flags (without replacement)
  __shared__ int bad;
  __shared__ uint64_t total;
  __shared__ int64_t npos;
  __shared__ uint64_t wave_tot[DRAW_THREADS / 64];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  if (tid == 0) {
    bad = 0;
    npos = 0;
  }
  __syncthreads();

  // weights, block sums, positive count
  for (int64_t b = wave; b < nb; b += DRAW_THREADS / 64) {
    const int64_t e = b * 64 + lane;
    uint64_t w = 0;
    bool inv = false;
    if (e < n) {
      const double p = probs[e];
      inv = !(p >= 0.0 && p <= 1.0);
      w = inv ? 0ull : (uint64_t)(p * 0x1p60);
    }
    if (repl) cnt[e] = 0u;
    else taken[e] = 0;
    bool ovf = false;
    uint64_t s = wave_sum_u64(w, ovf);
    wl[e] = wave_incl_scan_u64(w);  // exact: the block total did not overflow
    unsigned long long posm = __ballot(w > 0);
    unsigned long long invm = __ballot(inv);
    if (lane == 0) {
      L1[b] = s;
      if (ovf || invm) atomicOr(&bad, 1);
      atomicAdd((unsigned long long*)&npos, (unsigned long long)__popcll(posm));
    }
  }
  __syncthreads();
  for (int64_t sb = wave; sb < nsb; sb += DRAW_THREADS / 64) {
    const int64_t b = sb * 64 + lane;
    uint64_t v = b < nb ? L1[b] : 0ull;
    bool ovf = false;
    uint64_t s = wave_sum_u64(v, ovf);
    if (lane == 0) {
      L2[sb] = s;
      if (ovf) atomicOr(&bad, 1);
    }
  }
  __syncthreads();
  if (wave == 0) {
    uint64_t v = lane < nsb ? L2[lane] : 0ull;
    bool ovf = false;
    uint64_t s = wave_sum_u64(v, ovf);
    if (lane == 0) {
      total = s;
      if (ovf || s == 0ull || (!repl && npos < count)) atomicOr(&bad, 1);
    }
  }
  __syncthreads();
  if (bad) {
    for (int64_t t = tid; t < count; t += DRAW_THREADS) idx[t] = -1;
    if (tid == 0) atomicOr(status, ST_SAMPLE);
    return;
  }

  // the draws, one wave.  Every level keeps inclusive prefix sums: the
  // superblock sums (one per lane) and the block sums within each superblock
  // (lane b % 64, register b / 64) in registers, the weights of each block in
  // LDS.  A draw picks at each level the first entry whose prefix exceeds
  // tau (a ballot) and lowers tau by the prefix before it; without
  // replacement it then subtracts the drawn weight from the prefixes at and
  // after its position, so no scan is needed per draw.  LDS operations of one
  // wave complete in order; the memory clobber makes every lane reload the
  // weights of the next draw's block.
  if (wave == 0) {
    uint64_t l2p = wave_incl_scan_u64(lane < nsb ? L2[lane] : 0ull);
    uint64_t l1p[NB1];
#pragma unroll
    for (int m = 0; m < NB1; ++m) l1p[m] = wave_incl_scan_u64((m * 64 + lane < nb) ? L1[m * 64 + lane] : 0ull);
    // first lane whose prefix x exceeds tau (lane 0 if none: the sums are
    // kept consistent, so this only keeps indices in range), and the prefix
    // before it
    auto pick = [&](uint64_t x, uint64_t& tau_) -> int {
      const unsigned long long mask = __ballot(x > tau_);
      const int k = mask ? __ffsll((unsigned long long)mask) - 1 : 0;
      if (k > 0) tau_ -= readlane_u64(x, k - 1);
      return k;
    };
    uint64_t T = total;
    const uint64_t base = (set_id & 0xFFFFFFFFull) << 32;
    uint64_t uvec = 0;  // u_{t..t+63}, one per lane, made 64 draws at a time
    for (int64_t t = 0; t < count; ++t) {
      if ((t & 63) == 0) uvec = splitmix64_nth(seed, base + (uint64_t)(t + lane));
      const uint64_t u = readlane_u64(uvec, (int)(t & 63));
      uint64_t tau = __umul64hi(u, T);
      int sb = 0;
      uint64_t v1 = l1p[0];
      if (nsb > 1) {  // more than one superblock (n > 4096)
        sb = pick(l2p, tau);
#pragma unroll
        for (int m = 1; m < NB1; ++m)
          if (sb == m) v1 = l1p[m];
      }
      const int eb = pick(v1, tau);
      const int64_t b = (int64_t)sb * 64 + eb;
      const uint64_t pe = wl[b * 64 + lane];
      const int e = pick(pe, tau);
      const int64_t j = b * 64 + e;
      const uint64_t wj = readlane_u64(pe, e) - (e > 0 ? readlane_u64(pe, e - 1) : 0ull);
      if (repl) {
        if (lane == 0) cnt[j] = cnt[j] + 1u;
      } else {
        wl[b * 64 + lane] = pe - (lane >= e ? wj : 0ull);
        if (lane == 0) taken[j] = 1;
#pragma unroll
        for (int m = 0; m < NB1; ++m)
          if (sb == m && lane >= eb) l1p[m] -= wj;
        if (lane >= sb) l2p -= wj;
        T -= wj;
      }
      __asm__ __volatile__("" ::: "memory");
    }
  }
  __syncthreads();

  // sorted output: compaction of picked elements in index order (each
  // thread counts its chunk; a workgroup-wide exclusive scan gives offsets)
  const int64_t per = (npad + DRAW_THREADS - 1) / DRAW_THREADS;
  const int64_t e0 = min(npad, tid * per), e1 = min(npad, e0 + per);
  int64_t mine = 0;
  for (int64_t e = e0; e < e1; ++e) mine += repl ? (int64_t)cnt[e] : (int64_t)taken[e];
  const uint64_t incl = wave_incl_scan_u64((uint64_t)mine);
  if (lane == 63) wave_tot[wave] = incl;
  __syncthreads();
  int64_t o = (int64_t)(incl - (uint64_t)mine);
  for (int w = 0; w < wave; ++w) o += (int64_t)wave_tot[w];
  for (int64_t e = e0; e < e1; ++e) {
    int64_t k = repl ? (int64_t)cnt[e] : (int64_t)taken[e];
    for (int64_t r = 0; r < k && o < count; ++r) idx[o++] = e;
  }
}

__global__ __launch_bounds__(DRAW_THREADS) void k_draw(DrawJobs jobs, int repl, unsigned* status) {
  extern __shared__ uint64_t lds[];
  const DrawJob& job = jobs.j[blockIdx.x];
  draw_body(job.probs, job.n, job.count, job.seed, job.set_id, repl, job.idx, status, lds);
}

size_t draw_lds(int64_t n, int repl) {
  const int64_t npad = (n + 63) / 64 * 64;
  const int64_t nb = npad / 64;
  return (size_t)(npad + nb + 64) * 8 + (size_t)npad * (repl ? 4 : 1);
}

static hipError_t draw_jobs(const Ctx& c, DrawJobs jobs, int njobs, int repl, size_t lds) {
  hipError_t e = hipFuncSetAttribute((const void*)k_draw, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)(156 * 1024));  // 160 KiB less the static LDS
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_draw, dim3(njobs), dim3(DRAW_THREADS), lds, c.stream, jobs, repl, c.status);
  return hipGetLastError();
}

hipError_t launch_draw(const Ctx& c, const double* probs, int64_t n, int64_t count, uint64_t seed,
                       uint64_t set_id, int with_replacement, int64_t* idx) {
  DrawJobs jobs{};
  jobs.j[0] = DrawJob{probs, n, count, seed, set_id, idx};
  return draw_jobs(c, jobs, 1, with_replacement, draw_lds(n, with_replacement));
}

// Two independent draws (e.g. J from the column and I from the row
// probabilities) in one launch of two workgroups.
hipError_t launch_draw_pair(const Ctx& c, const double* p0, int64_t n0, int64_t count0, uint64_t set0,
                            int64_t* idx0, const double* p1, int64_t n1, int64_t count1, uint64_t set1,
                            int64_t* idx1, uint64_t seed, int with_replacement) {
  DrawJobs jobs{};
  jobs.j[0] = DrawJob{p0, n0, count0, seed, set0, idx0};
  jobs.j[1] = DrawJob{p1, n1, count1, seed, set1, idx1};
  const size_t lds = std::max(draw_lds(n0, with_replacement), draw_lds(n1, with_replacement));
  return draw_jobs(c, jobs, 2, with_replacement, lds);
}

// Batched draws: workgroup (set, b) draws J_b (set 0: c_b indices from the
// column probabilities) or I_b (set 1: r_b indices from the row
// probabilities) of problem b with the seed seed + b, so that problem b
// repeats the single solve seeded with seed + b.  Length probabilities are
// folded here from the batched norm pass: col2_j sums the row tiles and
// row2_i the column tiles in index order, ||A_b||_F^2 is a fixed-order sum
// of col2 (computed alike by both workgroups of a problem), and
// p_j = col2_j / ||A_b||_F^2 (Section 3.1).  Uniform: p_j = 1/n_b.
__global__ __launch_bounds__(DRAW_THREADS) void kb_draw(DrawBatch d, unsigned* status) {
  extern __shared__ uint64_t lds[];
  __shared__ double red[DRAW_THREADS];
  const int set = blockIdx.x, b = blockIdx.y, tid = threadIdx.x;
  const int64_t m = d.dm[b], n = d.dn[b];
  const int64_t len = set == 0 ? n : m;
  double* pr = set == 0 ? d.p + (int64_t)b * d.nx : d.q + (int64_t)b * d.mx;
  if (d.sampling == QCUR_UNIFORM) {
    const double u = 1.0 / (double)len;
    for (int64_t j = tid; j < len; j += DRAW_THREADS) pr[j] = u;
  } else {
    const int64_t nrbx = (d.mx + BATCH_RB - 1) / BATCH_RB, ncbx = (d.nx + BATCH_CB - 1) / BATCH_CB;
    const int64_t nrb = (m + BATCH_RB - 1) / BATCH_RB, ncb = (n + BATCH_CB - 1) / BATCH_CB;
    const double* cp = d.colpart + (int64_t)b * nrbx * d.nx;
    double s = 0.0;
    for (int64_t j = tid; j < n; j += DRAW_THREADS) {
      double c2 = 0.0;
      for (int64_t r = 0; r < nrb; ++r) c2 += cp[r * d.nx + j];
      s += c2;
    }
    red[tid] = s;
    __syncthreads();
    for (int w = DRAW_THREADS / 2; w >= 1; w >>= 1) {
      if (tid < w) red[tid] += red[tid + w];
      __syncthreads();
    }
    const double fro2 = red[0];
    if (tid == 0 && set == 0 && !(fro2 > 0.0 && fro2 < INFINITY)) atomicOr(status, ST_NUMERIC);
    if (set == 0) {
      for (int64_t j = tid; j < n; j += DRAW_THREADS) {
        double c2 = 0.0;
        for (int64_t r = 0; r < nrb; ++r) c2 += cp[r * d.nx + j];
        pr[j] = c2 / fro2;
      }
    } else {
      const double* rp = d.rowpart + (int64_t)b * ncbx * d.mx;
      for (int64_t i = tid; i < m; i += DRAW_THREADS) {
        double r2 = 0.0;
        for (int64_t cb = 0; cb < ncb; ++cb) r2 += rp[cb * d.mx + i];
        pr[i] = r2 / fro2;
      }
    }
  }
  __syncthreads();  // the probabilities written above are read back by the whole workgroup
  const int64_t count = set == 0 ? d.dc[b] : d.dr[b];
  int64_t* idx = set == 0 ? d.J + (int64_t)b * d.cx : d.I + (int64_t)b * d.rx;
  draw_body(pr, len, count, d.seed + (uint64_t)b, (uint64_t)set, d.repl, idx, status, lds);
}

hipError_t launch_draw_batch(const Ctx& c, int count, const DrawBatch& d) {
  if (count <= 0) return hipSuccess;
  const size_t lds = draw_lds(std::max(d.mx, d.nx), d.repl);
  hipLaunchKernelGGL(kb_draw, dim3(2, (unsigned)count), dim3(DRAW_THREADS), lds, c.stream, d, c.status);
  return hipGetLastError();
}

}  // namespace qcur
