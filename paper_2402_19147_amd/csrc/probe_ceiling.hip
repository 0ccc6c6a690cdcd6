// Measured ceilings (declared in qcur_probe.h): an MFMA loop per dtype and a
// streaming copy.  Measurement only; the QMCUR path does not use this file.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "../../include/qcur_probe.h"

namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int CHAINS = 8;  // independent accumulators per wave
constexpr int PROBE_BLOCKS = 4096, PROBE_THREADS = 256;

// Operands come from the lane index so that nothing is constant-folded; the
// accumulators are summed into out[] so that nothing is dead.
__global__ __launch_bounds__(PROBE_THREADS) void k_mfma_f64(double* out, int iters) {
  const double a = 1.0 + 1e-3 * (threadIdx.x & 7), b = 1.0 - 1e-3 * (threadIdx.x & 3);
  f64x4 acc[CHAINS];
#pragma unroll
  for (int c = 0; c < CHAINS; ++c) acc[c] = (f64x4){0, 0, 0, 0};
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int c = 0; c < CHAINS; ++c) acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[c], 0, 0, 0);
  }
  double s = 0;
#pragma unroll
  for (int c = 0; c < CHAINS; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
  out[(size_t)blockIdx.x * PROBE_THREADS + threadIdx.x] = s;
}

__global__ __launch_bounds__(PROBE_THREADS) void k_mfma_f32(float* out, int iters) {
  const float a = 1.0f + 1e-3f * (threadIdx.x & 7), b = 1.0f - 1e-3f * (threadIdx.x & 3);
  f32x4 acc[CHAINS];
#pragma unroll
  for (int c = 0; c < CHAINS; ++c) acc[c] = (f32x4){0, 0, 0, 0};
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int c = 0; c < CHAINS; ++c) acc[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[c], 0, 0, 0);
  }
  float s = 0;
#pragma unroll
  for (int c = 0; c < CHAINS; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
  out[(size_t)blockIdx.x * PROBE_THREADS + threadIdx.x] = s;
}

__global__ __launch_bounds__(PROBE_THREADS) void k_mfma_bf16(float* out, int iters) {
  bf16x8 a, b;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    a[e] = (__bf16)(1.0f + 0.0078125f * ((threadIdx.x + e) & 3));
    b[e] = (__bf16)(1.0f - 0.0078125f * ((threadIdx.x + 2 * e) & 3));
  }
  f32x4 acc[CHAINS];
#pragma unroll
  for (int c = 0; c < CHAINS; ++c) acc[c] = (f32x4){0, 0, 0, 0};
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int c = 0; c < CHAINS; ++c) acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[c], 0, 0, 0);
  }
  float s = 0;
#pragma unroll
  for (int c = 0; c < CHAINS; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
  out[(size_t)blockIdx.x * PROBE_THREADS + threadIdx.x] = s;
}

// grid-stride copy of 16-byte words with nontemporal loads and stores (of
// the forms tried, 1024 workgroups of these was the fastest streaming copy)
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(256) void k_copy16(u32x4* __restrict__ dst, const u32x4* __restrict__ src, size_t n) {
  const size_t st = (size_t)gridDim.x * 256;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += st)
    __builtin_nontemporal_store(__builtin_nontemporal_load(&src[i]), &dst[i]);
}

}  // namespace

extern "C" int qcur_probe_mfma(int dtype, int iters, double* tflops) {
  if (dtype < 0 || dtype > 2 || iters <= 0 || !tflops) return (int)hipErrorInvalidValue;
  void* out = nullptr;
  hipError_t e = hipMalloc(&out, (size_t)PROBE_BLOCKS * PROBE_THREADS * 8);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  double best = 0.0;
  // flops of one MFMA: 2 * 16 * 16 * K
  const double per = dtype == 2 ? 2.0 * 16 * 16 * 32 : 2.0 * 16 * 16 * 4;
  const double flop = per * CHAINS * (double)iters * (PROBE_BLOCKS * (PROBE_THREADS / 64));
  for (int rep = 0; rep < 4 && e == hipSuccess; ++rep) {
    e = hipEventRecord(e0, 0);
    if (dtype == 0) hipLaunchKernelGGL(k_mfma_f64, dim3(PROBE_BLOCKS), dim3(PROBE_THREADS), 0, 0, (double*)out, iters);
    if (dtype == 1) hipLaunchKernelGGL(k_mfma_f32, dim3(PROBE_BLOCKS), dim3(PROBE_THREADS), 0, 0, (float*)out, iters);
    if (dtype == 2) hipLaunchKernelGGL(k_mfma_bf16, dim3(PROBE_BLOCKS), dim3(PROBE_THREADS), 0, 0, (float*)out, iters);
    if (e == hipSuccess) e = hipGetLastError();
    if (e == hipSuccess) e = hipEventRecord(e1, 0);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e == hipSuccess && rep > 0 && ms > 0.0f) best = std::max(best, flop / (ms * 1e-3) / 1e12);
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (out) (void)hipFree(out);
  *tflops = best;
  return (int)e;
}

extern "C" int qcur_probe_copy(void* dst, const void* src, size_t bytes, int reps, double* gbps) {
  if (!dst || !src || !gbps || reps <= 0 || bytes == 0 || bytes % 16 || ((uintptr_t)dst | (uintptr_t)src) % 16)
    return (int)hipErrorInvalidValue;
  const size_t n = bytes / 16;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  const unsigned grid = 1024;
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_copy16, dim3(grid), dim3(256), 0, 0, (u32x4*)dst, (const u32x4*)src, n);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipEventRecord(e0, 0);
  for (int r = 0; r < reps && e == hipSuccess; ++r) {
    hipLaunchKernelGGL(k_copy16, dim3(grid), dim3(256), 0, 0, (u32x4*)dst, (const u32x4*)src, n);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipEventRecord(e1, 0);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float ms = 0.0f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  *gbps = (e == hipSuccess && ms > 0.0f) ? 2.0 * (double)bytes * reps / (ms * 1e-3) / 1e9 : 0.0;
  return (int)e;
}
