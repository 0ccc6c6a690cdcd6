/* libqcur_probe: measured ceilings for the roofline fractions of libqcur.
 *
 * Measurement only, not part of the QMCUR path: the achievable matrix-core
 * rate of each product dtype (a loop of independent MFMAs on every compute
 * unit, no memory traffic) and the achievable HBM bandwidth (a streaming
 * copy), so that kernel rates can be reported against what the device
 * sustains as well as against its published peaks.
 *
 * Both calls run on the current HIP device and stream 0, synchronise the
 * device, and return 0 on success or a HIP error code.
 */
#ifndef QCUR_PROBE_H
#define QCUR_PROBE_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Dense MFMA rate in TFLOP/s for dtype 0 (FP64, 16x16x4), 1 (FP32,
 * 16x16x4) or 2 (BF16 operands with FP32 accumulation, 16x16x32): every
 * wave issues `iters` rounds of eight independent MFMAs; 4096 workgroups of
 * 256 threads.  *tflops receives the best of three timed launches.  An
 * unknown dtype returns hipErrorInvalidValue (1). */
int qcur_probe_mfma(int dtype, int iters, double* tflops);

/* Streaming copy of `bytes` bytes (a multiple of 16, both pointers 16-byte
 * aligned device memory, not overlapping), timed over `reps` launches after
 * one untimed one.  *gbps receives (bytes read + bytes written) / mean time,
 * in GB/s (1e9 bytes).  Misaligned or empty arguments return
 * hipErrorInvalidValue (1). */
int qcur_probe_copy(void* dst, const void* src, size_t bytes, int reps, double* gbps);

#ifdef __cplusplus
}
#endif

#endif
