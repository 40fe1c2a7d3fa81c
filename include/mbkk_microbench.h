/*
 * mbkk_microbench.h - throughput probes of the gfx950 units that bound the
 * mbkk kernels (measurement support, not part of the method).
 *
 * The roofline of the Laplacian (L1) cross term and of every kernel's fused
 * exp is set by the vector ALU rather than by HBM or MFMA; these probes
 * measure the attainable rates of those units on the running GPU, so the
 * fractions the benchmark reports can be set beside both the datasheet peak
 * and the measured one.
 *
 * mbkk_microbench runs one probe kernel grid-wide (256 workgroups of 4 waves
 * per wave level, waves_per_simd in [1, 8] waves on every SIMD), each lane
 * running 16 independent dependency chains (the MFMA probes: 4 accumulators
 * per wave, the chain probe 1) for `iters` steps, once to warm up
 * and once timed with HIP events on `stream` (a hipStream_t, NULL = default).
 *   kind MBKK_PROBE_SUBADD   : s += |x - y| (v_sub_f32, v_add_f32 with |.|),
 *                              2 lane operations per pair + 1 FMA per step
 *   kind MBKK_PROBE_FMA      : a = fma(a, b, c), 1 lane operation
 *   kind MBKK_PROBE_EXP2     : a = 2^-a (v_exp_f32), 1 lane operation
 *   kind MBKK_PROBE_MFMA_BF16: v_mfma_f32_32x32x16_bf16, 32768 flops each
 *   kind MBKK_PROBE_MFMA_F32 : v_mfma_f32_32x32x2_f32, 4096 flops each
 *   kind MBKK_PROBE_MFMA_BF16_CHAIN: v_mfma_f32_32x32x16_bf16 with ONE
 *                              accumulator per wave (every product depends
 *                              on the one before it in the wave)
 * sink_dev: a device float array of at least 256 elements (never written in
 * practice; it keeps the work observable).  Writes the timed launch's
 * duration (ms_host) and the lane operations or flops it performed
 * (ops_host).  Returns 0, -1 for a bad argument, -4 for a HIP error.
 * Synchronises the stream.
 */
#ifndef MBKK_MICROBENCH_H
#define MBKK_MICROBENCH_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MBKK_PROBE_SUBADD 0
#define MBKK_PROBE_FMA 1
#define MBKK_PROBE_EXP2 2
#define MBKK_PROBE_MFMA_BF16 3
#define MBKK_PROBE_MFMA_F32 4
#define MBKK_PROBE_MFMA_BF16_CHAIN 5

int mbkk_microbench(int32_t kind, int64_t iters, int32_t waves_per_simd, void *stream, float *sink_dev,
                    double *ms_host, double *ops_host);

#ifdef __cplusplus
}
#endif
#endif /* MBKK_MICROBENCH_H */
