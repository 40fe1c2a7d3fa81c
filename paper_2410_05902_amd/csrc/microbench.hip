// Throughput probes of the gfx950 units the hot path is bound by: FP32
// subtract + add-|.| (the Laplacian distance's inner pair), FP32 FMA, the
// exp2 transcendental, and BF16 / FP32 MFMA (BF16 also as one dependent
// chain per wave).  They give the attainable rates
// that the roofline fractions of the VALU-bound and MFMA-bound kernels are set
// beside (include/mbkk_microbench.h).
//
// Every probe runs independent dependency chains per lane (enough of them to
// cover the unit's latency), grid-wide at a fixed number of waves per SIMD,
// and writes its result only under a condition the chains never meet, so no
// memory traffic enters the timing while the compiler must keep the work.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/mbkk_microbench.h"

namespace {

constexpr int kChains = 16;
constexpr int kCUs = 256;

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ void sink_if(float v, float *sink)
{
    if (v == 1234.5f)  // never true for the chains below
        sink[threadIdx.x] = v;
}

// 2 lane operations per element and step: v_sub_f32, then v_add_f32 with an
// |.| source modifier (s += |x - y|); plus one FMA per step for y (counted).
__global__ __launch_bounds__(256) void k_probe_subadd(int64_t iters, float y0, float *sink)
{
    float x[kChains], s[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) {
        x[c] = (float)(threadIdx.x + c) * 1e-3f;
        s[c] = 0.0f;
    }
    float y = y0;
    for (int64_t it = 0; it < iters; ++it) {
#pragma unroll
        for (int c = 0; c < kChains; ++c)
            s[c] += fabsf(x[c] - y);
        y = fmaf(s[0], 1e-30f, y0);  // one FMA per kChains pairs keeps y a run-time value
    }
    float t = 0.0f;
#pragma unroll
    for (int c = 0; c < kChains; ++c)
        t += s[c];
    sink_if(t, sink);
}

// 1 lane operation (an FMA) per element and step.
__global__ __launch_bounds__(256) void k_probe_fma(int64_t iters, float b, float *sink)
{
    float a[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c)
        a[c] = (float)(threadIdx.x + c) * 1e-3f;
    for (int64_t it = 0; it < iters; ++it) {
#pragma unroll
        for (int c = 0; c < kChains; ++c)
            a[c] = fmaf(a[c], b, 0.25f);
    }
    float t = 0.0f;
#pragma unroll
    for (int c = 0; c < kChains; ++c)
        t += a[c];
    sink_if(t, sink);
}

// 1 transcendental per element and step: a <- 2^(-a) (v_exp_f32 with a
// negated source), which stays in (0.5, 1].
__global__ __launch_bounds__(256) void k_probe_exp2(int64_t iters, float *sink)
{
    float a[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c)
        a[c] = (float)(threadIdx.x + c) * 1e-3f;
    for (int64_t it = 0; it < iters; ++it) {
#pragma unroll
        for (int c = 0; c < kChains; ++c)
            a[c] = __builtin_amdgcn_exp2f(-a[c]);
    }
    float t = 0.0f;
#pragma unroll
    for (int c = 0; c < kChains; ++c)
        t += a[c];
    sink_if(t, sink);
}

// MFMA: 4 independent 32x32 accumulators per wave.
template <bool BF16>
__global__ __launch_bounds__(256) void k_probe_mfma(int64_t iters, float *sink)
{
    f32x16 acc[4];
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int i = 0; i < 16; ++i)
            acc[q][i] = 0.0f;
    const float av = (float)(threadIdx.x & 7) * 1e-3f;
    bf16x8 ab;
#pragma unroll
    for (int i = 0; i < 8; ++i)
        ab[i] = (__bf16)(av + (float)i * 1e-3f);
    for (int64_t it = 0; it < iters; ++it) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if constexpr (BF16)
                acc[q] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ab, ab, acc[q], 0, 0, 0);
            else
                acc[q] = __builtin_amdgcn_mfma_f32_32x32x2f32(av, av, acc[q], 0, 0, 0);
        }
    }
    float t = 0.0f;
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int i = 0; i < 16; ++i)
            t += acc[q][i];
    sink_if(t, sink);
}

// MFMA, one dependent chain per wave: every product of the wave accumulates
// into the same 32x32 block, as a batch-stationary kernel holding one block
// of batch rows per wave does (the matrix core then overlaps only the
// products of different waves).
__global__ __launch_bounds__(256) void k_probe_mfma_chain(int64_t iters, float *sink)
{
    f32x16 acc;
#pragma unroll
    for (int i = 0; i < 16; ++i)
        acc[i] = 0.0f;
    const float av = (float)(threadIdx.x & 7) * 1e-3f;
    bf16x8 ab;
#pragma unroll
    for (int i = 0; i < 8; ++i)
        ab[i] = (__bf16)(av + (float)i * 1e-3f);
    for (int64_t it = 0; it < iters; ++it) {
#pragma unroll
        for (int q = 0; q < 4; ++q)
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ab, ab, acc, 0, 0, 0);
    }
    float t = 0.0f;
#pragma unroll
    for (int i = 0; i < 16; ++i)
        t += acc[i];
    sink_if(t, sink);
}

}  // namespace

extern "C" int mbkk_microbench(int32_t kind, int64_t iters, int32_t waves_per_simd, void *stream, float *sink_dev,
                               double *ms_host, double *ops_host)
{
    if (iters < 1 || waves_per_simd < 1 || waves_per_simd > 8 || !sink_dev || !ms_host || !ops_host)
        return -1;
    hipStream_t st = (hipStream_t)stream;
    // 4 waves per workgroup, one workgroup per SIMD-set of the chip per wave level
    const int blocks = kCUs * waves_per_simd;
    const double lanes = (double)blocks * 256.0;
    double ops = 0.0;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess)
        return -4;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return -4;
    }
    int rc = 0;
    auto launch = [&]() {
        switch (kind) {
        case MBKK_PROBE_SUBADD:
            hipLaunchKernelGGL(k_probe_subadd, dim3(blocks), dim3(256), 0, st, iters, 0.5f, sink_dev);
            ops = lanes * (double)iters * (kChains * 2.0 + 1.0);
            break;
        case MBKK_PROBE_FMA:
            hipLaunchKernelGGL(k_probe_fma, dim3(blocks), dim3(256), 0, st, iters, 0.999f, sink_dev);
            ops = lanes * (double)iters * kChains;
            break;
        case MBKK_PROBE_EXP2:
            hipLaunchKernelGGL(k_probe_exp2, dim3(blocks), dim3(256), 0, st, iters, sink_dev);
            ops = lanes * (double)iters * kChains;
            break;
        case MBKK_PROBE_MFMA_BF16:
            hipLaunchKernelGGL(k_probe_mfma<true>, dim3(blocks), dim3(256), 0, st, iters, sink_dev);
            ops = (double)blocks * 4.0 * (double)iters * 4.0 * 32.0 * 32.0 * 16.0 * 2.0;
            break;
        case MBKK_PROBE_MFMA_BF16_CHAIN:
            hipLaunchKernelGGL(k_probe_mfma_chain, dim3(blocks), dim3(256), 0, st, iters, sink_dev);
            ops = (double)blocks * 4.0 * (double)iters * 4.0 * 32.0 * 32.0 * 16.0 * 2.0;
            break;
        case MBKK_PROBE_MFMA_F32:
            hipLaunchKernelGGL(k_probe_mfma<false>, dim3(blocks), dim3(256), 0, st, iters, sink_dev);
            ops = (double)blocks * 4.0 * (double)iters * 4.0 * 32.0 * 32.0 * 2.0 * 2.0;
            break;
        default:
            rc = -1;
        }
    };
    launch();  // warm-up (clocks, code object load)
    if (rc == 0 && hipEventRecord(e0, st) == hipSuccess) {
        launch();
        if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess)
            rc = -4;
    } else if (rc == 0) {
        rc = -4;
    }
    float ms = 0.0f;
    if (rc == 0 && (hipGetLastError() != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
        rc = -4;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc)
        return rc;
    *ms_host = ms;
    *ops_host = ops;
    return 0;
}
