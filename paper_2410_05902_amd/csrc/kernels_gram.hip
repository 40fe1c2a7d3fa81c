// Gram blocks of the implicit centers (kernel values summed in FP64).
//
// A center held over its support (Section 4.1, Eq. 1 with a window of W
// batches) has self-norm <C_j, C_j> = sum_{c,c'} coef_j[c] coef_j[c'] G_j[c][c'];
// when batch i enters slot rr only the blocks
//   G_j[1+rr][c] = G_j[c][1+rr] = sum_{a in slot rr, center j} sum_{e in column c, center j} K(a, e)
// against the live columns c are new.  Their pairs are cut into tasks of
// kGramTA rows of the slot by te rows of the column (gram_plan), so that a
// cluster holding most of the batch is spread over the whole GPU:
//   plan : task offsets goff over jc = j * C + c (fused into the grouping
//          kernel of a step, k_gram_plan elsewhere);
//   work : kGramWaves waves take equal contiguous task ranges; wave w sums
//          its tasks of one jc in FP64 in task order and stores the sum at
//          gpart[w + jc].  The (wave, jc) runs of a split into contiguous
//          ranges form a monotone staircase, so w + jc is distinct per run;
//   fold : per live (j, c), the partials of its waves in wave order.
// Every sum has a fixed order, so the blocks are bit-reproducible.
//   k_gram_valu : any kernel, FP32 or FP64 arithmetic; a task is 32 slot
//                 rows (wave-uniform) x 64 column rows (one per lane);
//   k_gram_mfma : Gaussian MFMA forms; FP32 MFMA products and exp fused in
//                 registers; a task is one 16 x 16 output block.  The BF16
//                 forms take their Gram blocks here too: the self norms keep
//                 FP32 kernel values (summed in FP64), so a row re-scored in
//                 FP64 carries only the FP32 error of N_j.
#include "gram_body.h"
#include "kernels.h"

namespace mbkk {

// ---------------------------------------------------------------------------
// VALU tasks
// ---------------------------------------------------------------------------
template <int KIND, typename KT>
__device__ __forceinline__ void gram_term(KT &s, KT x, KT y)
{
    if constexpr (KIND == MBKK_GAUSS) {
        const KT v = x - y;
        s = fma(v, v, s);
    } else if constexpr (KIND == MBKK_LAPLACE) {
        s += fabs(x - y);
    } else {
        s = fma(x, y, s);
    }
}

template <int KIND, typename KT>
__device__ __forceinline__ KT gram_finish(KT s, KT prm)
{
    if constexpr (KIND == MBKK_GAUSS || KIND == MBKK_LAPLACE)
        return (KT)exp(-s / prm);
    else if constexpr (KIND == MBKK_LINEAR)
        return s;
    else
        return (s + prm) * (s + prm);
}

// VALU tasks: RPL column rows per lane (two in FP32, one in FP64), so a
// task is 32 slot rows by 64 RPL column rows, and coordinates are held in
// registers 32 / RPL at a time (the pool stride is a multiple of 32).
template <typename KT>
__host__ __device__ constexpr int gram_valu_rpl()
{
    return sizeof(KT) == 4 ? 2 : 1;
}

// Column rows eb*64 RPL + 64 q + l (q < RPL) of lane l are held in registers,
// 32 / RPL coordinates at a time; the task's slot rows are read with
// wave-uniform addresses and each coordinate serves the RPL rows.  Pairs,
// sums and the kernel value in KT; the task sum in FP64.
template <int KIND, typename KT>
__global__ __launch_bounds__(kGramWG) void k_gram_valu(const GramWork A, int d, int dp, double param,
                                                       const float *__restrict__ pool32, int zero_row)
{
    constexpr int RPL = gram_valu_rpl<KT>();
    constexpr int DC = 32 / RPL;
    const int lane = threadIdx.x & 63;
    const KT prm = (KT)param;
    __shared__ int32_t stage[kGramStage];
    // (one column set per task: the VALU plan takes Q = 1)
    gram_wave_loop<64 * RPL, false>(A, stage, blockIdx.x, [&](const GramCol &a, const GramCol &ec, int ab, int eb, int,
                                                              double &lsum) {
        bool eok[RPL];
        int re[RPL];
#pragma unroll
        for (int q = 0; q < RPL; ++q) {
            const int qe = eb * 64 * RPL + q * 64 + lane;
            eok[q] = qe < ec.n;
            re[q] = eok[q] ? (int)gram_row(ec, qe) : zero_row;
        }
        const int na = min(kGramTA, a.n - ab * kGramTA);
        const int ral = lane < na ? (int)gram_row(a, ab * kGramTA + lane) : zero_row;
        KT acc[RPL][kGramTA];
#pragma unroll
        for (int q = 0; q < RPL; ++q)
#pragma unroll
            for (int i = 0; i < kGramTA; ++i)
                acc[q][i] = 0;
        for (int t0 = 0; t0 < d; t0 += DC) {
            KT ev[RPL][DC];
#pragma unroll
            for (int q = 0; q < RPL; ++q) {
                const float *pe = pool32 + (int64_t)re[q] * dp + t0;
#pragma unroll
                for (int u = 0; u < DC; u += 4) {
                    const f32x4 v = *(const f32x4 *)(pe + u);
                    ev[q][u] = (KT)v[0];
                    ev[q][u + 1] = (KT)v[1];
                    ev[q][u + 2] = (KT)v[2];
                    ev[q][u + 3] = (KT)v[3];
                }
            }
#pragma unroll
            for (int i = 0; i < kGramTA; ++i) {
                if (i < na) {  // wave uniform
                    const int ra = __builtin_amdgcn_readlane(ral, i);
                    const float *pa = pool32 + (int64_t)ra * dp + t0;
#pragma unroll
                    for (int u = 0; u < DC; ++u) {
                        const KT au = (KT)pa[u];
#pragma unroll
                        for (int q = 0; q < RPL; ++q)
                            gram_term<KIND, KT>(acc[q][i], au, ev[q][u]);
                    }
                }
            }
        }
#pragma unroll
        for (int q = 0; q < RPL; ++q) {
            if (eok[q]) {
#pragma unroll
                for (int i = 0; i < kGramTA; ++i)
                    if (i < na)
                        lsum += (double)gram_finish<KIND, KT>(acc[q][i], prm);
            }
        }
    });
}

// MFMA tasks (Gaussian): gram_mfma_work, 5 waves per SIMD.
template <int DP>
// (fixed row stride: a task's next column tile is loaded during the current
// one's products, so the register budget asks only for 3 waves per SIMD; the
// tasks seldom fill more, since a task takes at least 4 tiles)
__global__ __launch_bounds__(kGramWG) __attribute__((amdgpu_waves_per_eu(DP > 0 ? 3 : 5))) void k_gram_mfma(
    const GramWork A, int dp_rt, int zero_row, const float *__restrict__ pool32, const float *__restrict__ poolsq,
    float c2, float c1)
{
    gram_mfma_work<DP>(A, dp_rt, zero_row, pool32, poolsq, c2, c1, blockIdx.x);
}

// ---------------------------------------------------------------------------
// plan (outside a step) and fold
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void k_gram_plan(int k, int C, int rr, uint32_t mask, int ta, int te,
                                                    const int32_t *__restrict__ ring_off,
                                                    const double *__restrict__ coef, int32_t *__restrict__ goff)
{
    __shared__ int sint[16];
    gram_plan(k, C, rr, mask, ta, te, ring_off, nullptr, coef, goff, sint);
}

// One wave per jc (gram_fold_jc).  In a step the fold runs instead inside
// the next support layout (k_prepare), with the same summation.
__global__ __launch_bounds__(256) void k_gram_fold(int k, int C, int rr, uint32_t mask, int nwaves,
                                                   const int32_t *__restrict__ goff,
                                                   const double *__restrict__ gpart, double *__restrict__ G)
{
    const int lane = threadIdx.x & 63;
    const int jc = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (jc >= k * C)
        return;
    const int j = jc / C, c = jc - j * C;
    if (!((mask >> c) & 1u))
        return;
    const double s = gram_fold_jc(goff, gpart, k * C, jc, nwaves);
    if (lane == 0) {
        double *g = G + (int64_t)j * C * C;
        g[(1 + rr) * C + c] = s;
        g[c * C + 1 + rr] = s;
    }
}

int gram_task_cols(int mfma, int fp64)
{
    return mfma ? 16 : 64 * (fp64 ? gram_valu_rpl<double>() : gram_valu_rpl<float>());
}

int gram_task_rows(int mfma) { return mfma ? kGramTAMfma : kGramTA; }
// the MFMA task loads its 16 slot rows once for up to MBKK_GRAM_QMAX column
// tiles (a power of two, at most 2^(kGramTileSteps - 1)); the VALU task
// takes one column set
#ifndef MBKK_GRAM_QMAX
#define MBKK_GRAM_QMAX 8
#endif
static_assert(MBKK_GRAM_QMAX >= 1 && MBKK_GRAM_QMAX <= 1 << (kGramTileSteps - 1), "column tiles per task");
int gram_task_qmax(int mfma) { return mfma ? MBKK_GRAM_QMAX : 1; }

void launch_gram_plan(const Layout &L, const Buffers &B, int rr, uint32_t mask, int ta, int te, hipStream_t st)
{
    hipLaunchKernelGGL(k_gram_plan, dim3(1), dim3(1024), 0, st, L.k, L.C, rr, mask, ta, te, B.ring_off, B.coef,
                       B.goff);
}

template <typename KT>
static void launch_gram_valu(const Layout &L, const Buffers &B, const GramWork &A, int kind, double param,
                             hipStream_t st)
{
    const dim3 grid(kGramWaves / (kGramWG / 64));
    const int zr = (int)L.PR;
#define MBKK_GV(K) \
    hipLaunchKernelGGL((k_gram_valu<K, KT>), grid, dim3(kGramWG), 0, st, A, L.d, L.dp, param, B.pool32, zr)
    switch (kind) {
    case MBKK_GAUSS: MBKK_GV(MBKK_GAUSS); break;
    case MBKK_LAPLACE: MBKK_GV(MBKK_LAPLACE); break;
    case MBKK_LINEAR: MBKK_GV(MBKK_LINEAR); break;
    default: MBKK_GV(MBKK_POLY2); break;
    }
#undef MBKK_GV
}

static void launch_gram_mfma(const Layout &L, const Buffers &B, const GramWork &A, double kappa, hipStream_t st)
{
    const double l2e = 1.4426950408889634;
    const float c2 = (float)(2.0 * l2e / kappa), c1 = (float)(-l2e / kappa);
    const dim3 grid(kGramWavesMfma / (kGramWG / 64));
    const int zr = (int)L.PR;
#define MBKK_GM(DP) \
    hipLaunchKernelGGL((k_gram_mfma<DP>), grid, dim3(kGramWG), 0, st, A, L.dp, zr, B.pool32, B.poolsq, c2, c1)
    switch (L.dp) {
    case 32: MBKK_GM(32); break;
    case 64: MBKK_GM(64); break;
    case 96: MBKK_GM(96); break;
    case 128: MBKK_GM(128); break;
    default: MBKK_GM(0); break;
    }
#undef MBKK_GM
}

void launch_gram(const Layout &L, const Buffers &B, int rr, uint32_t mask, int kind, double param, int fp64,
                 int mfma, bool fold, hipStream_t st)
{
    GramWork A;
    A.k = L.k;
    A.C = L.C;
    A.bmax = L.bmax;
    A.rr = rr;
    A.ring_off = B.ring_off;
    A.ring_perm = B.ring_perm;
    A.goff = B.goff;
    A.gpart = B.gpart;
    A.nwaves = gram_waves(mfma);
    if (mfma) {
        // every MFMA form: FP32 products (the BF16 forms' cross term alone is split)
        launch_gram_mfma(L, B, A, param, st);
    } else if (fp64) {
        launch_gram_valu<double>(L, B, A, kind, param, st);
    } else {
        launch_gram_valu<float>(L, B, A, kind, param, st);
    }
    if (fold)
        launch_gram_fold(L, B, rr, mask, mfma, st);
}

void launch_gram_fold(const Layout &L, const Buffers &B, int rr, uint32_t mask, int mfma, hipStream_t st)
{
    const int njc = L.k * L.C;
    hipLaunchKernelGGL(k_gram_fold, dim3((njc + 3) / 4), dim3(256), 0, st, L.k, L.C, rr, mask, gram_waves(mfma),
                       B.goff, B.gpart, B.G);
}

int gram_waves(int mfma) { return mfma ? kGramWavesMfma : kGramWaves; }

}  // namespace mbkk
