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
#include "dev_common.h"
#include "kernels.h"

namespace mbkk {

struct GramWork {
    int k, C, bmax, rr;
    const int32_t *ring_off, *ring_perm;
    const int32_t *goff;  // [k*C + 1] task offsets
    double *gpart;        // [kGramWaves + k*C] per-run partials
    int nwaves;           // waves of the work kernel (sets the task ranges)
};

constexpr int kGramWG = 256;  // 4 waves per workgroup
// LDS copy of the task offsets and the ring offsets (ints), when both fit
constexpr int kGramStage = 4096;

// gram_col with the offsets read once per wave into scalar registers.
__device__ __forceinline__ GramCol gram_col_uniform(int k, int bmax, int j, int c, const int32_t *ring_off,
                                                    const int32_t *__restrict__ ring_perm)
{
    GramCol g;
    if (c == 0) {
        g.n = 1;
        g.perm = nullptr;
        g.row0 = j;
    } else {
        const int32_t *o = ring_off + (int64_t)(c - 1) * (k + 1);
        const int o0 = __builtin_amdgcn_readfirstlane(o[j]), o1 = __builtin_amdgcn_readfirstlane(o[j + 1]);
        g.n = o1 - o0;
        g.perm = ring_perm + (int64_t)(c - 1) * bmax + o0;
        g.row0 = (int64_t)k + (int64_t)(c - 1) * bmax;
    }
    return g;
}

// Runs `task(a, e, ab, eb, lsum)` over this wave's task range; a = the slot's
// rows of center j, e = column c's rows, (ab, eb) the task's row blocks.
// Every thread of the workgroup calls it: when the task offsets and the ring
// offsets fit in `stage`, the workgroup first copies them there with
// coalesced loads, so the segment search and the column lookups read LDS.
template <int TE, class Task>
__device__ __forceinline__ void gram_wave_loop(const GramWork &A, int32_t *stage, Task &&task)
{
    const int lane = threadIdx.x & 63;
    // wave-uniform values are moved to scalar registers (readfirstlane)
    const int w = __builtin_amdgcn_readfirstlane(blockIdx.x * (kGramWG / 64) + (threadIdx.x >> 6));
    const int nJC = A.k * A.C;
    const int nro = (A.C - 1) * (A.k + 1);
    const int32_t *goff = A.goff, *ring_off = A.ring_off;
    // the task count (a scalar load): a workgroup whose waves have no task
    // leaves at once
    const int T = A.goff[nJC];
    if (T == 0)
        return;
    const int chunk = (T + A.nwaves - 1) / A.nwaves;
    if ((int64_t)blockIdx.x * (kGramWG / 64) * chunk >= T)
        return;  // workgroup uniform
    if (nJC + 1 + nro <= kGramStage) {  // workgroup uniform
        for (int i = threadIdx.x; i < nJC + 1 + nro; i += kGramWG)
            stage[i] = i <= nJC ? A.goff[i] : A.ring_off[i - (nJC + 1)];
        __syncthreads();
        goff = stage;
        ring_off = stage + nJC + 1;
    }
    const int64_t t0l = (int64_t)w * chunk;
    if (t0l >= T)
        return;  // wave uniform
    const int t0 = (int)t0l, t1 = min(T, t0 + chunk);
    int jc = __builtin_amdgcn_readfirstlane(wave_segment_of(goff, nJC, t0));
    int t = t0;
    while (t < t1) {  // wave uniform
        const int g0 = __builtin_amdgcn_readfirstlane(goff[jc]), g1 = __builtin_amdgcn_readfirstlane(goff[jc + 1]);
        const int e = min(t1, g1);
        if (t < e) {
            const int j = jc / A.C, c = jc - j * A.C;
            const GramCol a = gram_col_uniform(A.k, A.bmax, j, 1 + A.rr, ring_off, A.ring_perm);
            const GramCol ec = gram_col_uniform(A.k, A.bmax, j, c, ring_off, A.ring_perm);
            const int nE = (ec.n + TE - 1) / TE;
            double lsum = 0.0;
            for (; t < e; ++t) {
                const int u = t - g0;
                const int ab = u / nE, eb = u - ab * nE;
                task(a, ec, ab, eb, lsum);
            }
            for (int o = 32; o > 0; o >>= 1)
                lsum += __shfl_xor(lsum, o);
            if (lane == 0)
                A.gpart[w + jc] = lsum;
        }
        ++jc;
    }
}

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
    gram_wave_loop<64 * RPL>(A, stage, [&](const GramCol &a, const GramCol &ec, int ab, int eb, double &lsum) {
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

// ---------------------------------------------------------------------------
// MFMA tasks (Gaussian): exp(-(||a||^2 + ||e||^2 - 2 a.e) / kappa) with a.e
// on FP32 MFMA 16x16x4 (every MFMA form, the BF16 ones included): a task is
// a 16 x 16 block of (slot row, column row) pairs, so a cluster of b_j rows
// pads to a multiple of 16 rather than 32.  Lane l = 16 g + n supplies
// A[n][g] (slot row n) and B[g][n] (column row n) with g the quarter of the
// coordinates it sums, [g dp/4, (g+1) dp/4); it holds D[4 g + i][n], i < 4.
// DP = 0 takes the row stride at run time.
// ---------------------------------------------------------------------------
template <int DP>
__global__ __launch_bounds__(kGramWG) __attribute__((amdgpu_waves_per_eu(5))) void k_gram_mfma(
    const GramWork A, int dp_rt, int zero_row, const float *__restrict__ pool32, const float *__restrict__ poolsq,
    float c2, float c1)
{
    const int dp = DP > 0 ? DP : dp_rt;
    const int KQ = dp / 4;
    __shared__ float sqa[kGramWG / 64][16];
    __shared__ int32_t stage[kGramStage];
    const int lane = threadIdx.x & 63, wl = threadIdx.x >> 6, n = lane & 15, g = lane >> 4;
    gram_wave_loop<16>(A, stage, [&](const GramCol &a, const GramCol &ec, int ab, int eb, double &lsum) {
        const int qa = ab * 16 + n, qe = eb * 16 + n;
        // both permutation loads, then every row load, in flight together:
        // clamped indices and selects, no branches (a is a slot column, so
        // a.perm is set; column 0 of ec has no permutation and one row)
        const int32_t *ep = ec.perm ? ec.perm : a.perm;
        const int32_t pa = a.perm[min(qa, a.n - 1)];
        const int32_t pe = ep[min(qe, ec.n - 1)];
        const int64_t ra = qa < a.n ? a.row0 + pa : zero_row;
        const int64_t re = qe < ec.n ? (ec.perm ? ec.row0 + pe : ec.row0) : zero_row;
        const float sqa_v = poolsq[ra], sqe_v = poolsq[re];
        f32x4 acc;
#pragma unroll
        for (int i = 0; i < 4; ++i)
            acc[i] = 0.0f;
        const float *sa = pool32 + ra * dp + g * KQ, *se = pool32 + re * dp + g * KQ;
        if constexpr (DP > 0) {
            // the task's coordinates are all loaded before the first product
            constexpr int NS = DP / 16;
            f32x4 av[NS], ev[NS];
#pragma unroll
            for (int q = 0; q < NS; ++q) {
                av[q] = *(const f32x4 *)(sa + 4 * q);
                ev[q] = *(const f32x4 *)(se + 4 * q);
            }
            __builtin_amdgcn_sched_barrier(0);  // keep the loads ahead of the products
#pragma unroll
            for (int q = 0; q < NS; ++q)
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av[q][u], ev[q][u], acc, 0, 0, 0);
        } else {
            for (int s4 = 0; s4 < KQ; s4 += 4) {
                const f32x4 av = *(const f32x4 *)(sa + s4), ev = *(const f32x4 *)(se + s4);
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av[u], ev[u], acc, 0, 0, 0);
            }
        }
        // lane n (g = 0) publishes the norm of slot row n for the output rows m
        if (g == 0)
            sqa[wl][n] = c1 * sqa_v;
        const float se_ = c1 * sqe_v;
        // lane: column n (column row), rows m = 4 g + i (slot rows); the row
        // norms were written by this wave (in-order LDS access)
        if (qe < ec.n) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int m = 4 * g + i;
                if (ab * 16 + m < a.n)
                    lsum += (double)__builtin_amdgcn_exp2f(fmaf(acc[i], c2, sqa[wl][m] + se_));
            }
        }
    });
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
