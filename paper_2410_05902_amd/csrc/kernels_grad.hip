// Differentiation form of the batch objective (Section 3's f_B, Gaussian
// kernel in the bandwidth form K_s(x, y) = exp(-||x - y||^2 / (2 s^2))):
//   f(X_B, s) = (1/b) sum_x [1 - 2 P_j(x) + N_j],  j = j*(x) the argmin label,
//   P_j(x) = sum_{e in C_j} w_e K_s(x, y_e),  N_j = sum_{e, e' in C_j} w_e w_e' K_s(y_e, y_e').
// With the support points y_e and weights w_e held constant and hard labels:
//   df/dx   = (2 / (b s^2)) sum_e w_e K_s(x, y_e) (x - y_e)
//   df/ds   = (1/b) sum_x [-2 sum_e w_e K_s(x, y_e) ||x - y_e||^2 / s^3 + dN_j/ds]
//   dN_j/ds = sum_{e, e'} w_e w_e' K_s(y_e, y_e') ||y_e - y_e'||^2 / s^3.
// Kernel values are recomputed here (nothing of size b x M is stored).  The
// Gaussian MFMA forms (FP32 / BF16 contexts) take the MFMA kernels below the
// VALU ones: FP32 products and kernel values, FP64 sums; the FP64 form (and
// layouts without the MFMA padding) take the VALU kernels, in FP64.
#include "dev_common.h"
#include "kernels.h"

namespace mbkk {

// ---------------------------------------------------------------------------
// N_j(s) and dN_j/ds over all ordered pairs of center j's support entries,
// split over kSnSplit workgroups per center (workgroup g takes the a tiles
// g, g + kSnSplit, ...), so that one large center is spread over the chip.
// Each writes its partial sums; k_selfnorm_fold adds them in workgroup order.
// The pairs are taken in tiles of 16 rows a by 64 rows e
// whose coordinates are staged in LDS (128 coordinates per pass), so each
// coordinate is read from global memory once per tile instead of once per
// pair; thread (ta, te) of a tile owns the pairs (ta, te + 16 q), q < 4.
// Every thread sums its pairs in a fixed order, and the tree reduction is
// fixed as well (deterministic).
// ---------------------------------------------------------------------------
struct SelfNormArgs {
    int k, d, dp;
    const int32_t *seg_off, *sup_row;
    const double *sup_w64;
    const float *pool32;
    double inv_kappa;  // 1 / (2 s^2)
    double inv_s3;     // 1 / s^3
    double *part;      // [k][kSnSplit][2]
    double *N, *dN;
};

constexpr int kSnTA = 16, kSnTE = 64, kSnDim = 128;

__global__ __launch_bounds__(256) void k_selfnorm_sigma(const SelfNormArgs A)
{
    __shared__ float sa[kSnTA][kSnDim + 1], se[kSnTE][kSnDim + 1];
    __shared__ double rn[256], rd[256];
    const int j = blockIdx.x, g = blockIdx.y, tid = threadIdx.x;
    const int ta = tid / kSnTA, te = tid % kSnTA;  // a row of the tile, first e row (then +16 q)
    const int s0 = A.seg_off[j], L = A.seg_off[j + 1] - s0;
    double sn = 0.0, sd = 0.0;
    for (int a0 = g * kSnTA; a0 < L; a0 += kSnSplit * kSnTA) {
        for (int e0 = 0; e0 < L; e0 += kSnTE) {
            double d2[4] = {0.0, 0.0, 0.0, 0.0};
            // pool rows are zero from d up to the stride dp, so passes run over dp
            for (int t0 = 0; t0 < A.dp; t0 += kSnDim) {
                const int nt = min(kSnDim, A.dp - t0);
                // this thread's 16-byte chunks of the tiles: all pool-row indices
                // first, then all coordinate loads, so each pass waits on two
                // rounds of independent loads
                constexpr int CPRow = kSnDim / 4, Q = (kSnTA + kSnTE) * CPRow / 256;
                int ridx[Q];
#pragma unroll
                for (int q = 0; q < Q; ++q) {
                    const int i = tid + 256 * q, r = i / CPRow, c4 = i % CPRow;
                    const int row = r < kSnTA ? a0 + r : e0 + (r - kSnTA);
                    ridx[q] = row < L && 4 * c4 < nt ? A.sup_row[s0 + row] : -1;
                }
                f32x4 v[Q];
#pragma unroll
                for (int q = 0; q < Q; ++q) {
                    const int c4 = (tid + 256 * q) % CPRow;
                    const f32x4 z = {0.0f, 0.0f, 0.0f, 0.0f};
                    v[q] = ridx[q] >= 0 ? *(const f32x4 *)(A.pool32 + (int64_t)ridx[q] * A.dp + t0 + 4 * c4) : z;
                }
                __syncthreads();  // the previous pass is done with the tiles
#pragma unroll
                for (int q = 0; q < Q; ++q) {
                    const int i = tid + 256 * q, r = i / CPRow, c4 = i % CPRow;
                    float *dst = r < kSnTA ? &sa[r][4 * c4] : &se[r - kSnTA][4 * c4];
                    dst[0] = v[q][0];
                    dst[1] = v[q][1];
                    dst[2] = v[q][2];
                    dst[3] = v[q][3];
                }
                __syncthreads();
                for (int t = 0; t < nt; ++t) {
                    const double x = (double)sa[ta][t];
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const double v = x - (double)se[te + 16 * q][t];
                        d2[q] = fma(v, v, d2[q]);
                    }
                }
            }
            const int a = a0 + ta;
            const double wa = a < L ? A.sup_w64[s0 + a] : 0.0;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int e = e0 + te + 16 * q;
                const double we = e < L ? A.sup_w64[s0 + e] : 0.0;
                if (wa != 0.0 && we != 0.0) {
                    const double kv = exp(-d2[q] * A.inv_kappa);
                    sn = fma(wa * we, kv, sn);
                    sd = fma(wa * we * kv, d2[q], sd);
                }
            }
        }
    }
    rn[tid] = sn;
    rd[tid] = sd;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (tid < s) {
            rn[tid] += rn[tid + s];
            rd[tid] += rd[tid + s];
        }
        __syncthreads();
    }
    if (tid == 0) {
        A.part[((int64_t)j * kSnSplit + g) * 2] = rn[0];
        A.part[((int64_t)j * kSnSplit + g) * 2 + 1] = rd[0];
    }
}

// N_j and dN_j/ds from the kSnSplit partial sums of center j, in order.
__global__ __launch_bounds__(256) void k_selfnorm_fold(const SelfNormArgs A)
{
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= A.k)
        return;
    double sn = 0.0, sd = 0.0;
    for (int g = 0; g < kSnSplit; ++g) {
        sn += A.part[((int64_t)j * kSnSplit + g) * 2];
        sd += A.part[((int64_t)j * kSnSplit + g) * 2 + 1];
    }
    A.N[j] = sn;
    A.dN[j] = sd * A.inv_s3;
}

void launch_selfnorm_sigma(const Layout &L, const Buffers &B, double sigma, double *N, double *dN, hipStream_t st)
{
    SelfNormArgs A;
    A.k = L.k;
    A.d = L.d;
    A.dp = L.dp;
    A.seg_off = B.seg_off;
    A.sup_row = B.sup_row;
    A.sup_w64 = B.sup_w64;
    A.pool32 = B.pool32;
    A.inv_kappa = 1.0 / (2.0 * sigma * sigma);
    A.inv_s3 = 1.0 / (sigma * sigma * sigma);
    A.part = B.sn_part;
    A.N = N;
    A.dN = dN;
    hipLaunchKernelGGL(k_selfnorm_sigma, dim3((unsigned)L.k, kSnSplit), dim3(256), 0, st, A);
    hipLaunchKernelGGL(k_selfnorm_fold, dim3((unsigned)((L.k + 255) / 256)), dim3(256), 0, st, A);
}

// ---------------------------------------------------------------------------
// Per-row gradient: one wave per batch row x, lane l holds coordinates
// l + 64 c (c < CH) of x and of the accumulated sum_e w_e K (x - y_e); each
// support entry of the row's center costs one wave reduction of ||x - y_e||^2.
// Writes dX (scaled) and the row's term of df/ds.
// ---------------------------------------------------------------------------
struct GradRowArgs {
    int b, d, dp, k;
    const float *xb;  // [b x d] dense
    const int32_t *labels;
    const int32_t *seg_off, *sup_row;
    const double *sup_w64;
    const float *pool32;
    const double *dN;
    double inv_kappa, inv_s3, cx, cs;  // cx = 2 g / (b s^2), cs = g / b
    float *dX;
    double *rowds;   // [b]
    int32_t *flags;  // flags[2]: a label outside [0, k)
};

template <int CH>
__global__ __launch_bounds__(256) void k_grad_rows(const GradRowArgs A)
{
    const int lane = threadIdx.x & 63;
    const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (row >= A.b)
        return;
    const int j = A.labels[row];
    if (j < 0 || j >= A.k) {
        if (lane == 0) {
            atomicOr(&A.flags[2], 1);
            A.rowds[row] = 0.0;
        }
        for (int t = lane; t < A.d; t += 64)
            A.dX[(int64_t)row * A.d + t] = 0.0f;
        return;
    }
    double x[CH], acc[CH];
#pragma unroll
    for (int c = 0; c < CH; ++c) {
        const int t = lane + 64 * c;
        x[c] = t < A.d ? (double)A.xb[(int64_t)row * A.d + t] : 0.0;
        acc[c] = 0.0;
    }
    double q = 0.0;
    // U entries at a time: their loads and wave reductions are independent
    // and overlap; the sums still take the entries in order, one by one
    constexpr int U = 4;
    const int s1 = A.seg_off[j + 1];
    for (int s = A.seg_off[j]; s < s1; s += U) {
        double w[U], part[U], diff[U][CH];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            w[u] = s + u < s1 ? A.sup_w64[s + u] : 0.0;
            part[u] = 0.0;
            const float *y = A.pool32 + (int64_t)A.sup_row[s + u < s1 ? s + u : s] * A.dp;
#pragma unroll
            for (int c = 0; c < CH; ++c) {
                const int t = lane + 64 * c;
                diff[u][c] = t < A.d ? x[c] - (double)y[t] : 0.0;
                part[u] = fma(diff[u][c], diff[u][c], part[u]);
            }
        }
        for (int o = 32; o > 0; o >>= 1)
#pragma unroll
            for (int u = 0; u < U; ++u)
                part[u] += __shfl_xor(part[u], o);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (w[u] == 0.0)
                continue;  // (wave uniform)
            const double wk = w[u] * exp(-part[u] * A.inv_kappa);
#pragma unroll
            for (int c = 0; c < CH; ++c)
                acc[c] = fma(wk, diff[u][c], acc[c]);
            q = fma(wk, part[u], q);
        }
    }
#pragma unroll
    for (int c = 0; c < CH; ++c) {
        const int t = lane + 64 * c;
        if (t < A.d)
            A.dX[(int64_t)row * A.d + t] = (float)(A.cx * acc[c]);
    }
    if (lane == 0)
        A.rowds[row] = A.cs * (-2.0 * q * A.inv_s3 + A.dN[j]);
}

// Sum of the per-row terms in a fixed order (one workgroup).
__global__ __launch_bounds__(1024) void k_sum_rows(const double *v, int n, double *out)
{
    __shared__ double r[1024];
    const int tid = threadIdx.x;
    double s = 0.0;
    for (int i = tid; i < n; i += 1024)
        s += v[i];
    r[tid] = s;
    __syncthreads();
    for (int o = 512; o > 0; o >>= 1) {
        if (tid < o)
            r[tid] += r[tid + o];
        __syncthreads();
    }
    if (tid == 0)
        *out = r[0];
}

// ===========================================================================
// The same quantities on FP32 MFMA (Gaussian MFMA forms, row stride <= 128):
// kernel tiles are recomputed from x.y products, as the forward's cross term
// is; sums that leave a tile are FP64.  A center's segment is cut into
// blocks of 32 entries; entries of the last block past the segment's end
// (packed segments are not multiples of 32) take weight 0 and the zero row.
//
// 32 x 32 tiles on v_mfma_f32_32x32x2f32: lane l = 32 h + n supplies
// A[n][h] and B[h][n] of a k-step, and holds C[m][n] for
// m = 8 (i/4) + 4 h + i%4, i < 16.
// ===========================================================================

// Self norms at s: task (j, a, e) is the 32 x 32 block of entries a and e of
// center j (all ordered block pairs: nb_j^2 tasks, offsets toff); kGramWaves
// waves take equal contiguous task ranges and store one FP64 partial per
// (wave, center) run at part[w + j] (N) and part2[w + j] (the d2-weighted
// sum); the fold adds them in wave order (gram_fold_jc), as the Gram blocks.
struct SigmaGramArgs {
    int k, dp;
    int sup_cap;         // sup_row[sup_cap] is the zero pool row
    const int32_t *seg_off, *sup_row, *toff;
    const double *sup_w64;
    const float *pool32, *poolsq;
    float c;             // -log2(e) / (2 s^2)
    double inv_s3;
    double *part, *part2;
    double *N, *dN;
};

__global__ __launch_bounds__(1024) void k_sigma_plan(int k, const int32_t *__restrict__ seg_off,
                                                    int32_t *__restrict__ toff)
{
    __shared__ int sint[16];
    const int tid = threadIdx.x, per = (k + 1023) / 1024;
    const int j0 = min(k, tid * per), j1 = min(k, j0 + per);
    int local = 0;
    for (int j = j0; j < j1; ++j) {
        const int nb = (seg_off[j + 1] - seg_off[j] + 31) / 32;
        local += nb * nb;
    }
    int total;
    int run = block_exclusive_scan(local, sint, &total);
    for (int j = j0; j < j1; ++j) {
        toff[j] = run;
        const int nb = (seg_off[j + 1] - seg_off[j] + 31) / 32;
        run += nb * nb;
    }
    if (tid == 0)
        toff[k] = total;
}

template <int DP>
__global__ __launch_bounds__(256) void k_sigma_gram(const SigmaGramArgs A)
{
    __shared__ float sqa[4][32];
    __shared__ double wa[4][32];
    const int lane = threadIdx.x & 63, wl = threadIdx.x >> 6, n = lane & 31, h = lane >> 5;
    const int w = blockIdx.x * 4 + wl;
    const int T = A.toff[A.k];
    if (T == 0)
        return;
    const int chunk = (T + kGramWaves - 1) / kGramWaves;
    const int64_t t0l = (int64_t)w * chunk;
    if (t0l >= T)
        return;  // wave uniform
    const int t0 = (int)t0l, t1 = min(T, t0 + chunk);
    constexpr int KS = DP / 2;
    int j = wave_segment_of(A.toff, A.k, t0);
    int t = t0;
    while (t < t1) {  // wave uniform
        const int g0 = A.toff[j], g1 = A.toff[j + 1];
        const int e = min(t1, g1);
        if (t < e) {
            const int s0 = A.seg_off[j], s1 = A.seg_off[j + 1], nb = (s1 - s0 + 31) / 32;
            double ln = 0.0, ld = 0.0;
            for (; t < e; ++t) {
                const int u = t - g0, ab = u / nb, eb = u - ab * nb;
                const int sa = s0 + 32 * ab + n, se = s0 + 32 * eb + n;
                const bool oka = sa < s1, oke = se < s1;  // past the segment: weight 0, zero row
                const int64_t ra = A.sup_row[oka ? sa : A.sup_cap], re = A.sup_row[oke ? se : A.sup_cap];
                if (h == 0) {
                    sqa[wl][n] = A.poolsq[ra];
                    wa[wl][n] = oka ? A.sup_w64[sa] : 0.0;
                }
                const float sqe = A.poolsq[re];
                const double we = oke ? A.sup_w64[se] : 0.0;
                f32x16 acc;
#pragma unroll
                for (int i = 0; i < 16; ++i)
                    acc[i] = 0.0f;
                // the u-th MFMA of step q takes coordinate 8 q + 4 h + u: the
                // two lanes of a row read 32 contiguous bytes per step
                const float *pa = A.pool32 + ra * DP + 4 * h, *pe = A.pool32 + re * DP + 4 * h;
#pragma unroll
                for (int s4 = 0; s4 < KS; s4 += 4) {
                    const f32x4 av = *(const f32x4 *)(pa + 2 * s4), ev = *(const f32x4 *)(pe + 2 * s4);
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av[q], ev[q], acc, 0, 0, 0);
                }
                __builtin_amdgcn_wave_barrier();  // sqa / wa of this task were written by this wave
#pragma unroll
                for (int i = 0; i < 16; ++i) {
                    const int m = 8 * (i >> 2) + 4 * h + (i & 3);
                    const float d2 = fmaxf(fmaf(-2.0f, acc[i], sqa[wl][m] + sqe), 0.0f);
                    const double pk = wa[wl][m] * we * (double)__builtin_amdgcn_exp2f(A.c * d2);
                    ln += pk;
                    ld = fma(pk, (double)d2, ld);
                }
                __builtin_amdgcn_wave_barrier();  // before the next task's sqa / wa
            }
            for (int o = 32; o > 0; o >>= 1) {
                ln += __shfl_xor(ln, o);
                ld += __shfl_xor(ld, o);
            }
            if (lane == 0) {
                A.part[w + j] = ln;
                A.part2[w + j] = ld;
            }
        }
        ++j;
    }
}

__global__ __launch_bounds__(256) void k_sigma_fold(const SigmaGramArgs A)
{
    const int lane = threadIdx.x & 63;
    const int j = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (j >= A.k)
        return;
    const double sn = gram_fold_jc(A.toff, A.part, A.k, j, kGramWaves);
    const double sd = gram_fold_jc(A.toff, A.part2, A.k, j, kGramWaves);
    if (lane == 0) {
        A.N[j] = sn;
        A.dN[j] = sd * A.inv_s3;
    }
}

bool sigma_mfma_ok(const Layout &L)
{
    if (L.pad != kMfmaPad || !(L.dp == 32 || L.dp == 64 || L.dp == 96 || L.dp == 128))
        return false;
    const double nb = (double)L.Mcap / 32.0;  // at most this many blocks in one center
    return nb * nb < 2147483647.0;
}

void launch_sigma_norms(const Layout &L, const Buffers &B, double sigma, double *N, double *dN, hipStream_t st)
{
    SigmaGramArgs A;
    A.k = L.k;
    A.dp = L.dp;
    A.sup_cap = (int)L.Mcap;
    A.seg_off = B.seg_off;
    A.sup_row = B.sup_row;
    A.toff = B.sg_toff;
    A.sup_w64 = B.sup_w64;
    A.pool32 = B.pool32;
    A.poolsq = B.poolsq;
    A.c = (float)(-1.4426950408889634 / (2.0 * sigma * sigma));
    A.inv_s3 = 1.0 / (sigma * sigma * sigma);
    A.part = B.sg_part;
    A.part2 = B.sg_part + kGramWaves + L.k;
    A.N = N;
    A.dN = dN;
    hipLaunchKernelGGL(k_sigma_plan, dim3(1), dim3(1024), 0, st, L.k, (const int32_t *)B.seg_off, B.sg_toff);
    const dim3 grid(kGramWaves / 4);
    switch (L.dp) {
    case 32: hipLaunchKernelGGL(k_sigma_gram<32>, grid, dim3(256), 0, st, A); break;
    case 64: hipLaunchKernelGGL(k_sigma_gram<64>, grid, dim3(256), 0, st, A); break;
    case 96: hipLaunchKernelGGL(k_sigma_gram<96>, grid, dim3(256), 0, st, A); break;
    default: hipLaunchKernelGGL(k_sigma_gram<128>, grid, dim3(256), 0, st, A); break;
    }
    hipLaunchKernelGGL(k_sigma_fold, dim3((unsigned)((L.k + 3) / 4)), dim3(256), 0, st, A);
}

// ---------------------------------------------------------------------------
// Backward on MFMA.  The rows are grouped by label (k_group_labels: counts,
// offsets, a scatter; the order inside a group is immaterial, since every
// row's result depends on its own row only), and task (j, r) takes rows
// 32 r .. 32 r + 31 of center j's group against the whole support of j:
//   per 32-entry block of the support (the block's owner among 4 waves):
//     T   = X Y^T on MFMA, d2 = |x|^2 + |y|^2 - 2 T, P = w K(d2), Q = P d2,
//     R  += P 1, S += Q 1  (row sums, FP64),
//     G  += P Y            (32 x dp on MFMA, P through LDS into the A layout);
//   then, summed over the 4 waves in order,
//     dX  = (2 g / (b s^2)) (x R - G),
//     row term of df/ds = (g / b) (-2 S / s^3 + dN_j).
// ---------------------------------------------------------------------------
struct GroupArgs {
    int b, k, d;
    const int32_t *labels;
    int32_t *cnt, *cur;   // [k] counts and scatter cursors (cleared here)
    int32_t *loff;        // [k+1] row offsets of the groups
    int32_t *rtoff;       // [k+1] offsets of the 32-row tasks
    int32_t *perm;        // [b] rows grouped by label
    float *dX;            // rows with a bad label: zeroed
    double *rowds;
    int32_t *flags;       // flags[2]: a label outside [0, k)
    int32_t *ticket;      // cleared here for the grad kernel
};

// One workgroup.  With k <= kGroupLdsK the counters live in LDS (LDS
// atomics); otherwise in the workspace (device atomics, read back with atomic
// loads).  Every phase is separated by a barrier.
constexpr int kGroupLdsK = 8192;

template <bool LDS>
__global__ __launch_bounds__(1024) void k_group_labels(const GroupArgs A)
{
    __shared__ int sint[16];
    __shared__ int lcnt[LDS ? kGroupLdsK : 1], lcur[LDS ? kGroupLdsK : 1];
    int *cnt = LDS ? lcnt : A.cnt;
    int *cur = LDS ? lcur : A.cur;
    auto rd = [&](const int *p) -> int {
        if constexpr (LDS)
            return *p;
        else
            return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    };
    const int tid = threadIdx.x;
    for (int j = tid; j < A.k; j += 1024) {
        cnt[j] = 0;
        cur[j] = 0;
    }
    if (tid == 0)
        *A.ticket = 0;  // the grad kernel's count of finished tasks
    if constexpr (!LDS)
        __threadfence();
    __syncthreads();
    for (int r = tid; r < A.b; r += 1024) {
        const int j = A.labels[r];
        if (j >= 0 && j < A.k) {
            atomicAdd(&cnt[j], 1);
        } else {
            atomicOr(&A.flags[2], 1);
            A.rowds[r] = 0.0;
            for (int t = 0; t < A.d; ++t)
                A.dX[(int64_t)r * A.d + t] = 0.0f;
        }
    }
    if constexpr (!LDS)
        __threadfence();
    __syncthreads();
    const int per = (A.k + 1023) / 1024;
    const int j0 = min(A.k, tid * per), j1 = min(A.k, j0 + per);
    int lrow = 0, ltask = 0;
    for (int j = j0; j < j1; ++j) {
        const int c = rd(&cnt[j]);
        lrow += c;
        ltask += (c + 31) / 32;
    }
    int trow, ttask;
    int rrun = block_exclusive_scan(lrow, sint, &trow);
    int trun = block_exclusive_scan(ltask, sint, &ttask);
    for (int j = j0; j < j1; ++j) {
        const int c = rd(&cnt[j]);
        A.loff[j] = rrun;
        A.rtoff[j] = trun;
        cur[j] = rrun;  // (this thread's own centers: no other thread touched them yet)
        rrun += c;
        trun += (c + 31) / 32;
    }
    if (tid == 0) {
        A.loff[A.k] = trow;
        A.rtoff[A.k] = ttask;
    }
    if constexpr (!LDS)
        __threadfence();
    __syncthreads();
    for (int r = tid; r < A.b; r += 1024) {
        const int j = A.labels[r];
        if (j >= 0 && j < A.k)
            A.perm[atomicAdd(&cur[j], 1)] = r;
    }
}

struct GradMfmaArgs {
    int b, d, k;
    const int32_t *loff, *rtoff, *perm, *labels;
    const int32_t *seg_off, *sup_row;
    const float *sup_w;
    const float *pool32, *poolsq;
    const float *bat32, *batsq;  // the coordinates, gathered with row stride DP
    int64_t zero_row;            // pool row of zeros (rows past a group's end)
    int sup_cap;                 // sup_row[sup_cap] is the zero pool row, sup_w[sup_cap] = 0
    const double *dN;
    float c;                     // -log2(e) / (2 s^2)
    double inv_s3, cx, cs;       // cx = 2 g / (b s^2), cs = g / b
    float *dX;
    double *rowds;
    int32_t *ticket;             // tasks finished (cleared by k_group_labels)
    double *out;                 // df/ds: the sum of rowds, by the last task
};

// Each wave stages the 32 support rows of its block in LDS (row stride DP + 4
// floats: 16-byte reads at the k-steps' offsets hit distinct banks); the
// dot products read them there, and so does the contraction, whose operand
// is the same rows read down the columns.  The rows of a wave's next block
// are loaded into registers while the current one is multiplied, so one
// block's global latency hides behind the previous block's matrix work.
// NW waves per workgroup take the support blocks round robin.
template <int DP>
__host__ __device__ constexpr int grad_waves()
{
    return DP <= 64 ? 8 : 4;
}

template <int DP>
__global__ __launch_bounds__(64 * grad_waves<DP>()) void k_grad_mfma(const GradMfmaArgs A)
{
    constexpr int NW = grad_waves<DP>();
    constexpr int KS = DP / 2, NT = DP / 32, YS = DP + 4, NV = KS / 4;
    __shared__ __attribute__((aligned(16))) float Yl[NW][32][YS];
    __shared__ float Pl[NW][32][33];
    __shared__ float Gp[32][DP + 1];
    __shared__ double Rp[NW][32], Sp[NW][32];
    __shared__ double red[16];
    __shared__ float xsq[32];
    __shared__ int rows[32];
    __shared__ int last;
    const int lane = threadIdx.x & 63, wl = threadIdx.x >> 6, n = lane & 31, h = lane >> 5;
    const int task = blockIdx.x;
    const int ntask = A.rtoff[A.k];
    if (task >= ntask)
        return;  // block uniform
    const int j = wave_segment_of(A.rtoff, A.k, task);
    const int r0 = A.loff[j] + 32 * (task - A.rtoff[j]);
    const int nr = min(32, A.loff[j + 1] - r0);
    if (threadIdx.x < 32) {
        const int row = threadIdx.x < nr ? A.perm[r0 + threadIdx.x] : -1;
        rows[threadIdx.x] = row;
        xsq[threadIdx.x] = row >= 0 ? A.batsq[row] : 0.0f;
    }
    __syncthreads();
    // this lane's A fragments: row n of the task, coordinates 8 q + 4 h + u
    // (the u-th MFMA of step q), so the two lanes of a row read 32
    // contiguous bytes per step
    const int myrow = rows[n];
    const float *px = myrow >= 0 ? A.bat32 + (int64_t)myrow * DP + 4 * h : A.pool32 + A.zero_row * DP + 4 * h;
    f32x4 xf[NV];
#pragma unroll
    for (int q = 0; q < NV; ++q)
        xf[q] = *(const f32x4 *)(px + 8 * q);
    f32x16 G[NT];
#pragma unroll
    for (int tb = 0; tb < NT; ++tb)
#pragma unroll
        for (int i = 0; i < 16; ++i)
            G[tb][i] = 0.0f;
    double R = 0.0, S = 0.0;  // lanes < 32: row n's sum of P; lanes >= 32: of P d2
    const int s0 = A.seg_off[j], s1 = A.seg_off[j + 1], nb = (s1 - s0 + 31) / 32;
    float(*Y)[YS] = Yl[wl];
    float(*P)[33] = Pl[wl];
    // block eb's row n (this lane's coordinates 8 q + 4 h + u), weight and norm: loaded one block ahead
    f32x4 yv[NV];
    float we = 0.0f, sqe = 0.0f;
    auto fetch = [&](int eb) {
        const int se0 = s0 + 32 * eb + n;
        const int se = se0 < s1 ? se0 : A.sup_cap;  // past the segment: weight 0, zero row
        const int64_t re = A.sup_row[se];
        we = A.sup_w[se];
        sqe = A.poolsq[re];
        const float *pe = A.pool32 + re * DP + 4 * h;
#pragma unroll
        for (int q = 0; q < NV; ++q)
            yv[q] = *(const f32x4 *)(pe + 8 * q);
    };
    if (wl < nb)
        fetch(wl);
    for (int eb = wl; eb < nb; eb += NW) {  // wave uniform
        __builtin_amdgcn_wave_barrier();  // the previous block is done with the tiles
#pragma unroll
        for (int q = 0; q < NV; ++q)
            *(f32x4 *)&Y[n][8 * q + 4 * h] = yv[q];
        const float w_cur = we, sq_cur = sqe;
        if (eb + NW < nb)
            fetch(eb + NW);
        __builtin_amdgcn_wave_barrier();
        f32x16 acc;
#pragma unroll
        for (int i = 0; i < 16; ++i)
            acc[i] = 0.0f;
#pragma unroll
        for (int q = 0; q < NV; ++q) {
            const f32x4 ev = *(const f32x4 *)&Y[n][8 * q + 4 * h];
#pragma unroll
            for (int u = 0; u < 4; ++u)
                acc = __builtin_amdgcn_mfma_f32_32x32x2f32(xf[q][u], ev[u], acc, 0, 0, 0);
        }
        float qv[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int m = 8 * (i >> 2) + 4 * h + (i & 3);
            const float d2 = fmaxf(fmaf(-2.0f, acc[i], xsq[m] + sq_cur), 0.0f);
            const float p = w_cur * __builtin_amdgcn_exp2f(A.c * d2);
            P[m][n] = p;
            qv[i] = p * d2;
        }
        __builtin_amdgcn_wave_barrier();  // P is in LDS (one wave's in-order accesses)
        // G += P Y: k-steps over the block's entries, two per step; all operands
        // read first
        float pa[16], yb[16][NT];
#pragma unroll
        for (int s = 0; s < 16; ++s) {
            pa[s] = P[n][2 * s + h];
#pragma unroll
            for (int tb = 0; tb < NT; ++tb)
                yb[s][tb] = Y[2 * s + h][32 * tb + n];
        }
        if (h == 0) {  // row n's sum of P, four partial sums
            double t0 = 0.0, t1 = 0.0, t2 = 0.0, t3 = 0.0;
#pragma unroll
            for (int c = 0; c < 32; c += 4) {
                t0 += (double)P[n][c];
                t1 += (double)P[n][c + 1];
                t2 += (double)P[n][c + 2];
                t3 += (double)P[n][c + 3];
            }
            R += (t0 + t1) + (t2 + t3);
        }
#pragma unroll
        for (int s = 0; s < 16; ++s)
#pragma unroll
            for (int tb = 0; tb < NT; ++tb)
                G[tb] = __builtin_amdgcn_mfma_f32_32x32x2f32(pa[s], yb[s][tb], G[tb], 0, 0, 0);
        // P d2 into the tile (P's reads are done), then row n's sum of it
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int m = 8 * (i >> 2) + 4 * h + (i & 3);
            P[m][n] = qv[i];
        }
        __builtin_amdgcn_wave_barrier();
        if (h == 1) {
            double t0 = 0.0, t1 = 0.0, t2 = 0.0, t3 = 0.0;
#pragma unroll
            for (int c = 0; c < 32; c += 4) {
                t0 += (double)P[n][c];
                t1 += (double)P[n][c + 1];
                t2 += (double)P[n][c + 2];
                t3 += (double)P[n][c + 3];
            }
            S += (t0 + t1) + (t2 + t3);
        }
    }
    // the waves' partial sums, added in wave order through one LDS tile
    if (h == 0)
        Rp[wl][n] = R;
    else
        Sp[wl][n] = S;
    for (int q = 0; q < NW; ++q) {
        if (wl == q) {
#pragma unroll
            for (int tb = 0; tb < NT; ++tb)
#pragma unroll
                for (int i = 0; i < 16; ++i) {
                    const int m = 8 * (i >> 2) + 4 * h + (i & 3);
                    float *gp = &Gp[m][32 * tb + n];
                    *gp = q == 0 ? G[tb][i] : *gp + G[tb][i];
                }
        }
        __syncthreads();
    }
    for (int idx = threadIdx.x; idx < 32 * A.d; idx += 64 * NW) {
        const int m = idx / A.d, t = idx - m * A.d;
        const int row = rows[m];
        if (row < 0)
            continue;
        double Rm = 0.0;
#pragma unroll
        for (int q = 0; q < NW; ++q)
            Rm += Rp[q][m];
        const double x = (double)A.bat32[(int64_t)row * DP + t];
        A.dX[(int64_t)row * A.d + t] = (float)(A.cx * (x * Rm - (double)Gp[m][t]));
    }
    if (threadIdx.x < 32) {
        const int m = threadIdx.x, row = rows[m];
        if (row >= 0) {
            double Sm = 0.0;
#pragma unroll
            for (int q = 0; q < NW; ++q)
                Sm += Sp[q][m];
            A.rowds[row] = A.cs * (-2.0 * Sm * A.inv_s3 + A.dN[j]);
        }
    }
    // the last task to finish sums the row terms of df/ds in row order
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0)
        last = atomicAdd(A.ticket, 1) == ntask - 1;
    __syncthreads();
    if (last) {
        __threadfence();
        double v = 0.0;
        for (int r = threadIdx.x; r < A.b; r += 64 * NW)
            v += __hip_atomic_load(&A.rowds[r], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        v = block_sum(v, red);
        if (threadIdx.x == 0)
            *A.out = v;
    }
}

void launch_grad_mfma(const Layout &L, const Buffers &B, int b, double sigma, const int32_t *labels, double g,
                      const double *dN, float *dX, double *rowds, double *out, hipStream_t st)
{
    GroupArgs Gq;
    Gq.b = b;
    Gq.k = L.k;
    Gq.d = L.d;
    Gq.labels = labels;
    Gq.cnt = B.gr_cnt;
    Gq.cur = B.gr_cnt + L.k;
    Gq.loff = B.gr_loff;
    Gq.rtoff = B.gr_rtoff;
    Gq.perm = B.gr_perm;
    Gq.dX = dX;
    Gq.rowds = rowds;
    Gq.flags = B.flags;
    Gq.ticket = B.gr_cnt + 2 * L.k;
    if (L.k <= kGroupLdsK)
        hipLaunchKernelGGL(k_group_labels<true>, dim3(1), dim3(1024), 0, st, Gq);
    else
        hipLaunchKernelGGL(k_group_labels<false>, dim3(1), dim3(1024), 0, st, Gq);
    GradMfmaArgs A;
    A.b = b;
    A.d = L.d;
    A.k = L.k;
    A.loff = B.gr_loff;
    A.rtoff = B.gr_rtoff;
    A.perm = B.gr_perm;
    A.labels = labels;
    A.seg_off = B.seg_off;
    A.sup_row = B.sup_row;
    A.sup_w = B.sup_w;
    A.pool32 = B.pool32;
    A.poolsq = B.poolsq;
    A.bat32 = B.bat32;
    A.batsq = B.batsq;
    A.zero_row = L.PR;
    A.sup_cap = (int)L.Mcap;
    A.dN = dN;
    A.c = (float)(-1.4426950408889634 / (2.0 * sigma * sigma));
    A.inv_s3 = 1.0 / (sigma * sigma * sigma);
    A.cx = 2.0 * g / ((double)b * sigma * sigma);
    A.cs = g / (double)b;
    A.dX = dX;
    A.rowds = rowds;
    A.ticket = B.gr_cnt + 2 * L.k;
    A.out = out;
    // at most ceil(b / 32) + k tasks (each group adds at most one partial block)
    const dim3 grid((unsigned)((b + 31) / 32 + L.k));
    switch (L.dp) {
    case 32: hipLaunchKernelGGL(k_grad_mfma<32>, grid, dim3(64 * grad_waves<32>()), 0, st, A); break;
    case 64: hipLaunchKernelGGL(k_grad_mfma<64>, grid, dim3(64 * grad_waves<64>()), 0, st, A); break;
    case 96: hipLaunchKernelGGL(k_grad_mfma<96>, grid, dim3(64 * grad_waves<96>()), 0, st, A); break;
    default: hipLaunchKernelGGL(k_grad_mfma<128>, grid, dim3(64 * grad_waves<128>()), 0, st, A); break;
    }
}

int grad_max_dim() { return 64 * 16; }

void launch_grad_rows(const Layout &L, const Buffers &B, const float *xb, int b, double sigma, const int32_t *labels,
                      double g, const double *dN, float *dX, double *rowds, double *out, hipStream_t st)
{
    GradRowArgs A;
    A.b = b;
    A.d = L.d;
    A.dp = L.dp;
    A.k = L.k;
    A.xb = xb;
    A.labels = labels;
    A.seg_off = B.seg_off;
    A.sup_row = B.sup_row;
    A.sup_w64 = B.sup_w64;
    A.pool32 = B.pool32;
    A.dN = dN;
    A.inv_kappa = 1.0 / (2.0 * sigma * sigma);
    A.inv_s3 = 1.0 / (sigma * sigma * sigma);
    A.cx = 2.0 * g / ((double)b * sigma * sigma);
    A.cs = g / (double)b;
    A.dX = dX;
    A.rowds = rowds;
    A.flags = B.flags;
    const dim3 grid((unsigned)((b + 3) / 4));
    const int ch = (L.d + 63) / 64;
    if (ch <= 1)
        hipLaunchKernelGGL(k_grad_rows<1>, grid, dim3(256), 0, st, A);
    else if (ch <= 2)
        hipLaunchKernelGGL(k_grad_rows<2>, grid, dim3(256), 0, st, A);
    else if (ch <= 4)
        hipLaunchKernelGGL(k_grad_rows<4>, grid, dim3(256), 0, st, A);
    else if (ch <= 8)
        hipLaunchKernelGGL(k_grad_rows<8>, grid, dim3(256), 0, st, A);
    else
        hipLaunchKernelGGL(k_grad_rows<16>, grid, dim3(256), 0, st, A);
    hipLaunchKernelGGL(k_sum_rows, dim3(1), dim3(1024), 0, st, (const double *)rowds, b, out);
}

}  // namespace mbkk
