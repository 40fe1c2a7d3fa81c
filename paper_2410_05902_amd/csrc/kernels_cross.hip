// Cross term of the distance expansion, assignment and near-tie re-scoring.
//
// For a batch row x and center j (an implicit sparse combination of feature
// vectors, Section 4.1 / Eq. 1) the distance in feature space is
//     ||phi(x) - C_j||^2 = K(x,x) - 2 <phi(x), C_j> + <C_j, C_j>
// (Section 1, Lloyd in feature space; Section 4).  The cross term
//     P_j(x) = <phi(x), C_j> = sum_{s in S_j} w_s K(x, y_s)
// over the support S_j of center j is the hot loop.  Two implementations:
//   - k_cross_direct: VALU, one batch row per lane, support rows wave-uniform
//     (any kernel, FP32 or FP64; the Laplacian L1 path);
//   - k_cross_mfma  : Gaussian only, x.y on MFMA (FP32, or BF16 hi/lo split),
//     exp fused in registers, segmented weighted sums over the support rows.
#include "kernels.h"

namespace mbkk {

// ===========================================================================
// Direct VALU cross kernel
// ===========================================================================
// K(x, y) with x held in registers.  The loop runs over all DR entries: both
// the register row and the pool row are zero past d (DR <= padded stride), so
// the padding adds nothing, and the fixed trip count keeps x in registers.
template <int KIND, typename T, int DR>
__device__ __forceinline__ T kval_direct(const T (&x)[DR], const float *__restrict__ y, T cneg, T param)
{
    T s = 0;
#pragma unroll
    for (int t = 0; t < DR; ++t) {
        if constexpr (KIND == MBKK_GAUSS) {
            T v = x[t] - (T)y[t];
            s = fma(v, v, s);
        } else if constexpr (KIND == MBKK_LAPLACE) {
            s += fabs(x[t] - (T)y[t]);
        } else {
            s = fma(x[t], (T)y[t], s);
        }
    }
    if constexpr (KIND == MBKK_GAUSS || KIND == MBKK_LAPLACE) {
        if constexpr (sizeof(T) == 4)
            return exp2f(s * cneg);  // cneg = -log2(e) / bandwidth
        else
            return exp(-s / param);
    } else if constexpr (KIND == MBKK_LINEAR) {
        return s;
    } else {
        T u = s + param;
        return u * u;
    }
}

// Register-resident batch row (DR >= d), support rows read with wave-uniform
// addresses.  Grid: (row blocks of 256, center groups of cpg).
template <int KIND, typename T, int DR>
__global__ __launch_bounds__(256) void k_cross_direct(int nb, int d, int dp, int k, int cpg,
                                                       const float *__restrict__ bat32,
                                                       const float *__restrict__ pool32,
                                                       const int32_t *__restrict__ sup_row,
                                                       const float *__restrict__ sup_w,
                                                       const double *__restrict__ sup_w64,
                                                       const int32_t *__restrict__ seg_off, double param,
                                                       T *__restrict__ P, int ldp)
{
    const int row = blockIdx.x * 256 + threadIdx.x;
    const int rr = row < nb ? row : 0;
    const T prm = (T)param;
    const T cneg = (T)(-1.4426950408889634 / param);
    T x[DR > 0 ? DR : 1];
    static_assert(DR <= kDimAlign || DR % kDimAlign == 0, "register row must fit the padded stride");
    if constexpr (DR > 0) {
#pragma unroll
        for (int t = 0; t < DR; ++t)
            x[t] = t < d ? (T)bat32[(int64_t)rr * dp + t] : (T)0;
    }
    const int j0 = blockIdx.y * cpg, j1 = min(k, j0 + cpg);
    for (int j = j0; j < j1; ++j) {
        const int s0 = seg_off[j], s1 = seg_off[j + 1];
        T acc = 0;
        for (int s = s0; s < s1; ++s) {
            const float *y = pool32 + (int64_t)sup_row[s] * dp;
            T kv;
            if constexpr (DR > 0) {
                kv = kval_direct<KIND, T, DR>(x, y, cneg, prm);
            } else {
                // generic width: the batch row is re-read from memory
                T sacc = 0;
                const float *xr = bat32 + (int64_t)rr * dp;
                for (int t = 0; t < d; ++t) {
                    T xv = (T)xr[t], yv = (T)y[t];
                    if constexpr (KIND == MBKK_GAUSS) {
                        T v = xv - yv;
                        sacc = fma(v, v, sacc);
                    } else if constexpr (KIND == MBKK_LAPLACE) {
                        sacc += fabs(xv - yv);
                    } else {
                        sacc = fma(xv, yv, sacc);
                    }
                }
                if constexpr (KIND == MBKK_GAUSS || KIND == MBKK_LAPLACE) {
                    if constexpr (sizeof(T) == 4)
                        kv = exp2f(sacc * cneg);
                    else
                        kv = exp(-sacc / prm);
                } else if constexpr (KIND == MBKK_LINEAR) {
                    kv = sacc;
                } else {
                    T u = sacc + prm;
                    kv = u * u;
                }
            }
            if constexpr (sizeof(T) == 4)
                acc = fma(sup_w[s], kv, acc);
            else
                acc = fma(sup_w64[s], kv, acc);
        }
        if (row < nb)
            P[(int64_t)j * ldp + row] = acc;
    }
}

template <int KIND, typename T>
static void dispatch_direct_width(const Layout &L, const Buffers &B, int nb, int cpg, double param, T *P,
                                  hipStream_t st)
{
    dim3 grid((nb + 255) / 256, (L.k + cpg - 1) / cpg);
#define MBKK_DIRECT(DR)                                                                                       \
    hipLaunchKernelGGL((k_cross_direct<KIND, T, DR>), grid, dim3(256), 0, st, nb, L.d, L.dp, L.k, cpg,        \
                       B.bat32, B.pool32, B.sup_row, B.sup_w, B.sup_w64, B.seg_off, param, P, L.bmax)
    if (L.d <= 4)
        MBKK_DIRECT(4);
    else if (L.d <= 8)
        MBKK_DIRECT(8);
    else if (L.d <= 16)
        MBKK_DIRECT(16);
    else if (L.d <= 32)
        MBKK_DIRECT(32);
    else if (L.d <= 64)
        MBKK_DIRECT(64);
    else
        MBKK_DIRECT(0);
#undef MBKK_DIRECT
}

void launch_cross_direct(const Layout &L, const Buffers &B, int nb, int kind, double param, int fp64,
                         hipStream_t st)
{
    // enough workgroups to fill the chip: split the centers into groups
    const int rowblocks = (nb + 255) / 256;
    int cpg = (int)((int64_t)L.k * rowblocks / 2048);
    cpg = cpg < 1 ? 1 : cpg;
    if (fp64) {
        double *P = (double *)B.part;
        switch (kind) {
        case MBKK_GAUSS: dispatch_direct_width<MBKK_GAUSS, double>(L, B, nb, cpg, param, P, st); break;
        case MBKK_LAPLACE: dispatch_direct_width<MBKK_LAPLACE, double>(L, B, nb, cpg, param, P, st); break;
        case MBKK_LINEAR: dispatch_direct_width<MBKK_LINEAR, double>(L, B, nb, cpg, param, P, st); break;
        default: dispatch_direct_width<MBKK_POLY2, double>(L, B, nb, cpg, param, P, st); break;
        }
    } else {
        float *P = (float *)B.part;
        switch (kind) {
        case MBKK_GAUSS: dispatch_direct_width<MBKK_GAUSS, float>(L, B, nb, cpg, param, P, st); break;
        case MBKK_LAPLACE: dispatch_direct_width<MBKK_LAPLACE, float>(L, B, nb, cpg, param, P, st); break;
        case MBKK_LINEAR: dispatch_direct_width<MBKK_LINEAR, float>(L, B, nb, cpg, param, P, st); break;
        default: dispatch_direct_width<MBKK_POLY2, float>(L, B, nb, cpg, param, P, st); break;
        }
    }
}

// ===========================================================================
// MFMA cross kernel (Gaussian):  P_j(x) = sum_s w_s exp(-(||x||^2 + ||y_s||^2
// - 2 x.y_s) / kappa).  The product is computed transposed, support rows as
// the M dimension and batch rows as N, so that the 16 accumulator values a
// lane holds belong to ONE batch row and 16 support rows of one center; the
// weighted sum over the support is then an in-lane reduction plus one
// exchange between the two lane halves.
//
// Workgroup tile: 128 support rows x 128 batch rows, 4 waves in a 2x2 grid,
// each wave 64 x 64 = 2 x 2 MFMA blocks of 32 x 32; K staged through LDS in
// chunks of 32 (one LDS buffer, next chunk prefetched into registers).  Segments are padded to multiples of 32
// rows so that every 32-row block belongs to one center.  Output: one partial
// per (32-row block, batch row); the two blocks of a wave are merged when they
// belong to the same center.
//   MODE 0: FP32 MFMA 32x32x2 (plain form)
//   MODE 1: BF16 32x32x16, hi.hi + hi.lo + lo.hi (compensated split)
//   MODE 2: BF16 32x32x16, hi.hi only
// ===========================================================================
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef uint16_t u16x8 __attribute__((ext_vector_type(8)));

struct CrossArgs {
    int nb, dp, ntB;
    int64_t ntiles;           // support tiles * batch tiles
    int64_t zero_row;
    const int32_t *seg_total; // seg_off + k: used support rows
    const float *pool32;
    const uint16_t *poolhi, *poollo;
    const float *poolsq;
    const int32_t *sup_row;
    const float *sup_w;
    const int32_t *blk_center;
    const float *bat32;
    const uint16_t *bathi, *batlo;
    const float *batsq;
    float c2;   // 2 log2(e) / kappa
    float c1;   // -log2(e) / kappa
    float *part;
    int ldp;
};

constexpr int TS = 128, TB = 128, KC = 32;
constexpr int LDF = KC + 4;  // FP32 LDS row stride (floats): 144 B, conflict-free b128 reads
constexpr int LDH = KC + 8;  // BF16 LDS row stride (elements): 80 B

template <int MODE>
__global__ __launch_bounds__(256, 2) void k_cross_mfma(const CrossArgs A)
{
    constexpr bool F32 = MODE == 0;
    constexpr bool X3 = MODE == 1;
    // LDS (one buffer; the next K chunk is prefetched into registers):
    // FP32 -> As, Bs [TS][LDF] floats; BF16 -> hi (and lo) [TS][LDH] each
    constexpr int LDS_F = F32 ? 2 * TS * LDF : 4;
    constexpr int LDS_H = F32 ? 8 : TS * LDH;
    __shared__ __attribute__((aligned(16))) float smf[LDS_F];
    __shared__ __attribute__((aligned(16))) uint16_t sAh[LDS_H];
    __shared__ __attribute__((aligned(16))) uint16_t sAl[X3 ? LDS_H : 8];
    __shared__ __attribute__((aligned(16))) uint16_t sBh[LDS_H];
    __shared__ __attribute__((aligned(16))) uint16_t sBl[X3 ? LDS_H : 8];
    __shared__ __attribute__((aligned(16))) float sAy[TS];
    __shared__ __attribute__((aligned(16))) float sW[TS];

    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int wm = wid >> 1, wn = wid & 1;
    // XCD-aware tile order: consecutive tiles of one XCD share support rows
    const int64_t G8 = gridDim.x / 8;
    const int64_t t = (int64_t)(blockIdx.x % 8) * G8 + blockIdx.x / 8;
    if (t >= A.ntiles)
        return;
    const int st = (int)(t / A.ntB), bt = (int)(t % A.ntB);
    const int M = *A.seg_total;
    const int s0 = st * TS, b0 = bt * TB;
    if (s0 >= M)
        return;

    // per-tile support row metadata
    if (tid < TS) {
        const int s = s0 + tid;
        const int64_t prow = s < M ? (int64_t)A.sup_row[s] : A.zero_row;
        sAy[tid] = A.c1 * A.poolsq[prow];
        sW[tid] = s < M ? A.sup_w[s] : 0.0f;
    }

    const int nK = A.dp / KC;
    f32x16 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int bb = 0; bb < 2; ++bb)
#pragma unroll
            for (int i = 0; i < 16; ++i)
                acc[a][bb][i] = 0.0f;

    if constexpr (F32) {
        // loader: 4 rows per thread, one float4 each, for A and B
        const int lr = tid >> 3, lc = (tid & 7) * 4;
        const float *asrc[4];
        const float *bsrc[4];
        bool bok[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int r = lr + 32 * q;
            const int s = s0 + r;
            const int64_t prow = s < M ? (int64_t)A.sup_row[s] : A.zero_row;
            asrc[q] = A.pool32 + prow * A.dp + lc;
            bok[q] = b0 + r < A.nb;
            bsrc[q] = A.bat32 + (int64_t)(bok[q] ? b0 + r : 0) * A.dp + lc;
        }
        f32x4 ra[4], rb[4];
        auto gload = [&](int kc) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                ra[q] = *(const f32x4 *)(asrc[q] + kc * KC);
                rb[q] = bok[q] ? *(const f32x4 *)(bsrc[q] + kc * KC) : f32x4{0, 0, 0, 0};
            }
        };
        auto lstore = [&]() {
            float *As = smf;
            float *Bs = As + TS * LDF;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                *(f32x4 *)(As + (lr + 32 * q) * LDF + lc) = ra[q];
                *(f32x4 *)(Bs + (lr + 32 * q) * LDF + lc) = rb[q];
            }
        };
        gload(0);
        lstore();
        __syncthreads();
        const int frow = lane & 31, fh = lane >> 5;
        for (int kc = 0; kc < nK; ++kc) {
            if (kc + 1 < nK)
                gload(kc + 1);
            const float *As = smf;
            const float *Bs = As + TS * LDF;
            // K permutation inside the chunk: MFMA step s, lane half h -> column h*16 + s
            f32x4 af[2][4], bf[2][4];
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    af[a][v] = *(const f32x4 *)(As + (wm * 64 + a * 32 + frow) * LDF + fh * 16 + v * 4);
#pragma unroll
            for (int bb = 0; bb < 2; ++bb)
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    bf[bb][v] = *(const f32x4 *)(Bs + (wn * 64 + bb * 32 + frow) * LDF + fh * 16 + v * 4);
#pragma unroll
            for (int s = 0; s < 16; ++s)
#pragma unroll
                for (int a = 0; a < 2; ++a)
#pragma unroll
                    for (int bb = 0; bb < 2; ++bb)
                        acc[a][bb] = __builtin_amdgcn_mfma_f32_32x32x2f32(af[a][s >> 2][s & 3], bf[bb][s >> 2][s & 3],
                                                                           acc[a][bb], 0, 0, 0);
            if (kc + 1 < nK) {
                __syncthreads();
                lstore();
                __syncthreads();
            }
        }
    } else {
        // loader: 2 rows per thread, 8 bf16 (16 B) each, hi and lo, for A and B
        const int lr = tid >> 2, lc = (tid & 3) * 8;
        const uint16_t *ahs[2], *als[2], *bhs[2], *bls[2];
        bool bok[2];
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int r = lr + 64 * q;
            const int s = s0 + r;
            const int64_t prow = s < M ? (int64_t)A.sup_row[s] : A.zero_row;
            ahs[q] = A.poolhi + prow * A.dp + lc;
            als[q] = A.poollo + prow * A.dp + lc;
            bok[q] = b0 + r < A.nb;
            const int64_t brow = bok[q] ? b0 + r : 0;
            bhs[q] = A.bathi + brow * A.dp + lc;
            bls[q] = A.batlo + brow * A.dp + lc;
        }
        u16x8 rah[2], ral[2], rbh[2], rbl[2];
        const u16x8 z8 = {0, 0, 0, 0, 0, 0, 0, 0};
        auto gload = [&](int kc) {
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                rah[q] = *(const u16x8 *)(ahs[q] + kc * KC);
                rbh[q] = bok[q] ? *(const u16x8 *)(bhs[q] + kc * KC) : z8;
                if constexpr (X3) {
                    ral[q] = *(const u16x8 *)(als[q] + kc * KC);
                    rbl[q] = bok[q] ? *(const u16x8 *)(bls[q] + kc * KC) : z8;
                }
            }
        };
        auto lstore = [&]() {
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const int off = (lr + 64 * q) * LDH + lc;
                *(u16x8 *)(sAh + off) = rah[q];
                *(u16x8 *)(sBh + off) = rbh[q];
                if constexpr (X3) {
                    *(u16x8 *)(sAl + off) = ral[q];
                    *(u16x8 *)(sBl + off) = rbl[q];
                }
            }
        };
        gload(0);
        lstore();
        __syncthreads();
        const int frow = lane & 31, fh = lane >> 5;
        for (int kc = 0; kc < nK; ++kc) {
            if (kc + 1 < nK)
                gload(kc + 1);
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                bf16x8 ah[2], al[2], bh[2], bl[2];
#pragma unroll
                for (int a = 0; a < 2; ++a) {
                    const int off = (wm * 64 + a * 32 + frow) * LDH + s * 16 + fh * 8;
                    ah[a] = __builtin_bit_cast(bf16x8, *(const u16x8 *)(sAh + off));
                    if constexpr (X3)
                        al[a] = __builtin_bit_cast(bf16x8, *(const u16x8 *)(sAl + off));
                }
#pragma unroll
                for (int bb = 0; bb < 2; ++bb) {
                    const int off = (wn * 64 + bb * 32 + frow) * LDH + s * 16 + fh * 8;
                    bh[bb] = __builtin_bit_cast(bf16x8, *(const u16x8 *)(sBh + off));
                    if constexpr (X3)
                        bl[bb] = __builtin_bit_cast(bf16x8, *(const u16x8 *)(sBl + off));
                }
#pragma unroll
                for (int a = 0; a < 2; ++a)
#pragma unroll
                    for (int bb = 0; bb < 2; ++bb) {
                        acc[a][bb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[a], bh[bb], acc[a][bb], 0, 0, 0);
                        if constexpr (X3) {
                            acc[a][bb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[a], bl[bb], acc[a][bb], 0, 0, 0);
                            acc[a][bb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[a], bh[bb], acc[a][bb], 0, 0, 0);
                        }
                    }
            }
            if (kc + 1 < nK) {
                __syncthreads();
                lstore();
                __syncthreads();
            }
        }
    }

    // Epilogue.  Lane l holds batch column n = l % 32 of each 32-column block
    // and support rows m = 8 (i / 4) + 4 (l / 32) + i % 4, i = 0..15.
    const int n = lane & 31, h = lane >> 5;
    const int Mb = M / 32;
    float tot[2][2];
#pragma unroll
    for (int bb = 0; bb < 2; ++bb) {
        const int col = b0 + wn * 64 + bb * 32 + n;
        const float ax = col < A.nb ? A.c1 * A.batsq[col] : 0.0f;
#pragma unroll
        for (int a = 0; a < 2; ++a) {
            const int mbase = wm * 64 + a * 32;
            float sum = 0.0f;
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                const int m0 = mbase + 8 * g + 4 * h;
                const f32x4 ay = *(const f32x4 *)(sAy + m0);
                const f32x4 w = *(const f32x4 *)(sW + m0);
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const float arg = fmaf(acc[a][bb][4 * g + q], A.c2, ax + ay[q]);
                    sum = fmaf(w[q], __builtin_amdgcn_exp2f(arg), sum);
                }
            }
            sum += __shfl_xor(sum, 32);
            tot[a][bb] = sum;
        }
    }
    const int blk0 = (s0 + wm * 64) / 32;
    if (blk0 >= Mb)
        return;
    const bool has1 = blk0 + 1 < Mb;
    const bool merge = has1 && A.blk_center[blk0] == A.blk_center[blk0 + 1];
    if (h == 0) {
#pragma unroll
        for (int bb = 0; bb < 2; ++bb) {
            const int col = b0 + wn * 64 + bb * 32 + n;
            if (col >= A.nb)
                continue;
            if (merge) {
                A.part[(int64_t)blk0 * A.ldp + col] = tot[0][bb] + tot[1][bb];
            } else {
                A.part[(int64_t)blk0 * A.ldp + col] = tot[0][bb];
                if (has1)
                    A.part[(int64_t)(blk0 + 1) * A.ldp + col] = tot[1][bb];
            }
        }
    }
}

void launch_cross_mfma(const Layout &L, const Buffers &B, int nb, int precision, double kappa, hipStream_t st)
{
    CrossArgs A;
    A.nb = nb;
    A.dp = L.dp;
    A.ntB = (nb + TB - 1) / TB;
    const int64_t ntS = L.Mcap / TS;
    A.ntiles = ntS * A.ntB;
    A.zero_row = L.PR;
    A.seg_total = B.seg_off + L.k;
    A.pool32 = B.pool32;
    A.poolhi = B.poolhi;
    A.poollo = B.poollo;
    A.poolsq = B.poolsq;
    A.sup_row = B.sup_row;
    A.sup_w = B.sup_w;
    A.blk_center = B.blk_center;
    A.bat32 = B.bat32;
    A.bathi = B.bathi;
    A.batlo = B.batlo;
    A.batsq = B.batsq;
    const double l2e = 1.4426950408889634;
    A.c2 = (float)(2.0 * l2e / kappa);
    A.c1 = (float)(-l2e / kappa);
    A.part = (float *)B.part;
    A.ldp = L.bmax;
    const int64_t grid = (A.ntiles + 7) / 8 * 8;
    if (precision == MBKK_FP32)
        hipLaunchKernelGGL(k_cross_mfma<0>, dim3((unsigned)grid), dim3(256), 0, st, A);
    else if (precision == MBKK_BF16X3)
        hipLaunchKernelGGL(k_cross_mfma<1>, dim3((unsigned)grid), dim3(256), 0, st, A);
    else
        hipLaunchKernelGGL(k_cross_mfma<2>, dim3((unsigned)grid), dim3(256), 0, st, A);
}

// ===========================================================================
// Distances, argmin and margin.  One thread per batch row:
//   D_j = K(x,x) - 2 P_j + N_j  (FP64 assembly of the FP32/FP64 cross term)
// label = smallest j attaining the minimum; margin = second smallest - min.
// LAYOUT 0: P[j][row]; LAYOUT 1: per-32-block partials of the MFMA kernel.
// ===========================================================================
__device__ __forceinline__ double self_kernel(int kind, double param, double sq)
{
    if (kind == MBKK_LINEAR)
        return sq;
    if (kind == MBKK_POLY2)
        return (sq + param) * (sq + param);
    return 1.0;  // normalised kernels: K(x,x) = 1
}

template <typename T, int LAYOUT>
__device__ __forceinline__ double cross_of(const T *__restrict__ part, int ldp, int row, int j,
                                           const int32_t *__restrict__ seg_off)
{
    if constexpr (LAYOUT == 0) {
        return (double)part[(int64_t)j * ldp + row];
    } else {
        const int bs = seg_off[j] / 32, be = seg_off[j + 1] / 32;
        float s = 0.0f;
        for (int blk = bs; blk < be; ++blk) {
            if ((blk & 1) && blk - 1 >= bs)
                continue;  // merged into the even block of its pair
            s += part[(int64_t)blk * ldp + row];
        }
        return (double)s;
    }
}

template <typename T, int LAYOUT>
__global__ __launch_bounds__(256) void k_score(int nb, int k, const T *__restrict__ part, int ldp,
                                                const int32_t *__restrict__ seg_off, const double *__restrict__ N,
                                                int kind, double param, const double *__restrict__ batsq64,
                                                int32_t *__restrict__ labels, float *__restrict__ mind,
                                                float *__restrict__ margin, double *__restrict__ Dout, int64_t ldD)
{
    const int row = blockIdx.x * 256 + threadIdx.x;
    if (row >= nb)
        return;
    const double kxx = self_kernel(kind, param, batsq64[row]);
    double best = INFINITY, second = INFINITY;
    int lab = 0;
    for (int j = 0; j < k; ++j) {
        const double D = kxx - 2.0 * cross_of<T, LAYOUT>(part, ldp, row, j, seg_off) + N[j];
        if (Dout)
            Dout[(int64_t)row * ldD + j] = D;
        if (D < best) {
            second = best;
            best = D;
            lab = j;
        } else if (D < second) {
            second = D;
        }
    }
    labels[row] = lab;
    mind[row] = (float)best;
    margin[row] = (float)(second - best);
}

void launch_score(const Layout &L, const Buffers &B, int nb, int kind, double param, int fp64, int mfma,
                  double *D_out, int64_t ldD, hipStream_t st)
{
    dim3 grid((nb + 255) / 256);
    if (fp64)
        hipLaunchKernelGGL((k_score<double, 0>), grid, dim3(256), 0, st, nb, L.k, (const double *)B.part, L.bmax,
                           B.seg_off, B.N, kind, param, B.batsq64, B.labels, B.mind, B.margin, D_out, ldD);
    else if (mfma)
        hipLaunchKernelGGL((k_score<float, 1>), grid, dim3(256), 0, st, nb, L.k, (const float *)B.part, L.bmax,
                           B.seg_off, B.N, kind, param, B.batsq64, B.labels, B.mind, B.margin, D_out, ldD);
    else
        hipLaunchKernelGGL((k_score<float, 0>), grid, dim3(256), 0, st, nb, L.k, (const float *)B.part, L.bmax,
                           B.seg_off, B.N, kind, param, B.batsq64, B.labels, B.mind, B.margin, D_out, ldD);
}

// ===========================================================================
// FP64 re-scoring of near ties (BF16 forms).  One wave per batch row whose
// margin is below delta: candidates are the centers whose BF16-form distance
// is within delta of the best; for those the cross term is recomputed in
// FP64 from the FP32 coordinates (direct ||x - y||^2, FP64 exp, FP64
// weights), and the label, distance and margin are replaced.
// ===========================================================================
__global__ __launch_bounds__(256) void k_rescore(int nb, int k, int d, int dp, double kappa, double delta,
                                                  const float *__restrict__ part, int ldp,
                                                  const int32_t *__restrict__ seg_off, const double *__restrict__ N,
                                                  const float *__restrict__ bat32, const float *__restrict__ pool32,
                                                  const int32_t *__restrict__ sup_row,
                                                  const double *__restrict__ sup_w64, int32_t *__restrict__ labels,
                                                  float *__restrict__ mind, float *__restrict__ margin)
{
    const int lane = threadIdx.x & 63;
    const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (row >= nb)
        return;
    if (!(margin[row] < (float)delta))
        return;
    // best approximate distance (every lane scans a strided subset of centers)
    double best = INFINITY;
    for (int j = lane; j < k; j += 64) {
        const double D = 1.0 - 2.0 * cross_of<float, 1>(part, ldp, row, j, seg_off) + N[j];
        best = fmin(best, D);
    }
    for (int o = 32; o > 0; o >>= 1)
        best = fmin(best, __shfl_xor(best, o));
    const float *x = bat32 + (int64_t)row * dp;
    double b64 = INFINITY, s64 = INFINITY, outside = INFINITY;
    int lab = 0;
    for (int j = 0; j < k; ++j) {
        // wave-uniform candidate test
        double Dapprox = 0.0;
        if (lane == 0)
            Dapprox = 1.0 - 2.0 * cross_of<float, 1>(part, ldp, row, j, seg_off) + N[j];
        Dapprox = __shfl(Dapprox, 0);
        if (!(Dapprox <= best + delta)) {
            outside = fmin(outside, Dapprox);
            continue;
        }
        double p = 0.0;
        for (int s = seg_off[j] + lane; s < seg_off[j + 1]; s += 64) {
            const double w = sup_w64[s];
            if (w == 0.0)
                continue;
            const float *y = pool32 + (int64_t)sup_row[s] * dp;
            double d2 = 0.0;
            for (int t = 0; t < d; ++t) {
                const double v = (double)x[t] - (double)y[t];
                d2 += v * v;
            }
            p += w * exp(-d2 / kappa);
        }
        for (int o = 32; o > 0; o >>= 1)
            p += __shfl_xor(p, o);
        const double D = 1.0 - 2.0 * p + N[j];
        if (D < b64) {
            s64 = b64;
            b64 = D;
            lab = j;
        } else if (D < s64) {
            s64 = D;
        }
    }
    if (lane == 0) {
        labels[row] = lab;
        mind[row] = (float)b64;
        margin[row] = (float)(fmin(s64, outside) - b64);
    }
}

void launch_rescore(const Layout &L, const Buffers &B, int nb, int kind, double param, double delta,
                    hipStream_t st)
{
    (void)kind;
    hipLaunchKernelGGL(k_rescore, dim3((nb + 3) / 4), dim3(256), 0, st, nb, L.k, L.d, L.dp, param, delta,
                       (const float *)B.part, L.bmax, B.seg_off, B.N, B.bat32, B.pool32, B.sup_row, B.sup_w64,
                       B.labels, B.mind, B.margin);
}

// Sum of min distances of rows [0, nb) in FP64 (fixed order); adds to obj[1]
// when accumulate, else stores.
__global__ __launch_bounds__(1024) void k_sum_mind(int nb, const float *__restrict__ mind,
                                                    double *__restrict__ obj, int accumulate)
{
    __shared__ double red[1024];
    const int tid = threadIdx.x;
    double s = 0.0;
    for (int p = tid; p < nb; p += 1024)
        s += (double)mind[p];
    red[tid] = s;
    __syncthreads();
    for (int h = 512; h > 0; h >>= 1) {
        if (tid < h)
            red[tid] += red[tid + h];
        __syncthreads();
    }
    if (tid == 0)
        obj[1] = accumulate ? obj[1] + red[0] : red[0];
}

void launch_sum_mind(const Buffers &B, int nb, int accumulate, hipStream_t st)
{
    hipLaunchKernelGGL(k_sum_mind, dim3(1), dim3(1024), 0, st, nb, B.mind, B.obj, accumulate);
}

}  // namespace mbkk
