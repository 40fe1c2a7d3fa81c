// Cross term of the distance expansion (the scoring that consumes it is in
// kernels_score.hip).
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
#include <algorithm>
#include <type_traits>

#include "cross_layout.h"
#include "dev_common.h"
#include "kernels.h"

namespace mbkk {

// ===========================================================================
// Direct VALU cross kernel
// ===========================================================================
// K(x, y) with x held in registers.  The loop runs over all DR entries: both
// the register row and the pool row are zero past d (DR <= padded stride), so
// the padding adds nothing, and the fixed trip count keeps x in registers.
template <int KIND, typename T>
__device__ __forceinline__ T kfinish_direct(T s, T cneg, T param)
{
    if constexpr (KIND == MBKK_GAUSS || KIND == MBKK_LAPLACE) {
        if constexpr (sizeof(T) == 4)
            return __builtin_amdgcn_exp2f(s * cneg);  // cneg = -log2(e) / bandwidth
        else
            return exp(-s / param);
    } else if constexpr (KIND == MBKK_LINEAR) {
        return s;
    } else {
        T u = s + param;
        return u * u;
    }
}

// K(x_q, y) for RPL register rows at once: each coordinate of y is read once.
template <int KIND, typename T, int DR, int RPL>
__device__ __forceinline__ void kval_direct_rows(const T (&x)[RPL][DR], const float *__restrict__ y, T cneg,
                                                 T param, T (&kv)[RPL])
{
    T s[RPL];
#pragma unroll
    for (int q = 0; q < RPL; ++q)
        s[q] = 0;
#pragma unroll
    for (int t = 0; t < DR; ++t) {
        const T yt = (T)y[t];
#pragma unroll
        for (int q = 0; q < RPL; ++q) {
            if constexpr (KIND == MBKK_GAUSS) {
                T v = x[q][t] - yt;
                s[q] = fma(v, v, s[q]);
            } else if constexpr (KIND == MBKK_LAPLACE) {
                s[q] += fabs(x[q][t] - yt);
            } else {
                s[q] = fma(x[q][t], yt, s[q]);
            }
        }
    }
#pragma unroll
    for (int q = 0; q < RPL; ++q)
        kv[q] = kfinish_direct<KIND, T>(s[q], cneg, param);
}

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
            return __builtin_amdgcn_exp2f(s * cneg);  // cneg = -log2(e) / bandwidth
        else
            return exp(-s / param);
    } else if constexpr (KIND == MBKK_LINEAR) {
        return s;
    } else {
        T u = s + param;
        return u * u;
    }
}

// Broadcast of lane e's value to the wave (e wave-uniform).
__device__ __forceinline__ float wave_bcast(float v, int e)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), e));
}
__device__ __forceinline__ double wave_bcast(double v, int e)
{
    const int64_t b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffff), e);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), e);
    return __longlong_as_double(((int64_t)hi << 32) | (uint32_t)lo);
}

// Register-resident batch rows (DR >= d; RPL rows per lane, 256 apart).  The
// workgroup's range of support entries is taken 64 at a time: lane e of
// every wave loads entry c0 + e's pool row and weight (one coalesced load),
// and the entries are then broadcast one by one, their rows read with
// wave-uniform (scalar) loads, each used for the lane's RPL batch rows.  A
// run ends where a center's segment ends.  Grid: (row tiles of 256 RPL) x (ranges).
template <int KIND, typename T, int DR, int RPL>
__global__ __launch_bounds__(256) void k_cross_direct(int nb, int d, int dp, int k, int nranges,
                                                       const float *__restrict__ bat32,
                                                       const float *__restrict__ pool32,
                                                       const int32_t *__restrict__ sup_row,
                                                       const float *__restrict__ sup_w,
                                                       const double *__restrict__ sup_w64,
                                                       const int32_t *__restrict__ seg_off, double param,
                                                       T *__restrict__ P, int ldp)
{
    static_assert(RPL == 1 || DR > 0, "two rows per lane need a register-resident width");
    const int lane = threadIdx.x & 63;
    int row[RPL], rr[RPL];
#pragma unroll
    for (int q = 0; q < RPL; ++q) {
        row[q] = blockIdx.x * 256 * RPL + q * 256 + threadIdx.x;
        rr[q] = row[q] < nb ? row[q] : 0;
    }
    const int r = blockIdx.y;
    const int M = seg_off[k];
    const int RR = direct_range_rows(M, nranges);
    const int s0 = r * RR, s1 = min(M, s0 + RR);
    if (s0 >= s1)
        return;  // block uniform
    const T prm = (T)param;
    const T cneg = (T)(-1.4426950408889634 / param);
    T x[RPL][DR > 0 ? DR : 1];
    static_assert(DR <= kDimAlign || DR % kDimAlign == 0, "register row must fit the padded stride");
    if constexpr (DR > 0) {
#pragma unroll
        for (int q = 0; q < RPL; ++q)
#pragma unroll
            for (int t = 0; t < DR; ++t)
                x[q][t] = t < d ? (T)bat32[(int64_t)rr[q] * dp + t] : (T)0;
    }
    // the run being accumulated: center j up to cur_end, stored at id
    int j = wave_segment_of(seg_off, k, s0);
    int cur_end = min(s1, seg_off[j + 1]);
    int id = s0 == seg_off[j] ? j : k + r;
    T acc[RPL];
#pragma unroll
    for (int q = 0; q < RPL; ++q)
        acc[q] = 0;
    for (int c0 = s0; c0 < s1; c0 += 64) {
        const int n = min(64, s1 - c0);
        const int lrow = sup_row[c0 + (lane < n ? lane : 0)];
        T lw;
        if constexpr (sizeof(T) == 4)
            lw = lane < n ? sup_w[c0 + lane] : 0.0f;
        else
            lw = lane < n ? sup_w64[c0 + lane] : 0.0;
        for (int e = 0; e < n; ++e) {  // wave uniform
            const int s = c0 + e;
            if (s >= cur_end) {  // the run [.., cur_end) had entries: store it, move to s's center
#pragma unroll
                for (int q = 0; q < RPL; ++q) {
                    if (row[q] < nb)
                        P[(int64_t)id * ldp + row[q]] = acc[q];
                    acc[q] = 0;
                }
                do {
                    ++j;
                } while (seg_off[j + 1] <= s);
                cur_end = min(s1, seg_off[j + 1]);
                id = j;
            }
            const float *y = pool32 + (int64_t)__builtin_amdgcn_readlane(lrow, e) * dp;
            const T w = wave_bcast(lw, e);
            if constexpr (DR > 0) {
                if constexpr (RPL == 1) {
                    acc[0] = fma(w, kval_direct<KIND, T, DR>(x[0], y, cneg, prm), acc[0]);
                } else {
                    T kv[RPL];
                    kval_direct_rows<KIND, T, DR, RPL>(x, y, cneg, prm, kv);
#pragma unroll
                    for (int q = 0; q < RPL; ++q)
                        acc[q] = fma(w, kv[q], acc[q]);
                }
            } else {
                // generic width: the batch row is re-read from memory
                T sacc = 0;
                const float *xr = bat32 + (int64_t)rr[0] * dp;
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
                T kv;
                if constexpr (KIND == MBKK_GAUSS || KIND == MBKK_LAPLACE) {
                    if constexpr (sizeof(T) == 4)
                        kv = __builtin_amdgcn_exp2f(sacc * cneg);
                    else
                        kv = exp(-sacc / prm);
                } else if constexpr (KIND == MBKK_LINEAR) {
                    kv = sacc;
                } else {
                    T u = sacc + prm;
                    kv = u * u;
                }
                acc[0] = fma(w, kv, acc[0]);
            }
        }
    }
#pragma unroll
    for (int q = 0; q < RPL; ++q)
        if (row[q] < nb)
            P[(int64_t)id * ldp + row[q]] = acc[q];  // the last run (s0 < s1: it has entries)
}

template <int KIND, typename T>
static void dispatch_direct_width(const Layout &L, const Buffers &B, int nb, int nranges, double param, T *P,
                                  hipStream_t st)
{
    constexpr int R2 = sizeof(T) == 4 ? 2 : 1;  // rows per lane for d <= 32 (direct_rpl)
    const int rpl = direct_rpl(L.d, sizeof(T) == 8);
    dim3 grid((nb + 256 * rpl - 1) / (256 * rpl), nranges);
#define MBKK_DIRECT_R(DR, RPL)                                                                                 \
    hipLaunchKernelGGL((k_cross_direct<KIND, T, DR, RPL>), grid, dim3(256), 0, st, nb, L.d, L.dp, L.k, nranges, \
                       B.bat32, B.pool32, B.sup_row, B.sup_w, B.sup_w64, B.seg_off, param, P, L.bmax)
#define MBKK_DIRECT(DR) MBKK_DIRECT_R(DR, (DR > 0 && DR <= 32 ? R2 : 1))
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
#undef MBKK_DIRECT_R
}

void launch_cross_direct(const Layout &L, const Buffers &B, int nb, int kind, double param, int fp64,
                         hipStream_t st)
{
    const int nranges = direct_nranges(nb, direct_rpl(L.d, fp64));
    if (fp64) {
        double *P = (double *)B.part;
        switch (kind) {
        case MBKK_GAUSS: dispatch_direct_width<MBKK_GAUSS, double>(L, B, nb, nranges, param, P, st); break;
        case MBKK_LAPLACE: dispatch_direct_width<MBKK_LAPLACE, double>(L, B, nb, nranges, param, P, st); break;
        case MBKK_LINEAR: dispatch_direct_width<MBKK_LINEAR, double>(L, B, nb, nranges, param, P, st); break;
        default: dispatch_direct_width<MBKK_POLY2, double>(L, B, nb, nranges, param, P, st); break;
        }
    } else {
        float *P = (float *)B.part;
        switch (kind) {
        case MBKK_GAUSS: dispatch_direct_width<MBKK_GAUSS, float>(L, B, nb, nranges, param, P, st); break;
        case MBKK_LAPLACE: dispatch_direct_width<MBKK_LAPLACE, float>(L, B, nb, nranges, param, P, st); break;
        case MBKK_LINEAR: dispatch_direct_width<MBKK_LINEAR, float>(L, B, nb, nranges, param, P, st); break;
        default: dispatch_direct_width<MBKK_POLY2, float>(L, B, nb, nranges, param, P, st); break;
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

// ===========================================================================
// Batch-stationary MFMA cross kernel (d <= 128).  Each wave keeps the MFMA
// fragments of its NBK x 32 batch rows (all of K) in registers for the whole
// launch; the workgroup streams a range of RB support blocks (32 rows each)
// through two LDS buffers, SB blocks (one stage) at a time.
//  - Staging is by direct global->LDS loads (16 bytes per lane); each lane
//    gathers its pool row through sup_row, whose entries for the next stage
//    are fetched one stage ahead.  LDS rows are padded by one 16-byte chunk
//    (conflict-free 128-bit fragment reads); the pad positions load a
//    harmless chunk.  A stage is long enough (SB = 4 blocks) for the loads of
//    the next one to arrive while it computes.
//  - The accumulator of a block starts at -||x||^2 / 2 (exact), so the
//    exponent is c2 * acc + ay with ay = -log2(e) ||y||^2 / kappa staged per
//    row: exp(-||x-y||^2 / kappa) = exp2(c2 * (x.y - ||x||^2/2) + ay).
//  - The exp epilogue of block b-1 is issued between the MFMAs of block b,
//    in program order, each MFMA with its share of VALU work fenced off from
//    the scheduler: the VALU work then issues while the matrix core is busy.
//  - Segments are packed (a center's entries rounded up to a multiple of 8,
//    at least 32 when it has any), so a block holds at most one row where a
//    center starts (blk_split), a multiple of 8.  Consecutive rows of one
//    center are summed in registers; the epilogue of a block where a center
//    starts inside moves the finishing run's sums aside at that row group.  A run is written once, at slot 2 b of
//    the block b it starts at (a range start, or a center starting at the
//    block's first row) or at slot 2 b + 1 (a center starting inside block
//    b), so the partial buffer holds one value per (run, batch row).
// Grid: (#ranges x #batch tiles of 128 NBK rows), one round of workgroups
// (one per compute unit), XCD-aware: the workgroups of one XCD share support
// ranges.
// ===========================================================================
// Where the staging of the next stage is issued: spread between the MFMAs of
// the stage (one item every MBKK_BS_ITEM_STRIDE MFMAs, from the first), or
// all at the start of the stage.
#ifndef MBKK_BS_SPREAD
#define MBKK_BS_SPREAD 1
#endif
#ifndef MBKK_BS_XCD_BY_TILE
#define MBKK_BS_XCD_BY_TILE 1
#endif
constexpr bool kBsSpreadStaging = MBKK_BS_SPREAD != 0;
// MFMA positions between two staging items of the next stage
#ifndef MBKK_BS_ITEM_STRIDE
#define MBKK_BS_ITEM_STRIDE 10
#endif
// Wave priority by progress through the stage: priority 3 - k in block k,
// so that of the two waves of a SIMD the one behind issues first and both
// reach the end-of-stage barrier together (unprioritised, the older wave
// ran a block ahead and then idled at the barrier while the other ran
// alone)
#ifndef MBKK_BS_PRIO
#define MBKK_BS_PRIO 1
#endif

struct CrossBsArgs {
    int nb, nbt, nranges;
    int32_t sup_cap;      // Mcap: sup_row[Mcap] is the zero pool row, sup_w[Mcap] = sup_ay[Mcap] = 0
    int32_t pool_bytes;   // bytes of the pool in the staged form (the bound of its buffer resource)
    const int32_t *seg_total;
    const float *pool32;
    const uint16_t *poolhi, *poollo;
    const int32_t *sup_row;
    const float *sup_w, *sup_ay;
    const int32_t *blk_split;  // row of each block where a center starts (32: none)
    const char *batfrag;  // the batch in fragment order (see gather_rows_body), hi then lo
    int64_t frag_lo;      // byte offset of the lo fragments
    const float *batsq;
    float c2;
    float *part;
    int ldp;
};

typedef __attribute__((address_space(3))) void lds_void_t;

template <int MODE, int DP>
__global__ __launch_bounds__(256 * bs_wps(MODE, DP), kBsOcc) void k_cross_bs(const CrossBsArgs A)
{
    // buffer resources exist in the device pass only; the host pass keeps the launch stub
#if defined(__HIP_DEVICE_COMPILE__)
    constexpr bool F32 = MODE == 0;
    constexpr bool X3 = MODE == 1;
    constexpr int NBK = bs_nbk(MODE, DP);          // 32-row N-blocks (batch rows) per wave
    constexpr int NW = 4 * bs_wps(MODE, DP);       // waves per workgroup
    constexpr int SB = kBsStageBlocks;
    constexpr int KS = F32 ? DP / 2 : DP / 16;     // MFMA k-steps over K = DP
    constexpr int ES = F32 ? 4 : 2;                // element bytes
    constexpr int CPR = DP * ES / 16;              // 16-byte chunks per row
    constexpr int CPS = CPR + 1;                   // chunk positions per LDS row (one pad)
    constexpr int ROWS = 32 * SB;                  // support rows per stage
    constexpr int NPOS = ROWS * CPS;               // chunk positions per staged array
    constexpr int NINS = NPOS / 64;                // DMA instructions per array
    constexpr int NT = (NINS + NW - 1) / NW;       // per wave (waves take i = w, w+NW, ...)
    constexpr int NARR = X3 ? 2 : 1;
    constexpr int ABYTES = NPOS * 16;
    static_assert(NPOS % 64 == 0 && ROWS % 64 == 0 && ROWS / 64 * 2 == 4, "staging layout");
    // Two stage buffers, each its own object: every access below names its
    // buffer at compile time (the stage loop is unrolled by two), so the
    // compiler sees that the staging of one buffer cannot alias the reads of
    // the other and needs no wait between them.
    __shared__ __attribute__((aligned(16))) char sA0[NARR * ABYTES];
    __shared__ __attribute__((aligned(16))) char sA1[NARR * ABYTES];
    __shared__ __attribute__((aligned(16))) float sAy0[ROWS], sAy1[ROWS], sW0[ROWS], sW1[ROWS];
    __shared__ __attribute__((aligned(16))) int32_t sIdx0[ROWS], sIdx1[ROWS];  // pool rows of a stage
    using IC0 = std::integral_constant<int, 0>;
    using IC1 = std::integral_constant<int, 1>;
    auto bufA = [&](auto bc) -> char * {
        if constexpr (decltype(bc)::value == 0)
            return sA0;
        else
            return sA1;
    };
    auto bufAy = [&](auto bc) -> float * {
        if constexpr (decltype(bc)::value == 0)
            return sAy0;
        else
            return sAy1;
    };
    auto bufW = [&](auto bc) -> float * {
        if constexpr (decltype(bc)::value == 0)
            return sW0;
        else
            return sW1;
    };
    auto bufIdx = [&](auto bc) -> int32_t * {
        if constexpr (decltype(bc)::value == 0)
            return sIdx0;
        else
            return sIdx1;
    };

    const int tid = threadIdx.x, lane = tid & 63;
    const int wu = __builtin_amdgcn_readfirstlane(tid >> 6);
    // XCD-aware order: tiles t of XCD x are x*G8 .. x*G8+G8-1; consecutive t
    // share a support range
    const int64_t G8 = gridDim.x / 8;
    const int64_t t = (int64_t)(blockIdx.x % 8) * G8 + blockIdx.x / 8;
    if (t >= (int64_t)A.nranges * A.nbt)
        return;
#if MBKK_BS_XCD_BY_TILE
    const int range = (int)(t % A.nranges), bt = (int)(t / A.nranges);
#else
    const int range = (int)(t / A.nbt), bt = (int)(t % A.nbt);
#endif
    const int M = *A.seg_total;
    const int Mb = M / 32;
    const int RB = bs_range_blocks(Mb, A.nranges);
    const int blk0 = range * RB;
    if (blk0 >= Mb)
        return;
    const int blk1 = min(Mb, blk0 + RB);
    const int nst = (blk1 - blk0 + SB - 1) / SB;
    const int b0 = (bt * NW + wu) * (32 * NBK);  // this wave's batch rows
    const int n = lane & 31, h = lane >> 5;

    // ---- staging ---------------------------------------------------------
    // DMA slot q of this lane: instruction i = wave + NW q writes chunk
    // position 64 i + lane of a staged array, i.e. row dma_row(q), chunk
    // offset dma_coff(q) (recomputed when needed: registers are scarce)
    __builtin_assume(wu >= 0 && wu < NW);
    auto dma_row = [&](int q) { return min((64 * (wu + NW * q) + lane) / CPS, ROWS - 1); };
    auto dma_coff = [&](int q) {
        const int c = (64 * (wu + NW * q) + lane) % CPS;
        return (c < CPR ? c : 0) * 16;  // the pad position loads any valid chunk
    };
    int pidx[NT];
    // sup_row[Mcap] holds the zero pool row; entries past the support map there
    const int sentinel = A.sup_cap;
    // The staging goes through buffer resources (MUBUF loads into LDS) rather
    // than global_load_lds: the compiler treats a FLAT load that writes LDS as
    // touching both counters, and while one is outstanding every wait on LDS
    // reads becomes a full drain, which serialises the fragment reads that are
    // meant to run two k-steps ahead of their MFMAs.  A MUBUF load into LDS is
    // tracked on the vector-memory counter alone.
    constexpr int kRsrcWord3 = 0x00020000;  // raw buffer, 32-bit data format (gfx9)
    const int sup_bytes = 4 * (A.sup_cap + 1);
    const __amdgpu_buffer_rsrc_t rs_row =
        __builtin_amdgcn_make_buffer_rsrc((void *)A.sup_row, (short)0, sup_bytes, kRsrcWord3);
    const __amdgpu_buffer_rsrc_t rs_ay =
        __builtin_amdgcn_make_buffer_rsrc((void *)A.sup_ay, (short)0, sup_bytes, kRsrcWord3);
    const __amdgpu_buffer_rsrc_t rs_w =
        __builtin_amdgcn_make_buffer_rsrc((void *)A.sup_w, (short)0, sup_bytes, kRsrcWord3);
    const __amdgpu_buffer_rsrc_t rs_p0 = __builtin_amdgcn_make_buffer_rsrc(
        F32 ? (void *)A.pool32 : (void *)A.poolhi, (short)0, A.pool_bytes, kRsrcWord3);
    const __amdgpu_buffer_rsrc_t rs_p1 = __builtin_amdgcn_make_buffer_rsrc(
        F32 ? (void *)A.pool32 : (void *)A.poollo, (short)0, A.pool_bytes, kRsrcWord3);
    auto load_idx = [&](int s) {  // pool rows of this lane's DMA slots in stage s (from global)
        const int r0 = (blk0 + SB * s) * 32;
#pragma unroll
        for (int q = 0; q < NT; ++q) {
            const int srow = r0 + dma_row(q);
            pidx[q] = A.sup_row[srow < M ? srow : sentinel];
        }
    };
    // the pool rows of stage s, staged into index buffer bi by waves 0 and 1
    auto issue_idx = [&](int s, auto bi) {
        if (wu < 2) {
            const int srow = (blk0 + SB * s) * 32 + wu * 64 + lane;
            __builtin_amdgcn_raw_ptr_buffer_load_lds(rs_row, (lds_void_t *)(bufIdx(bi) + wu * 64), 4,
                                                     4 * (srow < M ? srow : sentinel), 0, 0, 0);
        }
    };
    auto read_idx = [&](auto bi) {  // this lane's DMA slot rows from index buffer bi
#pragma unroll
        for (int q = 0; q < NT; ++q)
            pidx[q] = bufIdx(bi)[dma_row(q)];
    };
    // where centers start in the range's blocks: lane l of spl_win holds the
    // row of block blk0 + cw0 + l where a center starts, 32 for none (blocks
    // past the range: none)
    int cw0 = 0, spl_win = 32;
    auto load_spl_win = [&](int base) {
        cw0 = base;
        const int b = blk0 + base + lane;
        spl_win = b < blk1 ? A.blk_split[b] : 32;
    };
    auto issue_slot = [&](auto bc, int q) {  // DMA slot q of every staged array (pidx[q] holds its row)
#pragma unroll
        for (int arr = 0; arr < NARR; ++arr) {
            const int i = wu + NW * q;
            if (NW * q + NW - 1 < NINS || i < NINS)
                __builtin_amdgcn_raw_ptr_buffer_load_lds(arr == 0 ? rs_p0 : rs_p1,
                                                         (lds_void_t *)(bufA(bc) + arr * ABYTES + i * 1024), 16,
                                                         pidx[q] * (DP * ES) + dma_coff(q), 0, 0, 0);
        }
    };
    auto issue_ayw = [&](int s, auto bc) {
        // exponent constants (waves 0, 1) and weights (waves 2, 3), 64 rows each
        if (wu >= 4)
            return;
        const int half = wu & 1;
        const int srow = (blk0 + SB * s) * 32 + half * 64 + lane;
        float *dst = (wu < 2 ? bufAy(bc) : bufW(bc)) + half * 64;
        __builtin_amdgcn_raw_ptr_buffer_load_lds(wu < 2 ? rs_ay : rs_w, (lds_void_t *)dst, 4,
                                                 4 * (srow < M ? srow : sentinel), 0, 0, 0);
    };
    auto issue = [&](int s, auto bc) {  // DMA of stage s into buffer bc
#pragma unroll
        for (int q = 0; q < NT; ++q)
            issue_slot(bc, q);
        issue_ayw(s, bc);
    };
    // The staging of stage s+1 (pool rows already in pidx) and the index
    // staging of stage s+2, as NT + 2 items placed after every IST-th MFMA of
    // stage s (positions k * NMF + mi), so that their issue overlaps
    // matrix-core work; all are issued before the end-of-stage barrier.
    auto stage_item = [&](int s, auto bc, auto bn, int pos) {  // bc / bn: the buffers of stages s / s+1
        // the stride, capped so that every item falls inside the stage
        constexpr int IST = std::min(MBKK_BS_ITEM_STRIDE, (SB * KS * NBK * (X3 ? 3 : 1) - 1) / (NT + 1));
        static_assert(IST >= 1, "staging items");
        if (pos % IST != 0)
            return;
        const int j = pos / IST;
        if (j < NT) {
            if (s + 1 < nst)
                issue_slot(bn, j);
        } else if (j == NT) {
            if (s + 1 < nst)
                issue_ayw(s + 1, bn);
        } else if (j == NT + 1) {
            if (s + 2 < nst)
                issue_idx(s + 2, bc);  // stage s+2 has the parity of stage s
        }
    };

    // ---- batch fragments into registers --------------------------------
    // The batch was written in fragment order when it was staged: the 16
    // bytes lane l = 32 h + n needs for k-step ks of a 32-row block are at
    // ((block * QPB + ks) * 64 + l) * 16 (QPB = KS, or KS / 4 in FP32), so
    // every fragment is one coalesced 1 KB load straight into its register,
    // and all of them are in flight together with the staging of stage 0.
    typedef typename std::conditional<F32, float, bf16x8>::type frag_t;
    frag_t bh[NBK][KS];
    frag_t bl[NBK][X3 ? KS : 1];
    float hx[NBK];
    {
        constexpr int QPB = F32 ? KS / 4 : KS;
        load_idx(0);
        load_spl_win(0);
#pragma unroll
        for (int nbk = 0; nbk < NBK; ++nbk) {
            const int row = b0 + nbk * 32 + n;
            const bool ok = row < A.nb;
            const int64_t blk = (b0 >> 5) + nbk;
            const char *src = A.batfrag + ((blk * QPB) * 64 + lane) * 16;
            if constexpr (F32) {
#pragma unroll
                for (int q = 0; q < QPB; ++q) {
                    const f32x4 z = {0.f, 0.f, 0.f, 0.f};
                    const f32x4 v = ok ? *(const f32x4 *)(src + q * 1024) : z;
                    bh[nbk][4 * q] = v[0];
                    bh[nbk][4 * q + 1] = v[1];
                    bh[nbk][4 * q + 2] = v[2];
                    bh[nbk][4 * q + 3] = v[3];
                }
            } else {
                const u16x8 z8 = {0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
                for (int ks = 0; ks < KS; ++ks) {
                    bh[nbk][ks] = __builtin_bit_cast(bf16x8, ok ? *(const u16x8 *)(src + ks * 1024) : z8);
                    if constexpr (X3)
                        bl[nbk][ks] =
                            __builtin_bit_cast(bf16x8, ok ? *(const u16x8 *)(src + A.frag_lo + ks * 1024) : z8);
                }
            }
            hx[nbk] = ok ? -0.5f * A.batsq[row] : 0.0f;
        }
        issue(0, IC0{});
        if (nst > 1)
            issue_idx(1, IC1{});
    }
    // fragment read of row n of a staged 32-row support block: byte offset in the padded layout
    const int aoff = n * (CPS * 16) + (F32 ? h * KS * 4 : h * 16);
    __syncthreads();  // stage 0 staged; buffer 1 is free for stage 1

    // ---- block products and epilogue ---------------------------------------
    // Epilogue element e of a lane: row i = e / NBK (m = 8 (i/4) + 4 h + i%4
    // of the block), N-block e % NBK.  eay / ew hold the exponent constants
    // and weights of the 16 rows of the block whose epilogue is running; the
    // block being multiplied reloads them for its own epilogue as soon as the
    // running epilogue is done with them (rows 0-7 at half time, rows 8-15 at
    // the end).  The first support fragments of the next block of the stage
    // are read during the last k-step.
    // run: the running center's sums; hold: those of the center that ended
    // inside the block whose epilogue ran last (a center started there)
    float run[NBK], hold[NBK];
#pragma unroll
    for (int nbk = 0; nbk < NBK; ++nbk) {
        run[nbk] = 0.0f;
        hold[nbk] = 0.0f;
    }
    const float c2 = A.c2;
    f32x4 eay[4], ew[4];
#pragma unroll
    for (int g = 0; g < 4; ++g) {
        eay[g] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
        ew[g] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    }
    auto load_ayw = [&](auto bc, int sub, int g0, int g1) {
#pragma unroll
        for (int g = g0; g < g1; ++g) {
            const int m0 = sub * 32 + 8 * g + 4 * h;
            eay[g] = *(const f32x4 *)(bufAy(bc) + m0);
            ew[g] = *(const f32x4 *)(bufW(bc) + m0);
        }
    };
    constexpr int NMF = KS * NBK * (X3 ? 3 : 1);  // MFMAs per block
    constexpr int NEL = 16 * NBK;                 // epilogue elements per lane
    constexpr int HALF = NMF / 2;                 // after it, rows 0-7 of the epilogue are done
    static_assert(NEL * HALF / NMF >= 8 * NBK || true, "");
    // rs: the block's row where a center starts (wave-uniform; 8, 16, 24 inside
    // the block).  The elements run in row-group order (e < 4 g NBK: rows below
    // 8 g, in both lane halves), so at the group where the new center starts
    // the finished center's sums move to hold and run restarts.
    auto epi_range = [&](const f32x16 (&accP)[NBK], int e0, int e1, int rs) {
#pragma unroll
        for (int e = e0; e < e1; ++e) {
            if (e > 0 && e % (4 * NBK) == 0 && rs == 2 * e / NBK) {  // rows 8 g .. : e = 4 g NBK
#pragma unroll
                for (int q = 0; q < NBK; ++q) {
                    hold[q] = run[q];
                    run[q] = 0.0f;
                }
            }
            const int i = e / NBK, nbk = e % NBK;
            run[nbk] = fmaf(ew[i / 4][i % 4], __builtin_amdgcn_exp2f(fmaf(accP[nbk][i], c2, eay[i / 4][i % 4])),
                            run[nbk]);
        }
    };
    // Carried support fragments of the next block: k-step 0 (a0h / a0l) and,
    // in the BF16 forms, k-step 1 (a1h / a1l): the BF16 fragments are read two
    // k-steps ahead of their MFMAs.
    typedef typename std::conditional<F32, f32x4, bf16x8>::type afrag_t;
    afrag_t a0h, a0l, a1h, a1l;
    auto load_a0 = [&](auto bc, int sub) {
        const char *base = bufA(bc) + sub * 32 * CPS * 16 + aoff;
        if constexpr (F32) {
            a0h = *(const f32x4 *)base;
        } else {
            a0h = __builtin_bit_cast(bf16x8, *(const u16x8 *)base);
            if constexpr (X3)
                a0l = __builtin_bit_cast(bf16x8, *(const u16x8 *)(base + ABYTES));
        }
    };
    auto load_a1 = [&](auto bc, int sub) {  // BF16: k-step 1 of block sub
        if constexpr (!F32) {
            const char *base = bufA(bc) + sub * 32 * CPS * 16 + aoff + 32;
            a1h = __builtin_bit_cast(bf16x8, *(const u16x8 *)base);
            if constexpr (X3)
                a1l = __builtin_bit_cast(bf16x8, *(const u16x8 *)(base + ABYTES));
        }
    };
    // The element range of MFMA mi: the epilogue is spread evenly; rows 0-7
    // (elements < 8 NBK) are finished by MFMA HALF - 1.
    auto share = [&](const f32x16 (&accP)[NBK], int mi, auto bc, int sub, int rs) {
        int e0 = mi * NEL / NMF, e1 = (mi + 1) * NEL / NMF;
        if (mi < HALF) {
            e1 = min(e1, 8 * NBK);
            e0 = min(e0, 8 * NBK);
            if (mi == HALF - 1)
                e1 = 8 * NBK;
        } else {
            e0 = max(e0, 8 * NBK);
        }
        epi_range(accP, e0, e1, rs);
        if (mi == HALF - 1)
            load_ayw(bc, sub, 0, 2);
        if (mi == NMF - 1)
            load_ayw(bc, sub, 2, 4);
    };
    // MFMAs of block `sub` of buffer bc into accN (k-step 0 fragments in
    // a0h / a0l), with the epilogue of the previous block (accP) spread
    // between them; reads the next block's k-step 0 fragments when `nsub` >= 0.
    auto fused_block = [&](f32x16 (&accN)[NBK], const f32x16 (&accP)[NBK], auto bc, int sub, int nsub,
                           auto hook, int rs) {
#pragma unroll
        for (int nbk = 0; nbk < NBK; ++nbk)
#pragma unroll
            for (int i = 0; i < 16; ++i)
                accN[nbk][i] = hx[nbk];
        const char *base = bufA(bc) + sub * 32 * CPS * 16 + aoff;
        if constexpr (F32) {
            f32x4 av = a0h, an;
#pragma unroll
            for (int s4 = 0; s4 < KS; s4 += 4) {
                if (s4 + 4 < KS)
                    an = *(const f32x4 *)(base + (s4 + 4) * 4);
                else if (nsub >= 0)
                    load_a0(bc, nsub);
#pragma unroll
                for (int u = 0; u < 4; ++u)
#pragma unroll
                    for (int nbk = 0; nbk < NBK; ++nbk) {
                        const int mi = ((s4 + u) * NBK + nbk);
                        accN[nbk] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[u], bh[nbk][s4 + u], accN[nbk], 0, 0, 0);
                        share(accP, mi, bc, sub, rs);
                        hook(mi);
                        __builtin_amdgcn_sched_barrier(0);
                    }
                av = an;
            }
        } else {
            static_assert(F32 || KS >= 2, "BF16 fragments are read two k-steps ahead");
            bf16x8 ah = a0h, ah1 = a1h, ahn = a0h;
            bf16x8 al = a0l, al1 = a1l, aln = a0l;  // lo fragments: BF16X3 only
            constexpr int NP = X3 ? 3 : 1;  // products per (k-step, N-block)
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) {
                if (ks + 2 < KS) {
                    ahn = __builtin_bit_cast(bf16x8, *(const u16x8 *)(base + (ks + 2) * 32));
                    if constexpr (X3)
                        aln = __builtin_bit_cast(bf16x8, *(const u16x8 *)(base + ABYTES + (ks + 2) * 32));
                } else if (nsub >= 0) {
                    if (ks + 2 == KS)
                        load_a0(bc, nsub);
                    else
                        load_a1(bc, nsub);
                }
#pragma unroll
                for (int pr = 0; pr < NP; ++pr)
#pragma unroll
                    for (int nbk = 0; nbk < NBK; ++nbk) {
                        const int mi = (ks * NP + pr) * NBK + nbk;
                        const bf16x8 aa = pr == 2 ? al : ah;
                        const bf16x8 bb = pr == 1 ? bl[nbk][ks] : bh[nbk][ks];
                        accN[nbk] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(aa, bb, accN[nbk], 0, 0, 0);
                        share(accP, mi, bc, sub, rs);
                        hook(mi);
                        __builtin_amdgcn_sched_barrier(0);
                    }
                ah = ah1;
                ah1 = ahn;
                if constexpr (X3) {
                    al = al1;
                    al1 = aln;
                }
            }
        }
    };
    // partial slots: 2 b for the run from block b's start, 2 b + 1 for the run
    // of a center that starts inside block b
    int run_slot = 2 * blk0;
    auto flush_vals = [&](float (&vals)[NBK]) {
        // lane l holds the half-sum (over rows with m % 8 in 4h..4h+3) of
        // column n of every N-block; swapping lanes 32-63 of block p with
        // lanes 0-31 of block p+1 puts both halves of block p in lanes < 32
        // and both halves of block p+1 in lanes >= 32
#pragma unroll
        for (int p = 0; p < NBK; p += 2) {
            const int q = p + 1 < NBK ? p + 1 : p;  // an unpaired last block pairs with itself
            const auto sw = __builtin_amdgcn_permlane32_swap(__float_as_uint(vals[p]), __float_as_uint(vals[q]), false,
                                                             false);
            const float tot = __uint_as_float(sw[0]) + __uint_as_float(sw[1]);
            const int col = b0 + (p + h) * 32 + n;
            if ((q != p || h == 0) && col < A.nb)
                A.part[(int64_t)run_slot * A.ldp + col] = tot;
        }
#pragma unroll
        for (int nbk = 0; nbk < NBK; ++nbk)
            vals[nbk] = 0.0f;
    };
    auto flush = [&]() { flush_vals(run); };

    // the block whose epilogue runs next, and its row where a center starts
    int prev_blk = blk0, prev_rs = 32;
    bool last_odd = false;
    auto split_over = [&]() {
        if (prev_rs > 0 && prev_rs < 32) {
            flush_vals(hold);  // the finished center, at its slot
            run_slot = 2 * prev_blk + 1;
        }
    };

    // ---- pipeline ----------------------------------------------------------
    static_assert(SB % 2 == 0, "blocks alternate between two accumulator sets");
    f32x16 acc0[NBK], acc1[NBK];  // even / odd blocks
#pragma unroll
    for (int nbk = 0; nbk < NBK; ++nbk)
#pragma unroll
        for (int i = 0; i < 16; ++i)
            acc1[nbk][i] = 0.0f;  // the "previous block" of the first one: weights 0
    // one stage in buffer bc; the next stage is staged into bn
    auto stage = [&](int s, auto bc, auto bn) {
        const int bp = blk0 + SB * s;
        if (SB * s + SB - 1 - cw0 >= 64)
            load_spl_win(SB * s);  // ranges of more than 64 blocks: next window
        int spl[SB];
#pragma unroll
        for (int k = 0; k < SB; ++k)
            spl[k] = __builtin_amdgcn_readlane(spl_win, SB * s + k - cw0);
        if (s + 1 < nst)
            read_idx(bn);  // pool rows of stage s+1, staged during stage s-1
        if constexpr (!kBsSpreadStaging) {
            if (s + 1 < nst) {
                issue(s + 1, bn);
                if (s + 2 < nst)
                    issue_idx(s + 2, bc);
            }
        }
        load_a0(bc, 0);
        if constexpr (!F32)
            load_a1(bc, 0);
#pragma unroll
        for (int k = 0; k < SB; ++k) {
            // block bp + k; epilogue of block bp + k - 1; staging items of the next stage
            if (bp + k >= blk1)
                continue;  // past the range (its last stage, which stages nothing more)
            const int nsub = k + 1 < SB ? k + 1 : -1;
            if constexpr (MBKK_BS_PRIO != 0) {
                switch (k) {  // (k is a constant once the loop is unrolled)
                case 0: __builtin_amdgcn_s_setprio(3); break;
                case 1: __builtin_amdgcn_s_setprio(2); break;
                case 2: __builtin_amdgcn_s_setprio(1); break;
                default: __builtin_amdgcn_s_setprio(0); break;
                }
            }
            auto hook = [&](int mi) {
                if constexpr (kBsSpreadStaging)
                    stage_item(s, bc, bn, k * NMF + mi);
            };
            if (k % 2 == 0)
                fused_block(acc0, acc1, bc, k, nsub, hook, prev_rs);
            else
                fused_block(acc1, acc0, bc, k, nsub, hook, prev_rs);
            last_odd = k % 2 == 1;
            // the previous block's epilogue is done: a center that started
            // inside it takes over (the finished center's sums are in hold)
            split_over();
            // a center that starts at this block's first row
            if (spl[k] == 0 && bp + k != blk0) {
                flush();
                run_slot = 2 * (bp + k);
            }
            prev_blk = bp + k;
            prev_rs = spl[k];
        }
        __syncthreads();
    };
    for (int s = 0; s < nst; s += 2) {
        stage(s, IC0{}, IC1{});
        if (s + 1 < nst)
            stage(s + 1, IC1{}, IC0{});
    }
    // the last block's epilogue (its accumulator set by its parity)
    if (last_odd)
        epi_range(acc1, 0, NEL, prev_rs);
    else
        epi_range(acc0, 0, NEL, prev_rs);
    split_over();
    flush();
#endif
}

void launch_cross_mfma(const Layout &L, const Buffers &B, int nb, int precision, double kappa, hipStream_t st)
{
    const double l2e = 1.4426950408889634;
    if (L.dp <= 128) {
        CrossBsArgs A;
        A.nb = nb;
        const int mode = bs_mode(precision), tr = bs_tile_rows(mode, L.dp);
        A.nbt = (nb + tr - 1) / tr;
        A.nranges = bs_nranges(nb, mode, L.dp);
        A.sup_cap = (int32_t)L.Mcap;
        A.seg_total = B.seg_off + L.k;
        A.pool32 = B.pool32;
        A.poolhi = B.poolhi;
        A.poollo = B.poollo;
        // at most (65536 + 31 * 8192 + 1) rows of 128 FP32 coordinates (164 MB): the
        // configuration limits on k, the window and b_max keep it within 31 bits
        A.pool_bytes = (int32_t)((L.PR + 1) * L.dp * (precision == MBKK_FP32 ? 4 : 2));
        A.sup_row = B.sup_row;
        A.sup_w = B.sup_w;
        A.sup_ay = B.sup_ay;
        A.blk_split = B.blk_split;
        A.batfrag = (const char *)B.batfrag;
        A.frag_lo = 2 * (int64_t)frag_rows(L) * L.dp;
        A.batsq = B.batsq;
        A.c2 = (float)(2.0 * l2e / kappa);
        A.part = (float *)B.part;
        A.ldp = L.bmax;
        const int64_t tiles = (int64_t)A.nranges * A.nbt;
        const dim3 grid((unsigned)((tiles + 7) / 8 * 8));
#define MBKK_BS(MODE, DP) hipLaunchKernelGGL((k_cross_bs<MODE, DP>), grid, dim3(256 * bs_wps(MODE, DP)), 0, st, A)
#define MBKK_BS_DP(MODE)                      \
    switch (L.dp) {                           \
    case 32: MBKK_BS(MODE, 32); break;        \
    case 64: MBKK_BS(MODE, 64); break;        \
    case 96: MBKK_BS(MODE, 96); break;        \
    default: MBKK_BS(MODE, 128); break;       \
    }
        if (precision == MBKK_FP32) {
            MBKK_BS_DP(0);
        } else if (precision == MBKK_BF16X3) {
            MBKK_BS_DP(1);
        } else {
            MBKK_BS_DP(2);
        }
#undef MBKK_BS_DP
#undef MBKK_BS
        return;
    }
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

}  // namespace mbkk
