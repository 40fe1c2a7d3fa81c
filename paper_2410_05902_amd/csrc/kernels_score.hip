// Distances, argmin and margin of each batch row, the FP64 re-scoring of
// near ties, and the grouping ranks of the update (Algorithm 2's assignment
// step).  For a batch row x and center j (an implicit sparse combination of
// feature vectors, Section 4.1 / Eq. 1) the distance in feature space is
//     ||phi(x) - C_j||^2 = K(x,x) - 2 <phi(x), C_j> + <C_j, C_j>
// with the cross term P_j(x) from the partial sums of the cross kernels
// (kernels_cross.hip) and the self norm N_j = <C_j, C_j> from the Gram blocks.
#include "cross_layout.h"
#include "dev_common.h"
#include "kernels.h"

namespace mbkk {

// ===========================================================================
// Distances, argmin and margin of each batch row:
//   D_j = K(x,x) - 2 P_j + N_j, the FP32 cross term added to the FP64 self
//   norm in FP64.  In a nearly orthogonal feature space (the Laplacian at
//   sigma = 4 in 32-D: kernel values of 1e-8 and below) the centers' P_j
//   differ far below an FP32 ulp of N_j, and an FP32 sum would tie them.
// label = smallest j attaining the minimum; margin = second smallest - min.
// LAYOUT 0: runs of the direct kernel; 1, 2: runs of the MFMA kernels (below).
// ===========================================================================
__device__ __forceinline__ double self_kernel(int kind, double param, double sq)
{
    if (kind == MBKK_LINEAR)
        return sq;
    if (kind == MBKK_POLY2)
        return (sq + param) * (sq + param);
    return 1.0;  // normalised kernels: K(x,x) = 1
}

// LAYOUT 0: the direct kernel's runs (ranges of RR rows): run j (the run at
// the center's first row) plus run k + r of every range r that starts
// strictly inside the center's segment.
// LAYOUT 1: the MFMA kernels write one partial per run of a center's blocks
// inside a range of RB blocks, at the run's first block: the center's first
// block and every range start inside the center.
// LAYOUT 2 (packed segments, which may start inside a block): two slots per
// block, 2 b for the run from block b's first row (a range start, or a center
// starting there) and 2 b + 1 for a center starting inside block b; a
// center's partials are its first slot and slot 2 b of every range start b
// after its first block and inside its segment.
// The direct kernel's runs are summed in FP64, the MFMA kernels' in FP32.
template <typename T, int LAYOUT>
__device__ __forceinline__ double cross_of(const T *__restrict__ part, int ldp, int row, int j,
                                           const int32_t *__restrict__ seg_off, int RB, int k = 0)
{
    if constexpr (LAYOUT == 0) {
        const int s0 = seg_off[j], s1 = seg_off[j + 1];
        if (s0 >= s1)
            return 0.0;
        double s = (double)part[(int64_t)j * ldp + row];
        for (int r = s0 / RB + 1; r * RB < s1; ++r)
            s += (double)part[(int64_t)(k + r) * ldp + row];
        return s;
    } else if constexpr (LAYOUT == 1) {
        const int bs = seg_off[j] / 32, be = seg_off[j + 1] / 32;
        if (bs >= be)
            return 0.0;
        float s = part[(int64_t)bs * ldp + row];
        for (int blk = (bs / RB + 1) * RB; blk < be; blk += RB)
            s += part[(int64_t)blk * ldp + row];
        return (double)s;
    } else {
        const int s0 = seg_off[j], s1 = seg_off[j + 1];
        if (s0 >= s1)
            return 0.0;
        const int b0 = s0 / 32;
        float s = part[(int64_t)(2 * b0 + (s0 % 32 != 0)) * ldp + row];
        for (int blk = (b0 / RB + 1) * RB; 32 * blk < s1; blk += RB)
            s += part[(int64_t)(2 * blk) * ldp + row];
        return (double)s;
    }
}

// cross_of in two phases, so that the loads of several centers are in
// flight together: cross_fetch issues the first two partials of the segment
// at clamped indices (no branch), cross_finish adds them in cross_of's order
// and, for a segment spanning more than two ranges, the rest in a loop.
template <typename T>
struct CrossFetch {
    T a, b;
    int lo, hi, next;  // LAYOUT 0, 2: segment [lo, hi) in entries; 1: blocks [lo, hi); next range or block
};

// s0, s1: seg_off[j], seg_off[j + 1]; mtot: seg_off[k]
template <typename T, int LAYOUT>
__device__ __forceinline__ CrossFetch<T> cross_fetch_at(const T *__restrict__ part, int ldp, int row, int j, int s0,
                                                        int s1, int mtot, int RB, int k)
{
    CrossFetch<T> f;
    if constexpr (LAYOUT == 0) {
        f.lo = s0;
        f.hi = s1;
        const int r1 = f.lo / RB + 1;
        const int nr = (mtot + RB - 1) / RB;  // ranges that hold partials
        f.a = part[(int64_t)j * ldp + row];
        f.b = part[(int64_t)(k + max(min(r1, nr - 1), 0)) * ldp + row];
        f.next = r1 * RB < f.hi ? r1 + 1 : -1;
    } else if constexpr (LAYOUT == 1) {
        f.lo = s0 / 32;
        f.hi = s1 / 32;
        const int b1 = (f.lo / RB + 1) * RB;
        const int top = max(f.hi - 1, 0);
        f.a = part[(int64_t)min(f.lo, top) * ldp + row];
        f.b = part[(int64_t)min(b1, top) * ldp + row];
        f.next = b1 < f.hi ? b1 + RB : -1;
    } else {
        f.lo = s0;
        f.hi = s1;
        const int b0 = s0 / 32, b1 = (b0 / RB + 1) * RB;
        const int top = max(2 * (mtot / 32) - 1, 0);  // last slot of the support
        f.a = part[(int64_t)min(2 * b0 + (s0 % 32 != 0), top) * ldp + row];
        f.b = part[(int64_t)min(2 * b1, top) * ldp + row];
        f.next = 32 * b1 < s1 ? b1 + RB : -1;
    }
    return f;
}

template <typename T, int LAYOUT>
__device__ __forceinline__ CrossFetch<T> cross_fetch(const T *__restrict__ part, int ldp, int row, int j,
                                                     const int32_t *__restrict__ seg_off, int RB, int k)
{
    return cross_fetch_at<T, LAYOUT>(part, ldp, row, j, seg_off[j], seg_off[j + 1], seg_off[k], RB, k);
}

template <typename T, int LAYOUT>
__device__ __forceinline__ double cross_finish(const CrossFetch<T> &f, const T *__restrict__ part, int ldp, int row,
                                               int RB, int k)
{
    if (f.lo >= f.hi)
        return 0.0;
    if constexpr (LAYOUT == 0) {
        double s = (double)f.a;
        if (f.next >= 0) {
            s += (double)f.b;
            for (int r = f.next; r * RB < f.hi; ++r)
                s += (double)part[(int64_t)(k + r) * ldp + row];
        }
        return s;
    } else if constexpr (LAYOUT == 1) {
        float s = f.a;
        if (f.next >= 0) {
            s += f.b;
            for (int blk = f.next; blk < f.hi; blk += RB)
                s += part[(int64_t)blk * ldp + row];
        }
        return (double)s;
    } else {
        float s = f.a;
        if (f.next >= 0) {
            s += f.b;
            for (int blk = f.next; 32 * blk < f.hi; blk += RB)
                s += part[(int64_t)(2 * blk) * ldp + row];
        }
        return (double)s;
    }
}

// One workgroup per 64 batch rows; its 16 waves split the centers (wave w
// takes j = w, w + 16, ...), each lane one row, then the 16 partial
// (best, label, second) triples of a row are merged in LDS.  Ties go to the
// lowest center index: comparisons are on (distance, label).
constexpr int kScoreWaves = 16;

__device__ __forceinline__ bool lex_less(double a, int la, double b, int lb)
{
    return a < b || (a == b && la < lb);
}

// One butterfly step of the per-row merge: the partner lane's (best, label,
// second) by the DPP pattern CTRL, then the lexicographically smaller best
// and the smallest remaining value as the second.
template <int CTRL>
__device__ __forceinline__ void score_merge_step(double &b0, int &l0, double &s0)
{
    const double bq = dpp_f64<CTRL>(b0), sq = dpp_f64<CTRL>(s0);
    const int lq = __builtin_amdgcn_update_dpp(0, l0, CTRL, 0xf, 0xf, false);
    if (lex_less(bq, lq, b0, l0)) {
        s0 = fmin(b0, sq);
        b0 = bq;
        l0 = lq;
    } else {
        s0 = fmin(s0, bq);
    }
}

struct ScoreArgs {
    int nb, k, ldp, RB, kind;
    int nranges;  // > 0: RB of the batch-stationary kernel, derived from the support size
    double param;
    const void *part;
    const int32_t *seg_off;
    const double *N;
    const double *batsq64;
    int32_t *labels;
    float *mind, *margin;
    double *Dout;
    int64_t ldD;
    // FP64 re-scoring of near ties (BF16 forms): a fixed threshold (delta > 0)
    // or the per-row bound from rel_dot, ymax2 and eN (the bound on the error
    // of a self norm N_j); nresc counts the re-scored rows
    double delta, kappa, rel_dot, ymax2, eN;
    unsigned long long *nresc;
    int d, dp;
    const float *bat32, *pool32;
    const int32_t *sup_row;
    const double *sup_w64;
    // grouping ranks (iteration only): rank of each row among the equal
    // labels before it in its chunk of 64 rows, and the chunk's label counts
    int32_t *rank, *gcnt;
};

// FP64 re-scoring of one batch row by one wave: candidates are the centers
// whose approximate distance is within delta of the best; for them the cross
// term is recomputed in FP64 from the FP32 coordinates (direct ||x - y||^2,
// FP64 exp, FP64 weights), and their distances (also in Dout when requested)
// then carry only the error of N_j (FP32 kernel values summed in FP64).
// best: the row's smallest approximate distance (from the scoring pass);
// seg_off / Nv: the segment offsets and self norms (LDS copies when staged).
template <int LAYOUT>
__device__ void rescore_row(const ScoreArgs &A, int row, int RB, double delta, double best,
                            const int32_t *__restrict__ seg_off, const double *__restrict__ Nv, int &lab_io,
                            float &mind_io, float &margin_io)
{
    const int lane = threadIdx.x & 63;
    const float *part = (const float *)A.part;
    const float *x = A.bat32 + (int64_t)row * A.dp;
    double b64 = INFINITY, s64 = INFINITY, outside = INFINITY;
    int lab = 0;
    for (int j0 = 0; j0 < A.k; j0 += 64) {
        const int jl = j0 + lane;
        const double Dap =
            jl < A.k ? 1.0 - 2.0 * cross_of<float, LAYOUT>(part, A.ldp, row, jl, seg_off, RB) + Nv[jl] : INFINITY;
        const bool cand = Dap <= best + delta;
        if (!cand)
            outside = fmin(outside, Dap);
        uint64_t mask = __ballot(cand);
        while (mask) {  // candidates in increasing center order (wave-uniform loop)
            const int bit = __ffsll((unsigned long long)mask) - 1;
            mask &= mask - 1;
            const int j = j0 + bit;
            double p = 0.0;
            for (int s = seg_off[j] + lane; s < seg_off[j + 1]; s += 64) {
                const double w = A.sup_w64[s];
                if (w == 0.0)
                    continue;
                // rows are zero past d up to the padded stride: 16-byte loads over dp
                const f32x4 *y4 = (const f32x4 *)(A.pool32 + (int64_t)A.sup_row[s] * A.dp);
                const f32x4 *x4 = (const f32x4 *)x;
                double d2 = 0.0;
#pragma unroll 4
                for (int t4 = 0; t4 < A.dp / 4; ++t4) {
                    const f32x4 a = x4[t4], c = y4[t4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const double v = (double)a[u] - (double)c[u];
                        d2 = fma(v, v, d2);
                    }
                }
                p += w * exp(-d2 / A.kappa);
            }
            for (int o = 32; o > 0; o >>= 1)
                p += __shfl_xor(p, o);
            const double D = 1.0 - 2.0 * p + Nv[j];
            if (A.Dout && lane == 0)
                A.Dout[(int64_t)row * A.ldD + j] = D;  // replaces the approximate value
            if (D < b64) {
                s64 = b64;
                b64 = D;
                lab = j;
            } else if (D < s64) {
                s64 = D;
            }
        }
    }
    for (int o = 32; o > 0; o >>= 1)
        outside = fmin(outside, __shfl_xor(outside, o));
    lab_io = lab;
    mind_io = (float)b64;
    margin_io = (float)(fmin(s64, outside) - b64);
}

// LK: the segment offsets and self norms are first copied to LDS (k <= kScoreLdsK).
constexpr int kScoreLdsK = 2048;

template <typename T, int LAYOUT, bool RESCORE, bool LK>
__global__ __launch_bounds__(64 * kScoreWaves) void k_score(const ScoreArgs A)
{
    // per-wave (best, second, label) of each row, row-major with one pad entry
    // so that neither the waves' stores nor the merge's loads share banks
    __shared__ double sb[64][kScoreWaves + 1], ss[64][kScoreWaves + 1];
    __shared__ int sl[64][kScoreWaves + 1];
    __shared__ int flab[64];
    __shared__ float fmin_[64], fmar[64];
    __shared__ double fdel[64], fbest[64], sep0[64];
    __shared__ int smax_seg, snresc;
    __shared__ int32_t lseg[LK ? kScoreLdsK + 1 : 1];
    __shared__ double lN[LK ? kScoreLdsK : 1];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int row = blockIdx.x * 64 + lane;
    const bool act = row < A.nb;
    const T *part = (const T *)A.part;
    const double x2row = A.batsq64[min(row, A.nb - 1)];
    // the merge below gives wave w rows 4w .. 4w + 3, 16 lanes each
    static_assert(kScoreWaves == 16, "16 partial triples per row, one per lane of a DPP row");
    const int mrow = w * 4 + (lane >> 4), mq = lane & 15;
    // loads in issue order: the LDS copy's first pass, then the partials of
    // the wave's first batch of centers (j = w, w + 16, ...), whose segment
    // bounds are scalar loads (the center index is wave-uniform), so that
    // the partials are requested before the barriers below.  Hoisted in the
    // FP32 forms only (the FP64 form has no registers left for it).
    constexpr int NB = 8;
    constexpr bool HOIST = sizeof(T) == 4;
    int sv0 = 0;
    double nv0 = 0.0;
    if constexpr (LK) {
        const int i = min((int)threadIdx.x, A.k);
        sv0 = A.seg_off[i];
        nv0 = A.N[min(i, A.k - 1)];
    }
    const int mtot = A.seg_off[A.k];
    const int RB = LAYOUT == 0 ? direct_range_rows(mtot, A.nranges)
                               : (A.nranges > 0 ? bs_range_blocks(mtot / 32, A.nranges) : A.RB);
    CrossFetch<T> fe0[HOIST ? NB : 1];
    if constexpr (HOIST) {
        int s0[NB], s1[NB];
#pragma unroll
        for (int u = 0; u < NB; ++u) {
            const int j = min(w + u * kScoreWaves, A.k - 1);
            s0[u] = A.seg_off[j];
            s1[u] = A.seg_off[j + 1];
        }
        __builtin_amdgcn_sched_barrier(0);  // every bound requested before the first partial
#pragma unroll
        for (int u = 0; u < NB; ++u)
            fe0[u] = cross_fetch_at<T, LAYOUT>(part, A.ldp, min(row, A.nb - 1), min(w + u * kScoreWaves, A.k - 1),
                                               s0[u], s1[u], mtot, RB, A.k);
    }
    const int32_t *seg_off = A.seg_off;
    const double *Nv = A.N;
    if constexpr (LK) {
        if ((int)threadIdx.x <= A.k) {
            lseg[threadIdx.x] = sv0;
            if ((int)threadIdx.x < A.k)
                lN[threadIdx.x] = nv0;
        }
        __builtin_amdgcn_sched_barrier(0);  // (these stores wait for the copy's loads only)
        for (int i = threadIdx.x + 64 * kScoreWaves; i <= A.k; i += 64 * kScoreWaves) {
            const int sv = A.seg_off[i];
            const double nv = A.N[min(i, A.k - 1)];
            __builtin_amdgcn_sched_barrier(0);  // both loads before either store
            lseg[i] = sv;
            if (i < A.k)
                lN[i] = nv;
        }
        __syncthreads();
        seg_off = lseg;
        Nv = lN;
    }
    const double kxx = act ? self_kernel(A.kind, A.param, x2row) : 0.0;
    if (RESCORE && w == kScoreWaves - 1 && !(A.delta > 0.0)) {
        // the row's part of the error bound below that needs no other wave,
        // taken while the partials are in flight
        const double x2 = act ? x2row : 0.0, y2 = A.ymax2;
        const double xn = sqrt(x2), yn = sqrt(y2);
        sep0[lane] = (2.0 * A.rel_dot * xn * yn + 0x1p-22 * (x2 + y2)) / A.kappa;
    }
    if constexpr (RESCORE) {
        // longest center segment: the length of the FP32 sums in the error bound
        if (threadIdx.x == 0) {
            smax_seg = 0;
            snresc = 0;
        }
        __syncthreads();
        int m = 0;
        for (int i = threadIdx.x; i < A.k; i += 64 * kScoreWaves)
            m = max(m, seg_off[i + 1] - seg_off[i]);
        m = wave_max(m);
        if (lane == 0)
            atomicMax(&smax_seg, m);
    }
    double best = INFINITY, second = INFINITY;
    int lab = 0x7fffffff;
    if (act) {
        // the wave's centers j = w, w + 16, ... in batches of 8 whose loads
        // are all in flight together (the first batch's since the start)
        for (int j0 = w; j0 < A.k; j0 += kScoreWaves * NB) {
            double P[NB], Nj[NB];
            CrossFetch<T> fe[NB];
            if (HOIST && j0 == w) {
#pragma unroll
                for (int u = 0; u < NB; ++u)
                    fe[u] = fe0[HOIST ? u : 0];
            } else {
#pragma unroll
                for (int u = 0; u < NB; ++u)
                    fe[u] = cross_fetch<T, LAYOUT>(part, A.ldp, row, min(j0 + u * kScoreWaves, A.k - 1), seg_off, RB,
                                                   A.k);
            }
#pragma unroll
            for (int u = 0; u < NB; ++u) {
                const int j = j0 + u * kScoreWaves;
                P[u] = j < A.k ? cross_finish<T, LAYOUT>(fe[u], part, A.ldp, row, RB, A.k) : 0.0;
                Nj[u] = j < A.k ? Nv[j] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < NB; ++u) {
                const int j = j0 + u * kScoreWaves;
                if (j < A.k) {
                    // in FP64, in the order K(x,x) - 2 P + N
                    const double D = kxx - 2.0 * P[u] + Nj[u];
                    if (A.Dout)
                        A.Dout[(int64_t)row * A.ldD + j] = D;
                    if (D < best) {  // j increases within a wave: strict < keeps the lowest index
                        second = best;
                        best = D;
                        lab = j;
                    } else if (D < second) {
                        second = D;
                    }
                }
            }
        }
    }
    sb[lane][w] = best;
    ss[lane][w] = second;
    sl[lane][w] = lab;
    __syncthreads();
    {
        // the 16 triples of row mrow, one per lane of a DPP row, merged by a
        // butterfly; the merge is an exact selection (the lexicographic
        // minimum of (distance, label), then the smallest other value), so
        // every order gives the sequential result
        double b0 = sb[mrow][mq], s0 = ss[mrow][mq];
        int l0 = sl[mrow][mq];
        score_merge_step<0xb1>(b0, l0, s0);   // quad_perm [1,0,3,2]
        score_merge_step<0x4e>(b0, l0, s0);   // quad_perm [2,3,0,1]
        score_merge_step<0x141>(b0, l0, s0);  // row_half_mirror
        score_merge_step<0x140>(b0, l0, s0);  // row_mirror
        if (mq == 0) {
            // a row whose distances are all NaN (non-finite input) matched no
            // center: it is assigned to center 0 so that every label is in range
            if (!(l0 >= 0 && l0 < A.k))
                l0 = 0;
            flab[mrow] = l0;
            fmin_[mrow] = (float)b0;
            fmar[mrow] = (float)(s0 - b0);
            if constexpr (RESCORE) {
                // Error bound of an approximate distance D_j (Gaussian, BF16 form):
                // the exponent a = (2 x.y - |x|^2 - |y|^2) / kappa has
                // |da| <= (2 rel_dot |x||y| + 2^-22 (|x|^2 + |y|^2)) / kappa = e(x, y)
                // (rel_dot: relative error of x.y against sum |x_t y_t| <= |x||y|;
                // 2^-22: the FP32 roundings of the norms and of the FMA), so a
                // kernel value has relative error <= e, and with weights summing
                // to at most 1 and kernel values at most 1
                //   |dP_j| <= e(x, Y) + S 2^-24,  |dN_j| <= e(Y, Y) + S 2^-24
                // (Y^2 = max |y|^2 over the data, S = longest segment: the FP32
                // sums).  N_j comes from FP32 kernel values summed in FP64: its
                // bound eN is the host's.  A margin above 2 (2 |dP| + |dN|) cannot
                // hide a swap.
                double dl = A.delta;
                if (!(dl > 0.0)) {
                    const double gS = (double)smax_seg * 0x1p-24;
                    const double eP = sep0[mrow] + gS;  // e(x, Y) from before the main loop
                    dl = 2.0 * (2.0 * eP + A.eN);
                }
                fdel[mrow] = dl;
                fbest[mrow] = b0;
            }
        }
    }
    __syncthreads();
    if constexpr (RESCORE) {
        // the wave's rows w, w + 16, w + 32, w + 48, tested by lanes 0-3 at once
        const int rt = w + kScoreWaves * (lane & 3);
        uint64_t todo = __ballot(lane < 4 && blockIdx.x * 64 + rt < A.nb && (double)fmar[rt] < fdel[rt]);
        while (todo) {  // wave-uniform row loop
            const int r = w + kScoreWaves * (__ffsll((unsigned long long)todo) - 1);
            todo &= todo - 1;
            const int rw = blockIdx.x * 64 + r;
            {
                int l;
                float m, g;
                rescore_row<LAYOUT>(A, rw, RB, fdel[r], fbest[r], seg_off, Nv, l, m, g);
                if (lane == 0) {
                    flab[r] = l;
                    fmin_[r] = m;
                    fmar[r] = g;
                    atomicAdd(&snresc, 1);
                }
            }
        }
        __syncthreads();
        if (threadIdx.x == 0 && snresc > 0 && A.nresc)
            atomicAdd(A.nresc, (unsigned long long)snresc);
    }
    if (w == 0 && act) {
        A.labels[row] = flab[lane];
        A.mind[row] = fmin_[lane];
        A.margin[row] = fmar[lane];
    }
    if (A.rank) {
        // rank of row r among the rows t < r of the chunk with its label, and
        // the chunk's count of that label (stored by the label's last row):
        // one ballot per row, rows spread over the waves
        int32_t *cnt = A.gcnt + (int64_t)blockIdx.x * A.k;
        for (int j = threadIdx.x; j < A.k; j += 64 * kScoreWaves)
            cnt[j] = 0;
        __syncthreads();
        const int nrow = min(64, A.nb - blockIdx.x * 64);
        const int Ll = lane < nrow ? flab[lane] : -1;
        for (int r = w; r < nrow; r += kScoreWaves) {  // wave uniform
            const int Lr = __builtin_amdgcn_readlane(Ll, r);
            const uint64_t m = __ballot(Ll == Lr);
            if (lane == 0) {
                const int rk = __popcll(m & ((1ull << r) - 1ull));
                const int c = __popcll(m);
                A.rank[blockIdx.x * 64 + r] = rk;
                if (rk == c - 1)
                    cnt[Lr] = c;
            }
        }
    }
}

// Bound on |N_j - <C_j, C_j>| for the Gaussian MFMA forms, whose Gram blocks
// hold FP32 kernel values summed in FP64 (u = 2^-24):
//  - a.e on FP32 MFMA over dp products: |d(a.e)| <= dp u |a||e| (+u: c2);
//  - the exponent's FP32 norms, scalings and sum: 4u (|a|^2 + |e|^2);
//  - so a kernel value has relative error <= (2 (dp+1) u Y^2 + 8u Y^2) / kappa
//    with Y^2 = max |y|^2 over the data, plus 2u for exp2 and the rounding of
//    its argument;
//  - the weights' products sum to at most 1 (FP64 coefficients and sums).
double selfnorm_error_bound(int dp, double ymax2, double kappa)
{
    const double u = 0x1p-24;
    return (2.0 * (dp + 1) * u * ymax2 + 8.0 * u * ymax2) / kappa + 2.0 * u;
}

void launch_score(const Layout &L, const Buffers &B, int nb, int kind, double param, int fp64, int mfma,
                  int precision, double tie_delta, double ymax2, double *D_out, int64_t ldD, bool with_rank,
                  hipStream_t st)
{
    ScoreArgs A;
    A.nb = nb;
    A.k = L.k;
    A.ldp = L.bmax;
    A.RB = 2;
    A.nranges = mfma ? (L.dp <= 128 ? bs_nranges(nb, bs_mode(precision), L.dp) : 0)
                     : direct_nranges(nb, direct_rpl(L.d, fp64));
    A.kind = kind;
    A.param = param;
    A.part = B.part;
    A.seg_off = B.seg_off;
    A.N = B.N;
    A.batsq64 = B.batsq64;
    A.labels = B.labels;
    A.mind = B.mind;
    A.margin = B.margin;
    A.Dout = D_out;
    A.ldD = ldD;
    A.delta = tie_delta;
    A.kappa = param;
    // relative error of the split product x.y against sum_t |x_t y_t|: bf16
    // rounding leaves |x - hi| <= 2^-8 |x| and |x - hi - lo| <= 2^-16 |x|;
    // hi.hi + hi.lo + lo.hi misses at most 3 * 2^-16 per term, hi.hi alone
    // 2^-7 + 2^-16; FP32 accumulation of the dp-long (x3: 3 dp) sum adds
    // n 2^-24
    A.rel_dot = precision == MBKK_BF16X1 ? 0x1p-7 + 0x1p-16 + (double)L.dp * 0x1p-24
                                         : 3.0 * 0x1p-16 + 3.0 * (double)L.dp * 0x1p-24;
    A.ymax2 = ymax2;
    A.eN = selfnorm_error_bound(L.dp, ymax2, param);
    A.nresc = B.nresc;
    A.d = L.d;
    A.dp = L.dp;
    A.bat32 = B.bat32;
    A.pool32 = B.pool32;
    A.sup_row = B.sup_row;
    A.sup_w64 = B.sup_w64;
    A.rank = with_rank ? B.rank : nullptr;
    A.gcnt = B.gcnt;
    const bool rescore = precision == MBKK_BF16X3 || precision == MBKK_BF16X1;
    dim3 grid((nb + 63) / 64), block(64 * kScoreWaves);
#define MBKK_SCORE(LK)                                                              \
    do {                                                                            \
        if (fp64)                                                                   \
            hipLaunchKernelGGL((k_score<double, 0, false, LK>), grid, block, 0, st, A); \
        else if (mfma && L.packed && rescore)                                       \
            hipLaunchKernelGGL((k_score<float, 2, true, LK>), grid, block, 0, st, A);   \
        else if (mfma && rescore)                                                   \
            hipLaunchKernelGGL((k_score<float, 1, true, LK>), grid, block, 0, st, A);   \
        else if (mfma && L.packed)                                                  \
            hipLaunchKernelGGL((k_score<float, 2, false, LK>), grid, block, 0, st, A);  \
        else if (mfma)                                                              \
            hipLaunchKernelGGL((k_score<float, 1, false, LK>), grid, block, 0, st, A);  \
        else                                                                        \
            hipLaunchKernelGGL((k_score<float, 0, false, LK>), grid, block, 0, st, A);  \
    } while (0)
    if (L.k <= kScoreLdsK)
        MBKK_SCORE(true);
    else
        MBKK_SCORE(false);
#undef MBKK_SCORE
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
