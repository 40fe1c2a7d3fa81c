// Untruncated mini-batch kernel k-means (Algorithm 1) run on the table of
// cross terms that Appendix A describes:
//     T[j][x] = <phi(x), C_i^j>  for every point x of X and every center j,
//     N[j]    = <C_i^j, C_i^j>.
// With the table the batch distances need no support at all,
//     ||phi(x) - C_i^j||^2 = K(x,x) - 2 T[j][x] + N[j],
// and one iteration updates, by the recursion of Section 4 (recursive
// distance update rule), with a = alpha_i^j and cm = cm(B_i^j):
//     N[j]    <- (1-a)^2 N[j] + 2 a (1-a) <C_i^j, cm> + a^2 <cm, cm>
//     T[j][x] <- (1-a) T[j][x] + a <phi(x), cm>                 for all x in X,
// where <C_i^j, cm> is the mean of the old T[j][y] over y in B_i^j and
// <cm, cm> the mean of K(y, y') over pairs of B_i^j.  Centers with no batch
// point keep T and N (a = 0).
//
// Table layout: center-major, T[j * ldT + x] (ldT = n rounded up to 64), so
// that the update, one lane per point, reads and writes whole lines.  FP32
// table (FP32 kernel values) or FP64 (FP64 kernel values).
//
// Kernels, in step order:
//   k_dp_score : distances of m rows from the table, argmin (lowest index on
//                ties), margin, the old T[label][x], per-center counts;
//   k_dp_plan  : segment offsets of the batch grouped by label, alpha, and
//                the pair tasks (64 x 64 tiles of each center's pairs);
//   k_dp_group : stable grouping (batch order inside a center);
//   k_dp_gram  : the pair tasks: partial sums of K(y, y') over 64 columns;
//   k_dp_rowsum: sum over B_i^j of K(y, y') for each grouped row y;
//   k_dp_norms : the N update and the per-center weights a / b_i^j;
//   k_dp_table : the table update over all of X (the O(n b) term) on the
//                VALU; the Gaussian in BF16X3, and in FP32 unless the
//                difference form is asked for, runs it on MFMA instead
//                (k_dp_mfma, then k_dp_blend).
#include <type_traits>

#include "dev_common.h"
#include "kernels.h"

namespace mbkk {

constexpr int kDpScoreWaves = 16;  // waves of a scoring workgroup; lane = row, waves split the centers
constexpr int kDpTableWG = 256;
constexpr int kDpTile = 64;         // rows and columns of a pair task
constexpr int kDpGramWGs = 1024;    // workgroups of the pair-task kernel (4 waves each, tasks grid-strided)

// Kernel value from the coordinate reduction s (squared distance, L1 distance
// or dot product) and the parameter.
template <int KIND, typename T>
__device__ __forceinline__ T dp_kfinish(T s, T cneg, T param)
{
    if constexpr (KIND == MBKK_GAUSS || KIND == MBKK_LAPLACE) {
        if constexpr (sizeof(T) == 4)
            return __builtin_amdgcn_exp2f(s * cneg);  // cneg = -log2(e) / param
        else
            return exp(-s / param);
    } else if constexpr (KIND == MBKK_LINEAR) {
        return s;
    } else {
        const T u = s + param;
        return u * u;
    }
}

template <int KIND, typename T>
__device__ __forceinline__ T dp_kstep(T x, T y, T s)
{
    if constexpr (KIND == MBKK_GAUSS) {
        const T v = x - y;
        return fma(v, v, s);
    } else if constexpr (KIND == MBKK_LAPLACE) {
        return s + fabs(x - y);
    } else {
        return fma(x, y, s);
    }
}

// K(x, x) of an X row in FP64 (1 for the Gaussian and Laplacian kernels).
template <int KIND>
__device__ __forceinline__ double dp_kself(const float *__restrict__ x, int d, double param)
{
    if constexpr (KIND == MBKK_GAUSS || KIND == MBKK_LAPLACE) {
        return 1.0;
    } else {
        double s = 0.0;
        for (int t = 0; t < d; ++t)
            s = fma((double)x[t], (double)x[t], s);
        if constexpr (KIND == MBKK_LINEAR)
            return s;
        else
            return (s + param) * (s + param);
    }
}

__device__ __forceinline__ bool dp_lex_less(double a, int ia, double b, int ib)
{
    return a < b || (a == b && ia < ib);
}

// ---------------------------------------------------------------------------
// Scoring from the table: 64 rows per workgroup (lane = row), wave w takes
// centers w, w + 16, ...  Rows [0, m) are X rows idx[r].
// ---------------------------------------------------------------------------
struct DpScoreArgs {
    const void *T;
    int64_t ldT;
    int k, m, d;
    int64_t n, ld;
    const float *X;
    const int32_t *idx;
    const double *N;
    double param;
    int32_t *labels;
    float *mind, *margin;
    void *tsel;       // [m] old T[label][x] in the table type (may be NULL)
    int32_t *counts;  // [k] incremented per label (may be NULL)
    double *Dout;     // [m x ldD] every distance (may be NULL)
    int64_t ldD;
    int32_t *flags;   // flags[0] raised for an index outside [0, n) (may be NULL)
};

template <int KIND, typename TT>
__global__ __launch_bounds__(64 * kDpScoreWaves) void k_dp_score(DpScoreArgs A)
{
    __shared__ double sb[kDpScoreWaves][64], ss[kDpScoreWaves][64];
    __shared__ int sl[kDpScoreWaves][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int r = blockIdx.x * 64 + lane;
    const bool act = r < A.m;
    // an index outside [0, n) is never dereferenced: its row is scored as row 0
    const int32_t xi = act ? A.idx[r] : 0;
    const bool inr = xi >= 0 && (int64_t)xi < A.n;
    const int64_t x = inr ? (int64_t)xi : 0;
    if (act && !inr && A.flags && w == 0)
        atomicOr(&A.flags[0], 1);
    const TT *__restrict__ T = (const TT *)A.T;
    double kxx = 0.0;
    if constexpr (KIND == MBKK_LINEAR || KIND == MBKK_POLY2)
        kxx = dp_kself<KIND>(A.X + x * A.ld, A.d, A.param);
    else
        kxx = 1.0;
    double best = INFINITY, second = INFINITY;
    int lab = -1;
    constexpr int NB = 8;  // table loads in flight per lane
    for (int j0 = w; j0 < A.k; j0 += kDpScoreWaves * NB) {
        double t[NB], nj[NB];
#pragma unroll
        for (int u = 0; u < NB; ++u) {
            const int j = j0 + u * kDpScoreWaves;
            t[u] = j < A.k ? (double)T[(int64_t)j * A.ldT + x] : 0.0;
            nj[u] = j < A.k ? A.N[j] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < NB; ++u) {
            const int j = j0 + u * kDpScoreWaves;
            if (j < A.k) {
                const double D = kxx - 2.0 * t[u] + nj[u];
                if (A.Dout && act)
                    A.Dout[(int64_t)r * A.ldD + j] = D;
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
    sb[w][lane] = best;
    ss[w][lane] = second;
    sl[w][lane] = lab;
    __syncthreads();
    if (w == 0) {
        double b0 = sb[0][lane], s0 = ss[0][lane];
        int l0 = sl[0][lane];
        for (int q = 1; q < kDpScoreWaves; ++q) {
            const double bq = sb[q][lane], sq = ss[q][lane];
            const int lq = sl[q][lane];
            if (lq >= 0 && (l0 < 0 || dp_lex_less(bq, lq, b0, l0))) {
                s0 = fmin(b0, sq);
                b0 = bq;
                l0 = lq;
            } else {
                s0 = fmin(s0, bq);
            }
        }
        if (!(l0 >= 0 && l0 < A.k))
            l0 = 0;  // every distance NaN: keep the label in range
        if (act) {
            A.labels[r] = l0;
            A.mind[r] = (float)b0;
            A.margin[r] = (float)(s0 - b0);
            if (A.tsel)
                ((TT *)A.tsel)[r] = T[(int64_t)l0 * A.ldT + x];
            if (A.counts)
                atomicAdd(&A.counts[l0], 1);
        }
    }
}

// ---------------------------------------------------------------------------
// Plan (one workgroup of 1024): seg[j] = exclusive prefix of the counts,
// alpha[j] by the learning-rate rule (beta: sqrt(b_j / b); full: 1 if b_j > 0;
// sklearn: b_j / sum of b_j over the iterations so far, cum updated).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void k_dp_plan(int k, int b, int lr, const int32_t *__restrict__ counts,
                                                  double *__restrict__ cum, double *__restrict__ alpha,
                                                  int32_t *__restrict__ seg, int32_t *__restrict__ toff)
{
    __shared__ int lds[16];
    int carry = 0, tcarry = 0;
    for (int j0 = 0; j0 < k; j0 += 1024) {
        const int j = j0 + threadIdx.x;
        const int c = j < k ? counts[j] : 0;
        const int nt = (c + kDpTile - 1) / kDpTile;
        int tot, ttot;
        const int ex = block_exclusive_scan(c, lds, &tot);
        const int tex = block_exclusive_scan(nt * nt, lds, &ttot);
        if (j < k) {
            seg[j] = carry + ex;
            toff[j] = tcarry + tex;
            double a;
            if (lr == MBKK_LR_FULL) {
                a = c > 0 ? 1.0 : 0.0;
            } else if (lr == MBKK_LR_SKLEARN) {
                const double s = cum[j] + (double)c;
                cum[j] = s;
                a = c > 0 ? (double)c / s : 0.0;
            } else {
                a = sqrt((double)c / (double)b);
            }
            alpha[j] = a;
        }
        carry += tot;
        tcarry += ttot;
    }
    if (threadIdx.x == 0) {
        seg[k] = carry;
        toff[k] = tcarry;
    }
}

// ---------------------------------------------------------------------------
// Stable grouping: grouped position of batch row r = seg[label] + number of
// rows before r with the same label.  Writes the pool row of every grouped
// entry (batch row r lives in pool row row0 + r), its center and its old
// table value.
// ---------------------------------------------------------------------------
template <typename TT>
__global__ __launch_bounds__(256) void k_dp_group(int b, const int32_t *__restrict__ labels,
                                                  const int32_t *__restrict__ seg, const TT *__restrict__ tsel,
                                                  int64_t row0, int32_t *__restrict__ sup_row,
                                                  int32_t *__restrict__ gctr, TT *__restrict__ gsel)
{
    __shared__ int lab[kMaxBatch];
    for (int q = threadIdx.x; q < b; q += 256)
        lab[q] = labels[q];
    __syncthreads();
    const int r = blockIdx.x * 256 + threadIdx.x;
    if (r >= b)
        return;
    const int l = lab[r];
    int before = 0;
    for (int q = 0; q < r; ++q)
        before += lab[q] == l;
    const int pos = seg[l] + before;
    sup_row[pos] = (int32_t)(row0 + r);
    gctr[pos] = l;
    gsel[pos] = tsel[r];
}

// ---------------------------------------------------------------------------
// Pair sums of the grouped batch.  Center j's pairs are cut into tiles of 64
// rows by 64 columns (nt_j^2 tasks, nt_j = ceil(b_j / 64), offsets toff from
// the plan); a wave takes one task at a time: lane = row (coordinates in
// registers), the columns broadcast one by one as in the table update.  The
// tile's row sums (kernel values in the table type, summed over at most 64
// columns) go to pp[column tile][row] in FP64.
// ---------------------------------------------------------------------------
template <int KIND, typename TT, int DR>
__global__ __launch_bounds__(256) void k_dp_gram(int k, int bmax, int dp, const float *__restrict__ pool32,
                                                 const int32_t *__restrict__ sup_row,
                                                 const int32_t *__restrict__ seg, const int32_t *__restrict__ toff,
                                                 double param, double *__restrict__ pp)
{
    const int lane = threadIdx.x & 63;
    const int nw = gridDim.x * 4;
    const int T = toff[k];
    const TT cneg = (TT)(-1.4426950408889634 / param), prm = (TT)param;
    for (int task = blockIdx.x * 4 + (threadIdx.x >> 6); task < T; task += nw) {  // wave uniform
        const int j = wave_segment_of(toff, k, task);
        const int s0 = seg[j], bj = seg[j + 1] - s0;
        const int nt = (bj + kDpTile - 1) / kDpTile;
        const int local = task - toff[j];
        const int rt = local / nt, ct = local - rt * nt;
        const int e = s0 + rt * kDpTile + lane;
        const bool act = e < s0 + bj;
        const float *__restrict__ xr = pool32 + (int64_t)sup_row[act ? e : s0] * dp;
        TT x[DR];
#pragma unroll
        for (int t = 0; t < DR; ++t)
            x[t] = (TT)xr[t];
        const int c0 = s0 + ct * kDpTile;
        const int cn = min(kDpTile, s0 + bj - c0);
        const int lrow = sup_row[c0 + (lane < cn ? lane : 0)];
        TT acc = 0;
        for (int q = 0; q < cn; ++q) {  // wave uniform
            const float *__restrict__ y = pool32 + (int64_t)__builtin_amdgcn_readlane(lrow, q) * dp;
            TT a = 0;
#pragma unroll
            for (int t = 0; t < DR; ++t)
                a = dp_kstep<KIND, TT>(x[t], (TT)y[t], a);
            acc += dp_kfinish<KIND, TT>(a, cneg, prm);
        }
        if (act)
            pp[(int64_t)ct * bmax + e] = (double)acc;
    }
}

// Row sums over the column tiles, in tile order.
__global__ __launch_bounds__(256) void k_dp_rowsum(int b, int bmax, const int32_t *__restrict__ gctr,
                                                   const int32_t *__restrict__ seg, const double *__restrict__ pp,
                                                   double *__restrict__ s_out)
{
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= b)
        return;
    const int j = gctr[e];
    const int nt = (seg[j + 1] - seg[j] + kDpTile - 1) / kDpTile;
    double s = 0.0;
    for (int ct = 0; ct < nt; ++ct)
        s += pp[(int64_t)ct * bmax + e];
    s_out[e] = s;
}

// ---------------------------------------------------------------------------
// N update and table weights, one wave per center: lane-strided sums over
// the center's grouped entries, then a fixed-order tree across the wave.
// ---------------------------------------------------------------------------
template <typename TT>
__global__ __launch_bounds__(256) void k_dp_norms(int k, const int32_t *__restrict__ seg,
                                                  const double *__restrict__ alpha, const TT *__restrict__ gsel,
                                                  const double *__restrict__ s_pair, double *__restrict__ N,
                                                  double *__restrict__ wgt, int32_t *__restrict__ counts)
{
    const int lane = threadIdx.x & 63;
    const int j = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (j >= k)
        return;  // wave uniform
    const int s0 = seg[j], s1 = seg[j + 1];
    const double a = alpha[j];
    if (lane == 0)
        counts[j] = 0;  // consumed by the plan: ready for the next scoring
    if (s1 == s0) {
        if (lane == 0)
            wgt[j] = 0.0;
        return;
    }
    double cc = 0.0, mm = 0.0;
    for (int e = s0 + lane; e < s1; e += 64) {
        cc += (double)gsel[e];
        mm += s_pair[e];
    }
    for (int o = 32; o > 0; o >>= 1) {
        cc += __shfl_xor(cc, o);
        mm += __shfl_xor(mm, o);
    }
    if (lane == 0) {
        const double bj = (double)(s1 - s0);
        cc /= bj;
        mm /= bj * bj;
        N[j] = (1.0 - a) * (1.0 - a) * N[j] + 2.0 * a * (1.0 - a) * cc + a * a * mm;
        wgt[j] = a / bj;
    }
}

// ---------------------------------------------------------------------------
// Table update over all of X on the VALU (every kernel; the Gaussian in FP64,
// with cross_impl DIRECT, or at d < 16).  Lane = RPL rows of X (256 apart), held in
// registers; every workgroup runs over all grouped entries, 64 at a time
// (lane e loads entry e's pool row, then the entries are broadcast one by
// one and their coordinates read with wave-uniform loads).  At the end of a
// center's segment the row's sum of kernel values is blended into the table:
//     T[j][x] <- (1 - alpha_j) T[j][x] + (alpha_j / b_j) * sum,
// or, when init is set, T[j][x] <- wgt_j * sum without reading T.
// ---------------------------------------------------------------------------
template <int KIND, typename TT, int DR, int RPL>
__global__ __launch_bounds__(kDpTableWG) void k_dp_table(int64_t n, int d, int64_t ld, const float *__restrict__ X,
                                                         int dp, const float *__restrict__ pool32, int k,
                                                         const int32_t *__restrict__ seg,
                                                         const int32_t *__restrict__ sup_row,
                                                         const double *__restrict__ alpha,
                                                         const double *__restrict__ wgt, double param, int init,
                                                         TT *__restrict__ T, int64_t ldT)
{
    const int lane = threadIdx.x & 63;
    int64_t row[RPL], rr[RPL];
#pragma unroll
    for (int q = 0; q < RPL; ++q) {
        row[q] = (int64_t)blockIdx.x * kDpTableWG * RPL + q * kDpTableWG + threadIdx.x;
        rr[q] = row[q] < n ? row[q] : 0;
    }
    const TT prm = (TT)param;
    const TT cneg = (TT)(-1.4426950408889634 / param);
    TT x[RPL][DR];
#pragma unroll
    for (int q = 0; q < RPL; ++q)
#pragma unroll
        for (int t = 0; t < DR; ++t)
            x[q][t] = t < d ? (TT)X[rr[q] * ld + t] : (TT)0;
    const int M = seg[k];
    if (M == 0)
        return;
    // The current center j: the end of its segment, its weight and rate are
    // loaded when j becomes current (the rows' old table values are read at
    // the blend: holding them would cost the registers of a wave per SIMD).
    int j = wave_segment_of(seg, k, 0);
    int cur_end;
    TT wj, keep;
    auto begin = [&]() {
        cur_end = seg[j + 1];
        wj = (TT)wgt[j];
        keep = (TT)(1.0 - alpha[j]);
    };
    begin();
    TT acc[RPL];
#pragma unroll
    for (int q = 0; q < RPL; ++q)
        acc[q] = 0;
    auto flush = [&]() {
        TT *__restrict__ Tj = T + (int64_t)j * ldT;
#pragma unroll
        for (int q = 0; q < RPL; ++q) {
            if (row[q] < n) {
                const TT old = init ? (TT)0 : Tj[row[q]];
                Tj[row[q]] = init ? wj * acc[q] : fma(wj, acc[q], keep * old);
            }
            acc[q] = 0;
        }
    };
    for (int c0 = 0; c0 < M; c0 += 64) {
        const int cnt = min(64, M - c0);
        const int lrow = sup_row[c0 + (lane < cnt ? lane : 0)];
        for (int e = 0; e < cnt; ++e) {  // wave uniform
            const int s = c0 + e;
            if (s >= cur_end) {
                flush();
                do {
                    ++j;
                } while (seg[j + 1] <= s);
                begin();
            }
            const float *__restrict__ y = pool32 + (int64_t)__builtin_amdgcn_readlane(lrow, e) * dp;
            TT sacc[RPL];
#pragma unroll
            for (int q = 0; q < RPL; ++q)
                sacc[q] = 0;
#pragma unroll
            for (int t = 0; t < DR; ++t) {
                const TT yt = (TT)y[t];
#pragma unroll
                for (int q = 0; q < RPL; ++q)
                    sacc[q] = dp_kstep<KIND, TT>(x[q][t], yt, sacc[q]);
            }
#pragma unroll
            for (int q = 0; q < RPL; ++q)
                acc[q] += dp_kfinish<KIND, TT>(sacc[q], cneg, prm);
        }
    }
    flush();
}

// ---------------------------------------------------------------------------
// Table update of the Gaussian on MFMA.  FP32 form: v_mfma_f32_32x32x2f32;
// BF16X3 form: v_mfma_f32_32x32x16_bf16 on the compensated split
// x = hi + lo (hi = bf16(x), lo = bf16(x - hi)), x.y ~ hi.hi + hi.lo + lo.hi,
// the batch entries' hi / lo from the pool and the points' split in registers.
// The product form S = x.y - |x|^2 / 2 is a dense contraction over the
// coordinates: A = 32 grouped batch entries (rows m), B = 32 points of X
// (columns n), K(x, y) = exp2(c2 S + ay) with c2 = 2 log2(e) / kappa and
// ay = -log2(e) |y|^2 / kappa.  Lane l = 32 h + n holds point n's column of a
// 32 x 32 tile: output rows 8 (i / 4) + 4 h + i % 4, i = 0..15, which the
// staging fills with the tile's entries 16 h + i (so a lane's 16 values are
// consecutive entries, and a segment is a range of them per lane half).  Lane half
// h contracts the coordinates h DP/2 .. (h + 1) DP/2 - 1 (k-step s: the next
// one (FP32) or eight (BF16) of them), so each lane reads consecutive
// coordinates of its rows.
//
// A wave holds two 32-point blocks of X in registers (64 points, 256 per
// workgroup) and runs over all grouped entries, staged 64 at a time through
// LDS (double-buffered; rows padded by 16 bytes so that the 16-byte reads of
// 16 lanes fall in distinct banks).  After each 32-entry tile the lane sums
// its kernel values per center segment (masks on i); at the end of a segment
// the two lane halves are combined (permlane32 swap) and
//     S[j][x] = (alpha_j / b_j) sum_{y in B^j} K(x, y)
// is stored; k_dp_blend then forms T <- (1 - alpha) T + S for the touched
// centers.  Entries past the support are zero rows outside every segment.
// ---------------------------------------------------------------------------
constexpr int kDpMfmaStage = 64;  // grouped entries per LDS stage

// NBX blocks of 32 points per wave: two (four waves per workgroup) up to
// DP = 64, one (eight waves) from DP = 96, so that two waves share each SIMD
// and one wave's epilogue runs beside the other's matrix work.
template <int DP, bool X3, int NBX>
__global__ __launch_bounds__(NBX == 2 ? 256 : 512, 2) void k_dp_mfma(int64_t n, int d, int64_t ld, const float *__restrict__ X,
                                                    const float *__restrict__ pool32,
                                                    const uint16_t *__restrict__ poolhi,
                                                    const uint16_t *__restrict__ poollo,
                                                    const float *__restrict__ poolsq, int k,
                                                    const int32_t *__restrict__ seg,
                                                    const int32_t *__restrict__ sup_row,
                                                    const double *__restrict__ wgt, float c2,
                                                    float *__restrict__ S, int64_t ldT)
{
    constexpr int HD = DP / 2;              // coordinates per lane half
    constexpr int KS = X3 ? DP / 16 : HD;   // MFMA k-steps
    constexpr int ES = X3 ? 2 : 4;          // element bytes in LDS
    constexpr int RS = DP + 16 / ES;        // LDS row stride (elements): 16 bytes of padding
    constexpr int NE = kDpMfmaStage;
    constexpr int NTH = 64 * 8 / NBX;       // threads of a workgroup (256 points)
    constexpr int TPE = NTH / kDpMfmaStage; // staging threads per entry
    constexpr int UPT = NE * DP * ES / NTH / 16;  // 16-byte pieces per array staged per thread and stage
    constexpr int NARR = X3 ? 2 : 1;
    static_assert(UPT >= 1 && (X3 || KS % 4 == 0), "staging in 16-byte pieces");
    typedef typename std::conditional<X3, uint16_t, float>::type elem_t;
    __shared__ __attribute__((aligned(16))) elem_t sY[2][NARR][NE * RS];
    __shared__ __attribute__((aligned(16))) float sAy[2][NE];
    const int tid = threadIdx.x, lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int nn = lane & 31, h = lane >> 5;
    const int M = seg[k];
    if (M == 0)
        return;
    const float ayc = -0.5f * c2;  // ay = ayc |y|^2
    // ---- the wave's blocks of X in registers ---------------------------------
    const int64_t x0 = (int64_t)blockIdx.x * 256 + w * (32 * NBX);
    typedef typename std::conditional<X3, bf16x8, float>::type bfrag_t;
    bfrag_t bxh[NBX][KS], bxl[NBX][X3 ? KS : 1];
    float hx[NBX];
#pragma unroll
    for (int q = 0; q < NBX; ++q) {
        const int64_t row = x0 + q * 32 + nn;
        const float *xr = X + (row < n ? row : 0) * ld;
        float ss = 0.0f;
        if constexpr (X3) {
#pragma unroll
            for (int s = 0; s < KS; ++s) {
                u16x8 vh, vl;
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int t = h * HD + 8 * s + u;
                    const float v = t < d ? xr[t] : 0.0f;
                    ss = fmaf(v, v, ss);
                    const uint16_t hb = f32_to_bf16_rne(v);
                    vh[u] = hb;
                    vl[u] = f32_to_bf16_rne(v - bf16_to_f32(hb));
                }
                bxh[q][s] = __builtin_bit_cast(bf16x8, vh);
                bxl[q][s] = __builtin_bit_cast(bf16x8, vl);
            }
        } else {
#pragma unroll
            for (int s = 0; s < KS; ++s) {
                const int t = h * HD + s;
                bxh[q][s] = t < d ? xr[t] : 0.0f;
                ss = fmaf(bxh[q][s], bxh[q][s], ss);
            }
        }
        ss += __shfl_xor(ss, 32);
        hx[q] = -0.5f * ss;
    }
    // ---- staging of grouped entries [e0, e0 + 64) into buffer bb ------------
    // thread t stages entry t / TPE, 16-byte pieces (t % TPE) * UPT .. + UPT of its
    // row in every array (FP32 row, or the BF16 hi and lo rows)
    const int se = tid / TPE, sq = tid % TPE;
    f32x4 pre[NARR][UPT];
    float pay = 0.0f;
    auto fetch = [&](int e0) {
        const int e = e0 + se;
        const int row = e < M ? sup_row[e] : -1;
        const int64_t r0 = (int64_t)(row < 0 ? 0 : row) * DP;
#pragma unroll
        for (int a = 0; a < NARR; ++a) {
            const char *src = X3 ? (const char *)((a == 0 ? poolhi : poollo) + r0)
                                 : (const char *)(pool32 + r0);
#pragma unroll
            for (int u = 0; u < UPT; ++u)
                pre[a][u] = row < 0 ? f32x4{0.f, 0.f, 0.f, 0.f} : *(const f32x4 *)(src + (sq * UPT + u) * 16);
        }
        pay = row < 0 ? 0.0f : ayc * poolsq[row];
    };
    // Entry e of a 32-entry tile goes to LDS row 8 ((e % 16) / 4) + 4 (e / 16)
    // + e % 4: the MFMA output row of element i of lane half h is then entry
    // 16 h + i, so each lane holds 16 consecutive entries of the tile.
    const int srow = (se & ~31) + 8 * ((se & 15) >> 2) + 4 * ((se >> 4) & 1) + (se & 3);
    auto commit = [&](int bb) {
#pragma unroll
        for (int a = 0; a < NARR; ++a) {
            char *dst = (char *)&sY[bb][a][srow * RS];
#pragma unroll
            for (int u = 0; u < UPT; ++u)
                *(f32x4 *)(dst + (sq * UPT + u) * 16) = pre[a][u];
        }
        if (sq == 0)
            sAy[bb][srow] = pay;
    };
    // ---- segment bookkeeping (wave uniform) ---------------------------------
    // The current center j, the end of its segment and its weight are held in
    // registers, loaded when j becomes current (a segment usually spans
    // tiles), so that the epilogue does not wait on memory.
    int j = wave_segment_of(seg, k, 0);
    int cur_end = seg[j + 1];
    float cur_w = (float)wgt[j];
    float run[NBX];
#pragma unroll
    for (int q = 0; q < NBX; ++q)
        run[q] = 0.0f;
    auto store = [&]() {
        if constexpr (NBX == 2) {
            const auto sw = __builtin_amdgcn_permlane32_swap(__float_as_uint(run[0]), __float_as_uint(run[1]),
                                                             false, false);
            const float tot = __uint_as_float(sw[0]) + __uint_as_float(sw[1]);
            const int64_t col = x0 + h * 32 + nn;  // lanes < 32: block 0, lanes >= 32: block 1
            if (col < n)
                S[(int64_t)j * ldT + col] = cur_w * tot;
        } else {
            const float tot = run[0] + __shfl_xor(run[0], 32);
            const int64_t col = x0 + nn;
            if (h == 0 && col < n)
                S[(int64_t)j * ldT + col] = cur_w * tot;
        }
#pragma unroll
        for (int q = 0; q < NBX; ++q)
            run[q] = 0.0f;
    };
    // segment sums of a tile of kernel values (entries [t0, t0 + 32))
    auto segments = [&](const f32x16 (&kv)[NBX], int t0) {
        int lo = t0;
        const int top = min(t0 + 32, M);
        while (lo < top) {  // wave uniform
            const int end = cur_end;
            const int hi = min(end, top);
            const int mlo = lo - t0, mhi = hi - t0;
            if (mlo == 0 && mhi == 32) {  // the whole tile in one segment: no masks
#pragma unroll
                for (int q = 0; q < NBX; ++q) {
                    float sq_ = 0.0f;
#pragma unroll
                    for (int i = 0; i < 16; ++i)
                        sq_ += kv[q][i];
                    run[q] += sq_;
                }
            } else {
                // element i of lane half h is entry 16 h + i: the segment's
                // elements are [a_h, b_h) with wave-uniform bounds per half
                const int a0 = min(max(mlo, 0), 16), b0 = min(max(mhi, 0), 16);
                const int a1 = min(max(mlo - 16, 0), 16), b1 = min(max(mhi - 16, 0), 16);
#pragma unroll
                for (int i = 0; i < 16; ++i) {
                    const bool in = h == 0 ? (i >= a0 && i < b0) : (i >= a1 && i < b1);
#pragma unroll
                    for (int q = 0; q < NBX; ++q)
                        run[q] += in ? kv[q][i] : 0.0f;
                }
            }
            if (end <= top) {
                store();
                if (end < M) {
                    int e1;
                    do {
                        ++j;
                        e1 = seg[j + 1];
                    } while (e1 <= end);
                    cur_end = e1;
                    cur_w = (float)wgt[j];
                }
            }
            lo = hi;
        }
    };
    // Software pipeline over tiles: the MFMAs of tile t go into one
    // accumulator set while the exponentials of tile t - 1 (the other set,
    // exponent constants in eay) are spread between them (BF16X3; FP32 takes
    // them after the MFMAs); the segment sums of tile t - 1 follow.  Tiles alternate between the sets by the
    // parity of t (two tiles per stage).
    constexpr int NMF = (X3 ? 3 : 1) * NBX * KS;  // MFMAs per tile
    constexpr int NEL = 16 * NBX;                 // kernel values per lane and tile
    f32x16 accA[NBX], accB[NBX];
    float eay[16];
#pragma unroll
    for (int q = 0; q < NBX; ++q)
#pragma unroll
        for (int i = 0; i < 16; ++i)
            accB[q][i] = 0.0f;
#pragma unroll
    for (int i = 0; i < 16; ++i)
        eay[i] = 0.0f;
    int prev = -1;  // first entry of the tile whose epilogue is pending
    // the exponentials due after MFMA mi of a tile, fenced from the scheduler
    // so that they issue while the matrix core is busy (MFMAs without a share
    // carry no fence)
    auto exp_share = [&](f32x16 (&kv)[NBX], int mi) {
        const int e0 = mi * NEL / NMF, e1 = (mi + 1) * NEL / NMF;
        if (e1 > e0) {
#pragma unroll
            for (int e = e0; e < e1; ++e)
                kv[e % NBX][e / NBX] = __builtin_amdgcn_exp2f(fmaf(kv[e % NBX][e / NBX], c2, eay[e / NBX]));
            __builtin_amdgcn_sched_barrier(0);
        }
    };
    auto tile = [&](f32x16 (&accN)[NBX], f32x16 (&accP)[NBX], int bb, int t32) {
#pragma unroll
        for (int q = 0; q < NBX; ++q)
#pragma unroll
            for (int i = 0; i < 16; ++i)
                accN[q][i] = hx[q];
        if constexpr (X3) {
            const uint16_t *arh = &sY[bb][0][(t32 * 32 + nn) * RS + h * HD];
            const uint16_t *arl = &sY[bb][1][(t32 * 32 + nn) * RS + h * HD];
            bf16x8 ah = __builtin_bit_cast(bf16x8, *(const u16x8 *)arh);
            bf16x8 al = __builtin_bit_cast(bf16x8, *(const u16x8 *)arl);
#pragma unroll
            for (int s = 0; s < KS; ++s) {
                bf16x8 ahn = ah, aln = al;
                if (s + 1 < KS) {
                    ahn = __builtin_bit_cast(bf16x8, *(const u16x8 *)(arh + 8 * (s + 1)));
                    aln = __builtin_bit_cast(bf16x8, *(const u16x8 *)(arl + 8 * (s + 1)));
                }
                // products hi.hi, hi.lo, lo.hi; the two point blocks alternate, so
                // consecutive MFMAs never wait on each other's accumulator
#pragma unroll
                for (int pr = 0; pr < 3; ++pr)
#pragma unroll
                    for (int q = 0; q < NBX; ++q) {
                        const bf16x8 aa = pr == 2 ? al : ah;
                        const bf16x8 bv = pr == 1 ? bxl[q][s] : bxh[q][s];
                        accN[q] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(aa, bv, accN[q], 0, 0, 0);
                        exp_share(accP, (s * 3 + pr) * NBX + q);
                    }
                ah = ahn;
                al = aln;
            }
        } else {
            const float *arow = &sY[bb][0][(t32 * 32 + nn) * RS + h * HD];
            f32x4 av = *(const f32x4 *)arow, an;
#pragma unroll
            for (int s4 = 0; s4 < KS; s4 += 4) {
                if (s4 + 4 < KS)
                    an = *(const f32x4 *)(arow + s4 + 4);
#pragma unroll
                for (int u = 0; u < 4; ++u)
#pragma unroll
                    for (int q = 0; q < NBX; ++q) {
                        accN[q] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[u], bxh[q][s4 + u], accN[q], 0, 0, 0);
                    }
                av = an;
            }
        }
        if constexpr (!X3) {
            // FP32: a tile's MFMAs take 4x longer than in BF16; its
            // exponentials run in one piece (fences would only constrain the
            // scheduling of the fragment reads)
#pragma unroll
            for (int mi = 0; mi < NMF; ++mi)
                exp_share(accP, mi);
        }
        if (prev >= 0)
            segments(accP, prev);
        // the new tile's exponent constants, for its epilogue during the next tile
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            const f32x4 a4 = *(const f32x4 *)&sAy[bb][t32 * 32 + 8 * g + 4 * h];
#pragma unroll
            for (int r = 0; r < 4; ++r)
                eay[4 * g + r] = a4[r];
        }
    };
    const int nst = (M + NE - 1) / NE;
    fetch(0);
    commit(0);
    __syncthreads();
    static_assert(NE == 64, "two tiles per stage: the tile parity selects the accumulator set");
    for (int st = 0; st < nst; ++st) {
        const int bb = st & 1;
        if (st + 1 < nst)
            fetch((st + 1) * NE);
        tile(accA, accB, bb, 0);
        prev = st * NE;
        if (st * NE + 32 < M) {  // wave uniform
            tile(accB, accA, bb, 1);
            prev = st * NE + 32;
        }
        if (st + 1 < nst)
            commit(bb ^ 1);
        __syncthreads();
    }
    // epilogue of the last tile
    if ((prev - (nst - 1) * NE) == 0) {
#pragma unroll
        for (int mi = 0; mi < NMF; ++mi)
            exp_share(accA, mi);
        segments(accA, prev);
    } else {
#pragma unroll
        for (int mi = 0; mi < NMF; ++mi)
            exp_share(accB, mi);
        segments(accB, prev);
    }
}

// T[j][x] <- (1 - alpha_j) T[j][x] + S[j][x] for the centers with batch points
// (init: T <- S).  A thread owns 4 consecutive points and runs over the
// centers, skipping (wave uniform) those the batch did not touch.
__global__ __launch_bounds__(256) void k_dp_blend(int64_t n, int k, const int32_t *__restrict__ seg,
                                                  const double *__restrict__ alpha, const float *__restrict__ S,
                                                  float *__restrict__ T, int64_t ldT, int init)
{
    const int64_t x = ((int64_t)blockIdx.x * 256 + threadIdx.x) * 4;
    if (x >= n)
        return;
    for (int j = 0; j < k; ++j) {
        if (seg[j + 1] == seg[j])
            continue;
        const f32x4 sv = *(const f32x4 *)(S + (int64_t)j * ldT + x);
        f32x4 *tp = (f32x4 *)(T + (int64_t)j * ldT + x);  // ldT is a multiple of 64: whole vectors
        if (init) {
            *tp = sv;
        } else {
            const float keep = (float)(1.0 - alpha[j]);
            const f32x4 tv = *tp;
            f32x4 r;
#pragma unroll
            for (int u = 0; u < 4; ++u)
                r[u] = fmaf(keep, tv[u], sv[u]);
            *tp = r;
        }
    }
}

static void launch_dp_mfma(const Layout &L, const Buffers &B, const int32_t *seg, const int32_t *sup_row,
                           double kappa, int init, hipStream_t st)
{
    const float c2 = (float)(2.0 * 1.4426950408889634 / kappa);
    const dim3 grid((unsigned)((L.n + 255) / 256));
#define MBKK_DP_MFMA(DPV, X3, NBX)                                                                                \
    hipLaunchKernelGGL((k_dp_mfma<DPV, X3, NBX>), grid, dim3(NBX == 2 ? 256 : 512), 0, st, L.n, L.d, B.ld, B.X,    \
                       B.pool32, B.poolhi, B.poollo, B.poolsq, L.k, seg, sup_row, B.dp_w, c2, B.dp_S, L.ldT)
#define MBKK_DP_MFMA_W(X3)                     \
    switch (L.dp) {                             \
    case 32: MBKK_DP_MFMA(32, X3, 2); break;    \
    case 64: MBKK_DP_MFMA(64, X3, 2); break;    \
    case 96: MBKK_DP_MFMA(96, X3, 1); break;    \
    default: MBKK_DP_MFMA(128, X3, 1); break;   \
    }
    if (L.bf16) {
        MBKK_DP_MFMA_W(true)
    } else {
        MBKK_DP_MFMA_W(false)
    }
#undef MBKK_DP_MFMA_W
#undef MBKK_DP_MFMA
    hipLaunchKernelGGL(k_dp_blend, dim3((unsigned)((L.n + 1023) / 1024)), dim3(256), 0, st, L.n, L.k, seg, B.alpha,
                       B.dp_S, (float *)B.dp_T, L.ldT, init);
}

// Rows per lane of the table update: two for FP32 rows of at most 32
// coordinates.  The register width DR of a row never exceeds the pool's
// padded stride dp (d rounded up to 32), so reading DR coordinates of a pool
// row stays inside it, and its entries past d are zero.
static int dp_rpl(int d, bool fp64) { return !fp64 && d <= 32 ? 2 : 1; }

int dp_max_dim() { return 128; }

template <int KIND, typename TT>
static void dispatch_dp_table(const Layout &L, const Buffers &B, const int32_t *seg, const int32_t *sup_row,
                              double param, int init, hipStream_t st)
{
    const int rpl = dp_rpl(L.d, sizeof(TT) == 8);
    const dim3 grid((unsigned)((L.n + (int64_t)kDpTableWG * rpl - 1) / ((int64_t)kDpTableWG * rpl)));
    TT *T = (TT *)B.dp_T;
#define MBKK_DP_TABLE(DR, RPL)                                                                                   \
    hipLaunchKernelGGL((k_dp_table<KIND, TT, DR, RPL>), grid, dim3(kDpTableWG), 0, st, L.n, L.d, B.ld, B.X, L.dp, \
                       B.pool32, L.k, seg, sup_row, B.alpha, B.dp_w, param, init, T, L.ldT)
    constexpr int R2 = sizeof(TT) == 4 ? 2 : 1;
    if (L.d <= 4)
        MBKK_DP_TABLE(4, R2);
    else if (L.d <= 8)
        MBKK_DP_TABLE(8, R2);
    else if (L.d <= 16)
        MBKK_DP_TABLE(16, R2);
    else if (L.d <= 32)
        MBKK_DP_TABLE(32, R2);
    else if (L.d <= 64)
        MBKK_DP_TABLE(64, 1);
    else if (L.d <= 96)
        MBKK_DP_TABLE(96, 1);
    else
        MBKK_DP_TABLE(128, 1);
#undef MBKK_DP_TABLE
}

template <typename TT>
static void dp_table_kind(const Layout &L, const Buffers &B, int kind, const int32_t *seg, const int32_t *sup_row,
                          double param, int init, hipStream_t st)
{
    switch (kind) {
    case MBKK_GAUSS: dispatch_dp_table<MBKK_GAUSS, TT>(L, B, seg, sup_row, param, init, st); break;
    case MBKK_LAPLACE: dispatch_dp_table<MBKK_LAPLACE, TT>(L, B, seg, sup_row, param, init, st); break;
    case MBKK_LINEAR: dispatch_dp_table<MBKK_LINEAR, TT>(L, B, seg, sup_row, param, init, st); break;
    default: dispatch_dp_table<MBKK_POLY2, TT>(L, B, seg, sup_row, param, init, st); break;
    }
}

void launch_dp_table(const Layout &L, const Buffers &B, int kind, double param, int fp64, int init,
                     hipStream_t st)
{
    // init: one entry per center, the initial points (pool rows 0..k-1)
    const int32_t *seg = init ? B.dp_iseg : B.seg_off;
    const int32_t *sup = init ? B.dp_irow : B.sup_row;
    if (L.dp_mfma) {
        launch_dp_mfma(L, B, seg, sup, param, init, st);
        return;
    }
    if (fp64)
        dp_table_kind<double>(L, B, kind, seg, sup, param, init, st);
    else
        dp_table_kind<float>(L, B, kind, seg, sup, param, init, st);
}

template <int KIND, typename TT>
static void dp_score_kind(DpScoreArgs &A, hipStream_t st)
{
    const dim3 grid((unsigned)((A.m + 63) / 64));
    hipLaunchKernelGGL((k_dp_score<KIND, TT>), grid, dim3(64 * kDpScoreWaves), 0, st, A);
}

void launch_dp_score(const Layout &L, const Buffers &B, int kind, double param, int fp64, const int32_t *idx, int m,
                     bool step, double *D_out, int64_t ldD, int32_t *flags, hipStream_t st)
{
    DpScoreArgs A;
    A.T = B.dp_T;
    A.ldT = L.ldT;
    A.k = L.k;
    A.m = m;
    A.n = L.n;
    A.d = L.d;
    A.ld = B.ld;
    A.X = B.X;
    A.idx = idx;
    A.N = B.N;
    A.param = param;
    A.labels = B.labels;
    A.mind = B.mind;
    A.margin = B.margin;
    A.tsel = step ? B.dp_tsel : nullptr;
    A.counts = step ? B.counts : nullptr;
    A.Dout = D_out;
    A.ldD = ldD;
    A.flags = flags;
#define MBKK_DP_SCORE(TT)                                                             \
    switch (kind) {                                                                   \
    case MBKK_GAUSS: dp_score_kind<MBKK_GAUSS, TT>(A, st); break;                     \
    case MBKK_LAPLACE: dp_score_kind<MBKK_LAPLACE, TT>(A, st); break;                 \
    case MBKK_LINEAR: dp_score_kind<MBKK_LINEAR, TT>(A, st); break;                   \
    default: dp_score_kind<MBKK_POLY2, TT>(A, st); break;                             \
    }
    if (fp64) {
        MBKK_DP_SCORE(double)
    } else {
        MBKK_DP_SCORE(float)
    }
#undef MBKK_DP_SCORE
}

template <int KIND, typename TT>
static void dp_gram_kind(const Layout &L, const Buffers &B, double param, hipStream_t st)
{
#define MBKK_DP_GRAM(DR)                                                                                          \
    hipLaunchKernelGGL((k_dp_gram<KIND, TT, DR>), dim3(kDpGramWGs), dim3(256), 0, st, L.k, L.bmax, L.dp, B.pool32, \
                       B.sup_row, B.seg_off, B.dp_toff, param, B.dp_pp)
    if (L.d <= 4)
        MBKK_DP_GRAM(4);
    else if (L.d <= 8)
        MBKK_DP_GRAM(8);
    else if (L.d <= 16)
        MBKK_DP_GRAM(16);
    else if (L.d <= 32)
        MBKK_DP_GRAM(32);
    else if (L.d <= 64)
        MBKK_DP_GRAM(64);
    else if (L.d <= 96)
        MBKK_DP_GRAM(96);
    else
        MBKK_DP_GRAM(128);
#undef MBKK_DP_GRAM
}

template <typename TT>
static void dp_update_t(const Layout &L, const Buffers &B, int b, int kind, double param, int lr, hipStream_t st)
{
    hipLaunchKernelGGL(k_dp_plan, dim3(1), dim3(1024), 0, st, L.k, b, lr, B.counts, B.cum, B.alpha, B.seg_off,
                       B.dp_toff);
    const dim3 gb((unsigned)((b + 255) / 256));
    const int64_t row0 = slot_row(L, 0, 0);
    hipLaunchKernelGGL(k_dp_group<TT>, gb, dim3(256), 0, st, b, B.labels, B.seg_off, (const TT *)B.dp_tsel, row0,
                       B.sup_row, B.dp_gctr, (TT *)B.dp_gsel);
    switch (kind) {
    case MBKK_GAUSS: dp_gram_kind<MBKK_GAUSS, TT>(L, B, param, st); break;
    case MBKK_LAPLACE: dp_gram_kind<MBKK_LAPLACE, TT>(L, B, param, st); break;
    case MBKK_LINEAR: dp_gram_kind<MBKK_LINEAR, TT>(L, B, param, st); break;
    default: dp_gram_kind<MBKK_POLY2, TT>(L, B, param, st); break;
    }
    hipLaunchKernelGGL(k_dp_rowsum, gb, dim3(256), 0, st, b, L.bmax, B.dp_gctr, B.seg_off, B.dp_pp, B.dp_pair);
    hipLaunchKernelGGL(k_dp_norms<TT>, dim3((unsigned)((L.k + 3) / 4)), dim3(256), 0, st, L.k, B.seg_off, B.alpha,
                       (const TT *)B.dp_gsel, B.dp_pair, B.N, B.dp_w, B.counts);
}

void launch_dp_update(const Layout &L, const Buffers &B, int b, int kind, double param, int fp64, int lr,
                      hipStream_t st)
{
    if (fp64)
        dp_update_t<double>(L, B, b, kind, param, lr, st);
    else
        dp_update_t<float>(L, B, b, kind, param, lr, st);
}

// Initial state: N[j] = K(c_j, c_j) from the pool rows of the initial points,
// table weights 1 and alpha 1 (the init launch of the table kernel writes
// K(x, c_j) without reading the table), the one-entry segments of the
// initial centers.
template <int KIND>
__global__ __launch_bounds__(256) void k_dp_init(int k, int d, int dp, const float *__restrict__ pool32,
                                                 double param, double *__restrict__ N,
                                                 double *__restrict__ wgt, double *__restrict__ alpha,
                                                 double *__restrict__ cum, int32_t *__restrict__ iseg,
                                                 int32_t *__restrict__ irow, int32_t *__restrict__ counts)
{
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j > k)
        return;
    iseg[j] = j;
    if (j == k)
        return;
    irow[j] = j;
    counts[j] = 0;
    wgt[j] = 1.0;
    alpha[j] = 1.0;
    cum[j] = 0.0;
    const float *__restrict__ y = pool32 + (int64_t)j * dp;
    double s = 0.0;
    for (int t = 0; t < d; ++t)
        s = dp_kstep<KIND, double>((double)y[t], (double)y[t], s);
    const double v = dp_kfinish<KIND, double>(s, -1.4426950408889634 / param, param);
    N[j] = v;
}

void launch_dp_init(const Layout &L, const Buffers &B, int kind, double param, int fp64, hipStream_t st)
{
    const dim3 g((unsigned)((L.k + 1 + 255) / 256));
    switch (kind) {
    case MBKK_GAUSS:
        hipLaunchKernelGGL(k_dp_init<MBKK_GAUSS>, g, dim3(256), 0, st, L.k, L.d, L.dp, B.pool32, param, B.N,
                           B.dp_w, B.alpha, B.cum, B.dp_iseg, B.dp_irow, B.counts);
        break;
    case MBKK_LAPLACE:
        hipLaunchKernelGGL(k_dp_init<MBKK_LAPLACE>, g, dim3(256), 0, st, L.k, L.d, L.dp, B.pool32, param,
                           B.N, B.dp_w, B.alpha, B.cum, B.dp_iseg, B.dp_irow, B.counts);
        break;
    case MBKK_LINEAR:
        hipLaunchKernelGGL(k_dp_init<MBKK_LINEAR>, g, dim3(256), 0, st, L.k, L.d, L.dp, B.pool32, param,
                           B.N, B.dp_w, B.alpha, B.cum, B.dp_iseg, B.dp_irow, B.counts);
        break;
    default:
        hipLaunchKernelGGL(k_dp_init<MBKK_POLY2>, g, dim3(256), 0, st, L.k, L.d, L.dp, B.pool32, param, B.N,
                           B.dp_w, B.alpha, B.cum, B.dp_iseg, B.dp_irow, B.counts);
        break;
    }
    launch_dp_table(L, B, kind, param, fp64, 1, st);
}

}  // namespace mbkk
