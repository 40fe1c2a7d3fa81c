// Device helpers shared by the kernel translation units (internal).
#pragma once

#include "mbkk_internal.h"

namespace mbkk {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef uint16_t u16x8 __attribute__((ext_vector_type(8)));

// Lane i of the result takes x from lane i - n of its row of 16 lanes, 0
// where there is none (DPP row_shr; CTRL = 0x110 + n), or, for the row
// broadcasts (CTRL 0x142: lane 15 of each row, 0x143: lane 31), the
// broadcast value in the rows of ROWS and 0 in the others.
template <int CTRL, int ROWS = 0xf>
__device__ __forceinline__ int dpp_or_zero(int x)
{
    return __builtin_amdgcn_update_dpp(0, x, CTRL, ROWS, 0xf, false);
}

// Inclusive prefix sum over the 64 lanes of a wave (every lane active), on
// the DPP paths of the register file: shifts by 1, 2, 4 and 8 inside each row
// of 16 lanes, then row 0's total into row 1 and row 2's into row 3, then
// the first two rows' total into rows 2 and 3.  No LDS round trips.
__device__ __forceinline__ int wave_inclusive_sum(int x)
{
    x += dpp_or_zero<0x111>(x);
    x += dpp_or_zero<0x112>(x);
    x += dpp_or_zero<0x114>(x);
    x += dpp_or_zero<0x118>(x);
    x += dpp_or_zero<0x142, 0xa>(x);
    x += dpp_or_zero<0x143, 0xc>(x);
    return x;
}

// Maximum over the 64 lanes of a wave (every lane active), the same in every
// lane: exchanges inside quads and rows by DPP (partners 1 and 2 apart, then
// the mirrored half-row and row, whose lanes all hold the same value by then),
// then the four rows' maxima read as scalars.
__device__ __forceinline__ int wave_max(int x)
{
    x = max(x, __builtin_amdgcn_update_dpp(x, x, 0xb1, 0xf, 0xf, false));   // quad_perm [1,0,3,2]
    x = max(x, __builtin_amdgcn_update_dpp(x, x, 0x4e, 0xf, 0xf, false));   // quad_perm [2,3,0,1]
    x = max(x, __builtin_amdgcn_update_dpp(x, x, 0x141, 0xf, 0xf, false));  // row_half_mirror
    x = max(x, __builtin_amdgcn_update_dpp(x, x, 0x140, 0xf, 0xf, false));  // row_mirror
    return max(max(__builtin_amdgcn_readlane(x, 0), __builtin_amdgcn_readlane(x, 16)),
               max(__builtin_amdgcn_readlane(x, 32), __builtin_amdgcn_readlane(x, 48)));
}

// Sum over the 64 lanes of a wave (every lane active), the same in every
// lane and in a fixed order: lane pairs 1 and 2 apart inside quads, then the
// mirrored half-row and row (whose lanes hold equal values by then), all by
// DPP, then the four row sums as ((row 0 + row 1) + (row 2 + row 3)).
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v)
{
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)u, CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(u >> 32), CTRL, 0xf, 0xf, false);
    return __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}
__device__ __forceinline__ double readlane_f64(double v, int l)
{
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = __builtin_amdgcn_readlane((int)(uint32_t)u, l);
    const uint32_t hi = __builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), l);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ double wave_sum_f64(double v)
{
    v += dpp_f64<0xb1>(v);   // quad_perm [1,0,3,2]
    v += dpp_f64<0x4e>(v);   // quad_perm [2,3,0,1]
    v += dpp_f64<0x141>(v);  // row_half_mirror
    v += dpp_f64<0x140>(v);  // row_mirror
    return (readlane_f64(v, 0) + readlane_f64(v, 16)) + (readlane_f64(v, 32) + readlane_f64(v, 48));
}

// Block-wide exclusive scan of one int per thread (blockDim.x a multiple of
// 64, at most 1024): wave scans, then a scan of the wave totals.  `lds` holds
// at least 16 ints.  Returns the exclusive prefix; *total gets the sum.
__device__ __forceinline__ int block_exclusive_scan(int v, int *lds, int *total)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const int x = wave_inclusive_sum(v);
    if (lane == 63)
        lds[wid] = x;
    __syncthreads();
    if (wid == 0) {
        const int t = wave_inclusive_sum(lane < nw ? lds[lane] : 0);
        if (lane < nw)
            lds[lane] = t;
    }
    __syncthreads();
    const int res = (wid > 0 ? lds[wid - 1] : 0) + x - v;
    *total = lds[nw - 1];
    __syncthreads();
    return res;
}

// Two exclusive scans (of a and of b) with one set of barriers; returns a's
// scan, b's in *run_b, totals in *tot_a, *tot_b.  `lds` holds at least 32 ints.
__device__ __forceinline__ int block_exclusive_scan2(int a, int b, int *lds, int *tot_a, int *run_b, int *tot_b)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const int x = wave_inclusive_sum(a), y = wave_inclusive_sum(b);
    if (lane == 63) {
        lds[wid] = x;
        lds[16 + wid] = y;
    }
    __syncthreads();
    if (wid == 0) {
        const int t = wave_inclusive_sum(lane < nw ? lds[lane] : 0);
        const int u = wave_inclusive_sum(lane < nw ? lds[16 + lane] : 0);
        if (lane < nw) {
            lds[lane] = t;
            lds[16 + lane] = u;
        }
    }
    __syncthreads();
    const int ra = (wid > 0 ? lds[wid - 1] : 0) + x - a;
    *run_b = (wid > 0 ? lds[16 + wid - 1] : 0) + y - b;
    *tot_a = lds[nw - 1];
    *tot_b = lds[16 + nw - 1];
    __syncthreads();
    return ra;
}

// N exclusive scans with one set of barriers: run[q] = the scan of v[q],
// tot[q] its total.  `lds` holds at least 16 N ints (at most 16 waves).
template <int N>
__device__ __forceinline__ void block_exclusive_scan_n(const int (&v)[N], int *lds, int (&run)[N], int (&tot)[N])
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
    int x[N];
#pragma unroll
    for (int q = 0; q < N; ++q)
        x[q] = wave_inclusive_sum(v[q]);
    if (lane == 63) {
#pragma unroll
        for (int q = 0; q < N; ++q)
            lds[16 * q + wid] = x[q];
    }
    __syncthreads();
    if (wid == 0) {
        int t[N];
#pragma unroll
        for (int q = 0; q < N; ++q)
            t[q] = wave_inclusive_sum(lane < nw ? lds[16 * q + lane] : 0);
        if (lane < nw) {
#pragma unroll
            for (int q = 0; q < N; ++q)
                lds[16 * q + lane] = t[q];
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < N; ++q) {
        run[q] = (wid > 0 ? lds[16 * q + wid - 1] : 0) + x[q] - v[q];
        tot[q] = lds[16 * q + nw - 1];
    }
    __syncthreads();
}

// Block-wide sum of one double per thread, in a fixed order (wave sums,
// then the wave totals in order).  `lds` holds at least 16 doubles.
__device__ __forceinline__ double block_sum(double v, double *lds)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
    v = wave_sum_f64(v);
    if (lane == 0)
        lds[wid] = v;
    __syncthreads();
    double t = 0.0;
    for (int w = 0; w < nw; ++w)
        t += lds[w];
    __syncthreads();
    return t;
}

// Smallest i in [0, n) with off[i + 1] > s, for a non-decreasing off[0..n]
// with off[n] > s: the segment of entry s (empty segments skipped).  A 64-way
// search by one wave; every lane of the wave calls it with the same s.
__device__ __forceinline__ int wave_segment_of(const int32_t *__restrict__ off, int n, int s)
{
    const int lane = threadIdx.x & 63;
    int lo = 0, hi = n;
    while (hi - lo > 1) {
        const int step = (hi - lo + 63) / 64;
        const int q = lo + lane * step;
        const bool pred = q < hi && off[q + 1] > s;
        const uint64_t m = __ballot(pred);
        if (m & 1ull)
            return lo;  // pred(lo)
        if (m == 0ull) {
            const int last = min(63, (hi - 1 - lo) / step);
            lo = lo + last * step + 1;
        } else {
            const int f = __ffsll((unsigned long long)m) - 1;
            hi = lo + f * step + 1;
            lo = lo + (f - 1) * step + 1;
        }
    }
    return lo;
}

// ---------------------------------------------------------------------------
// Gram blocks of one slot, as tasks.  The self-norm of a center held over its
// support (Section 4.1) is a quadratic form in the blocks
//   G_j[c][c'] = sum_{a in column c of center j} sum_{e in column c' of center j} K(a, e)
// (column 0: the initial point, 1 + p: the center's rows of slot p).  The
// blocks of slot rr against a set of live columns are cut into tasks of
// `ta` rows of slot rr by `te` rows of the column:
//   tasks(j, c) = ceil(na_j / ta) * ceil(ne_jc / te),
// enumerated over jc = j * C + c with exclusive offsets goff[0 .. k*C].
// ---------------------------------------------------------------------------
constexpr int kGramTA = 32;      // slot rows per task of the VALU form
constexpr int kGramTAMfma = 16;  // ... and of the MFMA form (16 x 16 tiles)
// Column tiles per task that a plan may choose: 1, 2, ..., 2^(steps - 1).
// A plan whose tasks outnumber the work kernel's waves takes more tiles per
// task, so that a task's slot rows are loaded once for several tiles.
constexpr int kGramTileSteps = 4;

// Rows of center j in column c: the slot rows through the grouping
// permutation of their slot, column 0 the initial point (pool row j).
struct GramCol {
    int n;                 // rows
    const int32_t *perm;   // grouped position -> row within the slot (nullptr: column 0)
    int64_t row0;          // pool row of the slot's first row (column 0: j)
};

__device__ __forceinline__ GramCol gram_col(int k, int bmax, int j, int c, const int32_t *__restrict__ ring_off,
                                            const int32_t *__restrict__ ring_perm)
{
    GramCol g;
    if (c == 0) {
        g.n = 1;
        g.perm = nullptr;
        g.row0 = j;
    } else {
        const int32_t *o = ring_off + (int64_t)(c - 1) * (k + 1);
        g.n = o[j + 1] - o[j];
        g.perm = ring_perm + (int64_t)(c - 1) * bmax + o[j];
        g.row0 = (int64_t)k + (int64_t)(c - 1) * bmax;
    }
    return g;
}

__device__ __forceinline__ int64_t gram_row(const GramCol &g, int q) { return g.perm ? g.row0 + g.perm[q] : g.row0; }

// Length of a center's segment holding len entries: a multiple of pad, or
// (packed) the entries rounded up to a multiple of kPackAlign, at least pad
// when there are any; and the end of the whole support (packed: rounded up
// to a multiple of pad).
constexpr int kPackAlign = 8;
__host__ __device__ inline int seg_padded_len(int len, int pad, bool packed)
{
    return packed ? (len > 0 ? max((len + kPackAlign - 1) / kPackAlign * kPackAlign, pad) : 0)
                  : (len + pad - 1) / pad * pad;
}
__host__ __device__ inline int seg_padded_end(int total, int pad, bool packed)
{
    return packed ? (total + pad - 1) / pad * pad : total;
}

// Task offsets of the blocks of slot rr against the columns in `mask`, by
// one workgroup (blockDim.x a multiple of 64, at most 1024).  Thread t owns
// the centers [t * per, (t + 1) * per), per = ceil(k / blockDim.x); na_own,
// if given, holds the row counts of slot rr for those centers (written by the
// same threads), else they come from ring_off of slot rr; coef: the centers'
// column weights, columns of weight 0 having no tasks.  `sint`: 16 ints of LDS.
// With seg_next, the same pass also writes the segment offsets of the support
// whose columns are `mask` (each center's rows over those columns, padded to
// a multiple of pad): the layout of the next iteration when mask holds its
// live columns.
__device__ __forceinline__ void gram_plan(int k, int C, int rr, uint32_t mask, int ta, int te,
                                          const int32_t *__restrict__ ring_off, const int32_t *na_own,
                                          const double *coef, int32_t *__restrict__ goff, int *sint,
                                          int pad = 1, int32_t *__restrict__ seg_next = nullptr,
                                          bool packed = false)
{
    const int tid = threadIdx.x, nt = blockDim.x;
    const int per = (k + nt - 1) / nt;
    const int j0 = min(k, tid * per), j1 = min(k, j0 + per);
    const int32_t *orr = ring_off + (int64_t)rr * (k + 1);
    auto rows = [&](int j, int c, int na) -> int {  // rows of center j in live column c
        if (!((mask >> c) & 1u) || coef[(int64_t)j * C + c] == 0.0)
            return 0;  // (a column of weight 0 is left out of the support)
        if (c == 0)
            return 1;
        if (c - 1 == rr)
            return na;
        const int32_t *o = ring_off + (int64_t)(c - 1) * (k + 1);
        return o[j + 1] - o[j];
    };
    auto tasks = [&](int j, int c, int na) -> int {
        return ((na + ta - 1) / ta) * ((rows(j, c, na) + te - 1) / te);
    };
    int local = 0, slocal = 0;
    for (int j = j0; j < j1; ++j) {
        const int na = na_own ? na_own[j] : orr[j + 1] - orr[j];
        int len = 0;
        for (int c = 0; c < C; ++c) {
            local += tasks(j, c, na);
            len += rows(j, c, na);
        }
        slocal += seg_padded_len(len, pad, packed);
    }
    if (seg_next) {
        int stotal;
        int srun = block_exclusive_scan(slocal, sint, &stotal);
        for (int j = j0; j < j1; ++j) {
            const int na = na_own ? na_own[j] : orr[j + 1] - orr[j];
            int len = 0;
            for (int c = 0; c < C; ++c)
                len += rows(j, c, na);
            seg_next[j] = srun;
            srun += seg_padded_len(len, pad, packed);
        }
        if (threadIdx.x == 0)
            seg_next[k] = seg_padded_end(stotal, pad, packed);
    }
    int total;
    int run = block_exclusive_scan(local, sint, &total);
    for (int j = j0; j < j1; ++j) {
        const int na = na_own ? na_own[j] : orr[j + 1] - orr[j];
        for (int c = 0; c < C; ++c) {
            goff[(int64_t)j * C + c] = run;
            run += tasks(j, c, na);
        }
    }
    if (tid == 0) {
        goff[(int64_t)k * C] = total;
        goff[(int64_t)k * C + 1] = 1;  // column tiles per task
    }
}

// Block (j, c) of the Gram work just done (jc = j * C + c, njc = k * C): the
// partials of the waves whose task ranges met jc (stored at gpart[w + jc];
// nwaves: the wave count of the work kernel, which sets the ranges),
// lane-strided with eight independent sums, then across the wave; every lane
// returns the sum.  One fixed order, wherever the fold runs.  Split in two so
// that a caller can issue the offset loads early: the wave range [w0, w1]
// (empty when the block has no tasks), then the sum over it.
__device__ __forceinline__ void gram_fold_range(const int32_t *__restrict__ goff, int njc, int jc, int nwaves, int &w0,
                                                int &w1)
{
    const int g0 = goff[jc], g1 = goff[jc + 1], T = goff[njc];
    w0 = 1;
    w1 = 0;
    if (g1 > g0) {  // then T >= g1 > 0
        const int chunk = (T + nwaves - 1) / nwaves;
        w0 = g0 / chunk;
        w1 = (g1 - 1) / chunk;
    }
}

__device__ __forceinline__ double gram_fold_sum(const double *__restrict__ gpart, int jc, int w0, int w1)
{
    const int lane = threadIdx.x & 63;
    const double *gp = gpart + jc;
    double q[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    int w = w0 + lane;
    for (; w + 7 * 64 <= w1; w += 8 * 64) {
#pragma unroll
        for (int u = 0; u < 8; ++u)
            q[u] += gp[w + u * 64];
    }
    for (; w <= w1; w += 64)
        q[0] += gp[w];
    double s = ((q[0] + q[1]) + (q[2] + q[3])) + ((q[4] + q[5]) + (q[6] + q[7]));
    for (int o = 32; o > 0; o >>= 1)
        s += __shfl_xor(s, o);
    return s;
}

__device__ __forceinline__ double gram_fold_jc(const int32_t *__restrict__ goff, const double *__restrict__ gpart,
                                               int njc, int jc, int nwaves)
{
    int w0, w1;
    gram_fold_range(goff, njc, jc, nwaves, w0, w1);
    return gram_fold_sum(gpart, jc, w0, w1);
}

}  // namespace mbkk
