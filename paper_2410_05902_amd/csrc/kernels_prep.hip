// Data staging and center bookkeeping kernels of one iteration of the
// truncated mini-batch kernel k-means (Algorithm 2):
//   - ||x||^2 cache, batch staging (gather + FP32 / BF16 hi-lo copies),
//   - support layout of the implicit centers (Eq. 1 as a ring of slots),
//   - the update: deterministic grouping of the batch by center, counts
//     b_i^j, learning rates, coefficient decay by (1 - alpha), truncation,
//     and the task plan of the new slot's Gram blocks (computed in
//     kernels_gram.hip).
#include "dev_common.h"
#include "kernels.h"

namespace mbkk {

// ---------------------------------------------------------------------------
// Fill of n 32-bit words with one value: every clearing of device state goes
// through this kernel rather than a runtime memset, so that a caller may
// capture the library's calls in a HIP graph.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_fill32(uint32_t *__restrict__ p, uint32_t v, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        p[i] = v;
}

void launch_fill32(void *p, uint32_t v, int64_t nwords, hipStream_t st)
{
    if (nwords <= 0)
        return;
    int64_t blocks = (nwords + 255) / 256;
    blocks = blocks < 1024 ? blocks : 1024;
    hipLaunchKernelGGL(k_fill32, dim3((unsigned)blocks), dim3(256), 0, st, (uint32_t *)p, v, nwords);
}

// ---------------------------------------------------------------------------
// ||x||^2 for every row of X, summed in FP64, stored as FP32 (data norms),
// and their maximum over the finite ones (as FP32 bits in *sqmax, which the
// caller zeroes first; non-negative floats order like their bit patterns).
// 16 lanes per row, rows grid-strided; one atomic per workgroup.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_row_sqnorm(const float *__restrict__ X, int64_t n, int d,
                                                     int64_t ld, float *__restrict__ sqn,
                                                     unsigned int *__restrict__ sqmax)
{
    __shared__ float wmax[4];
    const int sub = threadIdx.x & 15;
    float m = 0.0f;
    for (int64_t row = (int64_t)blockIdx.x * 16 + (threadIdx.x >> 4); row < n; row += (int64_t)gridDim.x * 16) {
        const float *r = X + row * ld;
        double s = 0.0;
        for (int t = sub; t < d; t += 16) {
            double v = r[t];
            s += v * v;
        }
        for (int o = 8; o > 0; o >>= 1)
            s += __shfl_xor(s, o, 16);
        const float f = (float)s;
        if (sub == 0)
            sqn[row] = f;
        if (isfinite(f))
            m = fmaxf(m, f);
    }
    for (int o = 32; o > 0; o >>= 1)
        m = fmaxf(m, __shfl_xor(m, o));
    if ((threadIdx.x & 63) == 0)
        wmax[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0)
        atomicMax(sqmax, __float_as_uint(fmaxf(fmaxf(wmax[0], wmax[1]), fmaxf(wmax[2], wmax[3]))));
}

void launch_row_sqnorm(const float *X, int64_t n, int d, int64_t ld, float *sqn, unsigned int *sqmax,
                       hipStream_t st)
{
    int64_t blocks = (n + 15) / 16;
    blocks = blocks < 4096 ? blocks : 4096;
    hipLaunchKernelGGL(k_row_sqnorm, dim3((unsigned)blocks), dim3(256), 0, st, X, n, d, ld, sqn, sqmax);
}

// ---------------------------------------------------------------------------
// Gathers rows X[idx[r]] (or rows of a dense matrix when idx == nullptr) into
// a padded row-major buffer of stride dp (zeros past d), with optional BF16
// hi/lo copies and FP32/FP64 squared norms.  Out-of-range indices read as
// zero rows and raise flags[0]; non-finite values raise flags[1] (when
// check_finite).  One wave per row.
// ---------------------------------------------------------------------------
struct GatherArgs {
    const float *X;
    int64_t n;
    int d;
    int64_t ld;
    const int32_t *idx;
    int64_t cnt;
    int dp;
    float *out32;
    uint16_t *outhi, *outlo;
    float *outsq;
    double *outsq64;
    int32_t *idx_copy;
    int32_t *flags;
    int check_finite;
    int frag_mode;    // 1: BF16 hi/lo fragments, 2: FP32 fragments, 0: none
    char *frag;
    int64_t frag_lo;  // byte offset of the lo fragments
};

// Four rows per wave, 16 per workgroup (`blk` numbers groups of 16 rows):
// the index loads of the four rows, then every coordinate load of a stretch
// of 128 coordinates of the four rows, go out before the first store
// (clamped indices, selects; restrict pointers, so the stores do not order
// the loads).
constexpr int kGatherRowsPerWave = 4;
constexpr int kGatherRowsPerBlock = 4 * kGatherRowsPerWave;

__device__ __forceinline__ void gather_rows_body(const GatherArgs &A, int64_t blk)
{
    constexpr int RW = kGatherRowsPerWave;
    const int lane = threadIdx.x & 63;
    const int64_t row0 = blk * kGatherRowsPerBlock + (threadIdx.x >> 6) * RW;
    if (row0 >= A.cnt)
        return;
    const float *__restrict__ X = A.X;
    float *__restrict__ out32 = A.out32;
    uint16_t *__restrict__ outhi = A.outhi;
    uint16_t *__restrict__ outlo = A.outlo;
    int64_t p[RW];
    bool live[RW], ok[RW];
    if (A.idx) {  // (uniform)
        int32_t iv[RW];
#pragma unroll
        for (int q = 0; q < RW; ++q)
            iv[q] = A.idx[min(row0 + q, A.cnt - 1)];
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int q = 0; q < RW; ++q) {
            asm volatile("" : "+v"(iv[q]));  // the value is used here: no load is sunk into a branch
            p[q] = iv[q];
        }
    } else {
#pragma unroll
        for (int q = 0; q < RW; ++q)
            p[q] = min(row0 + q, A.cnt - 1);
    }
#pragma unroll
    for (int q = 0; q < RW; ++q)
        live[q] = row0 + q < A.cnt;
#pragma unroll
    for (int q = 0; q < RW; ++q) {
        ok[q] = p[q] >= 0 && p[q] < A.n;
        if (live[q] && lane == 0) {
            if (!ok[q])
                atomicOr(&A.flags[0], 1);
            if (A.idx_copy)
                A.idx_copy[row0 + q] = (int32_t)p[q];
        }
    }
    double s[RW];
    bool finite[RW];
#pragma unroll
    for (int q = 0; q < RW; ++q) {
        s[q] = 0.0;
        finite[q] = true;
    }
    for (int t0 = 0; t0 < A.dp; t0 += 128) {
        float v[RW][2];
#pragma unroll
        for (int q = 0; q < RW; ++q) {
            const float *src = X + (ok[q] ? p[q] : 0) * A.ld;
#pragma unroll
            for (int u = 0; u < 2; ++u)
                v[q][u] = src[min(t0 + lane + 64 * u, A.d - 1)];
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int q = 0; q < RW; ++q) {
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                asm volatile("" : "+v"(v[q][u]));  // (as above)
                v[q][u] = ok[q] && t0 + lane + 64 * u < A.d ? v[q][u] : 0.0f;
            }
        }
#pragma unroll
        for (int q = 0; q < RW; ++q) {
            if (!live[q])
                continue;  // (wave uniform)
            const int64_t row = row0 + q;
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int t = t0 + lane + 64 * u;
                if (t >= A.dp)
                    continue;
                const float x = v[q][u];
                finite[q] &= isfinite(x);
                out32[row * A.dp + t] = x;
                if (outhi) {
                    const uint16_t h = f32_to_bf16_rne(x);
                    const uint16_t l = f32_to_bf16_rne(x - bf16_to_f32(h));
                    outhi[row * A.dp + t] = h;
                    outlo[row * A.dp + t] = l;
                    if (A.frag_mode == 1) {
                        // 32x32x16 BF16 fragment order: k-step ks = t / 16 of block
                        // row / 32; lane 32 (t / 8 % 2) + row % 32, element t % 8
                        const int64_t f =
                            ((((row >> 5) * (A.dp >> 4) + (t >> 4)) * 64 + ((t >> 3) & 1) * 32 + (row & 31)) << 3) +
                            (t & 7);
                        ((uint16_t *)A.frag)[f] = h;
                        ((uint16_t *)(A.frag + A.frag_lo))[f] = l;
                    }
                }
                if (A.frag_mode == 2) {
                    // 32x32x2 FP32 fragment order: lane half hh = t / (dp/2) holds the
                    // coordinates hh dp/2 + 4 q + e of row row % 32, chunk q
                    const int ks = A.dp >> 1, hh = t / ks, r2 = t - hh * ks;
                    const int64_t f =
                        ((((row >> 5) * (ks >> 2) + (r2 >> 2)) * 64 + hh * 32 + (row & 31)) << 2) + (r2 & 3);
                    ((float *)A.frag)[f] = x;
                }
                s[q] += (double)x * (double)x;
            }
        }
    }
#pragma unroll
    for (int q = 0; q < RW; ++q) {
        if (!live[q])
            continue;
        if (A.check_finite && !finite[q])
            atomicOr(&A.flags[1], 1);
        double sq = s[q];
        for (int o = 32; o > 0; o >>= 1)
            sq += __shfl_xor(sq, o);
        if (lane == 0) {
            A.outsq[row0 + q] = (float)sq;
            if (A.outsq64)
                A.outsq64[row0 + q] = sq;
        }
    }
}

__global__ __launch_bounds__(256) void k_gather_rows(const GatherArgs A) { gather_rows_body(A, blockIdx.x); }

void launch_gather_rows(const float *X, int64_t n, int d, int64_t ld, const int32_t *idx, int64_t cnt,
                        int dp, float *out32, uint16_t *outhi, uint16_t *outlo, float *outsq,
                        double *outsq64, int32_t *idx_copy, int32_t *flags, int check_finite,
                        hipStream_t st, int frag_mode, char *frag, int64_t frag_lo)
{
    if (cnt <= 0)
        return;
    const GatherArgs A{X,        n,     d,         ld,    idx,          cnt,       dp,   out32,
                       outhi,    outlo, outsq,     outsq64, idx_copy,   flags,     check_finite,
                       frag_mode, frag, frag_lo};
    const int64_t blocks = (cnt + kGatherRowsPerBlock - 1) / kGatherRowsPerBlock;
    hipLaunchKernelGGL(k_gather_rows, dim3((unsigned)blocks), dim3(256), 0, st, A);
}

// ---------------------------------------------------------------------------
// Kernel value helper for the bookkeeping kernels (FP32 or FP64).
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T kernel_value(int kind, T param, const float *__restrict__ a,
                                          const float *__restrict__ e, int d)
{
    T s = 0;
    if (kind == MBKK_GAUSS) {
        for (int t = 0; t < d; ++t) {
            T v = (T)a[t] - (T)e[t];
            s += v * v;
        }
        return (T)exp(-s / param);
    } else if (kind == MBKK_LAPLACE) {
        for (int t = 0; t < d; ++t)
            s += fabs((T)a[t] - (T)e[t]);
        return (T)exp(-s / param);
    } else if (kind == MBKK_LINEAR) {
        for (int t = 0; t < d; ++t)
            s += (T)a[t] * (T)e[t];
        return s;
    } else {
        for (int t = 0; t < d; ++t)
            s += (T)a[t] * (T)e[t];
        s += param;
        return s * s;
    }
}

// ---------------------------------------------------------------------------
// Initial centers: coef[j][0] = 1, other coefficients 0, running counts 0,
// G_j = 0 except G_j[0][0] = K(x_j, x_j) (pool rows [0, k) hold the points).
// With set_coef == 0 only G is reset (state import).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_init_state(int k, int C, int kind, double param, int d, int dp,
                                                     const float *__restrict__ pool32, double *__restrict__ coef,
                                                     double *__restrict__ cum, double *__restrict__ G, int fp64,
                                                     int set_coef)
{
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= k)
        return;
    if (set_coef) {
        for (int c = 0; c < C; ++c)
            coef[(int64_t)j * C + c] = c == 0 ? 1.0 : 0.0;
        cum[j] = 0.0;
    }
    double *g = G + (int64_t)j * C * C;
    for (int c = 0; c < C * C; ++c)
        g[c] = 0.0;
    const float *x = pool32 + (int64_t)j * dp;
    g[0] = fp64 ? kernel_value<double>(kind, param, x, x, d)
                : (double)kernel_value<float>(kind, (float)param, x, x, d);
}

void launch_init_state(const Layout &L, const Buffers &B, int kind, double param, int fp64, int set_coef,
                       hipStream_t st)
{
    hipLaunchKernelGGL(k_init_state, dim3((L.k + 255) / 256), dim3(256), 0, st, L.k, L.C, kind, param, L.d, L.dp,
                       B.pool32, B.coef, B.cum, B.G, fp64, set_coef);
}

// ---------------------------------------------------------------------------
// Support layout of C_i (one workgroup per center j).  Center j's segment is
// [seg_off[j], seg_off[j+1]): its initial point (while alive), then its points
// in every live slot, oldest batch first, padded with the zero pool row to a
// multiple of `pad`.  Each entry carries its pool row and the weight
// coef[j][column].  The workgroup also computes
//   N_j = <C_j, C_j> = sum_{c,c'} coef[j][c] coef[j][c'] G_j[c][c']
// over the live columns (FP64).
// ---------------------------------------------------------------------------
// Rows of center j's support: the initial point while alive and the center's
// rows of every live slot, columns of weight 0 left out (their terms are zero).
__device__ __forceinline__ int seg_len(int j, int k, int C, const int32_t *__restrict__ ring_off,
                                       const double *__restrict__ coef, const SlotList &live, int init_alive)
{
    const double *cf = coef + (int64_t)j * C;
    int len = init_alive && cf[0] != 0.0 ? 1 : 0;
    for (int s = 0; s < live.n; ++s) {
        if (cf[1 + live.r[s]] == 0.0)
            continue;
        const int32_t *o = ring_off + (int64_t)live.r[s] * (k + 1);
        len += o[j + 1] - o[j];
    }
    return len;
}

struct SupportArgs {
    int k, C, bmax, pad;
    int64_t zero_row;
    const int32_t *ring_off, *ring_perm;
    SlotList live;
    int init_alive;
    const double *coef;
    double *G;
    const int32_t *seg_next;  // non-null: segment offsets already computed by the update
    int fold_rr;          // >= 0: fold the Gram work of this slot into G first
    uint32_t fold_mask;
    const int32_t *goff;
    const double *gpart;
    int gram_waves;       // waves of the Gram work kernel that wrote gpart
    int32_t *seg_off, *sup_row;
    float *sup_w;
    double *sup_w64;
    int32_t *blk_center;  // padded segments: the center of each block (else null)
    int32_t *blk_split;   // packed segments: the row of each block where a center starts, 32 for none (else null)
    int packed;
    double *N;
    float *sup_ay;        // MFMA path only (else null)
    const float *poolsq;
    float ay_scale;       // -log2(e) / kappa
};

// 256 threads.  Every load that depends on no other is issued first,
// unconditionally at clamped indices (a load under a condition is waited on
// before the next one goes out): the fold's task offsets, the coefficients,
// the slot offsets of center j, the segment offsets and the old Gram blocks.
// The fold then takes 16 lanes per column, so the partials of every column
// are loaded in one round (before the barrier), every thread lays out
// entries (permutations, then row norms), and N_j is taken from LDS.
__device__ void support_fill_body(const SupportArgs &A, int j)
{
    const int k = A.k, C = A.C, bmax = A.bmax, pad = A.pad;
    const int64_t zero_row = A.zero_row;
    const int32_t *__restrict__ ring_off = A.ring_off;
    const int32_t *__restrict__ ring_perm = A.ring_perm;
    const SlotList &live = A.live;
    const int init_alive = A.init_alive;
    const double *__restrict__ coef = A.coef;
    double *__restrict__ G = A.G;
    int32_t *__restrict__ seg_off = A.seg_off;
    int32_t *__restrict__ sup_row = A.sup_row;
    float *__restrict__ sup_w = A.sup_w;
    double *__restrict__ sup_w64 = A.sup_w64;
    int32_t *__restrict__ blk_center = A.blk_center;
    int32_t *__restrict__ blk_split = A.blk_split;
    float *__restrict__ sup_ay = A.sup_ay;
    const float *__restrict__ poolsq = A.poolsq;
    const float ay_scale = A.ay_scale;
    constexpr int MC = kMaxSlots + 1;  // columns at most
    constexpr int FL = 16;             // fold lanes per column (columns [4 wv, 4 wv + 4) per wave)
    __shared__ int red[256];
    __shared__ int sh_start;
    __shared__ double scf[MC];              // coef[j][c]
    __shared__ double sG[MC * MC];          // G_j, with the folded blocks
    __shared__ int sA0[kMaxSlots], sN[kMaxSlots];  // live slot s: first grouped row of j, rows (0: weight 0)
    __shared__ int sSeg[2];
    __shared__ int sBig[MC];                // column whose fold has more than FL partials
    __shared__ double sNt[MC * MC];         // the terms of N_j
    const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
    const double *cfj = coef + (int64_t)j * C;
    double *gj = G + (int64_t)j * C * C;
    const int rr = A.fold_rr;
    const bool fold = rr >= 0;
    const bool lane_fold = C <= 4 * 4;  // every column in one 16-lane group
    // ---- round 1
    // the fold's task offsets: column fc of this 16-lane group
    const int fcu = 4 * wv + lane / FL, fc = min(fcu, C - 1), fi = lane & (FL - 1);
    const int fjc = j * C + fc;
    const int fg0 = A.goff[fjc], fg1 = A.goff[fjc + 1], fT = A.goff[k * C];
    // coefficient c = lane (wave 0)
    const double v_cf = cfj[min(lane, C - 1)];
    // live slot s = lane (wave 1): the offsets of center j and the weight
    const int s1 = min(lane, max(live.n - 1, 0));
    int p1 = 0;
#pragma unroll
    for (int s = 0; s < kMaxSlots; ++s)  // scalar reads of the slot list, then a select
        p1 = s < live.n && s == s1 ? live.r[s] : p1;
    const int32_t *o1p = ring_off + (int64_t)p1 * (k + 1);
    const int a0v = o1p[j], a1v = o1p[j + 1];
    const double w1v = cfj[1 + p1];
    // segment offsets written by the update (seg_off itself when there are none)
    const int32_t *snp = A.seg_next ? A.seg_next : seg_off;
    const int sg0 = snp[j], sg1 = snp[j + 1];
    // the old Gram blocks (waves 2-3)
    const double v_g = gj[min(max(tid - 128, 0), C * C - 1)];
    // ---- round 2 of the fold: its partials, one per lane
    // wave range of the column (as gram_fold_range; branch-free, so that the
    // task count's load is not sunk into a branch)
    const int fchunk = max(1, (fT + A.gram_waves - 1) / A.gram_waves);
    const bool fany = fg1 > fg0;
    const int fw0 = fany ? fg0 / fchunk : 1, fw1 = fany ? (fg1 - 1) / fchunk : 0;
    // (goff holds no plan before the first update: the index is formed only
    // for a pending fold and kept inside the partials either way)
    const int fwi = fold ? min(max(min(fw0 + fi, max(fw0, fw1)), 0), A.gram_waves - 1) : 0;
    const double fv = A.gpart[fjc + fwi];
    // ---- LDS
    if (tid < C)
        scf[tid] = v_cf;
    if (tid >= 64 && tid < 64 + live.n) {
        const int s = tid - 64;
        sA0[s] = a0v;
        sN[s] = w1v == 0.0 ? 0 : a1v - a0v;
    }
    if (tid == 0) {
        sSeg[0] = sg0;
        sSeg[1] = sg1;
    }
    if (tid >= 128) {
        if (tid - 128 < C * C)
            sG[tid - 128] = v_g;
        for (int q = tid; q < C * C; q += 128)  // C > 11
            sG[q] = gj[q];
    }
    if (fi == 0 && fcu < C) {
        sBig[fcu] = fw1 - fw0 >= FL;
    }
    __syncthreads();
    // ---- segment of center j
    int start, plen;
    if (A.seg_next) {
        // offsets written by the last update for this support
        start = sSeg[0];
        plen = sSeg[1] - start;
    } else {
        // exclusive prefix of the padded lengths of centers < j
        int acc = 0;
        for (int q = tid; q < j; q += 256) {
            const int l = seg_len(q, k, C, ring_off, coef, live, init_alive);
            acc += seg_padded_len(l, pad, A.packed);
        }
        red[tid] = acc;
        __syncthreads();
        for (int s = 128; s > 0; s >>= 1) {
            if (tid < s)
                red[tid] += red[tid + s];
            __syncthreads();
        }
        int len = init_alive && scf[0] != 0.0 ? 1 : 0;
        for (int s = 0; s < live.n; ++s)
            len += sN[s];
        plen = seg_padded_len(len, pad, A.packed);
        if (tid == 0)
            sh_start = red[0];
        __syncthreads();
        start = sh_start;
        if (j == k - 1)  // the last segment reaches the support's end
            plen = seg_padded_end(start + plen, pad, A.packed) - start;
    }
    if (tid == 0) {
        seg_off[j] = start;
        if (j == k - 1)
            seg_off[k] = start + plen;
    }
    {
        // ---- entries: the initial point (while alive, weight != 0), then the
        // center's rows of every live slot with weight != 0, oldest first, then
        // the zero row up to the padded length
        // (FU entries per thread per round, whose permutation and norm loads
        // are issued together at clamped indices: a large center's entries
        // then cost two load round trips, not two per 256 entries)
        constexpr int FU = 4;
        const int ni = init_alive && scf[0] != 0.0 ? 1 : 0;
        for (int qb = tid; qb < plen; qb += 256 * FU) {
            int64_t row[FU];
            double w[FU];
            int64_t pidx[FU];  // index into ring_perm, -1 for the initial point and padding
#pragma unroll
            for (int u = 0; u < FU; ++u) {
                const int q = qb + 256 * u;
                row[u] = zero_row;
                w[u] = 0.0;
                pidx[u] = -1;
                if (q < plen) {
                    if (q < ni) {
                        row[u] = j;
                        w[u] = scf[0];
                    } else {
                        int r = q - ni;
                        for (int s = 0; s < live.n; ++s) {
                            const int ns = sN[s];
                            if (r < ns) {
                                const int p = live.r[s];
                                row[u] = (int64_t)k + (int64_t)p * bmax;
                                pidx[u] = (int64_t)p * bmax + sA0[s] + r;
                                w[u] = scf[1 + p];
                                break;
                            }
                            r -= ns;
                        }
                    }
                }
            }
            int pv[FU];
#pragma unroll
            for (int u = 0; u < FU; ++u)
                pv[u] = ring_perm[max(pidx[u], (int64_t)0)];
#pragma unroll
            for (int u = 0; u < FU; ++u)
                row[u] += pidx[u] >= 0 ? pv[u] : 0;
            float ya[FU];
            if (sup_ay) {
#pragma unroll
                for (int u = 0; u < FU; ++u)
                    ya[u] = poolsq[row[u]];  // the zero row's entry exists (and is 0)
            }
#pragma unroll
            for (int u = 0; u < FU; ++u) {
                const int q = qb + 256 * u;
                if (q < plen) {
                    sup_row[start + q] = (int32_t)row[u];
                    sup_w[start + q] = (float)w[u];
                    sup_w64[start + q] = w[u];
                    if (sup_ay)
                        sup_ay[start + q] = row[u] == zero_row ? 0.0f : ay_scale * ya[u];
                }
            }
        }
        if (blk_center) {
            for (int q = start / 32 + tid; q < (start + plen) / 32; q += 256)
                blk_center[q] = j;
        }
        if (blk_split && plen > 0) {
            // the block holding the segment's first entry records where it
            // starts; the blocks wholly inside the segment record no start
            // (every block gets one writer: a segment is at least 32 entries)
            if (tid == 0)
                blk_split[start / 32] = start % 32;
            for (int q = start / 32 + 1 + tid; 32 * q + 32 <= start + plen; q += 256)
                blk_split[q] = 32;
        }
    }
    // ---- Gram blocks of the last update's slot (gram_fold_jc's sums: up to
    // FL partials in 16 lanes give the same additions as its 64-lane form,
    // whose other lanes hold exact zeros)
    if (fold) {
        if (lane_fold) {
            double q[8] = {0, 0, 0, 0, 0, 0, 0, 0};
            if (fw0 + fi <= fw1)
                q[0] += fv;
            double sm = ((q[0] + q[1]) + (q[2] + q[3])) + ((q[4] + q[5]) + (q[6] + q[7]));
            for (int o = FL / 2; o > 0; o >>= 1)
                sm += __shfl_xor(sm, o);
            if (fi == 0 && fcu < C && ((A.fold_mask >> fcu) & 1u) && fw1 - fw0 < FL) {
                sG[(1 + rr) * C + fcu] = sm;
                sG[fcu * C + 1 + rr] = sm;
                gj[(1 + rr) * C + fcu] = sm;
                gj[fcu * C + 1 + rr] = sm;
            }
        }
        // columns with more partials, or beyond the lane groups: one wave each
        for (int c = wv; c < C; c += 4) {  // wave uniform
            if (((A.fold_mask >> c) & 1u) && (!lane_fold || sBig[c])) {
                const double g = gram_fold_jc(A.goff, A.gpart, k * C, j * C + c, A.gram_waves);
                if (lane == 0) {
                    sG[(1 + rr) * C + c] = g;
                    sG[c * C + 1 + rr] = g;
                    gj[(1 + rr) * C + c] = g;
                    gj[c * C + 1 + rr] = g;
                }
            }
        }
    }
    __syncthreads();
    // ---- N_j from the Gram blocks (FP64), in a fixed order: the products of
    // the live columns' pairs (a, e) by one thread each, then their sum, a
    // major and e minor, by one thread
    const int nc = (init_alive ? 1 : 0) + live.n;
    auto col_of = [&](int i) { return init_alive ? (i == 0 ? 0 : 1 + live.r[i - 1]) : 1 + live.r[i]; };
    for (int t = tid; t < nc * nc; t += 256) {
        const int ca = col_of(t / nc), ce = col_of(t % nc);
        sNt[t] = scf[ca] * scf[ce] * sG[ca * C + ce];
    }
    __syncthreads();
    if (tid == 0) {
        double nn = 0.0;
        for (int t = 0; t < nc * nc; ++t)
            nn += sNt[t];
        A.N[j] = nn;
    }
}

// One launch prepares an iteration: workgroups [0, nsup) lay out the support
// of C_i (one per center), the others stage the batch rows (16 per workgroup).
__global__ __launch_bounds__(256) void k_prepare(const SupportArgs S, int nsup, const GatherArgs Gth)
{
    if ((int)blockIdx.x < nsup)
        support_fill_body(S, blockIdx.x);
    else
        gather_rows_body(Gth, (int64_t)blockIdx.x - nsup);
}

void launch_prepare(const Layout &L, const Buffers &B, bool with_support, const SlotList &live, int init_alive,
                    const int32_t *idx, int64_t cnt, int check_finite, float ay_scale, int fold_rr,
                    uint32_t fold_mask, bool seg_ready, hipStream_t st)
{
    SupportArgs S;
    S.k = L.k;
    S.C = L.C;
    S.bmax = L.bmax;
    S.pad = L.pad;
    S.zero_row = L.PR;
    S.ring_off = B.ring_off;
    S.ring_perm = B.ring_perm;
    S.live = live;
    S.init_alive = init_alive;
    S.coef = B.coef;
    S.G = B.G;
    S.seg_next = seg_ready ? B.seg_next : nullptr;
    S.fold_rr = with_support ? fold_rr : -1;
    S.fold_mask = fold_mask;
    S.goff = B.goff;
    S.gpart = B.gpart;
    S.gram_waves = gram_waves(L.pad == kMfmaPad);
    S.seg_off = B.seg_off;
    S.sup_row = B.sup_row;
    S.sup_w = B.sup_w;
    S.sup_w64 = B.sup_w64;
    S.blk_center = L.pad == kMfmaPad && !L.packed ? B.blk_center : nullptr;
    S.blk_split = L.packed ? B.blk_split : nullptr;
    S.packed = L.packed;
    S.N = B.N;
    S.sup_ay = L.pad == kMfmaPad ? B.sup_ay : nullptr;
    S.poolsq = B.poolsq;
    S.ay_scale = ay_scale;
    const GatherArgs Gth{B.X,       L.n,       L.d,       B.ld,      idx,       cnt,
                         L.dp,      B.bat32,   B.bathi,   B.batlo,   B.batsq,   B.batsq64,
                         B.batidx,  B.flags,   check_finite, L.frag_mode, B.batfrag,
                         2 * (int64_t)frag_rows(L) * L.dp};
    const int nsup = with_support ? L.k : 0;
    const int64_t ngat = cnt > 0 ? (cnt + kGatherRowsPerBlock - 1) / kGatherRowsPerBlock : 0;
    if (nsup + ngat > 0)
        hipLaunchKernelGGL(k_prepare, dim3((unsigned)(nsup + ngat)), dim3(256), 0, st, S, nsup, Gth);
}

// ---------------------------------------------------------------------------
// Update of Algorithm 2.  The batch is grouped by center in a deterministic,
// stable order (each center's points in batch order):
//   the scoring kernel ranks each row among the equal labels before it in its
//   chunk of 64 rows and counts the chunk's labels; then one workgroup
//   computes the counts b_i^j, the offsets of the centers in the new slot,
//   per-(chunk, label) bases, the learning rates alpha, the coefficient
//   update and truncation, the task offsets of the new slot's Gram blocks,
//   the batch objective, and scatters every row to base + rank.
// ---------------------------------------------------------------------------
// LDS variant (per-chunk counts held in LDS) when nchunk * k is at most this.
constexpr int kGroupLdsMax = 8192;

// For the variant with counts in global memory: per label j (one thread
// each, over as many workgroups as the labels need), the exclusive prefix of
// its counts over the chunks, in gbase (the base of (chunk, label) within the
// label), and its total b_j in counts.  The chunk loads of a thread are issued
// kLabelU at a time; consecutive threads read consecutive labels.
constexpr int kLabelU = 32;
__global__ __launch_bounds__(64) void k_label_bases(int k, int nchunk, const int32_t *__restrict__ gcnt,
                                                     int32_t *__restrict__ gbase, int32_t *__restrict__ counts)
{
    const int j = blockIdx.x * 64 + threadIdx.x;
    if (j >= k)
        return;
    int run = 0;
    for (int g0 = 0; g0 < nchunk; g0 += kLabelU) {
        int c[kLabelU];
#pragma unroll
        for (int u = 0; u < kLabelU; ++u)
            c[u] = gcnt[(int64_t)min(g0 + u, nchunk - 1) * k + j];
#pragma unroll
        for (int u = 0; u < kLabelU; ++u) {
            if (g0 + u < nchunk) {
                gbase[(int64_t)(g0 + u) * k + j] = run;
                run += c[u];
            }
        }
    }
    counts[j] = run;
}

template <bool LDS>
__global__ __launch_bounds__(1024) void k_group_offsets(
    int b, int k, int nchunk, int C, int p_new, int p_expired, int init_alive_before, int init_keep,
    SlotList live, WindowRank win, int lr, const int32_t *__restrict__ gcnt, int32_t *__restrict__ gbase,
    const float *__restrict__ mind,
    double *__restrict__ coef, double *__restrict__ cum, int32_t *__restrict__ counts,
    double *__restrict__ alpha, int32_t *__restrict__ off, double *__restrict__ obj,
    const int32_t *__restrict__ labels, const int32_t *__restrict__ rank, const int32_t *__restrict__ pts,
    int32_t *__restrict__ ring_idx, int32_t *__restrict__ ring_perm, uint32_t gram_mask, int gram_ta, int gram_te,
    const int32_t *__restrict__ ring_off, int32_t *__restrict__ goff, int pad, int packed,
    int32_t *__restrict__ seg_next)
{
    __shared__ int sint[16];
    __shared__ double sdbl[16];
    __shared__ int scnt[LDS ? kGroupLdsMax : 1], sbase[LDS ? kGroupLdsMax : 1];
    const int tid = threadIdx.x, nt = blockDim.x;
    // per-(chunk, label) counts: staged in LDS with coalesced loads
    const int32_t *cnt = gcnt;
    int32_t *base = gbase;
    if constexpr (LDS) {
        constexpr int CPT = kGroupLdsMax / 1024;  // blockDim.x == 1024
        int v[CPT];
#pragma unroll
        for (int q = 0; q < CPT; ++q) {
            const int i = tid + q * nt;
            v[q] = i < nchunk * k ? gcnt[i] : 0;
        }
#pragma unroll
        for (int q = 0; q < CPT; ++q) {
            const int i = tid + q * nt;
            if (i < nchunk * k)
                scnt[i] = v[q];
        }
        __syncthreads();
        cnt = scnt;
        base = sbase;
    }
    const int per = (k + nt - 1) / nt;
    const int j0 = tid * per, j1 = min(k, j0 + per);
    // totals of this thread's labels, block-wide exclusive scan -> offsets
    // (counts in global memory: k_label_bases has put the totals in counts
    // and the bases within each label in gbase)
    int local = 0;
    for (int j = j0; j < j1; ++j) {
        if constexpr (LDS) {
#pragma unroll 8
            for (int g = 0; g < nchunk; ++g)
                local += cnt[(int64_t)g * k + j];
        } else {
            local += counts[j];
        }
    }
    int total;
    int run = block_exclusive_scan(local, sint, &total);
    for (int j = j0; j < j1; ++j) {
        off[j] = run;
        int bj;
        if constexpr (LDS) {
            int gb = run;
#pragma unroll 8
            for (int g = 0; g < nchunk; ++g) {
                base[(int64_t)g * k + j] = gb;  // base of label j in chunk g
                gb += cnt[(int64_t)g * k + j];
            }
            bj = gb - run;
        } else {
            bj = counts[j];
        }
        run += bj;
        counts[j] = bj;
        double a;
        if (lr == MBKK_LR_FULL)
            a = bj > 0 ? 1.0 : 0.0;
        else if (lr == MBKK_LR_SKLEARN) {
            const double cs = cum[j] + (double)bj;
            cum[j] = cs;
            a = bj > 0 ? (double)bj / cs : 0.0;
        } else
            a = sqrt((double)bj / (double)b);
        alpha[j] = a;
        // C_{i+1} = (1 - a) C_i + a cm(B_i^j), truncated to the window
        double *cf = coef + (int64_t)j * C;
        if (init_alive_before)
            cf[0] *= (1.0 - a);
        for (int s = 0; s < live.n; ++s)
            cf[1 + live.r[s]] *= (1.0 - a);
        cf[1 + p_new] = bj > 0 ? a / (double)bj : 0.0;
        if (p_expired >= 0)
            cf[1 + p_expired] = 0.0;
        if (!init_keep)
            cf[0] = 0.0;
        // and by count (Section 4.1), as in the small variant
        if (win.tau > 0) {
            int sum = 0, q0 = -1;
            for (int q = win.n - 1; q >= 0 && q0 < 0; --q) {
                for (int p = 0; p < C - 1; ++p) {
                    if (win.rank[p] == q) {
                        const int32_t *o = ring_off + (int64_t)p * (k + 1);
                        sum += p == p_new ? bj : o[j + 1] - o[j];
                    }
                }
                if (sum >= win.tau)
                    q0 = q;
            }
            if (q0 >= 0 && win.first + q0 > 1) {
                cf[0] = 0.0;
                for (int p = 0; p < C - 1; ++p)
                    if (win.rank[p] >= 0 && win.rank[p] < q0)
                        cf[1 + p] = 0.0;
            }
        }
    }
    if (tid == 0)
        off[k] = b;
    // task offsets of the Gram blocks of the new slot (its counts are this
    // thread's b_i^j above; the other live slots' offsets are settled)
    gram_plan(k, C, p_new, gram_mask, gram_ta, gram_te, ring_off, counts, coef, goff, sint, pad, seg_next, packed);
    // sum of min distances (FP64), fixed order
    double sm = 0.0;
    for (int p = tid; p < b; p += nt)
        sm += (double)mind[p];
    sm = block_sum(sm, sdbl);  // (its barriers also publish the bases above)
    if (tid == 0)
        obj[0] = sm;
    // scatter: grouped position of every row = base of (chunk, label) + rank
    for (int p = tid; p < b; p += nt) {
        const int lab = min(max(labels[p], 0), k - 1);
        const int pos = base[(int64_t)(p / kChunk) * k + lab] + (LDS ? 0 : off[lab]) + rank[p];
        ring_perm[pos] = p;
        ring_idx[pos] = pts[p];
    }
}

// Variant for k <= kGroupSmallK, nchunk * k <= kGroupLdsMax, C <= kGroupSmallC
// and Gram task shapes that are powers of two (each thread owns at most one
// center; one workgroup, so the per-center work is a serial chain of a wave's
// instructions, and divisions are shifts): every global load that does not
// depend on a result of this kernel is issued at its start (the rows' labels,
// ranks, points and distances, the center's coefficient row and the ring
// offsets the Gram plan needs), so the phases below wait on LDS only.  The
// chunk sums of the counts are split over kGroupThreads / k slices of chunks.
constexpr int kGroupSmallK = 512, kGroupSmallC = 8, kGroupThreads = 1024;

__global__ __launch_bounds__(kGroupThreads) void k_group_offsets_small(
    int b, int k, int nchunk, int C, int p_new, int p_expired, int init_alive_before, int init_keep,
    SlotList live, WindowRank win, int lr, const int32_t *__restrict__ gcnt, const float *__restrict__ mind,
    double *__restrict__ coef, double *__restrict__ cum, int32_t *__restrict__ counts,
    double *__restrict__ alpha, int32_t *__restrict__ off, double *__restrict__ obj,
    const int32_t *__restrict__ labels, const int32_t *__restrict__ rank, const int32_t *__restrict__ pts,
    int32_t *__restrict__ ring_idx, int32_t *__restrict__ ring_perm, uint32_t gram_mask, int gram_ta, int gram_te,
    int gram_qmax, int gram_nwaves, const int32_t *__restrict__ ring_off, int32_t *__restrict__ goff, int pad,
    int packed, int32_t *__restrict__ seg_next)
{
    constexpr int RPT = kMaxBatch / kGroupThreads;  // batch rows per thread
    // the task rows and columns are powers of two (the launch checks it)
    const int lta = __builtin_ctz((unsigned)gram_ta), lte = __builtin_ctz((unsigned)gram_te);
    __shared__ int sint[16 * (1 + kGramTileSteps)];
    __shared__ double sdbl[16];
    __shared__ int scnt[kGroupLdsMax];    // per-(chunk, label) counts, then bases, then the grouped rows
    __shared__ int sidx[kMaxBatch];       // the grouped rows' points
    __shared__ int spart[kGroupThreads];  // per-(slice, label) sums, then slice starts
    __shared__ int soff[kGroupSmallK];
    const int tid = threadIdx.x, nt = kGroupThreads;
    // ---- independent loads: unconditional, at clamped indices, and selected
    // afterwards, so that none waits for another (a load under a condition
    // is waited on before the next one is issued)
    int r_lab[RPT], r_rank[RPT], r_pt[RPT];
    float r_md[RPT];
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
        const int pc = min(tid + i * nt, b - 1);  // b >= 1
        r_lab[i] = labels[pc];
        r_rank[i] = rank[pc];
        r_pt[i] = pts[pc];
        r_md[i] = mind[pc];
    }
    const bool own = tid < k;
    const int j = tid, jc = min(tid, k - 1);
    double cf[kGroupSmallC];
    int o0[kGroupSmallC], o1[kGroupSmallC];
    double cumv = 0.0;
    if ((tid & ~63) < k) {  // waves holding a center (one branch around every load)
#pragma unroll
        for (int c = 0; c < kGroupSmallC; ++c) {
            const int cc = min(c, C - 1), sc = max(cc - 1, 0);
            cf[c] = coef[(int64_t)jc * C + cc];
            const int32_t *o = ring_off + (int64_t)sc * (k + 1);
            o0[c] = o[jc];
            o1[c] = o[jc + 1];
        }
        cumv = cum[jc];
    } else {
#pragma unroll
        for (int c = 0; c < kGroupSmallC; ++c) {
            cf[c] = 0.0;
            o0[c] = o1[c] = 0;
        }
    }
    constexpr int CPT = kGroupLdsMax / kGroupThreads;
    int v[CPT];
#pragma unroll
    for (int q = 0; q < CPT; ++q)
        v[q] = gcnt[min(tid + q * nt, nchunk * k - 1)];
    // ---- selections
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
        if (tid + i * nt >= b) {
            r_lab[i] = 0;
            r_rank[i] = 0;
            r_pt[i] = 0;
            r_md[i] = 0.0f;
        }
    }
    int ne[kGroupSmallC];  // rows of center j in column c (other slots than the new one)
#pragma unroll
    for (int c = 0; c < kGroupSmallC; ++c) {
        const bool colok = own && c < C;
        cf[c] = colok ? cf[c] : 0.0;
        ne[c] = colok && c >= 1 && c - 1 != p_new && ((gram_mask >> c) & 1u) ? o1[c] - o0[c] : 0;
    }
    const double cumj = own && lr == MBKK_LR_SKLEARN ? cumv : 0.0;
#pragma unroll
    for (int q = 0; q < CPT; ++q) {
        const int i = tid + q * nt;
        if (i < nchunk * k)
            scnt[i] = v[q];
    }
    __syncthreads();
    // ---- label totals: slice sums over chunks, then per label over slices
    const int TG = nt / k;  // >= 2
    const int gs = (nchunk + TG - 1) / TG;
    if (tid < TG * k) {
        const int jj = tid % k, sl = tid / k;
        const int g1 = min(nchunk, (sl + 1) * gs);
        int sum = 0;
        for (int g = sl * gs; g < g1; ++g)
            sum += scnt[g * k + jj];
        spart[sl * k + jj] = sum;
    }
    __syncthreads();
    int bj = 0;
    if (own) {
        for (int sl = 0; sl < TG; ++sl) {
            const int v = spart[sl * k + j];
            spart[sl * k + j] = bj;  // start of slice sl within label j
            bj += v;
        }
    }
    int total;
    const int offj = block_exclusive_scan(own ? bj : 0, sint, &total);
    if (own) {
        soff[j] = offj;
        off[j] = offj;
        counts[j] = bj;
    }
    if (tid == 0)
        off[k] = b;
    __syncthreads();
    // ---- bases of (chunk, label), in place of the counts
    if (tid < TG * k) {
        const int jj = tid % k, sl = tid / k;
        const int g1 = min(nchunk, (sl + 1) * gs);
        int gb = soff[jj] + spart[sl * k + jj];
        for (int g = sl * gs; g < g1; ++g) {
            const int v = scnt[g * k + jj];
            scnt[g * k + jj] = gb;
            gb += v;
        }
    }
    // ---- learning rate and the coefficient update of center j
    int tasks[kGramTileSteps] = {};  // Gram tasks of 1, 2, 4, ... column tiles
    int slen = 0;
    int nA = 0, ntl[kGroupSmallC];  // slot-row tiles, and column tiles of the counted columns (else 0)
#pragma unroll
    for (int c = 0; c < kGroupSmallC; ++c)
        ntl[c] = 0;
    if (own) {
        double a;
        if (lr == MBKK_LR_FULL)
            a = bj > 0 ? 1.0 : 0.0;
        else if (lr == MBKK_LR_SKLEARN) {
            const double cs = cumj + (double)bj;
            cum[j] = cs;
            a = bj > 0 ? (double)bj / cs : 0.0;
        } else
            a = sqrt((double)bj / (double)b);
        alpha[j] = a;
        uint32_t livem = 0;
        for (int q = 0; q < live.n; ++q)
            livem |= 1u << live.r[q];
        // C_{i+1} = (1 - a) C_i + a cm(B_i^j), truncated to the window
#pragma unroll
        for (int c = 0; c < kGroupSmallC; ++c) {
            if (c >= C)
                break;
            double v = cf[c];
            if (c == 0) {
                if (init_alive_before)
                    v *= (1.0 - a);
                if (!init_keep)
                    v = 0.0;
            } else {
                const int p = c - 1;
                if ((livem >> p) & 1u)
                    v *= (1.0 - a);
                if (p == p_new)
                    v = bj > 0 ? a / (double)bj : 0.0;
                if (p == p_expired)
                    v = 0.0;
            }
            cf[c] = v;
        }
        // and by count (Section 4.1): the newest batches up to the one at
        // which the counts reach tau stay; older ones and the initial point
        // go when that batch is not the first
        if (win.tau > 0) {
            int sum = 0, q0 = -1;
            for (int q = win.n - 1; q >= 0 && q0 < 0; --q) {
                int cq = 0;
#pragma unroll
                for (int c = 1; c < kGroupSmallC; ++c)
                    if (c < C && win.rank[c - 1] == q)
                        cq = c - 1 == p_new ? bj : ne[c];
                sum += cq;
                if (sum >= win.tau)
                    q0 = q;
            }
            if (q0 >= 0 && win.first + q0 > 1) {
#pragma unroll
                for (int c = 0; c < kGroupSmallC; ++c)
                    if (c < C && (c == 0 || win.rank[c - 1] < q0))
                        cf[c] = 0.0;
            }
        }
#pragma unroll
        for (int c = 0; c < kGroupSmallC; ++c)
            if (c < C)
                coef[(int64_t)j * C + c] = cf[c];
        // Gram tasks of the new slot against the live columns that keep a
        // weight (for each number of column tiles per task), and the padded
        // segment of center j in the next support
        nA = (bj + gram_ta - 1) >> lta;
#pragma unroll
        for (int c = 0; c < kGroupSmallC; ++c) {
            if (c < C && ((gram_mask >> c) & 1u) && cf[c] != 0.0) {
                const int nec = c == 0 ? 1 : (c - 1 == p_new ? bj : ne[c]);
                ntl[c] = (nec + gram_te - 1) >> lte;
#pragma unroll
                for (int qi = 0; qi < kGramTileSteps; ++qi)
                    tasks[qi] += nA * ((ntl[c] + (1 << qi) - 1) >> qi);
                slen += nec;
            }
        }
        slen = seg_padded_len(slen, pad, packed);
    }
    int sv[1 + kGramTileSteps], srun_[1 + kGramTileSteps], stot[1 + kGramTileSteps];
    sv[0] = slen;
#pragma unroll
    for (int qi = 0; qi < kGramTileSteps; ++qi)
        sv[1 + qi] = tasks[qi];
    block_exclusive_scan_n<1 + kGramTileSteps>(sv, sint, srun_, stot);  // (its barriers also publish the bases)
    // column tiles per task: the fewest (a power of two up to gram_qmax) whose
    // tasks fit in the work kernel's waves, else the most (workgroup uniform)
    int qi = 0;
    while (qi + 1 < kGramTileSteps && (2 << qi) <= min(kGramQMin, gram_qmax))
        ++qi;
    while (qi + 1 < kGramTileSteps && (2 << qi) <= gram_qmax && stot[1 + qi] > gram_nwaves)
        ++qi;
    const int Q = 1 << qi;
    if (own)
        seg_next[j] = srun_[0];
    if (tid == 0)
        seg_next[k] = seg_padded_end(stot[0], pad, packed);
    if (own) {
        int trun = srun_[1 + qi];
#pragma unroll
        for (int c = 0; c < kGroupSmallC; ++c) {
            if (c < C) {
                goff[(int64_t)j * C + c] = trun;
                trun += nA * ((ntl[c] + Q - 1) >> qi);
            }
        }
    }
    if (tid == 0) {
        goff[(int64_t)k * C] = stot[1 + qi];
        goff[(int64_t)k * C + 1] = Q;
    }
    // ---- sum of min distances (FP64), in the order of the general variant
    double sm = 0.0;
#pragma unroll
    for (int i = 0; i < RPT; ++i)
        sm += (double)r_md[i];
    sm = block_sum(sm, sdbl);
    if (tid == 0)
        obj[0] = sm;
    // ---- scatter: grouped position of every row = base of (chunk, label) +
    // rank, through LDS (the bases' array, then sidx), then written out in
    // grouped order with coalesced stores
    int pos[RPT];
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
        const int p = tid + i * nt;
        const int lab = min(max(r_lab[i], 0), k - 1);
        pos[i] = p < b ? scnt[(p / kChunk) * k + lab] + r_rank[i] : -1;
    }
    __syncthreads();  // every base read before scnt is reused
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
        if (pos[i] >= 0) {
            scnt[pos[i]] = tid + i * nt;
            sidx[pos[i]] = r_pt[i];
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
        const int q = tid + i * nt;
        if (q < b) {
            ring_perm[q] = scnt[q];
            ring_idx[q] = sidx[q];
        }
    }
}

void launch_update(const Layout &L, const Buffers &B, int b, int p_new, int p_expired, int init_alive_before,
                   int init_keep, const SlotList &live, const WindowRank &win, int lr, uint32_t gram_mask,
                   int gram_ta, int gram_te, int gram_qmax, int gram_nwaves, hipStream_t st)
{
    const int nchunk = (b + kChunk - 1) / kChunk;
#define MBKK_GO(LDS)                                                                                             \
    hipLaunchKernelGGL(k_group_offsets<LDS>, dim3(1), dim3(1024), 0, st, b, L.k, nchunk, L.C, p_new, p_expired,  \
                       init_alive_before, init_keep, live, win, lr, B.gcnt, B.gbase, B.mind, B.coef, B.cum,      \
                       B.counts,                                                                                 \
                       B.alpha, B.ring_off + (int64_t)p_new * (L.k + 1), B.obj, B.labels, B.rank,                 \
                       B.slot_pts + (int64_t)p_new * L.bmax, B.ring_idx + (int64_t)p_new * L.bmax,               \
                       B.ring_perm + (int64_t)p_new * L.bmax, gram_mask, gram_ta, gram_te, B.ring_off, B.goff, L.pad,  \
                       (int)L.packed, B.seg_next)
    const bool pow2 = (gram_ta & (gram_ta - 1)) == 0 && (gram_te & (gram_te - 1)) == 0;
    if (L.k <= kGroupSmallK && (int64_t)nchunk * L.k <= kGroupLdsMax && L.C <= kGroupSmallC && pow2)
        hipLaunchKernelGGL(k_group_offsets_small, dim3(1), dim3(kGroupThreads), 0, st, b, L.k, nchunk, L.C, p_new,
                           p_expired, init_alive_before, init_keep, live, win, lr, B.gcnt, B.mind, B.coef, B.cum,
                           B.counts, B.alpha, B.ring_off + (int64_t)p_new * (L.k + 1), B.obj, B.labels, B.rank,
                           B.slot_pts + (int64_t)p_new * L.bmax, B.ring_idx + (int64_t)p_new * L.bmax,
                           B.ring_perm + (int64_t)p_new * L.bmax, gram_mask, gram_ta, gram_te, gram_qmax,
                           gram_nwaves, B.ring_off, B.goff, L.pad, (int)L.packed, B.seg_next);
    else if ((int64_t)nchunk * L.k <= kGroupLdsMax)
        MBKK_GO(true);
    else {
        hipLaunchKernelGGL(k_label_bases, dim3((unsigned)((L.k + 63) / 64)), dim3(64), 0, st, L.k, nchunk, B.gcnt,
                           B.gbase, B.counts);
        MBKK_GO(false);
    }
#undef MBKK_GO
}

}  // namespace mbkk
