// Data staging and center bookkeeping kernels of one iteration of the
// truncated mini-batch kernel k-means (Algorithm 2):
//   - ||x||^2 cache, batch staging (gather + FP32 / BF16 hi-lo copies),
//   - support layout of the implicit centers (Eq. 1 as a ring of slots),
//   - the update: deterministic grouping of the batch by center, counts
//     b_i^j, learning rates, coefficient decay by (1 - alpha), truncation,
//   - the FP64 Gram blocks that give <C_j, C_j> incrementally.
#include "kernels.h"

namespace mbkk {

// ---------------------------------------------------------------------------
// ||x||^2 for every row of X, summed in FP64, stored as FP32 (data norms).
// 16 lanes per row.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_row_sqnorm(const float *__restrict__ X, int64_t n, int d,
                                                     int64_t ld, float *__restrict__ sqn)
{
    const int sub = threadIdx.x & 15;
    const int64_t row = (int64_t)blockIdx.x * 16 + (threadIdx.x >> 4);
    if (row >= n)
        return;
    const float *r = X + row * ld;
    double s = 0.0;
    for (int t = sub; t < d; t += 16) {
        double v = r[t];
        s += v * v;
    }
    for (int o = 8; o > 0; o >>= 1)
        s += __shfl_xor(s, o, 16);
    if (sub == 0)
        sqn[row] = (float)s;
}

void launch_row_sqnorm(const float *X, int64_t n, int d, int64_t ld, float *sqn, hipStream_t st)
{
    int64_t blocks = (n + 15) / 16;
    hipLaunchKernelGGL(k_row_sqnorm, dim3((unsigned)blocks), dim3(256), 0, st, X, n, d, ld, sqn);
}

// ---------------------------------------------------------------------------
// Gathers rows X[idx[r]] (or rows of a dense matrix when idx == nullptr) into
// a padded row-major buffer of stride dp (zeros past d), with optional BF16
// hi/lo copies and FP32/FP64 squared norms.  Out-of-range indices read as
// zero rows and raise flags[0]; non-finite values raise flags[1] (when
// check_finite).  One wave per row.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_gather_rows(
    const float *__restrict__ X, int64_t n, int d, int64_t ld, const int32_t *__restrict__ idx,
    int64_t cnt, int dp, float *__restrict__ out32, uint16_t *__restrict__ outhi,
    uint16_t *__restrict__ outlo, float *__restrict__ outsq, double *__restrict__ outsq64,
    int32_t *__restrict__ idx_copy, int32_t *__restrict__ flags, int check_finite)
{
    const int lane = threadIdx.x & 63;
    const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (row >= cnt)
        return;
    int64_t p = idx ? (int64_t)idx[row] : row;
    bool ok = p >= 0 && p < n;
    if (!ok && lane == 0)
        atomicOr(&flags[0], 1);
    if (idx_copy && lane == 0)
        idx_copy[row] = (int32_t)p;
    const float *src = X + (ok ? p : 0) * ld;
    double s = 0.0;
    bool finite = true;
    for (int t = lane; t < dp; t += 64) {
        float v = (ok && t < d) ? src[t] : 0.0f;
        finite &= isfinite(v);
        out32[row * dp + t] = v;
        if (outhi) {
            uint16_t h = f32_to_bf16_rne(v);
            uint16_t l = f32_to_bf16_rne(v - bf16_to_f32(h));
            outhi[row * dp + t] = h;
            outlo[row * dp + t] = l;
        }
        s += (double)v * (double)v;
    }
    if (check_finite && !finite)
        atomicOr(&flags[1], 1);
    for (int o = 32; o > 0; o >>= 1)
        s += __shfl_xor(s, o);
    if (lane == 0) {
        outsq[row] = (float)s;
        if (outsq64)
            outsq64[row] = s;
    }
}

void launch_gather_rows(const float *X, int64_t n, int d, int64_t ld, const int32_t *idx, int64_t cnt,
                        int dp, float *out32, uint16_t *outhi, uint16_t *outlo, float *outsq,
                        double *outsq64, int32_t *idx_copy, int32_t *flags, int check_finite,
                        hipStream_t st)
{
    if (cnt <= 0)
        return;
    int64_t blocks = (cnt + 3) / 4;
    hipLaunchKernelGGL(k_gather_rows, dim3((unsigned)blocks), dim3(256), 0, st, X, n, d, ld, idx, cnt,
                       dp, out32, outhi, outlo, outsq, outsq64, idx_copy, flags, check_finite);
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
__device__ __forceinline__ int seg_len(int j, int k, const int32_t *__restrict__ ring_off, const SlotList &live,
                                       int init_alive)
{
    int len = init_alive;
    for (int s = 0; s < live.n; ++s) {
        const int32_t *o = ring_off + (int64_t)live.r[s] * (k + 1);
        len += o[j + 1] - o[j];
    }
    return len;
}

__global__ __launch_bounds__(256) void k_support_fill(
    int k, int C, int bmax, int pad, int64_t zero_row, const int32_t *__restrict__ ring_off,
    const int32_t *__restrict__ ring_perm, SlotList live, int init_alive, const double *__restrict__ coef,
    const double *__restrict__ G, int32_t *__restrict__ seg_off, int32_t *__restrict__ sup_row,
    float *__restrict__ sup_w, double *__restrict__ sup_w64, int32_t *__restrict__ blk_center,
    double *__restrict__ N)
{
    __shared__ int red[256];
    __shared__ int sh_start;
    const int j = blockIdx.x;
    const int tid = threadIdx.x;
    // exclusive prefix of the padded lengths of centers < j
    int acc = 0;
    for (int q = tid; q < j; q += 256) {
        const int l = seg_len(q, k, ring_off, live, init_alive);
        acc += (l + pad - 1) / pad * pad;
    }
    red[tid] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (tid < s)
            red[tid] += red[tid + s];
        __syncthreads();
    }
    const int len = seg_len(j, k, ring_off, live, init_alive);
    const int plen = (len + pad - 1) / pad * pad;
    if (tid == 0) {
        sh_start = red[0];
        seg_off[j] = red[0];
        if (j == k - 1)
            seg_off[k] = red[0] + plen;
    }
    __syncthreads();
    const int start = sh_start;
    int pos = start;
    if (init_alive) {
        if (tid == 0) {
            const double w = coef[(int64_t)j * C + 0];
            sup_row[pos] = j;
            sup_w[pos] = (float)w;
            sup_w64[pos] = w;
        }
        ++pos;
    }
    for (int s = 0; s < live.n; ++s) {
        const int p = live.r[s];
        const int32_t *o = ring_off + (int64_t)p * (k + 1);
        const int32_t *perm = ring_perm + (int64_t)p * bmax;
        const int a0 = o[j], a1 = o[j + 1];
        const double w = coef[(int64_t)j * C + 1 + p];
        const int64_t row0 = (int64_t)k + (int64_t)p * bmax;
        for (int q = tid; q < a1 - a0; q += 256) {
            sup_row[pos + q] = (int32_t)(row0 + perm[a0 + q]);
            sup_w[pos + q] = (float)w;
            sup_w64[pos + q] = w;
        }
        pos += a1 - a0;
    }
    for (int q = pos + tid; q < start + plen; q += 256) {
        sup_row[q] = (int32_t)zero_row;
        sup_w[q] = 0.0f;
        sup_w64[q] = 0.0;
    }
    if (blk_center) {
        for (int q = start / 32 + tid; q < (start + plen) / 32; q += 256)
            blk_center[q] = j;
    }
    // N_j from the Gram blocks (FP64), in a fixed order
    if (tid == 0) {
        int cols[kMaxSlots + 1];
        int nc = 0;
        if (init_alive)
            cols[nc++] = 0;
        for (int s = 0; s < live.n; ++s)
            cols[nc++] = 1 + live.r[s];
        const double *g = G + (int64_t)j * C * C;
        const double *cf = coef + (int64_t)j * C;
        double nn = 0.0;
        for (int a = 0; a < nc; ++a)
            for (int e = 0; e < nc; ++e)
                nn += cf[cols[a]] * cf[cols[e]] * g[cols[a] * C + cols[e]];
        N[j] = nn;
    }
}

void launch_support_fill(const Layout &L, const Buffers &B, const SlotList &live, int init_alive, hipStream_t st)
{
    hipLaunchKernelGGL(k_support_fill, dim3(L.k), dim3(256), 0, st, L.k, L.C, L.bmax, L.pad, L.PR, B.ring_off,
                       B.ring_perm, live, init_alive, B.coef, B.G, B.seg_off, B.sup_row, B.sup_w, B.sup_w64,
                       L.pad == kMfmaPad ? B.blk_center : nullptr, B.N);
}

// ---------------------------------------------------------------------------
// Gram work items of one slot: center j's grouped positions split into
// chunks of `rows`.  Single workgroup.
// ---------------------------------------------------------------------------
__device__ void build_chunks(int k, int rows, const int32_t *__restrict__ off, int32_t *__restrict__ chunk_off,
                             int32_t *__restrict__ chunk_j, int32_t *__restrict__ chunk_a0,
                             int32_t *__restrict__ chunk_a1, int32_t *__restrict__ nchunks, int *scratch)
{
    // scratch: blockDim.x ints; off must be complete before the call
    __syncthreads();
    const int tid = threadIdx.x, nt = blockDim.x;
    const int per = (k + nt - 1) / nt;
    const int j0 = tid * per, j1 = min(k, j0 + per);
    int local = 0;
    for (int j = j0; j < j1; ++j)
        local += (off[j + 1] - off[j] + rows - 1) / rows;
    scratch[tid] = local;
    __syncthreads();
    for (int s = 1; s < nt; s <<= 1) {
        const int v = tid >= s ? scratch[tid - s] : 0;
        __syncthreads();
        scratch[tid] += v;
        __syncthreads();
    }
    int base = scratch[tid] - local;
    for (int j = j0; j < j1; ++j) {
        chunk_off[j] = base;
        const int a0 = off[j], a1 = off[j + 1];
        for (int a = a0; a < a1; a += rows) {
            chunk_j[base] = j;
            chunk_a0[base] = a;
            chunk_a1[base] = min(a1, a + rows);
            ++base;
        }
    }
    if (tid == nt - 1) {
        chunk_off[k] = scratch[nt - 1];
        *nchunks = scratch[nt - 1];
    }
    __syncthreads();
}

__global__ __launch_bounds__(1024) void k_chunks(int k, int rows, const int32_t *__restrict__ off,
                                                  int32_t *__restrict__ chunk_off, int32_t *__restrict__ chunk_j,
                                                  int32_t *__restrict__ chunk_a0, int32_t *__restrict__ chunk_a1,
                                                  int32_t *__restrict__ nchunks)
{
    __shared__ int scratch[1024];
    build_chunks(k, rows, off, chunk_off, chunk_j, chunk_a0, chunk_a1, nchunks, scratch);
}

void launch_chunks(const Layout &L, const Buffers &B, int p, hipStream_t st)
{
    hipLaunchKernelGGL(k_chunks, dim3(1), dim3(1024), 0, st, L.k, L.gram_rows, B.ring_off + (int64_t)p * (L.k + 1),
                       B.chunk_off, B.chunk_j, B.chunk_a0, B.chunk_a1, B.nchunks);
}

// ---------------------------------------------------------------------------
// Update of Algorithm 2, in three launches that group the batch by center in
// a deterministic, stable order (each center's points in batch order):
//   rank    : per chunk of 256 rows, each row's rank among the equal labels
//             before it, and the chunk's count of every label;
//   offsets : (one workgroup) counts b_i^j, offsets of the centers in the new
//             slot, per-(chunk, label) bases, learning rates alpha, the
//             coefficient update and truncation, the batch objective, the
//             Gram work items;
//   scatter : grouped position of every row = base + rank.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kChunk) void k_group_rank(int b, int k, const int32_t *__restrict__ labels,
                                                        int32_t *__restrict__ rank, int32_t *__restrict__ gcnt)
{
    __shared__ int sl[kChunk];
    const int g = blockIdx.x, tid = threadIdx.x;
    const int p = g * kChunk + tid;
    // labels outside [0, k) are clamped so that every index below stays in range
    const int lab = p < b ? min(max(labels[p], 0), k - 1) : -1;
    sl[tid] = lab;
    int32_t *cnt = gcnt + (int64_t)g * k;
    for (int j = tid; j < k; j += kChunk)
        cnt[j] = 0;
    __syncthreads();
    int r = 0, c = 0;
    for (int t = 0; t < kChunk; ++t) {
        const int v = sl[t];  // wave-uniform address: LDS broadcast
        const int eq = v == lab;
        c += eq;
        r += eq & (t < tid);
    }
    if (p < b) {
        rank[p] = r;
        if (r == c - 1)
            cnt[lab] = c;
    }
}

__global__ __launch_bounds__(1024) void k_group_offsets(
    int b, int k, int nchunk, int C, int p_new, int p_expired, int init_alive_before, int init_keep,
    SlotList live, int lr, int gram_rows, int32_t *__restrict__ gcnt, const float *__restrict__ mind,
    double *__restrict__ coef, double *__restrict__ cum, int32_t *__restrict__ counts,
    double *__restrict__ alpha, int32_t *__restrict__ off, int32_t *__restrict__ chunk_off,
    int32_t *__restrict__ chunk_j, int32_t *__restrict__ chunk_a0, int32_t *__restrict__ chunk_a1,
    int32_t *__restrict__ nchunks, double *__restrict__ obj)
{
    __shared__ int scratch[1024];
    __shared__ double red[1024];
    const int tid = threadIdx.x, nt = blockDim.x;
    const int per = (k + nt - 1) / nt;
    const int j0 = tid * per, j1 = min(k, j0 + per);
    // totals of this thread's labels, block-wide exclusive scan -> offsets
    int local = 0;
    for (int j = j0; j < j1; ++j)
        for (int g = 0; g < nchunk; ++g)
            local += gcnt[(int64_t)g * k + j];
    scratch[tid] = local;
    __syncthreads();
    for (int s = 1; s < nt; s <<= 1) {
        const int v = tid >= s ? scratch[tid - s] : 0;
        __syncthreads();
        scratch[tid] += v;
        __syncthreads();
    }
    int run = scratch[tid] - local;
    for (int j = j0; j < j1; ++j) {
        off[j] = run;
        int gb = run;
        for (int g = 0; g < nchunk; ++g) {
            const int c = gcnt[(int64_t)g * k + j];
            gcnt[(int64_t)g * k + j] = gb;  // base of label j in chunk g
            gb += c;
        }
        const int bj = gb - run;
        run = gb;
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
    }
    if (tid == nt - 1)
        off[k] = b;
    // sum of min distances (FP64), fixed-order tree
    double sm = 0.0;
    for (int p = tid; p < b; p += nt)
        sm += (double)mind[p];
    red[tid] = sm;
    __syncthreads();
    for (int h = nt / 2; h > 0; h >>= 1) {
        if (tid < h)
            red[tid] += red[tid + h];
        __syncthreads();
    }
    if (tid == 0)
        obj[0] = red[0];
    build_chunks(k, gram_rows, off, chunk_off, chunk_j, chunk_a0, chunk_a1, nchunks, scratch);
}

__global__ __launch_bounds__(kChunk) void k_group_scatter(int b, int k, const int32_t *__restrict__ labels,
                                                           const int32_t *__restrict__ rank,
                                                           const int32_t *__restrict__ gbase,
                                                           const int32_t *__restrict__ pts,
                                                           int32_t *__restrict__ ring_idx,
                                                           int32_t *__restrict__ ring_perm)
{
    const int g = blockIdx.x;
    const int p = g * kChunk + threadIdx.x;
    if (p >= b)
        return;
    const int lab = min(max(labels[p], 0), k - 1);
    const int pos = gbase[(int64_t)g * k + lab] + rank[p];
    ring_perm[pos] = p;
    ring_idx[pos] = pts[p];
}

void launch_update(const Layout &L, const Buffers &B, int b, int p_new, int p_expired, int init_alive_before,
                   int init_keep, const SlotList &live, int lr, hipStream_t st)
{
    const int nchunk = (b + kChunk - 1) / kChunk;
    hipLaunchKernelGGL(k_group_rank, dim3(nchunk), dim3(kChunk), 0, st, b, L.k, B.labels, B.rank, B.gcnt);
    hipLaunchKernelGGL(k_group_offsets, dim3(1), dim3(1024), 0, st, b, L.k, nchunk, L.C, p_new, p_expired,
                       init_alive_before, init_keep, live, lr, L.gram_rows, B.gcnt, B.mind, B.coef, B.cum,
                       B.counts, B.alpha, B.ring_off + (int64_t)p_new * (L.k + 1), B.chunk_off, B.chunk_j,
                       B.chunk_a0, B.chunk_a1, B.nchunks, B.obj);
    hipLaunchKernelGGL(k_group_scatter, dim3(nchunk), dim3(kChunk), 0, st, b, L.k, B.labels, B.rank, B.gcnt,
                       B.slot_pts + (int64_t)p_new * L.bmax, B.ring_idx + (int64_t)p_new * L.bmax,
                       B.ring_perm + (int64_t)p_new * L.bmax);
}

// ---------------------------------------------------------------------------
// Gram blocks of slot rr against every live column (FP32 or FP64 kernel
// values, FP64 sums):  for each work item q = (j, grouped positions a0..a1 of
// slot rr) and column c,
//   Gpart[q][c] = sum_{a in q} sum_{e in column c, center j} K(a, e).
// Column 0 is the initial point of center j; column 1+p is slot p.
// Grid: (maxchunks, C); work items past *nchunks exit.  Each workgroup walks
// the column's rows in tiles of 16; a thread owns one (a, e) pair, and both
// row sets are staged through LDS 64 coordinates at a time, so any d works.
// ---------------------------------------------------------------------------
constexpr int kGramTile = 16, kGramK = 64, kGramLd = kGramK + 4;  // 272-byte LDS rows

template <int KIND, typename KT>
__device__ __forceinline__ void gram_acc4(KT &s, const float4 a, const float4 e)
{
    const float av[4] = {a.x, a.y, a.z, a.w}, ev[4] = {e.x, e.y, e.z, e.w};
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const KT x = (KT)av[u], y = (KT)ev[u];
        if constexpr (KIND == MBKK_GAUSS) {
            const KT v = x - y;
            s = fma(v, v, s);
        } else if constexpr (KIND == MBKK_LAPLACE) {
            s += fabs(x - y);
        } else {
            s = fma(x, y, s);
        }
    }
}

template <int KIND, typename KT>
__global__ __launch_bounds__(256) void k_gram(int k, int C, int bmax, int d, int dp, double param, int rr,
                                               uint32_t col_mask, const int32_t *__restrict__ ring_off,
                                               const int32_t *__restrict__ ring_perm,
                                               const float *__restrict__ pool32,
                                               const int32_t *__restrict__ nchunks,
                                               const int32_t *__restrict__ chunk_j,
                                               const int32_t *__restrict__ chunk_a0,
                                               const int32_t *__restrict__ chunk_a1, double *__restrict__ Gpart)
{
    __shared__ __attribute__((aligned(16))) float sa[kGramTile][kGramLd];
    __shared__ __attribute__((aligned(16))) float se[kGramTile][kGramLd];
    __shared__ double red[256];
    const int q = blockIdx.x, c = blockIdx.y, tid = threadIdx.x;
    if (q >= *nchunks)
        return;
    if (!((col_mask >> c) & 1u)) {
        if (tid == 0)
            Gpart[(int64_t)q * C + c] = 0.0;
        return;
    }
    const int j = chunk_j[q], a0 = chunk_a0[q];
    const int na = chunk_a1[q] - a0;
    const int pa = tid >> 4, pe = tid & 15;      // this thread's pair
    const int lr = tid >> 4, lc = (tid & 15) * 4;  // loader: row, 4 columns
    // pool rows of the loader's a-row and of the column's rows
    const int64_t arow = lr < na ? (int64_t)k + (int64_t)rr * bmax + ring_perm[(int64_t)rr * bmax + a0 + lr] : 0;
    int ne;
    int64_t erow0 = 0;
    const int32_t *eperm = nullptr;
    if (c == 0) {
        ne = 1;
        erow0 = j;
    } else {
        const int pc = c - 1;
        const int32_t *o = ring_off + (int64_t)pc * (k + 1);
        ne = o[j + 1] - o[j];
        eperm = ring_perm + (int64_t)pc * bmax + o[j];
        erow0 = (int64_t)k + (int64_t)pc * bmax;
    }
    const KT prm = (KT)param;
    double acc = 0.0;
    for (int et = 0; et < ne; et += kGramTile) {
        const bool eok = et + lr < ne;
        const int64_t erow = eok ? (c == 0 ? erow0 : erow0 + eperm[et + lr]) : 0;
        KT sacc = 0;
        // coordinates past d are zero in the pool, so whole 64-wide chunks
        // can be processed
        for (int t0 = 0; t0 < d; t0 += kGramK) {
            __syncthreads();
            {
                const int col = t0 + lc;
                float4 va = make_float4(0.f, 0.f, 0.f, 0.f), ve = va;
                if (lr < na && col < dp)
                    va = *(const float4 *)(pool32 + arow * dp + col);
                if (eok && col < dp)
                    ve = *(const float4 *)(pool32 + erow * dp + col);
                *(float4 *)&sa[lr][lc] = va;
                *(float4 *)&se[lr][lc] = ve;
            }
            __syncthreads();
#pragma unroll
            for (int t = 0; t < kGramK; t += 4)
                gram_acc4<KIND, KT>(sacc, *(const float4 *)&sa[pa][t], *(const float4 *)&se[pe][t]);
        }
        if (pa < na && et + pe < ne) {
            KT kv;
            if constexpr (KIND == MBKK_GAUSS || KIND == MBKK_LAPLACE)
                kv = (KT)exp(-sacc / prm);
            else if constexpr (KIND == MBKK_LINEAR)
                kv = sacc;
            else
                kv = (sacc + prm) * (sacc + prm);
            acc += (double)kv;
        }
    }
    red[tid] = acc;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (tid < h)
            red[tid] += red[tid + h];
        __syncthreads();
    }
    if (tid == 0)
        Gpart[(int64_t)q * C + c] = red[0];
}

template <typename KT>
static void launch_gram_t(const Layout &L, const Buffers &B, int rr, uint32_t col_mask, int kind, double param,
                          hipStream_t st)
{
    dim3 grid((unsigned)L.maxchunks, L.C);
#define MBKK_GRAM(K)                                                                                             \
    hipLaunchKernelGGL((k_gram<K, KT>), grid, dim3(256), 0, st, L.k, L.C, L.bmax, L.d, L.dp, param, rr, col_mask, \
                       B.ring_off, B.ring_perm, B.pool32, B.nchunks, B.chunk_j, B.chunk_a0, B.chunk_a1, B.Gpart)
    switch (kind) {
    case MBKK_GAUSS: MBKK_GRAM(MBKK_GAUSS); break;
    case MBKK_LAPLACE: MBKK_GRAM(MBKK_LAPLACE); break;
    case MBKK_LINEAR: MBKK_GRAM(MBKK_LINEAR); break;
    default: MBKK_GRAM(MBKK_POLY2); break;
    }
#undef MBKK_GRAM
}

void launch_gram(const Layout &L, const Buffers &B, int rr, uint32_t col_mask, int kind, double param, int fp64,
                 hipStream_t st)
{
    if (fp64)
        launch_gram_t<double>(L, B, rr, col_mask, kind, param, st);
    else
        launch_gram_t<float>(L, B, rr, col_mask, kind, param, st);
}

// Folds the work-item partials of slot rr into G_j[1+rr][c] = G_j[c][1+rr]
// (fixed order over the work items of center j).  One thread per center.
__global__ __launch_bounds__(256) void k_gram_fold(int k, int C, int rr, uint32_t col_mask,
                                                    const int32_t *__restrict__ chunk_off,
                                                    const double *__restrict__ Gpart, double *__restrict__ G)
{
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= k)
        return;
    double *g = G + (int64_t)j * C * C;
    const int q0 = chunk_off[j], q1 = chunk_off[j + 1];
    for (int c = 0; c < C; ++c) {
        if (!((col_mask >> c) & 1u))
            continue;
        double s = 0.0;
        for (int q = q0; q < q1; ++q)
            s += Gpart[(int64_t)q * C + c];
        g[(1 + rr) * C + c] = s;
        g[c * C + 1 + rr] = s;
    }
}

void launch_gram_fold(const Layout &L, const Buffers &B, int rr, uint32_t col_mask, hipStream_t st)
{
    hipLaunchKernelGGL(k_gram_fold, dim3((L.k + 255) / 256), dim3(256), 0, st, L.k, L.C, rr, col_mask,
                       B.chunk_off, B.Gpart, B.G);
}

}  // namespace mbkk
