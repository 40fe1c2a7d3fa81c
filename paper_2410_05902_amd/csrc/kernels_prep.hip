// Data staging and center bookkeeping kernels of one iteration of the
// truncated mini-batch kernel k-means (Algorithm 2):
//   - ||x||^2 cache, batch staging (gather + FP32 / BF16 hi-lo copies),
//   - support layout of the implicit centers (Eq. 1 as a ring of W slots),
//   - the update: grouping of the batch by center, counts b_i^j, learning
//     rates, coefficient decay by (1 - alpha) and truncation,
//   - the FP64 Gram blocks that give <C_j, C_j> incrementally.
#include "kernels.h"

namespace mbkk {

// ---------------------------------------------------------------------------
// ||x||^2 for every row of X, summed in FP64, stored as FP32 (data norms).
// One wave per row.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_row_sqnorm(const float *__restrict__ X, int64_t n, int d,
                                                     int64_t ld, float *__restrict__ sqn)
{
    const int lane = threadIdx.x & 63;
    const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (row >= n)
        return;
    const float *r = X + row * ld;
    double s = 0.0;
    for (int t = lane; t < d; t += 64) {
        double v = r[t];
        s += v * v;
    }
    for (int o = 32; o > 0; o >>= 1)
        s += __shfl_xor(s, o);
    if (lane == 0)
        sqn[row] = (float)s;
}

void launch_row_sqnorm(const float *X, int64_t n, int d, int64_t ld, float *sqn, hipStream_t st)
{
    int64_t blocks = (n + 3) / 4;
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
// Initial centers: pool rows [0,k) <- X[idx], coef[j][0] = 1, other
// coefficients 0, running counts 0, G[j][0][0] = K(x_j, x_j).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_init_state(int k, int W, int kind, double param, int d,
                                                     int dp, const float *__restrict__ pool32,
                                                     double *__restrict__ coef, double *__restrict__ cum,
                                                     double *__restrict__ G, int fp64)
{
    int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= k)
        return;
    const int C = W + 1;
    for (int c = 0; c < C; ++c)
        coef[(int64_t)j * C + c] = c == 0 ? 1.0 : 0.0;
    cum[j] = 0.0;
    double *g = G + (int64_t)j * C * C;
    for (int c = 0; c < C * C; ++c)
        g[c] = 0.0;
    const float *x = pool32 + (int64_t)j * dp;
    g[0] = fp64 ? kernel_value<double>(kind, param, x, x, d)
                : (double)kernel_value<float>(kind, (float)param, x, x, d);
}

void launch_init_state(int k, int W, int kind, double param, int d, int dp, const float *pool32,
                       double *coef, double *cum, double *G, int fp64, hipStream_t st)
{
    hipLaunchKernelGGL(k_init_state, dim3((k + 255) / 256), dim3(256), 0, st, k, W, kind, param, d, dp,
                       pool32, coef, cum, G, fp64);
}

// ---------------------------------------------------------------------------
// Support layout of C_i (one workgroup per center j).  Center j's segment is
// [seg_off[j], seg_off[j+1]): its initial point (while alive), then the
// points of every live ring slot, oldest batch first, padded with the zero
// pool row to a multiple of `pad`.  Each entry carries its pool row and its
// weight coef[j][column].  The workgroup also computes
//   N_j = <C_j, C_j> = sum_{c,c'} coef[j][c] coef[j][c'] G_j[c][c']
// over the live columns (FP64).
// ---------------------------------------------------------------------------
__device__ __forceinline__ int seg_len(int j, int k, int bmax, const int32_t *__restrict__ ring_off,
                                       const SlotList &live, int init_alive)
{
    int len = init_alive;
    for (int s = 0; s < live.n; ++s) {
        const int32_t *o = ring_off + (int64_t)live.r[s] * (k + 1);
        len += o[j + 1] - o[j];
    }
    return len;
}

__global__ __launch_bounds__(256) void k_support_fill(
    int k, int W, int bmax, int pad, int64_t zero_row, const int32_t *__restrict__ ring_off,
    SlotList live, int init_alive, const double *__restrict__ coef, const double *__restrict__ G,
    int32_t *__restrict__ seg_off, int32_t *__restrict__ sup_row, float *__restrict__ sup_w,
    double *__restrict__ sup_w64, int32_t *__restrict__ blk_center, double *__restrict__ N)
{
    __shared__ int red[256];
    __shared__ int sh_start;
    const int j = blockIdx.x;
    const int tid = threadIdx.x;
    // exclusive prefix of the padded lengths of centers < j
    int acc = 0;
    for (int q = tid; q < j; q += 256) {
        int l = seg_len(q, k, bmax, ring_off, live, init_alive);
        acc += (l + pad - 1) / pad * pad;
    }
    red[tid] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (tid < s)
            red[tid] += red[tid + s];
        __syncthreads();
    }
    const int len = seg_len(j, k, bmax, ring_off, live, init_alive);
    const int plen = (len + pad - 1) / pad * pad;
    if (tid == 0) {
        sh_start = red[0];
        seg_off[j] = red[0];
        if (j == k - 1)
            seg_off[k] = red[0] + plen;
    }
    __syncthreads();
    const int start = sh_start;
    const int C = W + 1;
    // entries
    int pos = start;
    if (init_alive) {
        if (tid == 0) {
            double w = coef[(int64_t)j * C + 0];
            sup_row[pos] = j;
            sup_w[pos] = (float)w;
            sup_w64[pos] = w;
        }
        ++pos;
    }
    for (int s = 0; s < live.n; ++s) {
        const int r = live.r[s];
        const int32_t *o = ring_off + (int64_t)r * (k + 1);
        const int a0 = o[j], a1 = o[j + 1];
        const double w = coef[(int64_t)j * C + 1 + r];
        for (int q = tid; q < a1 - a0; q += 256) {
            sup_row[pos + q] = (int32_t)(k + (int64_t)r * bmax + a0 + q);
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
        int cols[kMaxWindow + 1];
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

void launch_support_fill(const Layout &L, const Buffers &B, const SlotList &live, int init_alive,
                         int pad, hipStream_t st)
{
    hipLaunchKernelGGL(k_support_fill, dim3(L.k), dim3(256), 0, st, L.k, L.W, L.bmax, pad, L.PR,
                       B.ring_off, live, init_alive, B.coef, B.G, B.seg_off, B.sup_row, B.sup_w, B.sup_w64,
                       pad == kMfmaPad ? B.blk_center : nullptr, B.N);
}

// ---------------------------------------------------------------------------
// Gram work items of one ring slot r: center j's rows of slot r split into
// chunks of `rows` rows.  Single workgroup; shared by the update kernel.
// ---------------------------------------------------------------------------
__device__ void build_chunks(int k, int rows, const int32_t *__restrict__ off, int32_t *__restrict__ chunk_off,
                             int32_t *__restrict__ chunk_j, int32_t *__restrict__ chunk_a0,
                             int32_t *__restrict__ chunk_a1, int32_t *__restrict__ nchunks, int *scratch)
{
    // scratch: blockDim.x ints
    const int tid = threadIdx.x, nt = blockDim.x;
    const int per = (k + nt - 1) / nt;
    const int j0 = tid * per, j1 = min(k, j0 + per);
    int local = 0;
    for (int j = j0; j < j1; ++j)
        local += (off[j + 1] - off[j] + rows - 1) / rows;
    scratch[tid] = local;
    __syncthreads();
    // inclusive scan (Hillis-Steele) over threads
    for (int s = 1; s < nt; s <<= 1) {
        int v = tid >= s ? scratch[tid - s] : 0;
        __syncthreads();
        scratch[tid] += v;
        __syncthreads();
    }
    int base = scratch[tid] - local;
    for (int j = j0; j < j1; ++j) {
        chunk_off[j] = base;
        int a0 = off[j], a1 = off[j + 1];
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

void launch_chunks(const Layout &L, const Buffers &B, int r, hipStream_t st)
{
    hipLaunchKernelGGL(k_chunks, dim3(1), dim3(1024), 0, st, L.k, L.gram_rows, B.ring_off + (int64_t)r * (L.k + 1),
                       B.chunk_off, B.chunk_j, B.chunk_a0, B.chunk_a1, B.nchunks);
}

// ---------------------------------------------------------------------------
// Update of Algorithm 2 (single workgroup of 1024 threads):
//  1. group the batch by label: sort keys (label << 14 | position), a bitonic
//     sort in LDS, so each center's points keep batch order;
//  2. offsets of every center in the new slot, counts b_i^j;
//  3. learning rates alpha (beta: sqrt(b_i^j/b), full, or count-based);
//  4. coefficients: every live term times (1 - alpha); the new slot gets
//     alpha / b_i^j per point (0 for an empty cluster); the initial term is
//     dropped once i > W; the expired slot is the one overwritten;
//  5. the new slot's point indices, the permutation for the coordinate copy,
//     the Gram work items, and sum of the batch min-distances (FP64).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void k_update(
    int b, int k, int W, int r_new, int init_alive_before, int init_keep, SlotList live, int lr, int gram_rows,
    const int32_t *__restrict__ labels, const int32_t *__restrict__ batidx, const float *__restrict__ mind,
    int32_t *__restrict__ ring_idx, int32_t *__restrict__ ring_off, int bmax, double *__restrict__ coef,
    double *__restrict__ cum, int32_t *__restrict__ counts, double *__restrict__ alpha,
    int32_t *__restrict__ perm, int32_t *__restrict__ chunk_off, int32_t *__restrict__ chunk_j,
    int32_t *__restrict__ chunk_a0, int32_t *__restrict__ chunk_a1, int32_t *__restrict__ nchunks,
    double *__restrict__ obj)
{
    extern __shared__ uint32_t keys[];  // [P2] followed by 1024 ints of scratch
    const int tid = threadIdx.x, nt = blockDim.x;
    int P2 = 1;
    while (P2 < b)
        P2 <<= 1;
    int *scratch = (int *)(keys + P2);
    for (int p = tid; p < P2; p += nt)
        keys[p] = p < b ? (((uint32_t)labels[p]) << 14) | (uint32_t)p : 0xFFFFFFFFu;
    __syncthreads();
    // bitonic sort, ascending
    for (int size = 2; size <= P2; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int p = tid; p < P2 / 2; p += nt) {
                int lo = 2 * p - (p & (stride - 1));
                int hi = lo + stride;
                bool up = ((lo & size) == 0);
                uint32_t a = keys[lo], c = keys[hi];
                if ((a > c) == up) {
                    keys[lo] = c;
                    keys[hi] = a;
                }
            }
            __syncthreads();
        }
    }
    int32_t *off = ring_off + (int64_t)r_new * (k + 1);
    int32_t *slot = ring_idx + (int64_t)r_new * bmax;
    for (int p = tid; p < b; p += nt) {
        uint32_t key = keys[p];
        int lab = (int)(key >> 14);
        int pos = (int)(key & 0x3FFFu);
        perm[p] = pos;
        slot[p] = batidx[pos];
        int prev = p == 0 ? -1 : (int)(keys[p - 1] >> 14);
        for (int j = prev + 1; j <= lab; ++j)
            off[j] = p;
        if (p == b - 1)
            for (int j = lab + 1; j <= k; ++j)
                off[j] = b;
    }
    __syncthreads();
    const int C = W + 1;
    for (int j = tid; j < k; j += nt) {
        int bj = off[j + 1] - off[j];
        counts[j] = bj;
        double a;
        if (lr == MBKK_LR_FULL)
            a = bj > 0 ? 1.0 : 0.0;
        else if (lr == MBKK_LR_SKLEARN) {
            double c = cum[j] + (double)bj;
            cum[j] = c;
            a = bj > 0 ? (double)bj / c : 0.0;
        } else
            a = sqrt((double)bj / (double)b);
        alpha[j] = a;
        double *cf = coef + (int64_t)j * C;
        if (init_alive_before)
            cf[0] *= (1.0 - a);
        for (int s = 0; s < live.n; ++s)
            cf[1 + live.r[s]] *= (1.0 - a);
        cf[1 + r_new] = bj > 0 ? a / (double)bj : 0.0;
        if (!init_keep)
            cf[0] = 0.0;
    }
    // sum of min distances (FP64), fixed-order tree
    double s = 0.0;
    for (int p = tid; p < b; p += nt)
        s += (double)mind[p];
    __shared__ double red[1024];
    red[tid] = s;
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

void launch_update(const Layout &L, const Buffers &B, int b, int r_new, int init_alive_before,
                   int init_keep, const SlotList &live, int lr, hipStream_t st)
{
    int P2 = 1;
    while (P2 < b)
        P2 <<= 1;
    size_t shmem = (size_t)P2 * 4 + 1024 * 4;
    hipLaunchKernelGGL(k_update, dim3(1), dim3(1024), shmem, st, b, L.k, L.W, r_new, init_alive_before,
                       init_keep, live, lr, L.gram_rows, B.labels, B.batidx, B.mind, B.ring_idx, B.ring_off, L.bmax,
                       B.coef, B.cum, B.counts, B.alpha, B.perm, B.chunk_off, B.chunk_j, B.chunk_a0,
                       B.chunk_a1, B.nchunks, B.obj);
}

// ---------------------------------------------------------------------------
// Copies staged batch rows into ring slot r in grouped order:
// pool row k + r*bmax + p <- batch row perm[p].  One wave per row.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_slot_copy(int b, int dp, int64_t row0, const int32_t *__restrict__ perm,
                                                    const float *__restrict__ bat32, const uint16_t *__restrict__ bathi,
                                                    const uint16_t *__restrict__ batlo, const float *__restrict__ batsq,
                                                    const double *__restrict__ batsq64, float *__restrict__ pool32,
                                                    uint16_t *__restrict__ poolhi, uint16_t *__restrict__ poollo,
                                                    float *__restrict__ poolsq, double *__restrict__ poolsq64)
{
    const int lane = threadIdx.x & 63;
    const int p = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (p >= b)
        return;
    const int src = perm[p];
    const int64_t dst = row0 + p;
    for (int t = lane; t < dp; t += 64) {
        pool32[dst * dp + t] = bat32[(int64_t)src * dp + t];
        if (poolhi) {
            poolhi[dst * dp + t] = bathi[(int64_t)src * dp + t];
            poollo[dst * dp + t] = batlo[(int64_t)src * dp + t];
        }
    }
    if (lane == 0) {
        poolsq[dst] = batsq[src];
        poolsq64[dst] = batsq64[src];
    }
}

void launch_slot_copy(const Layout &L, const Buffers &B, int b, int r, hipStream_t st)
{
    hipLaunchKernelGGL(k_slot_copy, dim3((b + 3) / 4), dim3(256), 0, st, b, L.dp, (int64_t)L.k + (int64_t)r * L.bmax,
                       B.perm, B.bat32, B.bathi, B.batlo, B.batsq, B.batsq64, B.pool32, B.poolhi, B.poollo,
                       B.poolsq, B.poolsq64);
}

// ---------------------------------------------------------------------------
// Pool rows of a ring slot straight from X (set_state): pool row
// k + r*bmax + p <- X[ring_idx[r][p]].
// ---------------------------------------------------------------------------
void launch_pool_slot_from_X(const Layout &L, const Buffers &B, int r, int cnt, hipStream_t st)
{
    const int64_t row0 = (int64_t)L.k + (int64_t)r * L.bmax;
    launch_gather_rows(B.X, L.n, L.d, B.ld, B.ring_idx + (int64_t)r * L.bmax, cnt, L.dp,
                       B.pool32 + row0 * L.dp, B.poolhi ? B.poolhi + row0 * L.dp : nullptr,
                       B.poollo ? B.poollo + row0 * L.dp : nullptr, B.poolsq + row0, B.poolsq64 + row0,
                       nullptr, B.flags, 0, st);
}

// ---------------------------------------------------------------------------
// Gram blocks of ring slot rr against every live column (FP32 or FP64 kernel
// values, FP64 sums):  for each work item q = (j, rows a0..a1 of slot rr) and
// column c,  Gpart[q][c] = sum_{a in q} sum_{e in column c, center j} K(a, e).
// Column 0 is the initial point of center j; column 1+r is slot r.
// Grid: (maxchunks, W+1).  Work items past *nchunks exit.
// ---------------------------------------------------------------------------
template <typename KT>
__global__ __launch_bounds__(256) void k_gram(int k, int W, int bmax, int d, int dp, int kind, double param,
                                               int rr, uint32_t col_mask, const int32_t *__restrict__ ring_off,
                                               const float *__restrict__ pool32,
                                               const int32_t *__restrict__ nchunks,
                                               const int32_t *__restrict__ chunk_j,
                                               const int32_t *__restrict__ chunk_a0,
                                               const int32_t *__restrict__ chunk_a1, double *__restrict__ Gpart)
{
    extern __shared__ float arows[];  // [gram_rows * dp]
    __shared__ double red[256];
    const int q = blockIdx.x, c = blockIdx.y, tid = threadIdx.x;
    if (q >= *nchunks)
        return;
    const int C = W + 1;
    if (!((col_mask >> c) & 1u)) {
        if (tid == 0)
            Gpart[(int64_t)q * C + c] = 0.0;
        return;
    }
    const int j = chunk_j[q], a0 = chunk_a0[q], a1 = chunk_a1[q];
    const int na = a1 - a0;
    const int64_t arow0 = (int64_t)k + (int64_t)rr * bmax + a0;
    for (int t = tid; t < na * dp; t += 256)
        arows[t] = pool32[arow0 * dp + t];
    int64_t e0;
    int ne;
    if (c == 0) {
        e0 = j;
        ne = 1;
    } else {
        const int32_t *o = ring_off + (int64_t)(c - 1) * (k + 1);
        e0 = (int64_t)k + (int64_t)(c - 1) * bmax + o[j];
        ne = o[j + 1] - o[j];
    }
    __syncthreads();
    const KT prm = (KT)param;
    double s = 0.0;
    for (int pr = tid; pr < na * ne; pr += 256) {
        const int a = pr / ne, e = pr % ne;
        s += (double)kernel_value<KT>(kind, prm, arows + a * dp, pool32 + (e0 + e) * dp, d);
    }
    red[tid] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (tid < h)
            red[tid] += red[tid + h];
        __syncthreads();
    }
    if (tid == 0)
        Gpart[(int64_t)q * C + c] = red[0];
}

void launch_gram(const Layout &L, const Buffers &B, int rr, uint32_t col_mask, int kind, double param,
                 int fp64, hipStream_t st)
{
    dim3 grid((unsigned)L.maxchunks, L.W + 1);
    size_t shmem = (size_t)L.gram_rows * L.dp * sizeof(float);
    if (fp64)
        hipLaunchKernelGGL(k_gram<double>, grid, dim3(256), shmem, st, L.k, L.W, L.bmax, L.d, L.dp, kind, param,
                           rr, col_mask, B.ring_off, B.pool32, B.nchunks, B.chunk_j, B.chunk_a0, B.chunk_a1,
                           B.Gpart);
    else
        hipLaunchKernelGGL(k_gram<float>, grid, dim3(256), shmem, st, L.k, L.W, L.bmax, L.d, L.dp, kind, param,
                           rr, col_mask, B.ring_off, B.pool32, B.nchunks, B.chunk_j, B.chunk_a0, B.chunk_a1,
                           B.Gpart);
}

// Folds the work-item partials of slot rr into G_j[1+rr][c] = G_j[c][1+rr]
// (fixed order over the work items of center j).  One thread per center.
__global__ __launch_bounds__(256) void k_gram_fold(int k, int W, int rr, uint32_t col_mask,
                                                    const int32_t *__restrict__ chunk_off,
                                                    const double *__restrict__ Gpart, double *__restrict__ G)
{
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= k)
        return;
    const int C = W + 1;
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
    hipLaunchKernelGGL(k_gram_fold, dim3((L.k + 255) / 256), dim3(256), 0, st, L.k, L.W, rr, col_mask,
                       B.chunk_off, B.Gpart, B.G);
}

}  // namespace mbkk
