// Kernel k-means++ seeding on the device (FP64).  The paper initialises with
// "the kernel version of k-means++" (Sections 1 and 4), which keeps every
// initial center a single feature vector, hence a convex combination of X.
//   pick 0 : floor(u_0 n)
//   pick r : the first row p whose running sum of D2 (row order) exceeds
//            u_r * sum_p D2(p),  D2(p) = min over chosen c of
//            K(p,p) - 2 K(p,c) + K(c,c);
//            sum = 0 -> floor(u_r n); no crossing (rounding) -> the last p
//            with D2(p) > 0.
// Each round is two launches (D2 update + block sums, selection), with the
// pick kept on the device, so seeding needs no host round trip.
#include "kernels.h"

namespace mbkk {

constexpr int kKppBlock = 256;

// Partial kernel sums over the coordinates t = sub, sub + 16, ... of a row;
// the 16 lanes of a row then combine them and finish K (FP64).
template <int KIND>
__device__ __forceinline__ double kacc64(const float *__restrict__ a, const float *__restrict__ b, int d, int sub)
{
    double s = 0.0;
    for (int t = sub; t < d; t += 16) {
        const double x = (double)a[t], y = (double)b[t];
        if constexpr (KIND == MBKK_GAUSS) {
            const double v = x - y;
            s += v * v;
        } else if constexpr (KIND == MBKK_LAPLACE) {
            s += fabs(x - y);
        } else {
            s += x * y;
        }
    }
    for (int o = 8; o > 0; o >>= 1)
        s += __shfl_xor(s, o, 16);
    return s;
}

template <int KIND>
__device__ __forceinline__ double kfin64(double param, double s)
{
    if constexpr (KIND == MBKK_GAUSS || KIND == MBKK_LAPLACE)
        return exp(-s / param);
    else if constexpr (KIND == MBKK_LINEAR)
        return s;
    else
        return (s + param) * (s + param);
}

// K(p,p) for every row, D2 = +inf.  16 lanes per row.
template <int KIND>
__global__ __launch_bounds__(256) void k_kpp_self(const float *__restrict__ X, int64_t n, int d, int64_t ld,
                                                   double param, double *__restrict__ kself,
                                                   double *__restrict__ D2)
{
    const int sub = threadIdx.x & 15;
    const int64_t p = (int64_t)blockIdx.x * 16 + (threadIdx.x >> 4);
    if (p >= n)
        return;
    const float *x = X + p * ld;
    const double s = kacc64<KIND>(x, x, d, sub);
    if (sub == 0) {
        kself[p] = kfin64<KIND>(param, s);
        D2[p] = INFINITY;
    }
}

void launch_kpp_self(const Layout &L, const Buffers &B, int kind, double param, hipStream_t st)
{
    const dim3 grid((unsigned)((L.n + 15) / 16));
#define MBKK_KSELF(K) \
    hipLaunchKernelGGL(k_kpp_self<K>, grid, dim3(256), 0, st, B.X, L.n, L.d, B.ld, param, B.kself, B.D2)
    switch (kind) {
    case MBKK_GAUSS: MBKK_KSELF(MBKK_GAUSS); break;
    case MBKK_LAPLACE: MBKK_KSELF(MBKK_LAPLACE); break;
    case MBKK_LINEAR: MBKK_KSELF(MBKK_LINEAR); break;
    default: MBKK_KSELF(MBKK_POLY2); break;
    }
#undef MBKK_KSELF
}

// D2 <- min(D2, K(p,p) - 2K(p,c) + K(c,c)) with c = picks[r]; block sums over
// 256 consecutive rows (16 lanes per row, 16 rows at a time).
template <int KIND>
__global__ __launch_bounds__(256) void k_kpp_update(const float *__restrict__ X, int64_t n, int d, int64_t ld,
                                                     double param, const int32_t *__restrict__ picks,
                                                     int r, const double *__restrict__ kself,
                                                     double *__restrict__ D2, double *__restrict__ bsum)
{
    __shared__ double red[kKppBlock];
    const int tid = threadIdx.x, sub = tid & 15, grp = tid >> 4;
    const int64_t c = picks[r];
    const float *xc = X + c * ld;
    const double kcc = kself[c];
    for (int it = 0; it < kKppBlock / 16; ++it) {
        const int local = it * 16 + grp;
        const int64_t p = (int64_t)blockIdx.x * kKppBlock + local;
        double s = 0.0;
        if (p < n)
            s = kacc64<KIND>(X + p * ld, xc, d, sub);
        if (sub == 0) {
            double v = 0.0;
            if (p < n) {
                const double dd = kself[p] - 2.0 * kfin64<KIND>(param, s) + kcc;
                v = fmin(D2[p], dd);
                D2[p] = v;
            }
            red[local] = v;
        }
    }
    __syncthreads();
    for (int h = kKppBlock / 2; h > 0; h >>= 1) {
        if (tid < h)
            red[tid] += red[tid + h];
        __syncthreads();
    }
    if (tid == 0)
        bsum[blockIdx.x] = red[0];
}

// Selection of pick r (single workgroup of 1024 threads).
__global__ __launch_bounds__(1024) void k_kpp_select(int64_t n, int64_t nblocks, const double *__restrict__ u, int r,
                                                      const double *__restrict__ D2, const double *__restrict__ bsum,
                                                      int32_t *__restrict__ picks)
{
    __shared__ double part[1024];
    __shared__ int64_t found;
    const int tid = threadIdx.x;
    if (r == 0) {
        if (tid == 0) {
            int64_t p = (int64_t)floor(u[0] * (double)n);
            picks[0] = (int32_t)(p >= n ? n - 1 : p);
        }
        return;
    }
    const int64_t per = (nblocks + 1023) / 1024;
    const int64_t b0 = tid * per, b1 = min(nblocks, b0 + per);
    double s = 0.0;
    for (int64_t q = b0; q < b1; ++q)
        s += bsum[q];
    part[tid] = s;
    if (tid == 0)
        found = -1;
    __syncthreads();
    // exclusive prefix over threads (sequential by thread 0 keeps a fixed order)
    __shared__ double excl[1024];
    __shared__ double total;
    if (tid == 0) {
        double run = 0.0;
        for (int q = 0; q < 1024; ++q) {
            excl[q] = run;
            run += part[q];
        }
        total = run;
    }
    __syncthreads();
    const double tot = total;
    if (!(tot > 0.0)) {
        if (tid == 0) {
            int64_t p = (int64_t)floor(u[r] * (double)n);
            picks[r] = (int32_t)(p >= n ? n - 1 : p);
        }
        return;
    }
    const double target = u[r] * tot;
    // the thread whose block range contains the crossing walks its blocks, then the rows
    if (excl[tid] <= target && excl[tid] + part[tid] > target) {
        double run = excl[tid];
        for (int64_t q = b0; q < b1; ++q) {
            if (run + bsum[q] > target) {
                const int64_t p0 = q * kKppBlock, p1 = min(n, p0 + kKppBlock);
                int64_t hit = -1, lastpos = -1;
                for (int64_t p = p0; p < p1; ++p) {
                    run += D2[p];
                    if (D2[p] > 0.0)
                        lastpos = p;
                    if (run > target) {
                        hit = p;
                        break;
                    }
                }
                // the block's tree sum and the row-order sum can differ in the
                // last bits: then the block's last row with D2 > 0
                found = hit >= 0 ? hit : lastpos;
                break;
            }
            run += bsum[q];
        }
    }
    __syncthreads();
    if (tid == 0) {
        int64_t p = found;
        if (p < 0) {
            for (int64_t q = n - 1; q >= 0; --q)
                if (D2[q] > 0.0) {
                    p = q;
                    break;
                }
            if (p < 0)
                p = 0;
        }
        picks[r] = (int32_t)p;
    }
}

void launch_kpp_round(const Layout &L, const Buffers &B, int r, int kind, double param, hipStream_t st)
{
    // r == 0: select the first pick; r >= 1: update with pick r-1, then select pick r
    const int64_t nblocks = (L.n + kKppBlock - 1) / kKppBlock;
    if (r > 0) {
#define MBKK_KUPD(K)                                                                                     \
    hipLaunchKernelGGL(k_kpp_update<K>, dim3((unsigned)nblocks), dim3(kKppBlock), 0, st, B.X, L.n, L.d, B.ld, \
                       param, B.picks, r - 1, B.kself, B.D2, B.bsum)
        switch (kind) {
        case MBKK_GAUSS: MBKK_KUPD(MBKK_GAUSS); break;
        case MBKK_LAPLACE: MBKK_KUPD(MBKK_LAPLACE); break;
        case MBKK_LINEAR: MBKK_KUPD(MBKK_LINEAR); break;
        default: MBKK_KUPD(MBKK_POLY2); break;
        }
#undef MBKK_KUPD
    }
    hipLaunchKernelGGL(k_kpp_select, dim3(1), dim3(1024), 0, st, L.n, nblocks, B.u, r, B.D2, B.bsum, B.picks);
}

}  // namespace mbkk
