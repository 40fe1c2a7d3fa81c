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

__device__ __forceinline__ double kfun64(int kind, double param, const float *__restrict__ a,
                                         const float *__restrict__ b, int d)
{
    double s = 0.0;
    if (kind == MBKK_GAUSS) {
        for (int t = 0; t < d; ++t) {
            double v = (double)a[t] - (double)b[t];
            s += v * v;
        }
        return exp(-s / param);
    } else if (kind == MBKK_LAPLACE) {
        for (int t = 0; t < d; ++t)
            s += fabs((double)a[t] - (double)b[t]);
        return exp(-s / param);
    } else if (kind == MBKK_LINEAR) {
        for (int t = 0; t < d; ++t)
            s += (double)a[t] * (double)b[t];
        return s;
    }
    for (int t = 0; t < d; ++t)
        s += (double)a[t] * (double)b[t];
    s += param;
    return s * s;
}

__global__ __launch_bounds__(256) void k_kpp_self(const float *__restrict__ X, int64_t n, int d, int64_t ld,
                                                   int kind, double param, double *__restrict__ kself,
                                                   double *__restrict__ D2)
{
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= n)
        return;
    const float *x = X + p * ld;
    kself[p] = kfun64(kind, param, x, x, d);
    D2[p] = INFINITY;
}

void launch_kpp_self(const Layout &L, const Buffers &B, int kind, double param, hipStream_t st)
{
    hipLaunchKernelGGL(k_kpp_self, dim3((unsigned)((L.n + 255) / 256)), dim3(256), 0, st, B.X, L.n, L.d, B.ld,
                       kind, param, B.kself, B.D2);
}

// D2 <- min(D2, K(p,p) - 2K(p,c) + K(c,c)) with c = picks[r]; block sums.
__global__ __launch_bounds__(kKppBlock) void k_kpp_update(const float *__restrict__ X, int64_t n, int d, int64_t ld,
                                                           int kind, double param, const int32_t *__restrict__ picks,
                                                           int r, const double *__restrict__ kself,
                                                           double *__restrict__ D2, double *__restrict__ bsum)
{
    __shared__ double red[kKppBlock];
    const int tid = threadIdx.x;
    const int64_t p = (int64_t)blockIdx.x * kKppBlock + tid;
    const int64_t c = picks[r];
    double v = 0.0;
    if (p < n) {
        const double dd = kself[p] - 2.0 * kfun64(kind, param, X + p * ld, X + c * ld, d) + kself[c];
        v = fmin(D2[p], dd);
        D2[p] = v;
    }
    red[tid] = v;
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
    if (r > 0)
        hipLaunchKernelGGL(k_kpp_update, dim3((unsigned)nblocks), dim3(kKppBlock), 0, st, B.X, L.n, L.d, B.ld, kind,
                           param, B.picks, r - 1, B.kself, B.D2, B.bsum);
    hipLaunchKernelGGL(k_kpp_select, dim3(1), dim3(1024), 0, st, L.n, nblocks, B.u, r, B.D2, B.bsum, B.picks);
}

}  // namespace mbkk
