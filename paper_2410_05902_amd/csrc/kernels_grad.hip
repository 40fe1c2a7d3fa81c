// Differentiation form of the batch objective (Section 3's f_B, Gaussian
// kernel in the bandwidth form K_s(x, y) = exp(-||x - y||^2 / (2 s^2))):
//   f(X_B, s) = (1/b) sum_x [1 - 2 P_j(x) + N_j],  j = j*(x) the argmin label,
//   P_j(x) = sum_{e in C_j} w_e K_s(x, y_e),  N_j = sum_{e, e' in C_j} w_e w_e' K_s(y_e, y_e').
// With the support points y_e and weights w_e held constant and hard labels:
//   df/dx   = (2 / (b s^2)) sum_e w_e K_s(x, y_e) (x - y_e)
//   df/ds   = (1/b) sum_x [-2 sum_e w_e K_s(x, y_e) ||x - y_e||^2 / s^3 + dN_j/ds]
//   dN_j/ds = sum_{e, e'} w_e w_e' K_s(y_e, y_e') ||y_e - y_e'||^2 / s^3.
// Kernel values are recomputed here (nothing of size b x M is stored); the
// arithmetic is FP64 throughout.
#include "dev_common.h"
#include "kernels.h"

namespace mbkk {

// ---------------------------------------------------------------------------
// N_j(s) and dN_j/ds over all ordered pairs of center j's support entries,
// split over kSnSplit workgroups per center (workgroup g takes the a tiles
// g, g + kSnSplit, ...), so that one large center is spread over the chip.
// Each writes its partial sums; k_selfnorm_fold adds them in workgroup order.
// The pairs are taken in tiles of 16 rows a by 64 rows e
// whose coordinates are staged in LDS (128 coordinates per pass), so each
// coordinate is read from global memory once per tile instead of once per
// pair; thread (ta, te) of a tile owns the pairs (ta, te + 16 q), q < 4.
// Every thread sums its pairs in a fixed order, and the tree reduction is
// fixed as well (deterministic).
// ---------------------------------------------------------------------------
struct SelfNormArgs {
    int k, d, dp;
    const int32_t *seg_off, *sup_row;
    const double *sup_w64;
    const float *pool32;
    double inv_kappa;  // 1 / (2 s^2)
    double inv_s3;     // 1 / s^3
    double *part;      // [k][kSnSplit][2]
    double *N, *dN;
};

constexpr int kSnTA = 16, kSnTE = 64, kSnDim = 128;

__global__ __launch_bounds__(256) void k_selfnorm_sigma(const SelfNormArgs A)
{
    __shared__ float sa[kSnTA][kSnDim + 1], se[kSnTE][kSnDim + 1];
    __shared__ double rn[256], rd[256];
    const int j = blockIdx.x, g = blockIdx.y, tid = threadIdx.x;
    const int ta = tid / kSnTA, te = tid % kSnTA;  // a row of the tile, first e row (then +16 q)
    const int s0 = A.seg_off[j], L = A.seg_off[j + 1] - s0;
    double sn = 0.0, sd = 0.0;
    for (int a0 = g * kSnTA; a0 < L; a0 += kSnSplit * kSnTA) {
        for (int e0 = 0; e0 < L; e0 += kSnTE) {
            double d2[4] = {0.0, 0.0, 0.0, 0.0};
            // pool rows are zero from d up to the stride dp, so passes run over dp
            for (int t0 = 0; t0 < A.dp; t0 += kSnDim) {
                const int nt = min(kSnDim, A.dp - t0);
                // this thread's 16-byte chunks of the tiles: all pool-row indices
                // first, then all coordinate loads, so each pass waits on two
                // rounds of independent loads
                constexpr int CPRow = kSnDim / 4, Q = (kSnTA + kSnTE) * CPRow / 256;
                int ridx[Q];
#pragma unroll
                for (int q = 0; q < Q; ++q) {
                    const int i = tid + 256 * q, r = i / CPRow, c4 = i % CPRow;
                    const int row = r < kSnTA ? a0 + r : e0 + (r - kSnTA);
                    ridx[q] = row < L && 4 * c4 < nt ? A.sup_row[s0 + row] : -1;
                }
                f32x4 v[Q];
#pragma unroll
                for (int q = 0; q < Q; ++q) {
                    const int c4 = (tid + 256 * q) % CPRow;
                    const f32x4 z = {0.0f, 0.0f, 0.0f, 0.0f};
                    v[q] = ridx[q] >= 0 ? *(const f32x4 *)(A.pool32 + (int64_t)ridx[q] * A.dp + t0 + 4 * c4) : z;
                }
                __syncthreads();  // the previous pass is done with the tiles
#pragma unroll
                for (int q = 0; q < Q; ++q) {
                    const int i = tid + 256 * q, r = i / CPRow, c4 = i % CPRow;
                    float *dst = r < kSnTA ? &sa[r][4 * c4] : &se[r - kSnTA][4 * c4];
                    dst[0] = v[q][0];
                    dst[1] = v[q][1];
                    dst[2] = v[q][2];
                    dst[3] = v[q][3];
                }
                __syncthreads();
                for (int t = 0; t < nt; ++t) {
                    const double x = (double)sa[ta][t];
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const double v = x - (double)se[te + 16 * q][t];
                        d2[q] = fma(v, v, d2[q]);
                    }
                }
            }
            const int a = a0 + ta;
            const double wa = a < L ? A.sup_w64[s0 + a] : 0.0;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int e = e0 + te + 16 * q;
                const double we = e < L ? A.sup_w64[s0 + e] : 0.0;
                if (wa != 0.0 && we != 0.0) {
                    const double kv = exp(-d2[q] * A.inv_kappa);
                    sn = fma(wa * we, kv, sn);
                    sd = fma(wa * we * kv, d2[q], sd);
                }
            }
        }
    }
    rn[tid] = sn;
    rd[tid] = sd;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (tid < s) {
            rn[tid] += rn[tid + s];
            rd[tid] += rd[tid + s];
        }
        __syncthreads();
    }
    if (tid == 0) {
        A.part[((int64_t)j * kSnSplit + g) * 2] = rn[0];
        A.part[((int64_t)j * kSnSplit + g) * 2 + 1] = rd[0];
    }
}

// N_j and dN_j/ds from the kSnSplit partial sums of center j, in order.
__global__ __launch_bounds__(256) void k_selfnorm_fold(const SelfNormArgs A)
{
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= A.k)
        return;
    double sn = 0.0, sd = 0.0;
    for (int g = 0; g < kSnSplit; ++g) {
        sn += A.part[((int64_t)j * kSnSplit + g) * 2];
        sd += A.part[((int64_t)j * kSnSplit + g) * 2 + 1];
    }
    A.N[j] = sn;
    A.dN[j] = sd * A.inv_s3;
}

void launch_selfnorm_sigma(const Layout &L, const Buffers &B, double sigma, double *N, double *dN, hipStream_t st)
{
    SelfNormArgs A;
    A.k = L.k;
    A.d = L.d;
    A.dp = L.dp;
    A.seg_off = B.seg_off;
    A.sup_row = B.sup_row;
    A.sup_w64 = B.sup_w64;
    A.pool32 = B.pool32;
    A.inv_kappa = 1.0 / (2.0 * sigma * sigma);
    A.inv_s3 = 1.0 / (sigma * sigma * sigma);
    A.part = B.sn_part;
    A.N = N;
    A.dN = dN;
    hipLaunchKernelGGL(k_selfnorm_sigma, dim3((unsigned)L.k, kSnSplit), dim3(256), 0, st, A);
    hipLaunchKernelGGL(k_selfnorm_fold, dim3((unsigned)((L.k + 255) / 256)), dim3(256), 0, st, A);
}

// ---------------------------------------------------------------------------
// Per-row gradient: one wave per batch row x, lane l holds coordinates
// l + 64 c (c < CH) of x and of the accumulated sum_e w_e K (x - y_e); each
// support entry of the row's center costs one wave reduction of ||x - y_e||^2.
// Writes dX (scaled) and the row's term of df/ds.
// ---------------------------------------------------------------------------
struct GradRowArgs {
    int b, d, dp, k;
    const float *xb;  // [b x d] dense
    const int32_t *labels;
    const int32_t *seg_off, *sup_row;
    const double *sup_w64;
    const float *pool32;
    const double *dN;
    double inv_kappa, inv_s3, cx, cs;  // cx = 2 g / (b s^2), cs = g / b
    float *dX;
    double *rowds;   // [b]
    int32_t *flags;  // flags[2]: a label outside [0, k)
};

template <int CH>
__global__ __launch_bounds__(256) void k_grad_rows(const GradRowArgs A)
{
    const int lane = threadIdx.x & 63;
    const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (row >= A.b)
        return;
    const int j = A.labels[row];
    if (j < 0 || j >= A.k) {
        if (lane == 0) {
            atomicOr(&A.flags[2], 1);
            A.rowds[row] = 0.0;
        }
        for (int t = lane; t < A.d; t += 64)
            A.dX[(int64_t)row * A.d + t] = 0.0f;
        return;
    }
    double x[CH], acc[CH];
#pragma unroll
    for (int c = 0; c < CH; ++c) {
        const int t = lane + 64 * c;
        x[c] = t < A.d ? (double)A.xb[(int64_t)row * A.d + t] : 0.0;
        acc[c] = 0.0;
    }
    double q = 0.0;
    // U entries at a time: their loads and wave reductions are independent
    // and overlap; the sums still take the entries in order, one by one
    constexpr int U = 4;
    const int s1 = A.seg_off[j + 1];
    for (int s = A.seg_off[j]; s < s1; s += U) {
        double w[U], part[U], diff[U][CH];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            w[u] = s + u < s1 ? A.sup_w64[s + u] : 0.0;
            part[u] = 0.0;
            const float *y = A.pool32 + (int64_t)A.sup_row[s + u < s1 ? s + u : s] * A.dp;
#pragma unroll
            for (int c = 0; c < CH; ++c) {
                const int t = lane + 64 * c;
                diff[u][c] = t < A.d ? x[c] - (double)y[t] : 0.0;
                part[u] = fma(diff[u][c], diff[u][c], part[u]);
            }
        }
        for (int o = 32; o > 0; o >>= 1)
#pragma unroll
            for (int u = 0; u < U; ++u)
                part[u] += __shfl_xor(part[u], o);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (w[u] == 0.0)
                continue;  // (wave uniform)
            const double wk = w[u] * exp(-part[u] * A.inv_kappa);
#pragma unroll
            for (int c = 0; c < CH; ++c)
                acc[c] = fma(wk, diff[u][c], acc[c]);
            q = fma(wk, part[u], q);
        }
    }
#pragma unroll
    for (int c = 0; c < CH; ++c) {
        const int t = lane + 64 * c;
        if (t < A.d)
            A.dX[(int64_t)row * A.d + t] = (float)(A.cx * acc[c]);
    }
    if (lane == 0)
        A.rowds[row] = A.cs * (-2.0 * q * A.inv_s3 + A.dN[j]);
}

// Sum of the per-row terms in a fixed order (one workgroup).
__global__ __launch_bounds__(1024) void k_sum_rows(const double *v, int n, double *out)
{
    __shared__ double r[1024];
    const int tid = threadIdx.x;
    double s = 0.0;
    for (int i = tid; i < n; i += 1024)
        s += v[i];
    r[tid] = s;
    __syncthreads();
    for (int o = 512; o > 0; o >>= 1) {
        if (tid < o)
            r[tid] += r[tid + o];
        __syncthreads();
    }
    if (tid == 0)
        *out = r[0];
}

int grad_max_dim() { return 64 * 16; }

void launch_grad_rows(const Layout &L, const Buffers &B, const float *xb, int b, double sigma, const int32_t *labels,
                      double g, const double *dN, float *dX, double *rowds, double *out, hipStream_t st)
{
    GradRowArgs A;
    A.b = b;
    A.d = L.d;
    A.dp = L.dp;
    A.k = L.k;
    A.xb = xb;
    A.labels = labels;
    A.seg_off = B.seg_off;
    A.sup_row = B.sup_row;
    A.sup_w64 = B.sup_w64;
    A.pool32 = B.pool32;
    A.dN = dN;
    A.inv_kappa = 1.0 / (2.0 * sigma * sigma);
    A.inv_s3 = 1.0 / (sigma * sigma * sigma);
    A.cx = 2.0 * g / ((double)b * sigma * sigma);
    A.cs = g / (double)b;
    A.dX = dX;
    A.rowds = rowds;
    A.flags = B.flags;
    const dim3 grid((unsigned)((b + 3) / 4));
    const int ch = (L.d + 63) / 64;
    if (ch <= 1)
        hipLaunchKernelGGL(k_grad_rows<1>, grid, dim3(256), 0, st, A);
    else if (ch <= 2)
        hipLaunchKernelGGL(k_grad_rows<2>, grid, dim3(256), 0, st, A);
    else if (ch <= 4)
        hipLaunchKernelGGL(k_grad_rows<4>, grid, dim3(256), 0, st, A);
    else if (ch <= 8)
        hipLaunchKernelGGL(k_grad_rows<8>, grid, dim3(256), 0, st, A);
    else
        hipLaunchKernelGGL(k_grad_rows<16>, grid, dim3(256), 0, st, A);
    hipLaunchKernelGGL(k_sum_rows, dim3(1), dim3(1024), 0, st, (const double *)rowds, b, out);
}

}  // namespace mbkk
