// Contingency table of two labelings of the same rows, the input of the two
// agreement scores reported in Section 6 (adjusted Rand index, normalised
// mutual information): n_ij = number of rows r with labels[r] = i and
// truth[r] = j.  Counts are exact (integer atomics), so the table does not
// depend on the launch shape or the order of the rows.
#include "kernels.h"

namespace mbkk {

constexpr int kContWG = 256;
constexpr int kContLdsCells = 32768;  // tables up to this many cells are counted per workgroup in LDS (128 KB)
constexpr int kContRowsPerWG = 8192;  // rows per workgroup before the grid reaches its cap
constexpr int kContMaxWGs = 1024;

// LDS: each workgroup counts its rows into a private table, then adds the
// non-zero cells to the global table; else every row adds to the global table.
// A label outside [0, k) or truth outside [0, c) raises flags[2] and the row
// is not counted.
template <bool LDS>
__global__ __launch_bounds__(kContWG) void k_contingency(const int32_t *__restrict__ lab,
                                                         const int32_t *__restrict__ tru, int64_t m, int k, int c,
                                                         unsigned long long *__restrict__ table, int32_t *flags)
{
    extern __shared__ unsigned int h[];
    const int cells = k * c;
    if constexpr (LDS) {
        for (int q = threadIdx.x; q < cells; q += kContWG)
            h[q] = 0u;
        __syncthreads();
    }
    int bad = 0;
    const int64_t stride = (int64_t)gridDim.x * kContWG;
    for (int64_t r = (int64_t)blockIdx.x * kContWG + threadIdx.x; r < m; r += stride) {
        const int i = lab[r], j = tru[r];
        if ((unsigned)i >= (unsigned)k || (unsigned)j >= (unsigned)c) {
            bad = 1;
            continue;
        }
        if constexpr (LDS)
            atomicAdd(&h[i * c + j], 1u);
        else
            atomicAdd(&table[(int64_t)i * c + j], 1ull);
    }
    if (bad)
        atomicOr(&flags[2], 1);
    if constexpr (LDS) {
        __syncthreads();
        for (int q = threadIdx.x; q < cells; q += kContWG)
            if (h[q])
                atomicAdd(&table[q], (unsigned long long)h[q]);
    }
}

void launch_contingency(const int32_t *labels, const int32_t *truth, int64_t m, int k, int c, int64_t *table,
                        int32_t *flags, hipStream_t st)
{
    int64_t g = (m + kContRowsPerWG - 1) / kContRowsPerWG;
    g = g < 1 ? 1 : (g > kContMaxWGs ? kContMaxWGs : g);
    auto *t = reinterpret_cast<unsigned long long *>(table);
    const int64_t cells = (int64_t)k * c;
    if (cells <= kContLdsCells)
        hipLaunchKernelGGL(k_contingency<true>, dim3((unsigned)g), dim3(kContWG), (size_t)cells * 4, st, labels,
                           truth, m, k, c, t, flags);
    else
        hipLaunchKernelGGL(k_contingency<false>, dim3((unsigned)g), dim3(kContWG), 0, st, labels, truth, m, k, c,
                           t, flags);
}

}  // namespace mbkk
