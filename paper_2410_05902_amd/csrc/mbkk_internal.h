// Internal declarations of the mbkk library: context layout, launch helpers.
// Not part of the ABI (include/mbkk.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/mbkk.h"

namespace mbkk {

constexpr int kDimAlign = 32;     // pool / batch row stride is d rounded up to this
constexpr int kMfmaPad = 32;      // MFMA path: every center segment is a multiple of 32
constexpr int kMaxWindow = 30;    // ring slots W (G is (W+1)^2 per center)
constexpr int kMaxBatch = 8192;   // b_max; the update sorts (label, position) keys in LDS
constexpr int kGramRowsMax = 16;  // rows of the new slot per Gram work item (fewer for large d)

// Ordered list of ring slots (oldest batch first) that are live.
struct SlotList {
    int n;
    int r[kMaxWindow];
};

// Bit-level bf16 helpers (round to nearest even), shared by the staging
// kernels: hi = bf16(x), lo = bf16(x - hi).
__device__ __forceinline__ uint16_t f32_to_bf16_rne(float x)
{
    uint32_t u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }

struct Buffers {
    // data
    const float *X = nullptr;
    int64_t ld = 0;
    float *sqn = nullptr;        // [n] ||x||^2 (FP32 from an FP64 sum)
    // coordinate pool: rows [0,k) initial points, [k + r*bmax + p] ring slot r
    // position p, row PR = k + W*bmax is all zeros (padding target)
    float *pool32 = nullptr;     // [(PR+1) * dp]
    uint16_t *poolhi = nullptr;  // [(PR+1) * dp]  BF16 forms only
    uint16_t *poollo = nullptr;
    float *poolsq = nullptr;     // [PR+1]
    double *poolsq64 = nullptr;  // [PR+1]
    // staged batch rows
    int32_t *batidx = nullptr;   // [bmax] gathered indices (copy of the caller's)
    float *bat32 = nullptr;      // [bmax * dp]
    uint16_t *bathi = nullptr, *batlo = nullptr;
    float *batsq = nullptr;      // [bmax]
    double *batsq64 = nullptr;   // [bmax]
    // ring of W slots
    int32_t *ring_idx = nullptr; // [W * bmax]
    int32_t *ring_off = nullptr; // [W * (k+1)]
    int32_t *init_idx = nullptr; // [k]
    double *coef = nullptr;      // [k * (W+1)]
    double *cum = nullptr;       // [k]
    double *G = nullptr;         // [k * (W+1) * (W+1)]
    double *N = nullptr;         // [k]
    int32_t *counts = nullptr;   // [k]
    double *alpha = nullptr;     // [k]
    // Gram work items of the newest slot
    int32_t *chunk_j = nullptr, *chunk_a0 = nullptr, *chunk_a1 = nullptr;  // [maxchunks]
    int32_t *chunk_off = nullptr;  // [k+1]
    double *Gpart = nullptr;       // [maxchunks * (W+1)]
    // support of the current centers (padded segments)
    int32_t *seg_off = nullptr;  // [k+1]
    int32_t *sup_row = nullptr;  // [Mcap] pool row
    float *sup_w = nullptr;      // [Mcap]
    double *sup_w64 = nullptr;   // [Mcap]
    int32_t *blk_center = nullptr;  // [Mcap/32]
    // cross-term output and assignment
    void *part = nullptr;        // P[k][bmax] (direct) or per-32-block partials [Mcap/32][bmax]
    int32_t *labels = nullptr;   // [bmax]
    float *mind = nullptr;       // [bmax]
    float *margin = nullptr;     // [bmax]
    int32_t *perm = nullptr;     // [bmax]
    double *obj = nullptr;       // [4] device scalars
    int32_t *flags = nullptr;    // [4] error flags (index, non-finite)
    int32_t *nchunks = nullptr;  // [1]
    // k-means++
    double *D2 = nullptr;        // [n]
    double *kself = nullptr;     // [n]
    double *bsum = nullptr;      // [nblocks]
    int32_t *picks = nullptr;    // [k]
    double *u = nullptr;         // [k]
};

struct Layout {
    int64_t n;
    int d, dp, k, W, bmax, pad;
    int64_t PR;        // pool rows excluding the zero row
    int64_t Mcap;      // max padded support entries (multiple of 128)
    int64_t nblk;      // Mcap / 32
    int gram_rows;     // rows per Gram work item (its rows are staged in LDS)
    int64_t maxchunks; // Gram work items bound
    int64_t kpp_blocks;
    bool bf16;
    size_t bytes;
};

// Pieces of the layout computation and of every launch, implemented in the
// .hip files.
Layout make_layout(const mbkk_config &c);
void carve(const Layout &L, char *base, Buffers &B);

}  // namespace mbkk
