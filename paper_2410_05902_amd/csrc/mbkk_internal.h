// Internal declarations of the mbkk library: context layout, launch helpers.
// Not part of the ABI (include/mbkk.h is).
//
// Center representation (Eq. 1, sliding window): the points of each of the
// last W batches are kept in a ring of P = W + 1 physical slots; batch l lives
// in slot (l - 1) mod P.  Before iteration i the live slots hold batches
// max(1, i-W) .. i-1, so slot (i - 1) mod P is free and batch i is staged
// straight into it.  Within a slot the rows stay in batch order; the grouping
// by center is a permutation (ring_perm) plus per-center offsets (ring_off).
// Coefficients and Gram blocks are indexed by column c: 0 = initial point,
// 1 + p = physical slot p.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/mbkk.h"

namespace mbkk {

constexpr int kDimAlign = 32;     // pool row stride is d rounded up to this
constexpr int kMfmaPad = 32;      // MFMA path: every center segment is a multiple of 32
constexpr int kMaxWindow = 30;    // W; physical slots P = W + 1
constexpr int kMaxSlots = kMaxWindow + 1;
constexpr int kMaxBatch = 8192;   // b_max
constexpr int kChunk = 64;        // batch rows per grouping chunk (one scoring workgroup)
// batch-stationary MFMA cross kernel: workgroups per compute unit (waves per SIMD)
constexpr int kBsOcc = 1;
constexpr int kNumCU = 256;
constexpr int kDirectWGs = 2048;  // workgroups of the direct (VALU) cross kernel: ranges x row tiles (8 waves per SIMD)
constexpr int kSnSplit = 64;      // workgroups per center of the self norms at a bandwidth (differentiation form)
constexpr int kGramWaves = 5120;  // waves of the VALU Gram work kernel and the self norms at a bandwidth (5 per SIMD)
// fewest column tiles per task of the MFMA Gram form (the plan raises it to
// fit the waves): a task loads its slot rows once for all its tiles, and a
// compute unit's L1 traffic bounds the Gram work more than the task count
constexpr int kGramQMin = 4;
constexpr int kGramWavesMfma = 5120;  // waves of the MFMA Gram work kernel (5 per SIMD: its occupancy)

// Physical slots of the live batches, oldest batch first.
struct SlotList {
    int n;
    int r[kMaxSlots];
};

// The window after an update, for the count truncation (tau > 0): the rank
// (0 = oldest) of each physical slot in it, -1 outside; rank q holds batch
// first + q.
struct WindowRank {
    int n, tau;
    int64_t first;
    int rank[kMaxSlots];
};

// Bit-level bf16 helpers (round to nearest even): hi = bf16(x), lo = bf16(x - hi).
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
    unsigned int *sqmax = nullptr;  // [1] max of sqn over the finite rows (FP32 bits)
    // coordinate pool: rows [0,k) initial points, k + p*bmax + q: position q
    // (batch order) of physical slot p; row PR = k + P*bmax is all zeros
    float *pool32 = nullptr;     // [(PR+1) * dp]
    uint16_t *poolhi = nullptr;  // [(PR+1) * dp]  BF16 forms only
    uint16_t *poollo = nullptr;
    float *poolsq = nullptr;     // [PR+1]
    double *poolsq64 = nullptr;  // [PR+1]
    // the rows being scored: a view of one physical slot (set per call)
    int32_t *batidx = nullptr;   // [bmax] gathered indices of the staging slot
    float *bat32 = nullptr;
    uint16_t *bathi = nullptr, *batlo = nullptr;
    float *batsq = nullptr;
    double *batsq64 = nullptr;
    // the staged batch again in MFMA fragment order (batch-stationary cross
    // kernel): BF16 forms hi then lo (2 bytes each), FP32 form floats
    char *batfrag = nullptr;     // [frag_rows * dp * 4 bytes]
    // ring of P physical slots
    int32_t *slot_pts = nullptr;  // [P * bmax] point index of each row (batch order)
    int32_t *ring_idx = nullptr;  // [P * bmax] point indices, grouped by center
    int32_t *ring_perm = nullptr; // [P * bmax] grouped position -> batch-order row
    int32_t *ring_off = nullptr;  // [P * (k+1)]
    int32_t *init_idx = nullptr;  // [k]
    double *coef = nullptr;       // [k * C], C = P + 1
    double *cum = nullptr;        // [k]
    double *G = nullptr;          // [k * C * C]
    int32_t *goff = nullptr;      // [k * C + 2] task offsets of the Gram blocks being computed, their total, column tiles per task
    double *gpart = nullptr;      // [kGramWaves + k * C] their per-run partial sums
    double *N = nullptr;          // [k]
    int32_t *counts = nullptr;    // [k]
    double *alpha = nullptr;      // [k]
    // grouping of a batch by center
    int32_t *rank = nullptr;      // [bmax] rank of a row among equal labels of its chunk
    int32_t *gcnt = nullptr;      // [nchunk * k] per-chunk label counts
    int32_t *gbase = nullptr;     // [nchunk * k] per-chunk label bases in the new slot
    // support of the current centers (padded segments)
    int32_t *seg_off = nullptr;  // [k+1]
    int32_t *seg_next = nullptr; // [k+1] segment offsets of the next iteration's support (from the update)
    int32_t *sup_row = nullptr;  // [Mcap + 1] pool row; [Mcap] = the zero row
    float *sup_w = nullptr;      // [Mcap + 1]; [Mcap] = 0
    float *sup_ay = nullptr;     // [Mcap + 1], [Mcap] = 0; MFMA path: -log2(e) ||y||^2 / kappa of the entry's row
    double *sup_w64 = nullptr;   // [Mcap]
    double *sn_part = nullptr;   // [k][kSnSplit][2] partial sums of the self norms at a bandwidth
    int32_t *blk_center = nullptr;  // [Mcap/32] center of each 32-entry block (segments padded to 32)
    int32_t *blk_split = nullptr;   // [Mcap/32] packed segments: row of the block where a center starts (32: none)
    // cross-term output and assignment
    void *part = nullptr;        // P[k][bmax] (direct) or per-run partials [Mcap/32][bmax]
    int32_t *labels = nullptr;   // [bmax]
    float *mind = nullptr;       // [bmax]
    float *margin = nullptr;     // [bmax]
    double *obj = nullptr;       // [4] device scalars
    int32_t *flags = nullptr;    // [4] error flags (index, non-finite, label)
    unsigned long long *nresc = nullptr;  // [1] rows re-scored in FP64 (BF16 forms)
    // differentiation form
    double *Nsig = nullptr;      // [k] self norms at the bandwidth of the call
    double *dNsig = nullptr;     // [k] their derivative
    double *rowds = nullptr;     // [bmax] per-row terms of df/dsigma
    int32_t *sg_toff = nullptr;  // [k+1] task offsets of the self norms at a bandwidth (MFMA)
    double *sg_part = nullptr;   // [2 (kGramWaves + k)] their per-run partials (N, then d2-weighted)
    int32_t *gr_cnt = nullptr;   // [2k + 1] backward: group counts, scatter cursors, task ticket
    int32_t *gr_loff = nullptr;  // [k+1] row offsets of the groups
    int32_t *gr_rtoff = nullptr; // [k+1] offsets of the 32-row tasks
    int32_t *gr_perm = nullptr;  // [bmax] rows grouped by label
    // untruncated form (window 0): the table of cross terms of every point
    void *dp_T = nullptr;        // [k * ldT] T[j][x] = <phi(x), C_j>, FP32 or FP64
    void *dp_tsel = nullptr;     // [bmax] old T[label][x] of the batch rows
    void *dp_gsel = nullptr;     // [bmax] the same, grouped by center
    int32_t *dp_gctr = nullptr;  // [bmax] center of each grouped entry
    double *dp_pair = nullptr;   // [bmax] sum of K(y, y') over the entry's center
    int32_t *dp_toff = nullptr;  // [k+1] offsets of the centers' pair tasks
    double *dp_pp = nullptr;     // [ceil(bmax/64) * bmax] row sums of the pair tasks by column tile
    float *dp_S = nullptr;       // [k * ldT] MFMA form: (alpha_j / b_j) sum_y K(x, y) of the touched centers
    double *dp_w = nullptr;      // [k] alpha_j / b_j of the update (1 at init)
    int32_t *dp_iseg = nullptr;  // [k+1] one-entry segments of the initial centers
    int32_t *dp_irow = nullptr;  // [k] their pool rows
    // k-means++
    double *D2 = nullptr;        // [n]
    double *kself = nullptr;     // [n]
    double *bsum = nullptr;      // [nblocks]
    int32_t *picks = nullptr;    // [k]
    double *u = nullptr;         // [k]
};

struct Layout {
    int64_t n;
    int d, dp, k, W, P, C, bmax, pad;
    // packed segments (the batch-stationary MFMA kernel): a center's segment is
    // its entries, at least `pad` when it has any, the support's end rounded
    // up to a multiple of pad; else every segment is a multiple of pad
    bool packed;
    int64_t PR;        // pool rows excluding the zero row: k + P * bmax
    int64_t Mcap;      // max padded support entries (multiple of 128)
    int64_t nblk;      // Mcap / 32
    int nchunk;        // grouping chunks of a full batch: ceil(bmax / kChunk)
    int64_t kpp_blocks;
    bool bf16;
    int frag_mode;     // batch fragment copy: 0 none, 1 BF16 hi/lo, 2 FP32
    bool untrunc;      // window 0: untruncated, on the table of cross terms
    int64_t ldT;       // its row stride (n rounded up to 64)
    int tbytes;        // bytes of a table entry (4 or 8)
    bool dp_mfma;      // the table update on MFMA (Gaussian FP32, d >= 16)
    size_t bytes;
};

// Rows of the batch fragment copy (whole 32-row blocks).
inline int frag_rows(const Layout &L) { return (L.bmax + 31) / 32 * 32; }

Layout make_layout(const mbkk_config &c);
void carve(const Layout &L, char *base, Buffers &B);

// Row of physical slot p, position q, in the pool.
inline int64_t slot_row(const Layout &L, int p, int64_t q) { return (int64_t)L.k + (int64_t)p * L.bmax + q; }

}  // namespace mbkk
