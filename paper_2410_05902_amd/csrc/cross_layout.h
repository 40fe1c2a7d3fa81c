// Layout of the cross kernels' partial sums, shared by the cross kernels
// (kernels_cross.hip) and the scoring kernel that reads them
// (kernels_score.hip): the support ranges of the direct (VALU) kernel and of
// the batch-stationary MFMA kernel, and their launch shapes.
#pragma once

#include "mbkk_internal.h"

namespace mbkk {

// Ranges of the direct kernel: the concatenated support is cut into nranges
// ranges of RR rows (RR from the support size, so the scoring kernel derives
// the same cut); a run is a range's stretch of one center's segment.  Run id:
// the center j for the run that starts at the center's first row, k + r for
// the run that starts at the start of range r inside a center.
__host__ __device__ inline int direct_range_rows(int M, int nranges) { return (M + nranges - 1) / nranges; }

// Batch rows per lane of the direct kernel: two for FP32 rows of at most 32
// coordinates (each broadcast support row then feeds two evaluations).
inline int direct_rpl(int d, bool fp64) { return !fp64 && d <= 32 ? 2 : 1; }

// Ranges of the direct kernel for nb batch rows: about kDirectWGs workgroups
// (one round at 8 waves per SIMD), 3/4 of that with two rows per lane (whose
// registers allow 6 waves per SIMD).
inline int direct_nranges(int nb, int rpl)
{
    const int tiles = (nb + 256 * rpl - 1) / (256 * rpl);
    const int r = (rpl == 2 ? kDirectWGs * 3 / 4 : kDirectWGs) / tiles;
    return r < 1 ? 1 : r;
}

constexpr int kBsStageBlocks = 4;  // support blocks (32 rows) per stage of the MFMA kernel

// Blocks per range for Mb support blocks split over nranges ranges (the
// kernel's last stage of a range skips the blocks past it).
__host__ __device__ inline int bs_range_blocks(int Mb, int nranges) { return (Mb + nranges - 1) / nranges; }

// Waves per SIMD: two in the BF16X3 form with row stride above 64, whose
// two waves on a SIMD take turns, one issuing MFMAs while the other runs its
// exp epilogue or waits on LDS; one elsewhere (the FP32 MFMAs are twice as
// long, and at stride 64 the register file holds four N-blocks per wave).
__host__ __device__ constexpr int bs_wps(int mode, int dp) { return mode == 1 && dp > 64 ? 2 : 1; }
// Batch rows held in registers per wave, in 32-row N-blocks: as many as the
// register file allows (one wave per SIMD: 256 VGPRs + 256 AGPRs; two waves:
// half each) with two accumulator sets (the pipelined epilogue) and few
// copies between the two register kinds.  FP32 fragments are 2x larger and
// each FP32 MFMA is 2x longer, so two N-blocks already amortise the support
// reads.
__host__ __device__ constexpr int bs_nbk(int mode, int dp) { return mode == 0 ? 2 : (mode == 1 && dp > 64 ? 1 : 4); }
inline int bs_tile_rows(int mode, int dp) { return 4 * bs_wps(mode, dp) * 32 * bs_nbk(mode, dp); }
inline int bs_mode(int precision) { return precision == MBKK_FP32 ? 0 : (precision == MBKK_BF16X3 ? 1 : 2); }
// Ranges for nb batch rows: one round of workgroups (kBsOcc per compute unit).
inline int bs_nranges(int nb, int mode, int dp)
{
    const int tr = bs_tile_rows(mode, dp);
    const int nbt = (nb + tr - 1) / tr;
    const int r = kNumCU * kBsOcc / nbt;
    return r < 1 ? 1 : r;
}

}  // namespace mbkk
