// Gram work shared by the Gram kernels (kernels_gram.hip) and the support
// layout launch that runs a step's Gram work beside the next layout
// (kernels_prep.hip): the work description, the per-wave task loop and the
// MFMA task.
//
// A center held over its support (Section 4.1, Eq. 1 with a window of W
// batches) has self-norm <C_j, C_j> = sum_{c,c'} coef_j[c] coef_j[c'] G_j[c][c'];
// when batch i enters slot rr only the blocks
//   G_j[1+rr][c] = G_j[c][1+rr] = sum_{a in slot rr, center j} sum_{e in column c, center j} K(a, e)
// against the live columns c are new.  Their pairs are cut into tasks (the
// plan, gram_plan); kGramWaves-style equal contiguous task ranges go to the
// waves, wave w storing the FP64 sum of its tasks of one jc = j * C + c at
// gpart[w + jc] (the (wave, jc) runs form a staircase, so w + jc is distinct).
#pragma once

#include "dev_common.h"

namespace mbkk {

struct GramWork {
    int k, C, bmax, rr;
    const int32_t *ring_off, *ring_perm;
    const int32_t *goff;  // [k*C + 1] task offsets
    double *gpart;        // [kGramWaves + k*C] per-run partials
    int nwaves;           // waves of the work kernel (sets the task ranges)
};

constexpr int kGramWG = 256;  // 4 waves per workgroup
// LDS copy of the task offsets and the ring offsets (ints), when both fit
constexpr int kGramStage = 4096;

// gram_col with the offsets read once per wave into scalar registers.
__device__ __forceinline__ GramCol gram_col_uniform(int k, int bmax, int j, int c, const int32_t *ring_off,
                                                    const int32_t *__restrict__ ring_perm)
{
    GramCol g;
    if (c == 0) {
        g.n = 1;
        g.perm = nullptr;
        g.row0 = j;
    } else {
        const int32_t *o = ring_off + (int64_t)(c - 1) * (k + 1);
        const int o0 = __builtin_amdgcn_readfirstlane(o[j]), o1 = __builtin_amdgcn_readfirstlane(o[j + 1]);
        g.n = o1 - o0;
        g.perm = ring_perm + (int64_t)(c - 1) * bmax + o0;
        g.row0 = (int64_t)k + (int64_t)(c - 1) * bmax;
    }
    return g;
}

// XCD-aware order of the work workgroups (on by default)
#ifndef MBKK_GRAM_XCD
#define MBKK_GRAM_XCD 1
#endif

// Runs `task(a, e, ab, eb, Q, lsum)` over the task range of wave w = blk * 4 +
// (wave in the workgroup); a = the slot's rows of center j, e = column c's
// rows, (ab, eb) the task's row blocks: slot rows ab TA.., column tiles
// eb Q .. eb Q + Q - 1 of TE rows (Q, the plan's column tiles per task, is
// read after the task total when TQ, else 1).  Every thread of the workgroup calls
// it: when the task offsets and the ring offsets fit in `stage`, the
// workgroup first copies them there with coalesced loads, so the segment
// search and the column lookups read LDS.
// pblk: the physical workgroup index of a grid of nwaves / 4 workgroups
// (a multiple of 8).  Workgroups are handed to the 8 XCDs round robin
// (pblk % 8); the workgroups that have tasks are cut into 8 contiguous
// shares, share x taken by the workgroups of XCD x, so that the tasks of a
// center, which are contiguous, read their rows through one XCD's L2.
template <int TE, bool TQ, class Task>
__device__ __forceinline__ void gram_wave_loop(const GramWork &A, int32_t *stage, int pblk, Task &&task)
{
    const int lane = threadIdx.x & 63;
    const int nJC = A.k * A.C;
    const int nro = (A.C - 1) * (A.k + 1);
    const int32_t *goff = A.goff, *ring_off = A.ring_off;
    // the task count (a scalar load), and the loads of the LDS copy of the
    // offsets, which do not depend on it, in flight together; a workgroup
    // whose waves have no task leaves once they have arrived
    const int T = A.goff[nJC];
    const int Q = TQ ? A.goff[nJC + 1] : 1;
    const bool staged = nJC + 1 + nro <= kGramStage;  // workgroup uniform
    constexpr int SQ = kGramStage / kGramWG;
    const int tot = nJC + 1 + nro;
    int v[SQ];
    int vor = 0;
    if (staged) {
        // one address select each, no branch
#pragma unroll
        for (int q = 0; q < SQ; ++q) {
            const int i = min((int)threadIdx.x + q * kGramWG, tot - 1);
            v[q] = *(i <= nJC ? A.goff + i : A.ring_off + (i - (nJC + 1)));
            vor |= v[q];
        }
    }
    // (offsets are never negative, so the second test is false in every
    // thread and the exit stays workgroup uniform; it keeps the copy's loads
    // ahead of the exits below instead of sunk past them)
    if (T == 0 || vor < 0)
        return;
    const int chunk = (T + A.nwaves - 1) / A.nwaves;
    int blk = pblk;
    if constexpr (MBKK_GRAM_XCD != 0) {
        const int awg = ((T + chunk - 1) / chunk + kGramWG / 64 - 1) / (kGramWG / 64);  // workgroups with tasks
        const int share = (awg + 7) / 8;
        if (pblk / 8 >= share)
            return;  // workgroup uniform
        blk = (pblk % 8) * share + pblk / 8;
    }
    if ((int64_t)blk * (kGramWG / 64) * chunk >= T)
        return;  // workgroup uniform
    // wave-uniform values are moved to scalar registers (readfirstlane)
    const int w = __builtin_amdgcn_readfirstlane(blk * (kGramWG / 64) + (threadIdx.x >> 6));
    if (staged) {
#pragma unroll
        for (int q = 0; q < SQ; ++q) {
            const int i = threadIdx.x + q * kGramWG;
            if (i < tot)
                stage[i] = v[q];
        }
        __syncthreads();
        goff = stage;
        ring_off = stage + nJC + 1;
    }
    const int64_t t0l = (int64_t)w * chunk;
    if (t0l >= T)
        return;  // wave uniform
    const int t0 = (int)t0l, t1 = min(T, t0 + chunk);
    int jc = __builtin_amdgcn_readfirstlane(wave_segment_of(goff, nJC, t0));
    int t = t0;
    while (t < t1) {  // wave uniform
        const int g0 = __builtin_amdgcn_readfirstlane(goff[jc]), g1 = __builtin_amdgcn_readfirstlane(goff[jc + 1]);
        const int e = min(t1, g1);
        if (t < e) {
            const int j = jc / A.C, c = jc - j * A.C;
            const GramCol a = gram_col_uniform(A.k, A.bmax, j, 1 + A.rr, ring_off, A.ring_perm);
            const GramCol ec = gram_col_uniform(A.k, A.bmax, j, c, ring_off, A.ring_perm);
            const int nE = ((ec.n + TE - 1) / TE + Q - 1) / Q;
            double lsum = 0.0;
            for (; t < e; ++t) {
                const int u = t - g0;
                const int ab = u / nE, eb = u - ab * nE;
                task(a, ec, ab, eb, Q, lsum);
            }
            lsum = wave_sum_f64(lsum);
            if (lane == 0)
                A.gpart[w + jc] = lsum;
        }
        ++jc;
    }
}

// ---------------------------------------------------------------------------
// MFMA tasks (Gaussian): exp(-(||a||^2 + ||e||^2 - 2 a.e) / kappa) with a.e
// on FP32 MFMA 16x16x4 (every MFMA form, the BF16 ones included): a task is
// 16 slot rows by Q tiles of 16 column rows (the plan's Q: at least 4, more
// when the tasks would outnumber the waves), so a cluster of b_j rows pads
// to a multiple of 16 rather than 32, and a task loads its slot rows once
// for all its tiles.  Lane l = 16 g + n supplies
// A[n][g] (slot row n) and B[g][n] (column row n); the u-th MFMA of step t
// takes coordinate 16 t + 4 g + u, so one 16-byte load per lane and step
// serves four MFMAs and the four lanes of a row read 64 contiguous bytes
// (16 cache lines per wave load, not 64).  The lane holds D[4 g + i][n], i < 4.
// DP = 0 takes the row stride at run time.  blk: the physical workgroup index.
// ---------------------------------------------------------------------------
template <int DP>
__device__ __forceinline__ void gram_mfma_work(const GramWork &A, int dp_rt, int zero_row,
                                               const float *__restrict__ pool32, const float *__restrict__ poolsq,
                                               float c2, float c1, int blk)
{
    const int dp = DP > 0 ? DP : dp_rt;
    const int KQ = dp / 4;
    __shared__ __attribute__((aligned(16))) float sqa[kGramWG / 64][16];
    __shared__ int32_t stage[kGramStage];
    const int lane = threadIdx.x & 63, wl = threadIdx.x >> 6, n = lane & 15, g = lane >> 4;
    gram_wave_loop<16, true>(A, stage, blk, [&](const GramCol &a, const GramCol &ec, int ab, int eb, int Q,
                                                 double &lsum) {
        // the task: slot rows ab*16.., column tiles tile0 .. tile1-1 (wave uniform)
        const int qa = ab * 16 + n;
        const int tile0 = eb * Q, tile1 = min((ec.n + 15) / 16, tile0 + Q);
        // both permutation loads of the first tile, then every row load, in
        // flight together: clamped indices and selects, no branches (a is a
        // slot column, so a.perm is set; column 0 of ec has no permutation
        // and one row)
        const int32_t *ep = ec.perm ? ec.perm : a.perm;
        const int32_t pa = a.perm[min(qa, a.n - 1)];
        int32_t pe = ep[min(tile0 * 16 + n, ec.n - 1)];
        const int64_t ra = qa < a.n ? a.row0 + pa : zero_row;
        const float sqa_v = poolsq[ra];
        const float *sa = pool32 + ra * dp + 4 * g;
        // the slot rows' coordinates, loaded once for every tile of the task
        constexpr int NS = DP > 0 ? DP / 16 : 1;
        f32x4 av[NS];
        if constexpr (DP > 0) {
#pragma unroll
            for (int q = 0; q < NS; ++q)
                av[q] = *(const f32x4 *)(sa + 16 * q);
        }
        // lane: column n (column row), rows m = 4 g + i (slot rows); the
        // row norms were written by this wave (in-order LDS access) and are
        // read as one 16-byte load; rows past the cluster add an exact 0 (the
        // sum is positive, so no sign of zero changes)
        auto tile_sum = [&](int tile, const f32x4 &acc, float sqe_v) {
            const int qe_t = tile * 16 + n;
            if (tile == tile0 && g == 0)
                sqa[wl][n] = c1 * sqa_v;  // slot row n's norm for the output rows m, once per task
            const float se_ = c1 * sqe_v;
            if (qe_t < ec.n) {
                const f32x4 sq4 = *(const f32x4 *)&sqa[wl][4 * g];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int m = 4 * g + i;
                    const double t = (double)__builtin_amdgcn_exp2f(fmaf(acc[i], c2, sq4[i] + se_));
                    lsum += ab * 16 + m < a.n ? t : 0.0;
                }
            }
        };
        auto col_row = [&](int tile, int32_t pe_t) -> int64_t {
            const int qe_t = tile * 16 + n;
            return qe_t < ec.n ? (ec.perm ? ec.row0 + pe_t : ec.row0) : zero_row;
        };
        if constexpr (DP > 0) {
            // every tile's permutation entry at the start, then each tile's
            // rows requested before the previous tile's products (clamped
            // to the last tile, which then loads its rows twice)
            constexpr int QX = 1 << (kGramTileSteps - 1);
            int32_t pes[QX];
            pes[0] = pe;
#pragma unroll
            for (int q = 1; q < QX; ++q)
                pes[q] = ep[min(min(tile0 + q, tile1 - 1) * 16 + n, ec.n - 1)];
            int64_t re = col_row(tile0, pes[0]);
            float sqe_v = poolsq[re];
            f32x4 ev[NS];
#pragma unroll
            for (int q = 0; q < NS; ++q)
                ev[q] = *(const f32x4 *)(pool32 + re * dp + 4 * g + 16 * q);
#pragma unroll
            for (int t = 0; t < QX; ++t) {
                const int tile = tile0 + t;
                if (tile >= tile1)
                    break;  // wave uniform
                const int tn = min(tile + 1, tile1 - 1);
                const int64_t rn = col_row(tn, pes[t + 1 < QX ? t + 1 : t]);
                const float sqn = poolsq[rn];
                f32x4 en[NS];
#pragma unroll
                for (int q = 0; q < NS; ++q)
                    en[q] = *(const f32x4 *)(pool32 + rn * dp + 4 * g + 16 * q);
                // the slot row's norm is needed by this point (the products
                // wait for the row loads anyway), so its load is not sunk into
                // the branch that publishes it
                asm volatile("" ::"v"(sqa_v));
                f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
                for (int q = 0; q < NS; ++q)
#pragma unroll
                    for (int u = 0; u < 4; ++u)
                        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av[q][u], ev[q][u], acc, 0, 0, 0);
                tile_sum(tile, acc, sqe_v);
#pragma unroll
                for (int q = 0; q < NS; ++q)
                    ev[q] = en[q];
                sqe_v = sqn;
            }
        } else {
            for (int tile = tile0; tile < tile1; ++tile) {
                if (tile != tile0)
                    pe = ep[min(tile * 16 + n, ec.n - 1)];
                const int64_t re = col_row(tile, pe);
                const float sqe_v = poolsq[re];
                const float *se = pool32 + re * dp + 4 * g;
                f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
                // row stride at run time: 8 steps of 4 coordinates per round
                // of loads, all in flight before their products (clamped
                // indices; the steps past the row skip their products)
                constexpr int U = 8;
                for (int s0 = 0; s0 < KQ; s0 += 4 * U) {
                    f32x4 a4[U], e4[U];
#pragma unroll
                    for (int q = 0; q < U; ++q) {
                        const int s4 = min(s0 + 4 * q, KQ - 4);
                        a4[q] = *(const f32x4 *)(sa + 4 * s4);
                        e4[q] = *(const f32x4 *)(se + 4 * s4);
                    }
                    __builtin_amdgcn_sched_barrier(0);  // keep the loads ahead of the products
#pragma unroll
                    for (int q = 0; q < U; ++q)
                        if (s0 + 4 * q < KQ)  // wave uniform
#pragma unroll
                            for (int u = 0; u < 4; ++u)
                                acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a4[q][u], e4[q][u], acc, 0, 0, 0);
                }
                tile_sum(tile, acc, sqe_v);
            }
        }
    });
}

}  // namespace mbkk
