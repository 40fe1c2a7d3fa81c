// Host side of the mbkk C ABI: workspace layout, context, and the order of
// launches for one iteration of Algorithm 2 (truncated mini-batch kernel
// k-means).  Every device buffer lives in the caller's workspace; the library
// allocates no device memory.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <string>
#include <vector>

#include "kernels.h"

using namespace mbkk;

struct mbkk_ctx {
    mbkk_config cfg;
    Layout L;
    Buffers B;
    hipStream_t stream = nullptr;
    bool use_mfma = false;
    bool fp64 = false;
    bool data_set = false;
    double ymax2 = 0.0;         // max ||x||^2 over the data (bounds every support row)
    bool inited = false;
    int64_t iter = 1;           // index i of the next batch
    int64_t support_iter = -1;  // iteration for which the support layout is built
    // Gram work of the last step whose fold into G is left to the next support
    // layout (slot, column mask); fold_rr < 0: none pending
    int fold_rr = -1;
    uint32_t fold_mask = 0;
    // iteration whose support segment offsets the last update wrote to seg_next
    int64_t seg_next_iter = -1;
    // state version: bumped by every change of the centers; the support layout
    // (offsets, rows, weights) and the self norms at a bandwidth are valid for
    // the version they were made at
    int64_t version = 0;
    int64_t layout_version = -1;
    int64_t sig_version = -1;
    double sig_sigma = 0.0;
    int32_t slot_b[kMaxSlots] = {};  // points held by each physical slot
    int device = -1;                 // static workspace: the device whose array it uses (-1: none)
    // timing of the cross-term kernel
    bool timing = false;
    std::vector<hipEvent_t> ev;  // pairs (start, stop)
    size_t ev_used = 0;
    double ms_acc = 0.0;
    int64_t launches = 0;
    std::string err;
};

static std::string g_err;

static int fail(mbkk_ctx *c, int code, const std::string &msg)
{
    if (c)
        c->err = msg;
    else
        g_err = msg;
    return code;
}

#define HIPCHK(c, call)                                                                            \
    do {                                                                                           \
        hipError_t e_ = (call);                                                                    \
        if (e_ != hipSuccess)                                                                      \
            return fail((c), MBKK_E_HIP, std::string(#call) + ": " + hipGetErrorString(e_));     \
    } while (0)

namespace mbkk {

static size_t up(size_t x, size_t a) { return (x + a - 1) / a * a; }

static bool wants_mfma(const mbkk_config &c)
{
    if (c.window == 0)
        return false;  // the table form runs on the VALU
    if (c.cross_impl == MBKK_CROSS_MFMA)
        return true;
    if (c.cross_impl == MBKK_CROSS_DIRECT)
        return false;
    if (c.precision == MBKK_BF16X3 || c.precision == MBKK_BF16X1)
        return true;
    return c.kernel == MBKK_GAUSS && c.precision == MBKK_FP32 && c.d >= 16;
}

Layout make_layout(const mbkk_config &c)
{
    Layout L;
    L.n = c.n;
    L.d = c.d;
    L.dp = (int)up((size_t)c.d, kDimAlign);
    L.k = c.k;
    L.W = c.window;
    L.P = c.window + 1;
    L.C = L.P + 1;
    L.bmax = c.b_max;
    L.pad = wants_mfma(c) ? kMfmaPad : 1;
    L.packed = wants_mfma(c) && L.dp <= 128;
    L.bf16 = c.precision == MBKK_BF16X3 || c.precision == MBKK_BF16X1;
    // the batch-stationary MFMA cross kernel (row stride <= 128) reads the
    // batch from a fragment-order copy
    L.frag_mode = wants_mfma(c) && L.dp <= 128 ? (L.bf16 ? 1 : 2) : 0;
    L.PR = (int64_t)c.k + (int64_t)L.P * c.b_max;
    L.untrunc = c.window == 0;
    L.ldT = (int64_t)up((size_t)c.n, 64);
    L.tbytes = c.precision == MBKK_FP64 ? 8 : 4;
    // the Gaussian FP32 table update on MFMA (product form), as the FP32 cross
    // term of the truncated form with cross_impl AUTO / MFMA (d >= 16)
    L.dp_mfma = L.untrunc && c.kernel == MBKK_GAUSS &&
                (c.precision == MBKK_BF16X3 ||
                 (c.precision == MBKK_FP32 &&
                  (c.cross_impl == MBKK_CROSS_MFMA || (c.cross_impl == MBKK_CROSS_AUTO && c.d >= 16))));
    // live support: at most W slots of b_max points and the k initial points
    // (the table form: the grouped batch, or the k initial points)
    const int64_t Mlive = L.untrunc ? std::max<int64_t>(c.k, c.b_max) : (int64_t)c.k + (int64_t)c.window * c.b_max;
    L.Mcap = (int64_t)up((size_t)(Mlive + (int64_t)c.k * (L.pad - 1) + L.pad), 128);
    L.nblk = L.Mcap / 32;
    L.nchunk = (c.b_max + kChunk - 1) / kChunk;
    L.kpp_blocks = (c.n + 255) / 256;
    return L;
}

// Carves the workspace; with base == nullptr only sizes it (L.bytes).
void carve(const Layout &Lc, char *base, Buffers &B)
{
    Layout &L = const_cast<Layout &>(Lc);
    size_t off = 0;
    auto take = [&](size_t bytes) -> void * {
        off = up(off, 256);
        void *p = base ? base + off : nullptr;
        off += bytes == 0 ? 1 : bytes;
        return p;
    };
    const int64_t prows = L.PR + 1;
    const int C = L.C;
    B.sqn = (float *)take(sizeof(float) * L.n);
    B.sqmax = (unsigned int *)take(sizeof(unsigned int));
    B.pool32 = (float *)take(sizeof(float) * prows * L.dp);
    B.poolhi = L.bf16 ? (uint16_t *)take(2 * prows * L.dp) : nullptr;
    B.poollo = L.bf16 ? (uint16_t *)take(2 * prows * L.dp) : nullptr;
    B.poolsq = (float *)take(sizeof(float) * prows);
    B.poolsq64 = (double *)take(sizeof(double) * prows);
    B.batfrag = L.frag_mode ? (char *)take(4 * (size_t)frag_rows(L) * L.dp) : nullptr;
    B.slot_pts = (int32_t *)take(4 * (size_t)L.P * L.bmax);
    B.ring_idx = (int32_t *)take(4 * (size_t)L.P * L.bmax);
    B.ring_perm = (int32_t *)take(4 * (size_t)L.P * L.bmax);
    B.ring_off = (int32_t *)take(4 * (size_t)L.P * (L.k + 1));
    B.init_idx = (int32_t *)take(4 * (size_t)L.k);
    B.coef = (double *)take(8 * (size_t)L.k * C);
    B.cum = (double *)take(8 * (size_t)L.k);
    B.G = (double *)take(8 * (size_t)L.k * C * C);
    B.goff = (int32_t *)take(4 * ((size_t)L.k * C + 2));
    B.gpart = (double *)take(8 * ((size_t)kGramWaves + (size_t)L.k * C));
    B.N = (double *)take(8 * (size_t)L.k);
    B.counts = (int32_t *)take(4 * (size_t)L.k);
    B.alpha = (double *)take(8 * (size_t)L.k);
    B.rank = (int32_t *)take(4 * (size_t)L.bmax);
    B.gcnt = (int32_t *)take(4 * (size_t)L.nchunk * L.k);
    B.gbase = (int32_t *)take(4 * (size_t)L.nchunk * L.k);
    B.seg_off = (int32_t *)take(4 * (size_t)(L.k + 1));
    B.seg_next = (int32_t *)take(4 * (size_t)(L.k + 1));
    B.sup_row = (int32_t *)take(4 * (L.Mcap + 1));  // [Mcap] = zero pool row (sentinel)
    B.sup_w = (float *)take(4 * (L.Mcap + 1));   // [Mcap] = 0 (sentinel)
    B.sup_ay = (float *)take(4 * (L.Mcap + 1));  // [Mcap] = 0 (sentinel)
    B.sup_w64 = (double *)take(8 * L.Mcap);
    B.sn_part = (double *)take(8 * 2 * (size_t)L.k * kSnSplit);
    B.blk_center = (int32_t *)take(4 * L.nblk);
    B.blk_split = (int32_t *)take(4 * L.nblk);
    // cross-term partials of the kernel in use: runs of the direct kernel (FP32
    // or FP64), or FP32 values per (32-row block, batch row) on MFMA: one, or
    // two with packed segments (the run from the block's start, and the run of
    // a center that starts inside the block)
    const size_t part_direct = (size_t)(L.k + kDirectWGs) * L.bmax * L.tbytes;
    const size_t part_mfma = (size_t)L.nblk * (L.packed ? 2 : 1) * L.bmax * 4;
    B.part = take(L.untrunc ? 0 : (L.pad == kMfmaPad ? part_mfma : part_direct));
    if (L.untrunc) {
        B.dp_T = take((size_t)L.tbytes * (size_t)L.k * (size_t)L.ldT);
        B.dp_tsel = take(8 * (size_t)L.bmax);
        B.dp_gsel = take(8 * (size_t)L.bmax);
        B.dp_gctr = (int32_t *)take(4 * (size_t)L.bmax);
        B.dp_pair = (double *)take(8 * (size_t)L.bmax);
        B.dp_toff = (int32_t *)take(4 * ((size_t)L.k + 1));
        B.dp_pp = (double *)take(8 * (size_t)((L.bmax + 63) / 64) * L.bmax);
        B.dp_S = L.dp_mfma ? (float *)take(4 * (size_t)L.k * (size_t)L.ldT) : nullptr;
        B.dp_w = (double *)take(8 * (size_t)L.k);
        B.dp_iseg = (int32_t *)take(4 * ((size_t)L.k + 1));
        B.dp_irow = (int32_t *)take(4 * (size_t)L.k);
    }
    B.labels = (int32_t *)take(4 * (size_t)L.bmax);
    B.mind = (float *)take(4 * (size_t)L.bmax);
    B.margin = (float *)take(4 * (size_t)L.bmax);
    // device scalars and error flags, adjacent so that one copy reads both back
    B.obj = (double *)take(8 * 4 + 4 * 4);
    B.flags = (int32_t *)(B.obj + 4);
    B.nresc = (unsigned long long *)take(8);
    B.Nsig = (double *)take(8 * (size_t)L.k);
    B.dNsig = (double *)take(8 * (size_t)L.k);
    B.rowds = (double *)take(8 * (size_t)L.bmax);
    B.sg_toff = (int32_t *)take(4 * ((size_t)L.k + 1));
    B.sg_part = (double *)take(8 * 2 * ((size_t)kGramWaves + L.k));
    B.gr_cnt = (int32_t *)take(4 * (2 * (size_t)L.k + 1));  // counts, cursors, task ticket
    B.gr_loff = (int32_t *)take(4 * ((size_t)L.k + 1));
    B.gr_rtoff = (int32_t *)take(4 * ((size_t)L.k + 1));
    B.gr_perm = (int32_t *)take(4 * (size_t)L.bmax);
    B.D2 = (double *)take(8 * (size_t)L.n);
    B.kself = (double *)take(8 * (size_t)L.n);
    B.bsum = (double *)take(8 * (size_t)L.kpp_blocks);
    B.picks = (int32_t *)take(4 * (size_t)L.k);
    B.u = (double *)take(8 * (size_t)L.k);
    L.bytes = up(off, 256);
}

}  // namespace mbkk

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------
static int check_config(const mbkk_config *c, std::string &why)
{
    if (!c) {
        why = "config is NULL";
        return MBKK_E_INVALID;
    }
    if (c->n <= 0 || c->d <= 0 || c->k <= 0 || c->k > 65536 || c->k > c->n) {
        why = "need n > 0, d > 0, 0 < k <= min(n, 65536)";
        return MBKK_E_INVALID;
    }
    if (c->n > 2147483647LL) {
        why = "n must fit in int32 indices";
        return MBKK_E_INVALID;
    }
    if (c->b_max <= 0 || c->b_max > kMaxBatch) {
        why = "need 1 <= b_max <= 8192";
        return MBKK_E_INVALID;
    }
    if (c->tau < 0) {
        why = "need tau >= 0";
        return MBKK_E_INVALID;
    }
    if (c->window < 0 || c->window > kMaxWindow) {
        why = "need 0 <= window <= 30";
        return MBKK_E_INVALID;
    }
    if (c->window == 0) {
        if (c->tau != 0) {
            why = "window 0 (untruncated) takes no tau";
            return MBKK_E_INVALID;
        }
        if (c->precision == MBKK_BF16X1) {
            why = "window 0 (untruncated) runs in FP32, FP64 or BF16X3";
            return MBKK_E_INVALID;
        }
        if (c->d > dp_max_dim()) {
            why = "window 0 (untruncated) needs d <= 128";
            return MBKK_E_INVALID;
        }
        const double tb = (double)(c->precision == MBKK_FP64 ? 8 : 4) * (double)c->k * (double)(c->n + 63);
        if (tb > (double)((int64_t)1 << 42)) {
            why = "window 0 (untruncated): the n x k table exceeds 4 TiB";
            return MBKK_E_INVALID;
        }
    }
    if (c->kernel < MBKK_GAUSS || c->kernel > MBKK_POLY2) {
        why = "unknown kernel";
        return MBKK_E_INVALID;
    }
    if ((c->kernel == MBKK_GAUSS || c->kernel == MBKK_LAPLACE) && !(c->kernel_param > 0.0)) {
        why = "bandwidth must be > 0";
        return MBKK_E_INVALID;
    }
    if (c->precision < MBKK_FP32 || c->precision > MBKK_BF16X1) {
        why = "unknown precision";
        return MBKK_E_INVALID;
    }
    if (c->lr < MBKK_LR_BETA || c->lr > MBKK_LR_SKLEARN) {
        why = "unknown learning rate";
        return MBKK_E_INVALID;
    }
    if (c->cross_impl < MBKK_CROSS_AUTO || c->cross_impl > MBKK_CROSS_MFMA) {
        why = "unknown cross_impl";
        return MBKK_E_INVALID;
    }
    const bool bf = c->precision == MBKK_BF16X3 || c->precision == MBKK_BF16X1;
    if ((bf || c->cross_impl == MBKK_CROSS_MFMA) && c->kernel != MBKK_GAUSS) {
        why = "the MFMA / BF16 forms exist for the Gaussian kernel only";
        return MBKK_E_INVALID;
    }
    if (bf && c->cross_impl == MBKK_CROSS_DIRECT) {
        why = "BF16 forms run on MFMA only";
        return MBKK_E_INVALID;
    }
    if (c->cross_impl == MBKK_CROSS_MFMA && c->precision == MBKK_FP64) {
        why = "no FP64 MFMA form";
        return MBKK_E_INVALID;
    }
    return MBKK_OK;
}

// Physical slots of the batches live in C_i (the state before iteration i):
// batches max(1, i-W) .. i-1, oldest first; batch l lives in slot (l-1) mod P.
static int phys_of(int64_t l, int P) { return (int)((l - 1) % P); }

static SlotList live_before(int64_t i, int W)
{
    SlotList s;
    s.n = 0;
    const int64_t lo = i - W < 1 ? 1 : i - W;
    for (int64_t l = lo; l <= i - 1; ++l)
        s.r[s.n++] = phys_of(l, W + 1);
    return s;
}

static uint32_t col_mask_of(const SlotList &s, bool init_alive)
{
    uint32_t m = init_alive ? 1u : 0u;
    for (int q = 0; q < s.n; ++q)
        m |= 1u << (1 + s.r[q]);
    return m;
}

// Gram blocks of slot p against the live columns in `mask`: on FP32 MFMA for
// the Gaussian MFMA forms (BF16 ones included), else VALU.  In a step
// (`in_step`) the update kernel already wrote the task plan and the fold is
// left to the next support layout; elsewhere plan, work and fold run here.
static void gram(mbkk_ctx *c, int p, uint32_t mask, bool in_step)
{
    if (!in_step)
        launch_gram_plan(c->L, c->B, p, mask, gram_task_rows(c->use_mfma), gram_task_cols(c->use_mfma, c->fp64),
                         c->stream);
    launch_gram(c->L, c->B, p, mask, c->cfg.kernel, c->cfg.kernel_param, c->fp64, c->use_mfma, !in_step, c->stream);
    if (in_step) {
        c->fold_rr = p;
        c->fold_mask = mask;
    }
}

// Hands the pending fold to the caller's support layout (or runs it alone).
static int take_fold(mbkk_ctx *c, uint32_t *mask)
{
    const int rr = c->fold_rr;
    *mask = c->fold_mask;
    c->fold_rr = -1;
    return rr;
}

static int check_flags(mbkk_ctx *c)
{
    int32_t f[2] = {0, 0};
    HIPCHK(c, hipMemcpyAsync(f, c->B.flags, sizeof(f), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (f[0])
        return fail(c, MBKK_E_INDEX, "index outside [0, n)");
    if (f[1])
        return fail(c, MBKK_E_NONFINITE, "non-finite value in a gathered row");
    return MBKK_OK;
}

static int clear_flags(mbkk_ctx *c)
{
    launch_fill32(c->B.flags, 0, 4, c->stream);
    HIPCHK(c, hipGetLastError());
    return MBKK_OK;
}

// A positive tie_delta replaces the per-row error bound of the BF16 forms.
static double tie_delta(const mbkk_config &c) { return c.tie_delta > 0.0 ? c.tie_delta : 0.0; }

// Points the batch view at physical slot p (the free slot of the iteration).
static void set_batch_view(mbkk_ctx *c, int p)
{
    const Layout &L = c->L;
    Buffers &B = c->B;
    const int64_t r0 = slot_row(L, p, 0);
    B.batidx = B.slot_pts + (int64_t)p * L.bmax;
    B.bat32 = B.pool32 + r0 * L.dp;
    B.bathi = L.bf16 ? B.poolhi + r0 * L.dp : nullptr;
    B.batlo = L.bf16 ? B.poollo + r0 * L.dp : nullptr;
    B.batsq = B.poolsq + r0;
    B.batsq64 = B.poolsq64 + r0;
}

// One launch: stages rows idx[0..cnt) into the free slot of the current
// iteration and, when not done yet, lays out the support of C_i.
static void prepare(mbkk_ctx *c, const int32_t *idx, int64_t cnt)
{
    const Layout &L = c->L;
    set_batch_view(c, phys_of(c->iter, L.P));
    const bool need = c->support_iter != c->iter;
    const SlotList live = live_before(c->iter, L.W);
    const int init_alive = c->iter <= L.W + 1;
    const float ay_scale = (float)(-1.4426950408889634 / c->cfg.kernel_param);
    int fold_rr = -1;
    uint32_t fold_mask = 0;
    if (need)
        fold_rr = take_fold(c, &fold_mask);
    launch_prepare(L, c->B, need, live, init_alive, idx, cnt, c->cfg.validate, ay_scale, fold_rr, fold_mask,
                   c->seg_next_iter == c->iter, c->stream);
    if (need) {
        c->support_iter = c->iter;
        c->layout_version = c->version;
    }
}

// The next (start, stop) pair of timing events.
static int timing_pair(mbkk_ctx *c, hipEvent_t *e0, hipEvent_t *e1)
{
    if (c->ev_used + 2 > c->ev.size()) {
        for (int q = 0; q < 256; ++q) {
            hipEvent_t e;
            HIPCHK(c, hipEventCreate(&e));
            c->ev.push_back(e);
        }
    }
    *e0 = c->ev[c->ev_used];
    *e1 = c->ev[c->ev_used + 1];
    c->ev_used += 2;
    return MBKK_OK;
}

static int cross_and_score(mbkk_ctx *c, int nb, double *D_out, int64_t ldD, bool with_rank)
{
    const Layout &L = c->L;
    const mbkk_config &cf = c->cfg;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (c->timing) {
        int rc = timing_pair(c, &e0, &e1);
        if (rc)
            return rc;
        HIPCHK(c, hipEventRecord(e0, c->stream));
    }
    if (c->use_mfma)
        launch_cross_mfma(L, c->B, nb, cf.precision, cf.kernel_param, c->stream);
    else
        launch_cross_direct(L, c->B, nb, cf.kernel, cf.kernel_param, c->fp64, c->stream);
    if (c->timing) {
        HIPCHK(c, hipEventRecord(e1, c->stream));
        c->launches++;
    }
    launch_score(L, c->B, nb, cf.kernel, cf.kernel_param, c->fp64, c->use_mfma, cf.precision, tie_delta(cf), c->ymax2,
                 D_out, ldD, with_rank, c->stream);
    HIPCHK(c, hipGetLastError());
    return MBKK_OK;
}

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

int mbkk_workspace_size(const mbkk_config *cfg, size_t *bytes)
{
    std::string why;
    int rc = check_config(cfg, why);
    if (rc)
        return fail(nullptr, rc, why);
    if (!bytes)
        return fail(nullptr, MBKK_E_INVALID, "bytes is NULL");
    Layout L = make_layout(*cfg);
    Buffers B;
    carve(L, nullptr, B);
    *bytes = L.bytes;
    return MBKK_OK;
}

// Sets up context c over the workspace (already checked): carves it and
// writes the rows and sentinels that must start at fixed values.
static int setup(mbkk_ctx *c, const mbkk_config *cfg, void *workspace, void *stream)
{
    const Layout L = make_layout(*cfg);
    c->cfg = *cfg;
    c->L = L;
    carve(c->L, (char *)workspace, c->B);
    c->stream = (hipStream_t)stream;
    c->use_mfma = wants_mfma(*cfg);
    c->fp64 = cfg->precision == MBKK_FP64;
    std::fill(c->slot_b, c->slot_b + kMaxSlots, 0);
    // zero row of the pool (segment padding target), sentinels, error flags,
    // re-score count, ring offsets
    const int64_t zr = L.PR;
    launch_fill32(c->B.pool32 + zr * L.dp, 0, L.dp, c->stream);
    if (L.bf16) {
        launch_fill32(c->B.poolhi + zr * L.dp, 0, L.dp / 2, c->stream);
        launch_fill32(c->B.poollo + zr * L.dp, 0, L.dp / 2, c->stream);
    }
    launch_fill32(c->B.poolsq + zr, 0, 1, c->stream);
    launch_fill32(c->B.poolsq64 + zr, 0, 2, c->stream);
    launch_fill32(c->B.sup_row + L.Mcap, (uint32_t)L.PR, 1, c->stream);
    launch_fill32(c->B.sup_w + L.Mcap, 0, 1, c->stream);
    launch_fill32(c->B.sup_ay + L.Mcap, 0, 1, c->stream);
    launch_fill32(c->B.flags, 0, 4, c->stream);
    launch_fill32(c->B.nresc, 0, 2, c->stream);
    launch_fill32(c->B.ring_off, 0, (int64_t)L.P * (L.k + 1), c->stream);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return fail(nullptr, MBKK_E_HIP, std::string("workspace init: ") + hipGetErrorString(e));
    return MBKK_OK;
}

int mbkk_create(const mbkk_config *cfg, void *workspace, size_t bytes, void *stream, mbkk_ctx **out)
{
    std::string why;
    int rc = check_config(cfg, why);
    if (rc)
        return fail(nullptr, rc, why);
    if (!out)
        return fail(nullptr, MBKK_E_INVALID, "out is NULL");
    Layout L = make_layout(*cfg);
    Buffers B;
    carve(L, nullptr, B);
    if (!workspace || bytes < L.bytes || ((uintptr_t)workspace & 255))
        return fail(nullptr, MBKK_E_WORKSPACE, "workspace missing, smaller than mbkk_workspace_size or not 256-byte aligned");
    mbkk_ctx *c = new mbkk_ctx();
    rc = setup(c, cfg, workspace, stream);
    if (rc) {
        delete c;
        return rc;
    }
    *out = c;
    return MBKK_OK;
}

// ---------------------------------------------------------------------------
// Workspace in a static device array, for callers that cannot allocate.
// ---------------------------------------------------------------------------
// `scratch` is the device array.  In host code its name is only a stand-in
// for the symbol: the device address of each GPU's copy comes from
// hipGetSymbolAddress, taken once per device with that device current, and
// only that address is ever handed to kernels.  One context at a time may
// use a device's array; its host-side context is static as well, so that
// mbkk_create_static allocates nothing on the device or the host heap.
constexpr size_t kStaticWorkspaceBytes = (size_t)64 << 20;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kStaticWorkspaceBytes];

static std::mutex g_static_mu;
static void *g_scratch_dev[kMaxDevices];  // device address of `scratch` per device (nullptr: not looked up)
static bool g_static_busy[kMaxDevices];
static mbkk_ctx g_static_ctx[kMaxDevices];

int mbkk_create_static(const mbkk_config *cfg, void *stream, mbkk_ctx **out)
{
    std::string why;
    int rc = check_config(cfg, why);
    if (rc)
        return fail(nullptr, rc, why);
    if (!out)
        return fail(nullptr, MBKK_E_INVALID, "out is NULL");
    Layout L = make_layout(*cfg);
    Buffers B;
    carve(L, nullptr, B);
    if (L.bytes > kStaticWorkspaceBytes)
        return fail(nullptr, MBKK_E_WORKSPACE,
                    "configuration needs " + std::to_string(L.bytes) + " bytes of workspace; the static array holds " +
                        std::to_string(kStaticWorkspaceBytes));
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return fail(nullptr, MBKK_E_HIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices)
        return fail(nullptr, MBKK_E_INVALID, "device ordinal beyond the static table");
    std::lock_guard<std::mutex> lock(g_static_mu);
    if (g_static_busy[dev])
        return fail(nullptr, MBKK_E_STATE, "the static workspace of this device is in use by another context");
    if (!g_scratch_dev[dev]) {
        // once per device, with that device current
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(nullptr, MBKK_E_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_dev[dev] = ptr;
    }
    mbkk_ctx *c = &g_static_ctx[dev];
    c->data_set = false;
    c->inited = false;
    c->iter = 1;
    c->support_iter = -1;
    c->fold_rr = -1;
    c->fold_mask = 0;
    c->seg_next_iter = -1;
    c->layout_version = -1;
    c->sig_version = -1;
    c->ymax2 = 0.0;
    c->timing = false;
    c->ev_used = 0;
    c->ms_acc = 0.0;
    c->launches = 0;
    c->err.clear();
    rc = setup(c, cfg, g_scratch_dev[dev], stream);
    if (rc)
        return rc;
    c->device = dev;
    g_static_busy[dev] = true;
    *out = c;
    return MBKK_OK;
}

int mbkk_destroy(mbkk_ctx *c)
{
    if (!c)
        return MBKK_OK;
    for (hipEvent_t e : c->ev)
        (void)hipEventDestroy(e);
    c->ev.clear();
    if (c->device >= 0) {
        // a context over a static array: the array and the context go back to the device
        std::lock_guard<std::mutex> lock(g_static_mu);
        g_static_busy[c->device] = false;
        c->device = -1;
        return MBKK_OK;
    }
    delete c;
    return MBKK_OK;
}

const char *mbkk_last_error(const mbkk_ctx *c) { return c ? c->err.c_str() : g_err.c_str(); }

int mbkk_set_data(mbkk_ctx *c, const float *X, int64_t ld)
{
    if (!c)
        return fail(nullptr, MBKK_E_INVALID, "ctx is NULL");
    if (!X || ld < c->cfg.d)
        return fail(c, MBKK_E_INVALID, "X is NULL or ld < d");
    c->B.X = X;
    c->B.ld = ld;
    launch_fill32(c->B.sqmax, 0, 1, c->stream);
    launch_row_sqnorm(X, c->L.n, c->L.d, ld, c->B.sqn, c->B.sqmax, c->stream);
    HIPCHK(c, hipGetLastError());
    unsigned int bits = 0;
    HIPCHK(c, hipMemcpyAsync(&bits, c->B.sqmax, sizeof(bits), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    float f;
    memcpy(&f, &bits, sizeof(f));
    c->ymax2 = (double)f;
    c->version++;
    c->data_set = true;
    c->inited = false;
    return MBKK_OK;
}

static int init_common(mbkk_ctx *c, const int32_t *idx_dev)
{
    const Layout &L = c->L;
    Buffers &B = c->B;
    if (c->cfg.validate && clear_flags(c))
        return MBKK_E_HIP;
    // pool rows [0, k) <- X[idx]
    launch_gather_rows(B.X, L.n, L.d, B.ld, idx_dev, L.k, L.dp, B.pool32, L.bf16 ? B.poolhi : nullptr,
                       L.bf16 ? B.poollo : nullptr, B.poolsq, B.poolsq64, B.init_idx, B.flags, c->cfg.validate,
                       c->stream);
    if (L.untrunc) {
        launch_dp_init(L, B, c->cfg.kernel, c->cfg.kernel_param, c->fp64, c->stream);
    } else {
        launch_init_state(L, B, c->cfg.kernel, c->cfg.kernel_param, c->fp64, 1, c->stream);
        launch_fill32(B.ring_off, 0, (int64_t)L.P * (L.k + 1), c->stream);
    }
    HIPCHK(c, hipGetLastError());
    c->iter = 1;
    c->support_iter = -1;
    c->fold_rr = -1;
    c->seg_next_iter = -1;
    c->version++;
    std::fill(c->slot_b, c->slot_b + kMaxSlots, 0);
    if (c->cfg.validate) {
        int rc = check_flags(c);
        if (rc)
            return rc;
    }
    c->inited = true;
    return MBKK_OK;
}

int mbkk_init_centers(mbkk_ctx *c, const int32_t *idx_dev)
{
    if (!c)
        return fail(nullptr, MBKK_E_INVALID, "ctx is NULL");
    if (!c->data_set)
        return fail(c, MBKK_E_STATE, "set_data first");
    if (!idx_dev)
        return fail(c, MBKK_E_INVALID, "idx is NULL");
    return init_common(c, idx_dev);
}

int mbkk_init_kmeanspp(mbkk_ctx *c, const double *u_host, int32_t *idx_out_dev)
{
    if (!c)
        return fail(nullptr, MBKK_E_INVALID, "ctx is NULL");
    if (!c->data_set)
        return fail(c, MBKK_E_STATE, "set_data first");
    if (!u_host)
        return fail(c, MBKK_E_INVALID, "u is NULL");
    const Layout &L = c->L;
    for (int r = 0; r < L.k; ++r)
        if (!(u_host[r] >= 0.0 && u_host[r] < 1.0))
            return fail(c, MBKK_E_INVALID, "uniforms must lie in [0, 1)");
    HIPCHK(c, hipMemcpyAsync(c->B.u, u_host, sizeof(double) * L.k, hipMemcpyHostToDevice, c->stream));
    launch_kpp_self(L, c->B, c->cfg.kernel, c->cfg.kernel_param, c->stream);
    for (int r = 0; r < L.k; ++r)
        launch_kpp_round(L, c->B, r, c->cfg.kernel, c->cfg.kernel_param, c->stream);
    HIPCHK(c, hipGetLastError());
    if (idx_out_dev)
        HIPCHK(c, hipMemcpyAsync(idx_out_dev, c->B.picks, 4 * (size_t)L.k, hipMemcpyDeviceToDevice, c->stream));
    return init_common(c, c->B.picks);
}

// One iteration of Algorithm 1 on the table of cross terms (window 0): the
// batch is staged in slot 0 (pool rows for the pair sums and the table
// update, its indices for the last batch's objective), scored from the
// table, grouped, and T and N updated.
static int dp_step(mbkk_ctx *c, const int32_t *batch, int32_t b, int32_t *labels_dev, float *mind_dev,
                   double *fbefore_host)
{
    const Layout &L = c->L;
    Buffers &B = c->B;
    const mbkk_config &cf = c->cfg;
    if (cf.validate && clear_flags(c))
        return MBKK_E_HIP;
    set_batch_view(c, 0);
    launch_gather_rows(B.X, L.n, L.d, B.ld, batch, b, L.dp, B.bat32, B.bathi, B.batlo, B.batsq, B.batsq64, B.batidx,
                       B.flags, cf.validate, c->stream);
    launch_dp_score(L, B, cf.kernel, cf.kernel_param, c->fp64, B.batidx, b, true, nullptr, 0, nullptr, c->stream);
    launch_sum_mind(B, b, 0, c->stream);
    launch_dp_update(L, B, b, cf.kernel, cf.kernel_param, c->fp64, cf.lr, c->stream);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (c->timing) {
        int rc = timing_pair(c, &e0, &e1);
        if (rc)
            return rc;
        HIPCHK(c, hipEventRecord(e0, c->stream));
    }
    launch_dp_table(L, B, cf.kernel, cf.kernel_param, c->fp64, 0, c->stream);
    if (c->timing) {
        HIPCHK(c, hipEventRecord(e1, c->stream));
        c->launches++;
    }
    HIPCHK(c, hipGetLastError());
    c->slot_b[0] = b;
    c->iter += 1;
    c->version++;
    if (labels_dev)
        HIPCHK(c, hipMemcpyAsync(labels_dev, B.labels, 4 * (size_t)b, hipMemcpyDeviceToDevice, c->stream));
    if (mind_dev)
        HIPCHK(c, hipMemcpyAsync(mind_dev, B.mind, 4 * (size_t)b, hipMemcpyDeviceToDevice, c->stream));
    if (fbefore_host) {
        double s = 0.0;
        HIPCHK(c, hipMemcpyAsync(&s, B.obj + 1, sizeof(double), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        *fbefore_host = s / (double)b;
    }
    if (cf.validate)
        return check_flags(c);
    return MBKK_OK;
}

int mbkk_step(mbkk_ctx *c, const int32_t *batch, int32_t b, int32_t *labels_dev, float *mind_dev,
              double *fbefore_host)
{
    if (!c)
        return fail(nullptr, MBKK_E_INVALID, "ctx is NULL");
    if (!c->inited)
        return fail(c, MBKK_E_STATE, "init_centers / init_kmeanspp first");
    if (!batch || b <= 0 || b > c->L.bmax)
        return fail(c, MBKK_E_INVALID, "need a batch with 1 <= b <= b_max");
    if (c->L.untrunc)
        return dp_step(c, batch, b, labels_dev, mind_dev, fbefore_host);
    const Layout &L = c->L;
    Buffers &B = c->B;
    const int64_t i = c->iter;
    const int W = L.W;
    if (c->cfg.validate && clear_flags(c))
        return MBKK_E_HIP;
    prepare(c, batch, b);
    int rc = cross_and_score(c, b, nullptr, 0, true);
    if (rc)
        return rc;
    // update of the centers
    const int P = L.P;
    const SlotList live = live_before(i, W);
    const int init_alive_before = i <= W + 1;
    const int init_keep = i <= W;
    const int p_new = phys_of(i, P);
    const int p_expired = i - W >= 1 ? phys_of(i - W, P) : -1;
    const SlotList live_after = live_before(i + 1, W);
    const uint32_t mask = col_mask_of(live_after, init_keep);
    WindowRank win;
    win.n = live_after.n;
    win.tau = c->cfg.tau;
    win.first = i + 1 - W < 1 ? 1 : i + 1 - W;  // batch of live_after.r[0]
    for (int p = 0; p < kMaxSlots; ++p)
        win.rank[p] = -1;
    for (int q = 0; q < live_after.n; ++q)
        win.rank[live_after.r[q]] = q;
    launch_update(L, B, b, p_new, p_expired, init_alive_before, init_keep, live, win, c->cfg.lr, mask,
                  gram_task_rows(c->use_mfma), gram_task_cols(c->use_mfma, c->fp64), gram_task_qmax(c->use_mfma),
                  gram_waves(c->use_mfma), c->stream);
    gram(c, p_new, mask, true);
    c->seg_next_iter = i + 1;
    HIPCHK(c, hipGetLastError());
    c->slot_b[p_new] = b;
    c->iter = i + 1;
    c->version++;
    if (labels_dev)
        HIPCHK(c, hipMemcpyAsync(labels_dev, B.labels, 4 * (size_t)b, hipMemcpyDeviceToDevice, c->stream));
    if (mind_dev)
        HIPCHK(c, hipMemcpyAsync(mind_dev, B.mind, 4 * (size_t)b, hipMemcpyDeviceToDevice, c->stream));
    if (fbefore_host) {
        double s = 0.0;
        HIPCHK(c, hipMemcpyAsync(&s, B.obj, sizeof(double), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        *fbefore_host = s / (double)b;
    }
    if (c->cfg.validate)
        return check_flags(c);
    return MBKK_OK;
}

int mbkk_assign(mbkk_ctx *c, const int32_t *idx, int64_t m, int32_t *labels_dev, float *mind_dev,
                float *margin_dev, double *D_dev)
{
    if (!c)
        return fail(nullptr, MBKK_E_INVALID, "ctx is NULL");
    if (!c->inited)
        return fail(c, MBKK_E_STATE, "init_centers / init_kmeanspp first");
    if (m < 0 || (m > 0 && !idx))
        return fail(c, MBKK_E_INVALID, "bad index array");
    const Layout &L = c->L;
    Buffers &B = c->B;
    if (c->cfg.validate && clear_flags(c))
        return MBKK_E_HIP;
    if (m == 0 && !L.untrunc)
        prepare(c, nullptr, 0);
    for (int64_t m0 = 0; m0 < m; m0 += L.bmax) {
        const int nb = (int)((m - m0) < L.bmax ? (m - m0) : L.bmax);
        if (L.untrunc) {
            launch_dp_score(L, B, c->cfg.kernel, c->cfg.kernel_param, c->fp64, idx + m0, nb, false,
                            D_dev ? D_dev + m0 * L.k : nullptr, L.k, c->cfg.validate ? B.flags : nullptr, c->stream);
        } else {
            prepare(c, idx + m0, nb);
            int rc = cross_and_score(c, nb, D_dev ? D_dev + m0 * L.k : nullptr, L.k, false);
            if (rc)
                return rc;
        }
        if (labels_dev)
            HIPCHK(c, hipMemcpyAsync(labels_dev + m0, B.labels, 4 * (size_t)nb, hipMemcpyDeviceToDevice, c->stream));
        if (mind_dev)
            HIPCHK(c, hipMemcpyAsync(mind_dev + m0, B.mind, 4 * (size_t)nb, hipMemcpyDeviceToDevice, c->stream));
        if (margin_dev)
            HIPCHK(c, hipMemcpyAsync(margin_dev + m0, B.margin, 4 * (size_t)nb, hipMemcpyDeviceToDevice, c->stream));
    }
    if (c->cfg.validate)
        return check_flags(c);
    return MBKK_OK;
}

int mbkk_objective(mbkk_ctx *c, const int32_t *idx, int64_t m, double *out_host)
{
    if (!c)
        return fail(nullptr, MBKK_E_INVALID, "ctx is NULL");
    if (!c->inited)
        return fail(c, MBKK_E_STATE, "init_centers / init_kmeanspp first");
    if (m <= 0 || !idx || !out_host)
        return fail(c, MBKK_E_INVALID, "need m > 0 indices and an output");
    const Layout &L = c->L;
    if (c->cfg.validate && clear_flags(c))
        return MBKK_E_HIP;
    for (int64_t m0 = 0; m0 < m; m0 += L.bmax) {
        const int nb = (int)((m - m0) < L.bmax ? (m - m0) : L.bmax);
        if (L.untrunc) {
            launch_dp_score(L, c->B, c->cfg.kernel, c->cfg.kernel_param, c->fp64, idx + m0, nb, false, nullptr, 0,
                            c->cfg.validate ? c->B.flags : nullptr, c->stream);
        } else {
            prepare(c, idx + m0, nb);
            int rc = cross_and_score(c, nb, nullptr, 0, false);
            if (rc)
                return rc;
        }
        launch_sum_mind(c->B, nb, m0 > 0, c->stream);
    }
    double s = 0.0;
    HIPCHK(c, hipMemcpyAsync(&s, c->B.obj + 1, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    *out_host = s / (double)m;
    if (c->cfg.validate)
        return check_flags(c);
    return MBKK_OK;
}

int mbkk_last_batch_objective(mbkk_ctx *c, double *f_host)
{
    if (!c)
        return fail(nullptr, MBKK_E_INVALID, "ctx is NULL");
    if (!c->inited || c->iter < 2)
        return fail(c, MBKK_E_STATE, "no step yet");
    if (!f_host)
        return fail(c, MBKK_E_INVALID, "f is NULL");
    // batch i-1 lives in its ring slot with its point indices in slot_pts
    const int p = phys_of(c->iter - 1, c->L.P);
    const int b = c->slot_b[p];
    if (b < 1)
        return fail(c, MBKK_E_STATE, "the last batch's slot holds no points");
    return mbkk_objective(c, c->B.slot_pts + (int64_t)p * c->L.bmax, b, f_host);
}

// Adjusted Rand index and normalised mutual information (arithmetic-mean
// normalisation) of a contingency table n[k x c], in FP64 (each pair count
// C(n, 2) is exact for cells below 2^26 rows).
static void agreement_scores(const std::vector<int64_t> &n, int k, int c, double *ari, double *nmi)
{
    std::vector<double> a(k, 0.0), b(c, 0.0);
    double N = 0.0, sij = 0.0;
    for (int i = 0; i < k; ++i)
        for (int j = 0; j < c; ++j) {
            const double v = (double)n[(size_t)i * c + j];
            a[i] += v;
            b[j] += v;
            N += v;
            sij += v * (v - 1.0) * 0.5;
        }
    double sa = 0.0, sb = 0.0, hu = 0.0, hv = 0.0;
    for (int i = 0; i < k; ++i) {
        sa += a[i] * (a[i] - 1.0) * 0.5;
        if (a[i] > 0.0)
            hu -= a[i] / N * std::log(a[i] / N);
    }
    for (int j = 0; j < c; ++j) {
        sb += b[j] * (b[j] - 1.0) * 0.5;
        if (b[j] > 0.0)
            hv -= b[j] / N * std::log(b[j] / N);
    }
    // ARI: (index - expected index) / (max index - expected index), pairs
    const double expct = sa * sb / (N * (N - 1.0) * 0.5);
    const double den = 0.5 * (sa + sb) - expct;
    *ari = den == 0.0 ? 1.0 : (sij - expct) / den;
    double mi = 0.0;
    for (int i = 0; i < k; ++i)
        for (int j = 0; j < c; ++j) {
            const double v = (double)n[(size_t)i * c + j];
            if (v > 0.0)
                mi += v / N * (std::log(v) + std::log(N) - std::log(a[i]) - std::log(b[j]));
        }
    if (hu == 0.0 && hv == 0.0)
        *nmi = 1.0;  // one cluster on both sides: identical partitions
    else
        *nmi = std::max(0.0, mi) / (0.5 * (hu + hv));
}

int mbkk_agreement(mbkk_ctx *c, const int32_t *labels_dev, const int32_t *truth_dev, int64_t m, int32_t nc,
                   int64_t *table_dev, double *ari_host, double *nmi_host)
{
    if (!c)
        return fail(nullptr, MBKK_E_INVALID, "ctx is NULL");
    if (m < 2 || m >= ((int64_t)1 << 40) || !labels_dev || !truth_dev || !table_dev || !ari_host || !nmi_host)
        return fail(c, MBKK_E_INVALID, "need 2 <= m < 2^40 rows, both labelings, a table and two outputs");
    const int k = c->L.k;
    if (nc < 1 || (int64_t)k * nc > ((int64_t)1 << 26))
        return fail(c, MBKK_E_INVALID, "need 1 <= c and k * c <= 2^26");
    launch_fill32(c->B.flags, 0, 4, c->stream);
    launch_fill32(table_dev, 0, 2 * (int64_t)k * nc, c->stream);
    launch_contingency(labels_dev, truth_dev, m, k, nc, table_dev, c->B.flags, c->stream);
    HIPCHK(c, hipGetLastError());
    std::vector<int64_t> n((size_t)k * nc);
    int32_t f[3] = {0, 0, 0};
    HIPCHK(c, hipMemcpyAsync(n.data(), table_dev, sizeof(int64_t) * n.size(), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(f, c->B.flags, sizeof(f), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (f[2])
        return fail(c, MBKK_E_INVALID, "label outside [0, k) or truth outside [0, c)");
    agreement_scores(n, k, nc, ari_host, nmi_host);
    return MBKK_OK;
}

// ---------------------------------------------------------------------------
// Differentiation form (Gaussian kernel with bandwidth sigma, kappa = 2 sigma^2)
// ---------------------------------------------------------------------------
static int grad_args(mbkk_ctx *c, const float *xb, int32_t b, double sigma)
{
    if (!c)
        return fail(nullptr, MBKK_E_INVALID, "ctx is NULL");
    if (c->L.untrunc)
        return fail(c, MBKK_E_STATE, "the differentiation form needs the centers' support (window >= 1)");
    if (!c->inited)
        return fail(c, MBKK_E_STATE, "init_centers / init_kmeanspp first");
    if (c->cfg.kernel != MBKK_GAUSS)
        return fail(c, MBKK_E_INVALID, "the differentiation form needs the Gaussian kernel");
    if (!xb || b < 1 || b > c->L.bmax)
        return fail(c, MBKK_E_INVALID, "need 1 <= b <= b_max rows of coordinates");
    if (!(sigma > 0.0) || !std::isfinite(sigma))
        return fail(c, MBKK_E_INVALID, "sigma must be finite and > 0");
    return MBKK_OK;
}

// Lays out the support of C_i with the exponent constants of bandwidth kappa
// (the cross term at sigma needs them); the next call that scores at the
// model's own bandwidth lays the support out again.
static void layout_at_sigma(mbkk_ctx *c, double sigma)
{
    const Layout &L = c->L;
    const double kappa = 2.0 * sigma * sigma;
    const SlotList live = live_before(c->iter, L.W);
    const int init_alive = c->iter <= L.W + 1;
    uint32_t fold_mask = 0;
    const int fold_rr = take_fold(c, &fold_mask);
    launch_prepare(L, c->B, true, live, init_alive, nullptr, 0, 0, (float)(-1.4426950408889634 / kappa), fold_rr,
                   fold_mask, c->seg_next_iter == c->iter, c->stream);
    c->support_iter = -1;
    c->layout_version = c->version;
}

// Self norms at sigma and their derivative, once per (state, sigma): the
// backward that follows a forward at the same sigma reuses them.
static void norms_at_sigma(mbkk_ctx *c, double sigma)
{
    if (c->sig_version == c->version && c->sig_sigma == sigma)
        return;
    if (sigma_mfma_ok(c->L))
        launch_sigma_norms(c->L, c->B, sigma, c->B.Nsig, c->B.dNsig, c->stream);
    else
        launch_selfnorm_sigma(c->L, c->B, sigma, c->B.Nsig, c->B.dNsig, c->stream);
    c->sig_version = c->version;
    c->sig_sigma = sigma;
}

int mbkk_objective_fwd(mbkk_ctx *c, const float *xb_dev, int32_t b, double sigma, int32_t *labels_dev,
                       double *f_host)
{
    int rc = grad_args(c, xb_dev, b, sigma);
    if (rc)
        return rc;
    const Layout &L = c->L;
    Buffers &B = c->B;
    const mbkk_config &cf = c->cfg;
    const double kappa = 2.0 * sigma * sigma;
    if (clear_flags(c))
        return MBKK_E_HIP;
    // the rows go to the free slot of the current iteration
    set_batch_view(c, phys_of(c->iter, L.P));
    launch_gather_rows(xb_dev, b, L.d, L.d, nullptr, b, L.dp, B.bat32, B.bathi, B.batlo, B.batsq, B.batsq64, nullptr,
                       B.flags, 1, c->stream, L.frag_mode, B.batfrag, 2 * (int64_t)frag_rows(L) * L.dp);
    layout_at_sigma(c, sigma);
    norms_at_sigma(c, sigma);
    Buffers Bs = B;
    Bs.N = B.Nsig;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (c->timing) {
        rc = timing_pair(c, &e0, &e1);
        if (rc)
            return rc;
        HIPCHK(c, hipEventRecord(e0, c->stream));
    }
    if (c->use_mfma)
        launch_cross_mfma(L, Bs, b, cf.precision, kappa, c->stream);
    else
        launch_cross_direct(L, Bs, b, MBKK_GAUSS, kappa, c->fp64, c->stream);
    if (c->timing) {
        HIPCHK(c, hipEventRecord(e1, c->stream));
        c->launches++;
    }
    launch_score(L, Bs, b, MBKK_GAUSS, kappa, c->fp64, c->use_mfma, cf.precision, tie_delta(cf), c->ymax2, nullptr, 0,
                 false, c->stream);
    launch_sum_mind(B, b, 0, c->stream);
    HIPCHK(c, hipGetLastError());
    if (labels_dev)
        HIPCHK(c, hipMemcpyAsync(labels_dev, B.labels, 4 * (size_t)b, hipMemcpyDeviceToDevice, c->stream));
    // the device scalars and the flags in one read-back
    double io[6];
    HIPCHK(c, hipMemcpyAsync(io, B.obj, sizeof(io), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    int32_t f[4];
    memcpy(f, io + 4, sizeof(f));
    if (f[1])
        return fail(c, MBKK_E_NONFINITE, "non-finite value in the coordinates");
    if (f_host)
        *f_host = io[1] / (double)b;
    return MBKK_OK;
}

int mbkk_objective_bwd(mbkk_ctx *c, const float *xb_dev, int32_t b, double sigma, const int32_t *labels_dev,
                       double g, float *dX_dev, double *dsigma_host)
{
    int rc = grad_args(c, xb_dev, b, sigma);
    if (rc)
        return rc;
    if (!labels_dev || !dX_dev || !dsigma_host)
        return fail(c, MBKK_E_INVALID, "labels, dX and dsigma are required");
    if (c->L.d > grad_max_dim())
        return fail(c, MBKK_E_INVALID, "the backward supports d <= " + std::to_string(grad_max_dim()));
    if (!std::isfinite(g))
        return fail(c, MBKK_E_INVALID, "g must be finite");
    const Layout &L = c->L;
    Buffers &B = c->B;
    if (clear_flags(c))
        return MBKK_E_HIP;
    // the support layout and the self norms of a forward at this state and
    // sigma are still valid; otherwise they are made here
    if (c->layout_version != c->version)
        layout_at_sigma(c, sigma);
    norms_at_sigma(c, sigma);
    if (sigma_mfma_ok(L)) {
        // the coordinates go to the free slot, as in the forward
        set_batch_view(c, phys_of(c->iter, L.P));
        launch_gather_rows(xb_dev, b, L.d, L.d, nullptr, b, L.dp, B.bat32, nullptr, nullptr, B.batsq, B.batsq64,
                           nullptr, B.flags, 0, c->stream);
        launch_grad_mfma(L, B, b, sigma, labels_dev, g, B.dNsig, dX_dev, B.rowds, B.obj + 2, c->stream);
    } else {
        launch_grad_rows(L, B, xb_dev, b, sigma, labels_dev, g, B.dNsig, dX_dev, B.rowds, B.obj + 2, c->stream);
    }
    HIPCHK(c, hipGetLastError());
    double io[6];
    HIPCHK(c, hipMemcpyAsync(io, B.obj, sizeof(io), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    int32_t f[4];
    memcpy(f, io + 4, sizeof(f));
    if (f[2])
        return fail(c, MBKK_E_INVALID, "label outside [0, k)");
    *dsigma_host = io[2];
    return MBKK_OK;
}

int mbkk_center_norms(mbkk_ctx *c, double *N_host)
{
    if (!c)
        return fail(nullptr, MBKK_E_INVALID, "ctx is NULL");
    if (!c->inited)
        return fail(c, MBKK_E_STATE, "init_centers / init_kmeanspp first");
    if (!N_host)
        return fail(c, MBKK_E_INVALID, "N is NULL");
    if (!c->L.untrunc)
        prepare(c, nullptr, 0);
    HIPCHK(c, hipMemcpyAsync(N_host, c->B.N, 8 * (size_t)c->L.k, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return MBKK_OK;
}

int mbkk_get_state(mbkk_ctx *c, mbkk_state *s)
{
    if (!c)
        return fail(nullptr, MBKK_E_INVALID, "ctx is NULL");
    if (c->L.untrunc)
        return fail(c, MBKK_E_STATE, "window 0 keeps the centers as the table of cross terms: no state image");
    if (!c->inited)
        return fail(c, MBKK_E_STATE, "no state yet");
    const Layout &L = c->L;
    if (!s || s->k != L.k || s->window != L.W || s->b_max != L.bmax || !s->init_idx || !s->slot_b ||
        !s->slot_idx || !s->slot_off || !s->coef || !s->cum)
        return fail(c, MBKK_E_INVALID, "state buffers missing or shaped for another configuration");
    const int W = L.W, P = L.P, C = L.C, Cs = W + 1;
    const int64_t i = c->iter;
    std::vector<int32_t> ridx((size_t)P * L.bmax), roff((size_t)P * (L.k + 1));
    std::vector<double> coef((size_t)L.k * C);
    HIPCHK(c, hipMemcpyAsync(s->init_idx, c->B.init_idx, 4 * (size_t)L.k, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(ridx.data(), c->B.ring_idx, 4 * ridx.size(), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(roff.data(), c->B.ring_off, 4 * roff.size(), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(coef.data(), c->B.coef, 8 * coef.size(), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(s->cum, c->B.cum, 8 * (size_t)L.k, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    // physical slot of batch l -> logical slot (l-1) mod W of the state image
    s->iteration = i;
    for (int r = 0; r < W; ++r)
        s->slot_b[r] = 0;
    memset(s->slot_off, 0, sizeof(int32_t) * (size_t)W * (L.k + 1));
    for (int j = 0; j < L.k; ++j)
        for (int cc = 0; cc < Cs; ++cc)
            s->coef[(size_t)j * Cs + cc] = cc == 0 ? coef[(size_t)j * C] : 0.0;
    const int64_t lo = i - W < 1 ? 1 : i - W;
    for (int64_t l = lo; l <= i - 1; ++l) {
        const int p = phys_of(l, P), r = (int)((l - 1) % W);
        s->slot_b[r] = c->slot_b[p];
        memcpy(s->slot_idx + (size_t)r * L.bmax, ridx.data() + (size_t)p * L.bmax, 4 * (size_t)L.bmax);
        memcpy(s->slot_off + (size_t)r * (L.k + 1), roff.data() + (size_t)p * (L.k + 1), 4 * (size_t)(L.k + 1));
        for (int j = 0; j < L.k; ++j)
            s->coef[(size_t)j * Cs + 1 + r] = coef[(size_t)j * C + 1 + p];
    }
    return MBKK_OK;
}

int mbkk_set_state(mbkk_ctx *c, const mbkk_state *s)
{
    if (!c)
        return fail(nullptr, MBKK_E_INVALID, "ctx is NULL");
    if (c->L.untrunc)
        return fail(c, MBKK_E_STATE, "window 0 keeps the centers as the table of cross terms: no state image");
    if (!c->data_set)
        return fail(c, MBKK_E_STATE, "set_data first");
    const Layout &L = c->L;
    if (!s || s->k != L.k || s->window != L.W || s->b_max != L.bmax || !s->init_idx || !s->slot_b ||
        !s->slot_idx || !s->slot_off || !s->coef || !s->cum || s->iteration < 1)
        return fail(c, MBKK_E_INVALID, "state buffers missing or shaped for another configuration");
    const int W = L.W, P = L.P, C = L.C, Cs = W + 1;
    const int64_t i = s->iteration;
    const bool init_alive = i <= W + 1;
    const int64_t lo = i - W < 1 ? 1 : i - W;
    // host-side validation of the live logical slots (batch l in slot (l-1) mod W)
    for (int64_t l = lo; l <= i - 1; ++l) {
        const int r = (int)((l - 1) % W);
        const int32_t *off = s->slot_off + (int64_t)r * (L.k + 1);
        // (a live slot may hold no points: with tau every center can have
        // dropped that batch)
        if (s->slot_b[r] < 0 || s->slot_b[r] > L.bmax || off[0] != 0 || off[L.k] != s->slot_b[r])
            return fail(c, MBKK_E_INVALID, "slot offsets inconsistent with slot sizes");
        for (int j = 0; j < L.k; ++j)
            if (off[j + 1] < off[j])
                return fail(c, MBKK_E_INVALID, "slot offsets not monotone");
        for (int q = 0; q < s->slot_b[r]; ++q) {
            const int32_t v = s->slot_idx[(int64_t)r * L.bmax + q];
            if (v < 0 || v >= L.n)
                return fail(c, MBKK_E_INDEX, "slot index outside [0, n)");
        }
    }
    for (int j = 0; j < L.k; ++j)
        if (s->init_idx[j] < 0 || s->init_idx[j] >= L.n)
            return fail(c, MBKK_E_INDEX, "initial index outside [0, n)");
    Buffers &B = c->B;
    // physical images: batch l -> slot (l-1) mod P, rows in the image's
    // grouped order (identity permutation); dead columns get coefficient 0
    std::vector<double> coef((size_t)L.k * C, 0.0);
    std::vector<int32_t> offs((size_t)P * (L.k + 1), 0), idx((size_t)P * L.bmax, 0), perm((size_t)P * L.bmax, 0);
    std::vector<int32_t> sb(P, 0);
    for (int j = 0; j < L.k; ++j)
        coef[(size_t)j * C] = init_alive ? s->coef[(size_t)j * Cs] : 0.0;
    for (int64_t l = lo; l <= i - 1; ++l) {
        const int r = (int)((l - 1) % W), p = phys_of(l, P);
        sb[p] = s->slot_b[r];
        memcpy(offs.data() + (size_t)p * (L.k + 1), s->slot_off + (size_t)r * (L.k + 1), 4 * (size_t)(L.k + 1));
        memcpy(idx.data() + (size_t)p * L.bmax, s->slot_idx + (size_t)r * L.bmax, 4 * (size_t)sb[p]);
        for (int q = 0; q < sb[p]; ++q)
            perm[(size_t)p * L.bmax + q] = q;
        for (int j = 0; j < L.k; ++j)
            coef[(size_t)j * C + 1 + p] = s->coef[(size_t)j * Cs + 1 + r];
    }
    const SlotList live = live_before(i, W);
    const uint32_t mask = col_mask_of(live, init_alive);
    HIPCHK(c, hipMemcpyAsync(B.ring_idx, idx.data(), 4 * idx.size(), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(B.slot_pts, idx.data(), 4 * idx.size(), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(B.ring_perm, perm.data(), 4 * perm.size(), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(B.ring_off, offs.data(), 4 * offs.size(), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(B.coef, coef.data(), 8 * coef.size(), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(B.cum, s->cum, 8 * (size_t)L.k, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(B.picks, s->init_idx, 4 * (size_t)L.k, hipMemcpyHostToDevice, c->stream));
    // initial points, G reset with G[j][0][0] = K(x_j, x_j); a fold left by a
    // step of the replaced state is dropped
    c->fold_rr = -1;
    c->seg_next_iter = -1;
    launch_gather_rows(B.X, L.n, L.d, B.ld, B.picks, L.k, L.dp, B.pool32, L.bf16 ? B.poolhi : nullptr,
                       L.bf16 ? B.poollo : nullptr, B.poolsq, B.poolsq64, B.init_idx, B.flags, 0, c->stream);
    launch_init_state(L, B, c->cfg.kernel, c->cfg.kernel_param, c->fp64, 0, c->stream);
    // coordinates of the live slots
    for (int q = 0; q < live.n; ++q) {
        const int p = live.r[q];
        const int64_t r0 = slot_row(L, p, 0);
        launch_gather_rows(B.X, L.n, L.d, B.ld, B.ring_idx + (int64_t)p * L.bmax, sb[p], L.dp,
                           B.pool32 + r0 * L.dp, L.bf16 ? B.poolhi + r0 * L.dp : nullptr,
                           L.bf16 ? B.poollo + r0 * L.dp : nullptr, B.poolsq + r0, B.poolsq64 + r0, nullptr,
                           B.flags, 0, c->stream);
    }
    // Gram blocks of every live slot against every live column
    for (int q = 0; q < live.n; ++q) {
        const int p = live.r[q];
        gram(c, p, mask, false);
    }
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (int p = 0; p < P; ++p)
        c->slot_b[p] = sb[p];
    c->iter = i;
    c->support_iter = -1;
    c->version++;
    c->inited = true;
    return MBKK_OK;
}

int mbkk_rescore_count(mbkk_ctx *c, int64_t *rows_host, int32_t reset)
{
    if (!c)
        return fail(nullptr, MBKK_E_INVALID, "ctx is NULL");
    if (!rows_host)
        return fail(c, MBKK_E_INVALID, "rows is NULL");
    unsigned long long v = 0;
    HIPCHK(c, hipMemcpyAsync(&v, c->B.nresc, sizeof(v), hipMemcpyDeviceToHost, c->stream));
    if (reset)
        launch_fill32(c->B.nresc, 0, 2, c->stream);
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipStreamSynchronize(c->stream));
    *rows_host = (int64_t)v;
    return MBKK_OK;
}

int mbkk_selfnorm_error_bound(mbkk_ctx *c, double *bound_host)
{
    if (!c)
        return fail(nullptr, MBKK_E_INVALID, "ctx is NULL");
    if (!bound_host)
        return fail(c, MBKK_E_INVALID, "bound is NULL");
    if (!c->data_set)
        return fail(c, MBKK_E_STATE, "set_data first");
    if (!c->use_mfma || c->cfg.kernel != MBKK_GAUSS)
        return fail(c, MBKK_E_STATE, "the bound covers the Gaussian MFMA forms");
    *bound_host = selfnorm_error_bound(c->L.dp, c->ymax2, c->cfg.kernel_param);
    return MBKK_OK;
}

int mbkk_set_timing(mbkk_ctx *c, int32_t enable)
{
    if (!c)
        return fail(nullptr, MBKK_E_INVALID, "ctx is NULL");
    c->timing = enable != 0;
    c->ev_used = 0;
    c->ms_acc = 0.0;
    c->launches = 0;
    // events are created here, outside any timed loop
    while (c->timing && c->ev.size() < 1024) {
        hipEvent_t e;
        HIPCHK(c, hipEventCreate(&e));
        c->ev.push_back(e);
    }
    return MBKK_OK;
}

int mbkk_get_timing(mbkk_ctx *c, double *ms_host, int64_t *launches_host)
{
    if (!c)
        return fail(nullptr, MBKK_E_INVALID, "ctx is NULL");
    HIPCHK(c, hipStreamSynchronize(c->stream));
    double ms = 0.0;
    for (size_t q = 0; q + 1 < c->ev_used; q += 2) {
        float t = 0.0f;
        HIPCHK(c, hipEventElapsedTime(&t, c->ev[q], c->ev[q + 1]));
        ms += t;
    }
    if (ms_host)
        *ms_host = ms;
    if (launches_host)
        *launches_host = c->launches;
    return MBKK_OK;
}

}  // extern "C"
