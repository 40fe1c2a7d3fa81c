/*
 * mbkk.h - C ABI of the MI355X (gfx950) library for truncated mini-batch
 * kernel k-means (Jourdan & Schwartzman, "Mini-batch kernel k-means",
 * ICLR 2025).
 *
 * The library runs the per-iteration hot path of the paper's Algorithm 2 on
 * one GPU: batch-to-center distances in feature space by the kernel trick
 * (Section 1, "Lloyd's algorithm in feature space"; Section 4), argmin
 * assignment, the learning-rate update of the implicit centers and their
 * truncation to a window of recent batches (Section 4.1, Eq. 1 and the
 * unrolled recursion before it; sliding-window footnote).
 *
 * window = 0 selects the untruncated Algorithm 1 instead, run on the table
 * of cross terms that Appendix A describes: the context keeps
 * <phi(x), C_j> for every row x of X and every center j (a k x n table in the
 * workspace, FP32 or FP64 by the precision) and <C_j, C_j>, and each step
 * updates both by the recursion of Section 4 (O(n b) kernel evaluations and
 * one pass over the table).  In that form tau must be 0, the precision FP32,
 * FP64 or BF16X3 (Gaussian) and d <= 128; the Gaussian runs the update on
 * MFMA in BF16X3, and in FP32 with cross_impl AUTO and d >= 16 or MFMA (the
 * workspace then also holds a k x n FP32 array of the step's sums), else on
 * the VALU; BF16X3 has no FP64 re-scoring in this form; mbkk_get_state,
 * mbkk_set_state and the differentiation form return MBKK_E_STATE; an
 * out-of-range index in mbkk_step / mbkk_assign / mbkk_objective is scored
 * as row 0 (and reported under validate), see the conventions below.
 *
 * Conventions for every entry point:
 *  - Pointers named *_dev are device pointers (HIP / torch CUDA tensors on the
 *    ROCm build); pointers named *_host are host pointers.  Device arrays are
 *    dense, row-major, caller-owned; the library never frees them.
 *  - All GPU work is enqueued on the stream given to mbkk_create, in stream
 *    order.  Calls that write a *_host output synchronise that stream.
 *  - Return value: MBKK_OK (0) or a negative MBKK_E_* code; no C++ exception
 *    crosses the ABI.  mbkk_last_error() gives a message for the context (or
 *    for the last failed mbkk_create when called with NULL).
 *  - A context is not thread-safe; calls on one context must be serialised.
 *  - Index arrays are int32 row numbers of X in [0, n).  Out-of-range indices
 *    are never dereferenced, and when config.validate is non-zero the call
 *    returns MBKK_E_INDEX (this check synchronises the stream).  Without
 *    validate the result for such an entry is defined but meaningless, and
 *    differs between the forms: the truncated forms (window >= 1) score a
 *    row of zeros in its place; the table form (window = 0), which holds
 *    cross terms only for rows of X, scores row 0.
 */
#ifndef MBKK_H
#define MBKK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Return codes. */
#define MBKK_OK 0
#define MBKK_E_INVALID (-1)    /* bad argument or configuration            */
#define MBKK_E_STATE (-2)      /* call out of order (e.g. step before init) */
#define MBKK_E_WORKSPACE (-3)  /* workspace missing, too small or misaligned */
#define MBKK_E_HIP (-4)        /* a HIP runtime call failed                  */
#define MBKK_E_INDEX (-5)      /* index outside [0, n) (validate only)       */
#define MBKK_E_NONFINITE (-6)  /* NaN/Inf in gathered rows (validate only)   */

/* Kernel functions K(x, y) (the paper's K; kernel_param is its bandwidth).
 * GAUSS  : exp(-||x-y||_2^2 / kappa), kernel_param = kappa   (Section 6)
 * LAPLACE: exp(-||x-y||_1  / sigma), kernel_param = sigma    (abstract)
 * LINEAR : <x, y>                                             (test kernel)
 * POLY2  : (<x, y> + c)^2,            kernel_param = c        (test kernel) */
#define MBKK_GAUSS 0
#define MBKK_LAPLACE 1
#define MBKK_LINEAR 2
#define MBKK_POLY2 3

/* Arithmetic of the cross term <phi(x), C_j>.
 * FP32  : FP32 kernel values.  Gaussian via ||x||^2 + ||y||^2 - 2 x.y with x.y
 *         on FP32 MFMA (or direct VALU when cross_impl = DIRECT); the other
 *         kernels on the VALU.
 * FP64  : every kernel value and sum in FP64 (VALU).
 * BF16X3: Gaussian only; x.y of the cross term on BF16 MFMA as the
 *         compensated split product hi.hi + hi.lo + lo.hi with FP32
 *         accumulation, norms and the exp argument in FP32; the centers' self
 *         norms from FP32 MFMA kernel values summed in FP64.  Rows whose two
 *         best distances are closer than an error bound of the form are
 *         re-scored in FP64: the cross term of every candidate center (those
 *         within the bound of the best) is recomputed from the FP32
 *         coordinates, so a re-scored distance carries only the error of N_j
 *         (mbkk_selfnorm_error_bound).  The bound follows from the bf16 split
 *         (|x - hi| <= 2^-8 |x|, |x - hi - lo| <= 2^-16 |x|), the FP32 sums,
 *         ||x||, the largest ||y||^2 of the data and kappa; a positive
 *         tie_delta replaces it.  Ties are broken arbitrarily in Section 5;
 *         here, as in every form, by the lowest center index.
 * BF16X1: as BF16X3 with the single product hi.hi (information only). */
#define MBKK_FP32 0
#define MBKK_FP64 1
#define MBKK_BF16X3 2
#define MBKK_BF16X1 3

/* Learning-rate rules alpha_i^j (b_i^j = |B_i^j|). */
#define MBKK_LR_BETA 0     /* sqrt(b_i^j / b)           (Section 5)            */
#define MBKK_LR_FULL 1     /* 1 if b_i^j > 0, else 0     (b = n gives Lloyd)    */
#define MBKK_LR_SKLEARN 2  /* b_i^j / sum_{l<=i} b_l^j   (count rate, to 0)     */

/* Cross-term implementation choice. */
#define MBKK_CROSS_AUTO 0    /* MFMA for Gaussian FP32/BF16 when d >= 16, else direct */
#define MBKK_CROSS_DIRECT 1  /* VALU kernel, any kernel and precision              */
#define MBKK_CROSS_MFMA 2    /* MFMA kernel (Gaussian, FP32/BF16 only)             */

typedef struct {
    int64_t n;           /* rows of X                                            */
    int32_t d;           /* columns of X                                         */
    int32_t k;           /* number of centers, 1 <= k <= 65536, k <= n           */
    int32_t b_max;       /* largest batch or index chunk, 1 <= b_max <= 8192     */
    int32_t window;      /* W: a center keeps its last W batches, 1 <= W <= 30;  */
                         /* 0: untruncated, on the table of cross terms          */
    int32_t kernel;      /* MBKK_GAUSS ...                                       */
    double kernel_param; /* kappa / sigma / c; > 0 for GAUSS and LAPLACE         */
    int32_t precision;   /* MBKK_FP32 ...                                        */
    int32_t lr;          /* MBKK_LR_BETA ...                                     */
    int32_t cross_impl;  /* MBKK_CROSS_AUTO ...                                  */
    double tie_delta;    /* BF16 forms: FP64 re-scoring threshold; <= 0: bound   */
    int32_t validate;    /* non-zero: report bad indices / non-finite rows       */
    int32_t tau;         /* 0: the window alone truncates; > 0: also the count   */
                         /* rule of Section 4.1: a center keeps its newest       */
                         /* batches (within the window) up to the one at which   */
                         /* its counts reach tau, and drops the older ones and   */
                         /* its initial point unless that is batch 1             */
} mbkk_config;

typedef struct mbkk_ctx mbkk_ctx;

/* Host-side image of the iteration state (all arrays caller-allocated).
 * Before iteration i the centers are C_i^j = coef[j][0] phi(x_{init_idx[j]})
 * + sum over live ring slots r of coef[j][1+r] * sum_{p in slot r, center j}
 * phi(x_p)   (Eq. 1: per-point weight alpha_l^j / b_l^j times the product of
 * (1 - alpha) of the later iterations).  Slot r holds batch l with
 * (l - 1) mod W = r; its points are grouped by center, center j occupying
 * positions slot_off[r][j] .. slot_off[r][j+1]-1.  Slots live before
 * iteration i: batches max(1, i-W) .. i-1; the initial term is live while
 * i <= W + 1.  Coefficients of dead slots must be 0. */
typedef struct {
    int64_t iteration;  /* i, the index of the next batch (1 after init)    */
    int32_t k, window, b_max;
    int32_t *init_idx;  /* [k]                                               */
    int32_t *slot_b;    /* [W] number of points held by slot r (0 = empty)   */
    int32_t *slot_idx;  /* [W * b_max] point indices, grouped by center      */
    int32_t *slot_off;  /* [W * (k + 1)] center offsets within each slot      */
    double *coef;       /* [k * (W + 1)]                                     */
    double *cum;        /* [k] running counts (sklearn rate)                 */
} mbkk_state;

/* Bytes of device workspace that mbkk_create needs for this configuration. */
int mbkk_workspace_size(const mbkk_config *cfg, size_t *bytes);

/* Creates a context.  workspace_dev: device buffer of at least
 * mbkk_workspace_size bytes, 256-byte aligned, owned by the caller and kept
 * alive until mbkk_destroy (all device state lives there; the library does
 * not allocate device memory).  stream: a hipStream_t (NULL = default). */
int mbkk_create(const mbkk_config *cfg, void *workspace_dev, size_t bytes, void *stream,
                mbkk_ctx **out);
int mbkk_destroy(mbkk_ctx *ctx);
const char *mbkk_last_error(const mbkk_ctx *ctx);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): mbkk_create without a
 * workspace argument.  The context's device state lives in a static device
 * array of the library, 64 MiB (67108864 bytes) per GPU, held
 * from the library's first use on a GPU until the process ends; the host-side
 * context is static too, and neither call allocates device or heap memory.
 * The context works on the current device (stream must belong to it) and is
 * used with every other entry point exactly like one from mbkk_create.
 * Limits: one such context per device at a time (a second call before
 * mbkk_destroy of the first returns MBKK_E_STATE); a configuration whose
 * mbkk_workspace_size exceeds the array returns MBKK_E_WORKSPACE.  The array
 * keeps the previous context's contents; creation clears what must start at
 * fixed values, and everything else is written before it is read.  Work of
 * two contexts that overlaps in time on one device would race on the array,
 * which the one-context rule excludes. */
int mbkk_create_static(const mbkk_config *cfg, void *stream, mbkk_ctx **out);

/* Borrows X_dev (n x d FP32, row stride ld >= d elements, 16-byte aligned
 * rows when ld % 4 == 0) and caches ||x||^2 for every row.  X_dev must stay
 * valid and unchanged for the lifetime of the context. */
int mbkk_set_data(mbkk_ctx *ctx, const float *X_dev, int64_t ld);

/* Initial centers C_1^j = phi(x_{idx[j]}), single points, hence convex
 * combinations of X as Algorithm 1 requires.  idx_dev: [k] device int32.
 * Resets the iteration counter to 1. */
int mbkk_init_centers(mbkk_ctx *ctx, const int32_t *idx_dev);

/* Kernel k-means++ seeding (Section 1: "kernel version of k-means++"), all
 * on the device in FP64: first pick floor(u[0] n); pick r is the first row p
 * whose running sum of D2 exceeds u[r] * sum D2, D2(p) = min over chosen c of
 * K(p,p) - 2K(p,c) + K(c,c).  u_host: [k] uniforms in [0,1).  Writes the picks
 * to idx_out_dev ([k] int32, may be NULL) and initialises the centers. */
int mbkk_init_kmeanspp(mbkk_ctx *ctx, const double *u_host, int32_t *idx_out_dev);

/* One iteration of Algorithm 2 on the batch tuple B_i = batch_dev[0..b-1]
 * (indices, duplicates allowed, 1 <= b <= b_max): distances to C_i, argmin
 * (lowest center index on ties), counts b_i^j, learning rates, update and
 * truncation of the centers.  Optional outputs: labels_dev [b] int32,
 * mind_dev [b] FP32 (distance to the assigned center), fbefore_host (the
 * batch objective f_{B_i}(C_i), synchronises). */
int mbkk_step(mbkk_ctx *ctx, const int32_t *batch_dev, int32_t b, int32_t *labels_dev,
              float *mind_dev, double *fbefore_host);

/* Assignment of m points (any m >= 0, processed in chunks of b_max) to the
 * current centers, no state change.  Outputs (each may be NULL): labels_dev
 * [m] int32, mind_dev [m] FP32, margin_dev [m] FP32 (second smallest minus
 * smallest distance), D_dev [m * k] FP64 (all distances, row-major; in the
 * BF16 forms the candidates of a re-scored row hold their FP64 values). */
int mbkk_assign(mbkk_ctx *ctx, const int32_t *idx_dev, int64_t m, int32_t *labels_dev,
                float *mind_dev, float *margin_dev, double *D_dev);

/* f_A(C) = (1/m) sum_{x in A} min_j ||phi(x) - C_j||^2 (Section 3) for the m
 * points idx_dev[0..m-1]; synchronises. */
int mbkk_objective(mbkk_ctx *ctx, const int32_t *idx_dev, int64_t m, double *out_host);

/* f_{B_i}(C_{i+1}): the objective of the last step's batch B_i (its tuple of
 * points, duplicates included) on the centers after that step's update: the
 * second term of the early-stopping test of Algorithms 1 and 2, whose first
 * term f_{B_i}(C_i) is mbkk_step's fbefore.  Scores the batch again (one
 * assignment pass); synchronises.  MBKK_E_STATE before the first step. */
int mbkk_last_batch_objective(mbkk_ctx *ctx, double *f_host);

/* Agreement of a labeling with reference labels, the two quality scores of
 * Section 6: the adjusted Rand index (pair counting, corrected for chance)
 * and the normalised mutual information I(U; V) / ((H(U) + H(V)) / 2),
 * natural logarithms.  labels_dev [m] int32 in [0, k) (e.g. from
 * mbkk_assign), truth_dev [m] int32 in [0, c), 2 <= m < 2^40, 1 <= c,
 * k * c <= 2^26; table_dev [k x c] int64 row-major device array owned by the
 * caller, overwritten with the contingency table (cell (i, j) = rows with
 * label i and truth j).  Writes ari_host and nmi_host (FP64, computed on the
 * host from the table).  Conventions: ARI = 1 when both labelings are one
 * cluster, or both all singletons; NMI = 1 when both are one cluster.
 * Returns MBKK_E_INVALID for a value outside its range (the table then holds
 * the in-range rows only).  Synchronises. */
int mbkk_agreement(mbkk_ctx *ctx, const int32_t *labels_dev, const int32_t *truth_dev, int64_t m, int32_t c,
                   int64_t *table_dev, double *ari_host, double *nmi_host);

/* Copies the iteration state to / from host memory (checkpoint, resume,
 * lock-step comparison).  set_state recomputes the center Gram blocks. */
int mbkk_get_state(mbkk_ctx *ctx, mbkk_state *out_host);
int mbkk_set_state(mbkk_ctx *ctx, const mbkk_state *in_host);

/* Differentiation form, for tuning the bandwidth of the Gaussian kernel
 * (Section 6 sets it by hand; here it can follow a gradient).  With the
 * kernel in bandwidth form K_s(x, y) = exp(-||x - y||^2 / (2 s^2)) (kappa =
 * 2 s^2) and the current centers' support points and weights held constant,
 * the batch objective of Section 3 as a function of the batch coordinates xb
 * and of s:
 *   f(xb, s) = (1/b) sum_x min_j ||phi_s(x) - C_j||^2
 *            = (1/b) sum_x [1 - 2 sum_{e in C_j} w_e K_s(x, y_e) + <C_j, C_j>_s],
 * j the argmin (lowest index on ties), <C_j, C_j>_s re-evaluated at s.
 * Gaussian kernel only; no state change.
 *
 * mbkk_objective_fwd: xb_dev [b x d] FP32 row-major dense device array,
 * 1 <= b <= b_max, sigma > 0.  Writes labels_dev [b] int32 (may be NULL) and
 * f_host.  The cross term uses the context's precision form.  Returns
 * MBKK_E_NONFINITE for NaN/Inf coordinates. */
int mbkk_objective_fwd(mbkk_ctx *ctx, const float *xb_dev, int32_t b, double sigma, int32_t *labels_dev,
                       double *f_host);

/* mbkk_objective_bwd: gradient of g * f at fixed labels labels_dev [b] (those
 * of the forward: the hard assignment, a subgradient at ties):
 *   dX_dev [b x d] FP32 = g (2 / (b s^2)) sum_{e in C_j} w_e K_s(x, y_e) (x - y_e)
 *   dsigma_host        = g (1/b) sum_x [-2 sum_e w_e K_s(x, y_e) ||x - y_e||^2 / s^3
 *                                       + d<C_j, C_j>_s / ds].
 * Kernel values are recomputed (nothing of size b x M is stored); FP64
 * arithmetic; d <= 1024.  Returns MBKK_E_INVALID for a label outside [0, k). */
int mbkk_objective_bwd(mbkk_ctx *ctx, const float *xb_dev, int32_t b, double sigma, const int32_t *labels_dev,
                       double g, float *dX_dev, double *dsigma_host);

/* Self norms <C_j, C_j> of the current centers (FP64, accumulated from the
 * Gram blocks), N_host [k]; synchronises. */
int mbkk_center_norms(mbkk_ctx *ctx, double *N_host);

/* Near-tie re-scoring of the BF16 forms (the assignment step of Algorithm 2,
 * whose ties Section 5 leaves arbitrary).  mbkk_rescore_count: the number
 * of rows re-scored in FP64 by every scoring pass (step, assign, objective,
 * objective_fwd) since mbkk_create or the last reset; reset != 0 clears the
 * count after reading it; synchronises.  Always 0 in the FP32 and FP64
 * forms.  mbkk_selfnorm_error_bound: the bound on |N_j - <C_j, C_j>| of the
 * Gaussian MFMA forms (FP32 kernel values summed in FP64), from d, the
 * largest ||x||^2 of the data and kappa; after re-scoring, a row's label is
 * the exact argmin wherever the exact margin exceeds twice this bound.
 * MBKK_E_STATE before mbkk_set_data or for another form. */
int mbkk_rescore_count(mbkk_ctx *ctx, int64_t *rows_host, int32_t reset);
int mbkk_selfnorm_error_bound(mbkk_ctx *ctx, double *bound_host);

/* Accumulated device time of the cross-term kernel (the dominant kernel of
 * mbkk_step, mbkk_assign, mbkk_objective and mbkk_objective_fwd; for window 0
 * the table update) in milliseconds and the number of launches since the last
 * reset, measured with HIP events on the context's stream when timing is
 * enabled. */
int mbkk_set_timing(mbkk_ctx *ctx, int32_t enable);
int mbkk_get_timing(mbkk_ctx *ctx, double *ms_host, int64_t *launches_host);

#ifdef __cplusplus
}
#endif
#endif /* MBKK_H */
