// Launch helpers of the mbkk kernels (internal).
#pragma once

#include "mbkk_internal.h"

namespace mbkk {

// p[0 .. nwords) = v (32-bit words): the library's only way of clearing memory.
void launch_fill32(void *p, uint32_t v, int64_t nwords, hipStream_t st);
void launch_row_sqnorm(const float *X, int64_t n, int d, int64_t ld, float *sqn, unsigned int *sqmax,
                       hipStream_t st);
// frag_mode 1 / 2: also write the rows (as batch rows 0..cnt-1) in MFMA
// fragment order into frag (BF16 hi, then lo at byte offset frag_lo / FP32).
void launch_gather_rows(const float *X, int64_t n, int d, int64_t ld, const int32_t *idx, int64_t cnt,
                        int dp, float *out32, uint16_t *outhi, uint16_t *outlo, float *outsq,
                        double *outsq64, int32_t *idx_copy, int32_t *flags, int check_finite,
                        hipStream_t st, int frag_mode = 0, char *frag = nullptr, int64_t frag_lo = 0);
void launch_init_state(const Layout &L, const Buffers &B, int kind, double param, int fp64, int set_coef,
                       hipStream_t st);
// fold_rr >= 0: the Gram work of slot fold_rr against fold_mask is folded
// into G by the support layout (before the self norms use it).  seg_ready:
// B.seg_next holds the segment offsets of this support (from the update).
void launch_prepare(const Layout &L, const Buffers &B, bool with_support, const SlotList &live, int init_alive,
                    const int32_t *idx, int64_t cnt, int check_finite, float ay_scale, int fold_rr,
                    uint32_t fold_mask, bool seg_ready, hipStream_t st);
// The update also writes the task plan of the new slot's Gram blocks against
// the columns in gram_mask (tasks gram_ta slot rows by 1..gram_qmax tiles of
// gram_te column rows: the fewest tiles whose tasks fit in gram_nwaves
// waves), and the segment offsets of the support over those columns into
// B.seg_next.  win: the window after the update and tau (> 0: the count
// truncation of each center, whose dropped columns get coefficient 0).
void launch_update(const Layout &L, const Buffers &B, int b, int p_new, int p_expired, int init_alive_before,
                   int init_keep, const SlotList &live, const WindowRank &win, int lr, uint32_t gram_mask,
                   int gram_ta, int gram_te, int gram_qmax, int gram_nwaves, hipStream_t st);

// Gram blocks of slot rr against the columns in col_mask: plan (when not made
// by the update), then work and fold.  mfma: the Gaussian MFMA forms (FP32
// MFMA products in every precision form); else VALU in FP64 or FP32.
int gram_task_cols(int mfma, int fp64);  // te of the plan for the chosen Gram form
int gram_task_rows(int mfma);            // ta of the plan for the chosen Gram form
int gram_task_qmax(int mfma);            // most column tiles per task the Gram form takes
void launch_gram_plan(const Layout &L, const Buffers &B, int rr, uint32_t col_mask, int ta, int te, hipStream_t st);
void launch_gram(const Layout &L, const Buffers &B, int rr, uint32_t col_mask, int kind, double param, int fp64,
                 int mfma, bool fold, hipStream_t st);
void launch_gram_fold(const Layout &L, const Buffers &B, int rr, uint32_t col_mask, int mfma, hipStream_t st);
int gram_waves(int mfma);  // waves of the Gram work kernel of that form (its task ranges)

// Cross term P = <phi(x), C_j> for the staged batch rows [0, nb).
void launch_cross_direct(const Layout &L, const Buffers &B, int nb, int kind, double param, int fp64,
                         hipStream_t st);
void launch_cross_mfma(const Layout &L, const Buffers &B, int nb, int precision, double kappa,
                       hipStream_t st);
// Distances, argmin, margin (and optionally every distance) of rows [0, nb).
// BF16 forms: rows whose margin is below tie_delta (> 0), or below the
// per-row error bound of the form (tie_delta <= 0; ymax2 bounds ||y||^2 of
// every support row), are re-scored in FP64.
void launch_score(const Layout &L, const Buffers &B, int nb, int kind, double param, int fp64, int mfma,
                  int precision, double tie_delta, double ymax2, double *D_out, int64_t ldD, bool with_rank,
                  hipStream_t st);
void launch_sum_mind(const Buffers &B, int nb, int accumulate, hipStream_t st);
// Bound on the error of a self norm N_j of the Gaussian MFMA forms (FP32
// kernel values summed in FP64), for row stride dp, max ||y||^2 and kappa.
double selfnorm_error_bound(int dp, double ymax2, double kappa);

// Differentiation form (Gaussian, bandwidth s): self norms and their
// s-derivative for every center, and the per-row gradient plus the summed
// df/ds (written to *out).
void launch_selfnorm_sigma(const Layout &L, const Buffers &B, double sigma, double *N, double *dN, hipStream_t st);
void launch_grad_rows(const Layout &L, const Buffers &B, const float *xb, int b, double sigma, const int32_t *labels,
                      double g, const double *dN, float *dX, double *rowds, double *out, hipStream_t st);
int grad_max_dim();
// The same on FP32 MFMA for the MFMA layouts (padded segments, row stride
// 32, 64, 96 or 128): self norms and their derivative at s (task plan, work,
// fold), and the backward (grouping of the rows by label, per-group tiles,
// dsigma sum).  sigma_mfma_ok: whether the layout admits them.
bool sigma_mfma_ok(const Layout &L);
void launch_sigma_norms(const Layout &L, const Buffers &B, double sigma, double *N, double *dN, hipStream_t st);
void launch_grad_mfma(const Layout &L, const Buffers &B, int b, double sigma, const int32_t *labels, double g,
                      const double *dN, float *dX, double *rowds, double *out, hipStream_t st);

// Untruncated form on the table of cross terms (window 0).  init: N and the
// table of the initial centers (pool rows 0..k-1).  score: distances of rows
// idx[0..m) from the table into labels / mind / margin (step: also the old
// table value of the winner and the counts).  update: plan, grouping, pair
// sums, N and weights of batch rows [0, b) (staged in slot 0).  table: the
// update of T over all of X.
int dp_max_dim();
void launch_dp_init(const Layout &L, const Buffers &B, int kind, double param, int fp64, hipStream_t st);
void launch_dp_score(const Layout &L, const Buffers &B, int kind, double param, int fp64, const int32_t *idx, int m,
                     bool step, double *D_out, int64_t ldD, int32_t *flags, hipStream_t st);
void launch_dp_update(const Layout &L, const Buffers &B, int b, int kind, double param, int fp64, int lr,
                      hipStream_t st);
// L.dp_mfma: the Gaussian FP32 form on MFMA (k_dp_mfma + k_dp_blend).
void launch_dp_table(const Layout &L, const Buffers &B, int kind, double param, int fp64, int init,
                     hipStream_t st);

// Contingency table [k x c] (int64, zeroed by the caller) of labels in [0, k)
// against truth in [0, c); an out-of-range row raises flags[2].
void launch_contingency(const int32_t *labels, const int32_t *truth, int64_t m, int k, int c, int64_t *table,
                        int32_t *flags, hipStream_t st);

// k-means++
void launch_kpp_self(const Layout &L, const Buffers &B, int kind, double param, hipStream_t st);
void launch_kpp_round(const Layout &L, const Buffers &B, int r, int kind, double param, hipStream_t st);

}  // namespace mbkk
