/*
 * FP64 single-threaded CPU oracle for truncated mini-batch kernel k-means
 * (Jourdan & Schwartzman, "Mini-batch kernel k-means", ICLR 2025).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the checker that the GPU path is
 * compared against.  Only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load it; the product path never calls it and must
 * fail when its own HIP library is missing.  It shares no code, header, table
 * or constant with the GPU library.
 *
 * Everything is plain FP64 with direct loops: no BLAS, no blocking, no
 * incremental tricks.  Inputs are the caller's FP32 values widened to double.
 *
 * What it computes (paper references are to sections / equations / algorithms):
 *
 *  - Kernel k-means goal f_A(C) = (1/|A|) sum_{x in A} min_j ||phi(x) - C_j||^2
 *    (Section 3, "Kernel k-means").
 *  - Distances by the kernel trick, ||phi(x)-C||^2 = K(x,x) - 2<phi(x),C> + <C,C>,
 *    with every center an explicit sparse combination of feature vectors
 *    (Section 1 "Lloyd's algorithm in feature space"; Section 4.1).
 *  - One iteration of Algorithm 2 (truncated mini-batch kernel k-means):
 *    assign the batch by argmin (lowest center index on ties, the paper breaks
 *    ties arbitrarily, Section 5), learning rate alpha = sqrt(b_i^j / b)
 *    (Section 5), center update C <- (1-alpha) C + alpha cm(B_i^j), truncated
 *    to the batches of the retention window (Eq. 1 with the coefficients of
 *    the unrolled recursion in Section 4.1; the initial center is kept, scaled
 *    by the product of (1-alpha), while the window still reaches batch 1).
 *  - Kernel k-means++ seeding (Section 1/4: "kernel version of k-means++").
 *  - The batch objective and its gradient with respect to the Gaussian
 *    bandwidth and the batch coordinates (differentiation form).
 *
 * Readings of the paper that this file fixes (each listed in the design notes):
 *   window W >= 1: after iteration i a center keeps batches
 *     max(1, i-W+1) .. i, plus the initial term while i <= W; W = 0 keeps all.
 *   tau > 0 (the rule of Section 4.1, applied within the window): Q_i^j runs
 *     from batch i down to the newest batch l at which the counts
 *     b_i^j + ... + b_l^j (the paper's sum over Q, read with b_l^j) reach tau;
 *     batches older than l and the initial term are dropped when l > 1; if the
 *     counts reach tau only at batch 1, or never, the center is untruncated.
 *   no renormalisation after truncation (Eq. 1 drops terms, nothing rescales).
 *   empty cluster: b_i^j = 0 gives alpha = 0 and adds no term.
 *   batches are tuples: a point drawn twice counts twice.
 *
 * Parity status: the distance assembly, the coefficient bookkeeping and the
 * Gaussian / polynomial / linear kernels are pinned by the tests (explicit
 * feature maps, Lloyd, brute force, closed forms).  See tests/test_oracle_*.py.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_GAUSS 0
#define ORC_LAPLACE 1
#define ORC_LINEAR 2
#define ORC_POLY2 3

#define ORC_LR_BETA 0
#define ORC_LR_FULL 1
#define ORC_LR_SKLEARN 2

/* ------------------------------------------------------------------------ */
/* Kernel functions K(u, v).                                                 */
/* ------------------------------------------------------------------------ */

/* Gaussian exp(-||u-v||^2 / kappa) (Section 6), Laplacian exp(-||u-v||_1 / sigma)
 * (named as a normalised kernel in the abstract), linear <u,v>, and the
 * degree-2 polynomial (<u,v> + c)^2.  d2 and l1 are summed directly. */
double orc_kernel(int kind, double param, const double *u, const double *v, int d)
{
    double s = 0.0;
    int t;
    switch (kind) {
    case ORC_GAUSS:
        for (t = 0; t < d; ++t) {
            double e = u[t] - v[t];
            s += e * e;
        }
        return exp(-s / param);
    case ORC_LAPLACE:
        for (t = 0; t < d; ++t)
            s += fabs(u[t] - v[t]);
        return exp(-s / param);
    case ORC_LINEAR:
        for (t = 0; t < d; ++t)
            s += u[t] * v[t];
        return s;
    case ORC_POLY2:
        for (t = 0; t < d; ++t)
            s += u[t] * v[t];
        s += param;
        return s * s;
    default:
        return NAN;
    }
}

/* ------------------------------------------------------------------------ */
/* Model: every center is a list of terms; a term is a coefficient times the  */
/* sum of the feature vectors of a tuple of points.                          */
/* ------------------------------------------------------------------------ */

typedef struct {
    int64_t tag;    /* 0: initial-center term; l >= 1: the part of batch B_l */
    double coef;    /* weight of each feature vector of the term            */
    int32_t npts;
    int32_t *pts;
} orc_term;

typedef struct {
    int32_t nterms, cap;
    orc_term *t;
} orc_center;

typedef struct {
    const float *X;   /* borrowed (n x d) row-major FP32 */
    int64_t n;
    int32_t d, k, W, kind, lr;
    int32_t tau;      /* 0: window only; > 0: the per-center rule of Section 4.1 */
    double param;
    int64_t iter;     /* index i of the next batch (starts at 1) */
    orc_center *c;
    double *cum;      /* per-center running count, used by the sklearn rate */
    double *xa, *xb;  /* scratch rows */
} orc_model;

static void load_row(const orc_model *m, int64_t p, double *out)
{
    const float *r = m->X + p * (int64_t)m->d;
    for (int t = 0; t < m->d; ++t)
        out[t] = (double)r[t];
}

static double kpp(orc_model *m, int64_t p, int64_t q)
{
    load_row(m, p, m->xa);
    load_row(m, q, m->xb);
    return orc_kernel(m->kind, m->param, m->xa, m->xb, m->d);
}

static void center_clear(orc_center *c)
{
    for (int g = 0; g < c->nterms; ++g)
        free(c->t[g].pts);
    c->nterms = 0;
}

static void center_push(orc_center *c, int64_t tag, double coef, int32_t npts, const int32_t *pts)
{
    if (c->nterms == c->cap) {
        c->cap = c->cap ? 2 * c->cap : 8;
        c->t = (orc_term *)realloc(c->t, sizeof(orc_term) * (size_t)c->cap);
    }
    orc_term *t = &c->t[c->nterms++];
    t->tag = tag;
    t->coef = coef;
    t->npts = npts;
    t->pts = (int32_t *)malloc(sizeof(int32_t) * (size_t)(npts > 0 ? npts : 1));
    memcpy(t->pts, pts, sizeof(int32_t) * (size_t)npts);
}

/* The count threshold tau of Section 4.1 (0: the window alone truncates). */
int orc_set_tau(orc_model *m, int32_t tau)
{
    if (!m || tau < 0)
        return -1;
    m->tau = tau;
    return 0;
}

orc_model *orc_create(const float *X, int64_t n, int32_t d, int32_t k, int32_t W,
                      int32_t kind, double param, int32_t lr)
{
    if (!X || n <= 0 || d <= 0 || k <= 0 || W < 0)
        return NULL;
    orc_model *m = (orc_model *)calloc(1, sizeof(orc_model));
    m->X = X;
    m->n = n;
    m->d = d;
    m->k = k;
    m->W = W;
    m->kind = kind;
    m->param = param;
    m->lr = lr;
    m->iter = 1;
    m->c = (orc_center *)calloc((size_t)k, sizeof(orc_center));
    m->cum = (double *)calloc((size_t)k, sizeof(double));
    m->xa = (double *)malloc(sizeof(double) * (size_t)d);
    m->xb = (double *)malloc(sizeof(double) * (size_t)d);
    return m;
}

void orc_destroy(orc_model *m)
{
    if (!m)
        return;
    for (int j = 0; j < m->k; ++j) {
        center_clear(&m->c[j]);
        free(m->c[j].t);
    }
    free(m->c);
    free(m->cum);
    free(m->xa);
    free(m->xb);
    free(m);
}

/* Initial centers C_1^j = phi(x_{idx[j]}): a convex combination of X as
 * Algorithm 1 requires.  Resets the iteration counter to 1. */
int orc_init_centers(orc_model *m, const int32_t *idx)
{
    for (int j = 0; j < m->k; ++j) {
        if (idx[j] < 0 || idx[j] >= m->n)
            return -1;
        center_clear(&m->c[j]);
        center_push(&m->c[j], 0, 1.0, 1, &idx[j]);
        m->cum[j] = 0.0;
    }
    m->iter = 1;
    return 0;
}

/* Arbitrary centers given as entries (center, point, coefficient); each entry
 * becomes one initial term.  Used by the tests to place centers at cm(S) or
 * at random convex combinations.  Resets the iteration counter to 1. */
int orc_set_centers(orc_model *m, int64_t nent, const int32_t *ent_center,
                    const int32_t *ent_point, const double *ent_coef)
{
    for (int j = 0; j < m->k; ++j) {
        center_clear(&m->c[j]);
        m->cum[j] = 0.0;
    }
    for (int64_t e = 0; e < nent; ++e) {
        int32_t j = ent_center[e], p = ent_point[e];
        if (j < 0 || j >= m->k || p < 0 || p >= m->n)
            return -1;
        center_push(&m->c[j], 0, ent_coef[e], 1, &p);
    }
    m->iter = 1;
    return 0;
}

/* A whole iteration state: the counter i of the next batch, every term of
 * every center (the layout orc_state_export writes: term_center, term_tag
 * (0: the initial point, l >= 1: the part of batch B_l), term_coef,
 * term_npts, and the points of all terms concatenated) and the running
 * counts.  Resuming from an exported state continues the same run: the window
 * and the count rule act on the tags.  Returns -1 on a bad entry. */
int orc_set_terms(orc_model *m, int64_t iteration, int64_t nterms, const int32_t *term_center,
                  const int64_t *term_tag, const double *term_coef, const int32_t *term_npts,
                  const int32_t *points, const double *cum)
{
    if (iteration < 1)
        return -1;
    int64_t e = 0;
    for (int64_t a = 0; a < nterms; ++a) {
        if (term_center[a] < 0 || term_center[a] >= m->k || term_npts[a] < 1 || term_tag[a] < 0 ||
            term_tag[a] >= iteration)
            return -1;
        for (int32_t q = 0; q < term_npts[a]; ++q)
            if (points[e + q] < 0 || points[e + q] >= m->n)
                return -1;
        e += term_npts[a];
    }
    for (int j = 0; j < m->k; ++j) {
        center_clear(&m->c[j]);
        m->cum[j] = cum ? cum[j] : 0.0;
    }
    e = 0;
    for (int64_t a = 0; a < nterms; ++a) {
        center_push(&m->c[term_center[a]], term_tag[a], term_coef[a], term_npts[a], points + e);
        e += term_npts[a];
    }
    m->iter = iteration;
    return 0;
}

/* <C_j, C_j> = sum over all pairs of support points of coef*coef*K, directly. */
static double center_sqnorm(orc_model *m, int j)
{
    const orc_center *c = &m->c[j];
    double s = 0.0;
    for (int g = 0; g < c->nterms; ++g)
        for (int a = 0; a < c->t[g].npts; ++a)
            for (int h = 0; h < c->nterms; ++h)
                for (int e = 0; e < c->t[h].npts; ++e)
                    s += c->t[g].coef * c->t[h].coef * kpp(m, c->t[g].pts[a], c->t[h].pts[e]);
    return s;
}

/* <phi(x), C_j> for a point given by coordinates. */
static double center_cross(orc_model *m, int j, const double *x)
{
    const orc_center *c = &m->c[j];
    double s = 0.0;
    for (int g = 0; g < c->nterms; ++g)
        for (int a = 0; a < c->t[g].npts; ++a) {
            load_row(m, c->t[g].pts[a], m->xb);
            s += c->t[g].coef * orc_kernel(m->kind, m->param, x, m->xb, m->d);
        }
    return s;
}

/* Cross terms P[r*k+j] = <phi(x_r), C_j> and self norms N[j] = <C_j, C_j> for
 * the points idx[0..m-1].  Either output may be NULL. */
int orc_terms(orc_model *m, const int32_t *idx, int64_t cnt, double *P, double *N)
{
    double *x = (double *)malloc(sizeof(double) * (size_t)m->d);
    if (N)
        for (int j = 0; j < m->k; ++j)
            N[j] = center_sqnorm(m, j);
    if (P)
        for (int64_t r = 0; r < cnt; ++r) {
            if (idx[r] < 0 || idx[r] >= m->n) {
                free(x);
                return -1;
            }
            load_row(m, idx[r], x);
            for (int j = 0; j < m->k; ++j)
                P[r * m->k + j] = center_cross(m, j, x);
        }
    free(x);
    return 0;
}

/* Self norms N[j] = <C_j, C_j> for every center. */
void orc_center_norms(orc_model *m, double *N)
{
    for (int j = 0; j < m->k; ++j)
        N[j] = center_sqnorm(m, j);
}

/* Distances D[r*k+j] = K(x,x) - 2<phi(x),C_j> + N[j] for the points
 * idx[0..cnt-1], given the self norms N, plus the argmin (lowest index among
 * equal minima), the minimum and the margin between the two smallest
 * distances (0 on an exact tie, +inf when k = 1).  Any output may be NULL.
 * Rows are independent, so callers may split idx across threads. */
int orc_distances_n(orc_model *m, const double *N, const int32_t *idx, int64_t cnt,
                    double *D, int32_t *label, double *mind, double *margin)
{
    int k = m->k;
    double *row = (double *)malloc(sizeof(double) * (size_t)k);
    double *x = (double *)malloc(sizeof(double) * (size_t)m->d);
    double *y = (double *)malloc(sizeof(double) * (size_t)m->d);
    int rc = 0;
    for (int64_t r = 0; r < cnt; ++r) {
        if (idx[r] < 0 || idx[r] >= m->n) {
            rc = -1;
            break;
        }
        load_row(m, idx[r], x);
        double kxx = orc_kernel(m->kind, m->param, x, x, m->d);
        int best = 0;
        for (int j = 0; j < k; ++j) {
            /* <phi(x), C_j>, term by term */
            const orc_center *c = &m->c[j];
            double p = 0.0;
            for (int g = 0; g < c->nterms; ++g)
                for (int a = 0; a < c->t[g].npts; ++a) {
                    const float *src = m->X + (int64_t)c->t[g].pts[a] * m->d;
                    for (int t = 0; t < m->d; ++t)
                        y[t] = (double)src[t];
                    p += c->t[g].coef * orc_kernel(m->kind, m->param, x, y, m->d);
                }
            row[j] = kxx - 2.0 * p + N[j];
            if (row[j] < row[best])
                best = j;
        }
        double second = INFINITY;
        for (int j = 0; j < k; ++j)
            if (j != best && row[j] < second)
                second = row[j];
        if (D)
            memcpy(D + r * k, row, sizeof(double) * (size_t)k);
        if (label)
            label[r] = best;
        if (mind)
            mind[r] = row[best];
        if (margin)
            margin[r] = second - row[best];
    }
    free(row);
    free(x);
    free(y);
    return rc;
}

int orc_distances(orc_model *m, const int32_t *idx, int64_t cnt, double *D,
                  int32_t *label, double *mind, double *margin)
{
    double *N = (double *)malloc(sizeof(double) * (size_t)m->k);
    orc_center_norms(m, N);
    int rc = orc_distances_n(m, N, idx, cnt, D, label, mind, margin);
    free(N);
    return rc;
}

/* f_A(C) = (1/|A|) sum_{x in A} min_j ||phi(x) - C_j||^2 (Section 3). */
double orc_objective(orc_model *m, const int32_t *idx, int64_t cnt)
{
    double *mind = (double *)malloc(sizeof(double) * (size_t)(cnt > 0 ? cnt : 1));
    if (orc_distances(m, idx, cnt, NULL, NULL, mind, NULL) != 0) {
        free(mind);
        return NAN;
    }
    double s = 0.0;
    for (int64_t r = 0; r < cnt; ++r)
        s += mind[r];
    free(mind);
    return cnt > 0 ? s / (double)cnt : 0.0;
}

/* Center update of Algorithm 2 for iteration i = m->iter, given the batch
 * tuple B_i = batch[0..b-1] and its assignment labels (computed by
 * orc_distances on the centers C_i).  Outputs (nullable): the counts b_i^j
 * and learning rates alpha_i^j.  Advances the iteration counter. */
int orc_update(orc_model *m, const int32_t *batch, int32_t b, const int32_t *lab,
               int32_t *counts_out, double *alpha_out)
{
    int k = m->k;
    if (b <= 0)
        return -1;
    for (int r = 0; r < b; ++r)
        if (lab[r] < 0 || lab[r] >= k || batch[r] < 0 || batch[r] >= m->n)
            return -1;
    int64_t i = m->iter;
    int32_t *pts = (int32_t *)malloc(sizeof(int32_t) * (size_t)b);
    for (int j = 0; j < k; ++j) {
        /* B_i^j in batch order; duplicates stay. */
        int32_t bj = 0;
        for (int r = 0; r < b; ++r)
            if (lab[r] == j)
                pts[bj++] = batch[r];
        double alpha;
        if (m->lr == ORC_LR_FULL)
            alpha = bj > 0 ? 1.0 : 0.0;
        else if (m->lr == ORC_LR_SKLEARN) {
            m->cum[j] += (double)bj;
            alpha = bj > 0 ? (double)bj / m->cum[j] : 0.0;
        } else
            alpha = sqrt((double)bj / (double)b);
        if (counts_out)
            counts_out[j] = bj;
        if (alpha_out)
            alpha_out[j] = alpha;

        /* C_{i+1} = (1 - alpha) C_i + alpha cm(B_i^j): scale every kept term,
         * then add the new batch mean with weight alpha / b_i^j per point. */
        orc_center *c = &m->c[j];
        for (int g = 0; g < c->nterms; ++g)
            c->t[g].coef *= (1.0 - alpha);
        if (bj > 0)
            center_push(c, i, alpha / (double)bj, bj, pts);

        /* Truncation to the window: keep batches max(1, i-W+1)..i and the
         * initial term only while i <= W (W = 0 keeps everything). */
        if (m->W > 0) {
            int w = 0;
            for (int g = 0; g < c->nterms; ++g) {
                int64_t tag = c->t[g].tag;
                int keep = (tag == 0) ? (i <= m->W) : (tag > i - m->W);
                if (keep)
                    c->t[w++] = c->t[g];
                else
                    free(c->t[g].pts);
            }
            c->nterms = w;
        }
        /* Truncation by count (Section 4.1): Q_i^j = {i, i-1, ..., lmin} with
         * lmin the newest batch at which b_i^j + ... + b_lmin^j >= tau.  When
         * lmin > 1 the terms of batches older than lmin and the initial term
         * go; otherwise (lmin = 1, or the counts never reach tau) nothing. */
        if (m->tau > 0) {
            int64_t lmin = 0;  /* 0: tau not reached */
            int64_t sum = 0;
            for (int64_t l = i; l >= 1 && lmin == 0; --l) {
                for (int g = 0; g < c->nterms; ++g)
                    if (c->t[g].tag == l)
                        sum += c->t[g].npts;
                if (sum >= m->tau)
                    lmin = l;
            }
            if (lmin > 1) {
                int w = 0;
                for (int g = 0; g < c->nterms; ++g) {
                    if (c->t[g].tag >= lmin)
                        c->t[w++] = c->t[g];
                    else
                        free(c->t[g].pts);
                }
                c->nterms = w;
            }
        }
    }
    m->iter = i + 1;
    free(pts);
    return 0;
}

/* One iteration of Algorithm 2 on the batch tuple B_i = batch[0..b-1]:
 * assignment on C_i, then the update.  Outputs (each may be NULL): labels,
 * min distance, margin, the distance matrix (b x k), the batch objective
 * f_{B_i}(C_i) before the update, the counts b_i^j and the rates alpha_i^j. */
int orc_step(orc_model *m, const int32_t *batch, int32_t b, int32_t *labels_out,
             double *mind_out, double *margin_out, double *D_out, double *fbefore,
             int32_t *counts_out, double *alpha_out)
{
    if (b <= 0)
        return -1;
    int32_t *lab = (int32_t *)malloc(sizeof(int32_t) * (size_t)b);
    double *mind = (double *)malloc(sizeof(double) * (size_t)b);
    int rc = orc_distances(m, batch, b, D_out, lab, mind, margin_out);
    if (rc == 0) {
        double f = 0.0;
        for (int r = 0; r < b; ++r)
            f += mind[r];
        if (fbefore)
            *fbefore = f / (double)b;
        rc = orc_update(m, batch, b, lab, counts_out, alpha_out);
    }
    if (rc == 0 && labels_out)
        memcpy(labels_out, lab, sizeof(int32_t) * (size_t)b);
    if (rc == 0 && mind_out)
        memcpy(mind_out, mind, sizeof(double) * (size_t)b);
    free(lab);
    free(mind);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* State export: the iteration counter and every term of every center.       */
/* ------------------------------------------------------------------------ */

int64_t orc_iteration(const orc_model *m) { return m->iter; }

/* Running per-center counts used by the count-based (sklearn) rate. */
void orc_cum(const orc_model *m, double *out)
{
    memcpy(out, m->cum, sizeof(double) * (size_t)m->k);
}

/* Number of terms and of (term, point) entries, to size the export arrays. */
void orc_state_size(const orc_model *m, int64_t *nterms, int64_t *nentries)
{
    int64_t a = 0, e = 0;
    for (int j = 0; j < m->k; ++j) {
        a += m->c[j].nterms;
        for (int g = 0; g < m->c[j].nterms; ++g)
            e += m->c[j].t[g].npts;
    }
    *nterms = a;
    *nentries = e;
}

/* Terms in center order, and within a center in insertion order (oldest
 * first): term_center, term_tag, term_coef, term_npts; then all points of all
 * terms concatenated in the same order. */
void orc_state_export(const orc_model *m, int32_t *term_center, int64_t *term_tag,
                      double *term_coef, int32_t *term_npts, int32_t *points)
{
    int64_t a = 0, e = 0;
    for (int j = 0; j < m->k; ++j)
        for (int g = 0; g < m->c[j].nterms; ++g) {
            const orc_term *t = &m->c[j].t[g];
            term_center[a] = j;
            term_tag[a] = t->tag;
            term_coef[a] = t->coef;
            term_npts[a] = t->npts;
            ++a;
            memcpy(points + e, t->pts, sizeof(int32_t) * (size_t)t->npts);
            e += t->npts;
        }
}

/* ------------------------------------------------------------------------ */
/* Kernel k-means++ (plain, non-greedy).                                     */
/* ------------------------------------------------------------------------ */

/* Picks k indices.  u[0..k-1] are uniforms in [0,1) supplied by the caller.
 * First pick: floor(u0 * n).  Pick r: D2(p) = min over chosen c of
 * K(p,p) - 2K(p,c) + K(c,c); the first p whose running sum (index order)
 * exceeds u_r * sum_p D2(p).  If the sum is zero, floor(u_r * n); if rounding
 * leaves no running sum above the target, the last p with D2(p) > 0. */
int orc_kmeanspp(const float *X, int64_t n, int32_t d, int32_t kind, double param,
                 int32_t k, const double *u, int32_t *out)
{
    double *D2 = (double *)malloc(sizeof(double) * (size_t)n);
    double *kpp_self = (double *)malloc(sizeof(double) * (size_t)n);
    double *x = (double *)malloc(sizeof(double) * (size_t)d);
    double *c = (double *)malloc(sizeof(double) * (size_t)d);
    for (int64_t p = 0; p < n; ++p) {
        for (int t = 0; t < d; ++t)
            x[t] = X[p * d + t];
        kpp_self[p] = orc_kernel(kind, param, x, x, d);
        D2[p] = INFINITY;
    }
    for (int r = 0; r < k; ++r) {
        int64_t pick;
        if (r == 0) {
            pick = (int64_t)floor(u[0] * (double)n);
        } else {
            double total = 0.0;
            for (int64_t p = 0; p < n; ++p)
                total += D2[p];
            if (!(total > 0.0)) {
                pick = (int64_t)floor(u[r] * (double)n);
            } else {
                double target = u[r] * total, run = 0.0;
                pick = -1;
                for (int64_t p = 0; p < n; ++p) {
                    run += D2[p];
                    if (run > target) {
                        pick = p;
                        break;
                    }
                }
                if (pick < 0)
                    for (int64_t p = n - 1; p >= 0; --p)
                        if (D2[p] > 0.0) {
                            pick = p;
                            break;
                        }
            }
        }
        if (pick >= n)
            pick = n - 1;
        out[r] = (int32_t)pick;
        for (int t = 0; t < d; ++t)
            c[t] = X[pick * d + t];
        double kcc = orc_kernel(kind, param, c, c, d);
        for (int64_t p = 0; p < n; ++p) {
            for (int t = 0; t < d; ++t)
                x[t] = X[p * d + t];
            double dd = kpp_self[p] - 2.0 * orc_kernel(kind, param, x, c, d) + kcc;
            if (dd < D2[p])
                D2[p] = dd;
        }
    }
    free(D2);
    free(kpp_self);
    free(x);
    free(c);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Differentiation form: batch objective over free coordinates and its       */
/* gradient, Gaussian kernel K_sigma(u,v) = exp(-||u-v||^2 / (2 sigma^2)).    */
/* ------------------------------------------------------------------------ */

static double gauss_sigma(const double *u, const double *v, int d, double sigma, double *d2_out)
{
    double s = 0.0;
    for (int t = 0; t < d; ++t) {
        double e = u[t] - v[t];
        s += e * e;
    }
    if (d2_out)
        *d2_out = s;
    return exp(-s / (2.0 * sigma * sigma));
}

/* f_B(xb, sigma) = (1/b) sum_x min_j [K(x,x) - 2 sum_s w_s K(x,y_s) + N_j(sigma)]
 * with the support points y_s and weights w_s of the current centers held
 * fixed and xb a (b x d) row-major FP64 matrix.  labels_out (nullable) gets the
 * argmin of each row. */
double orc_fobj_coords(orc_model *m, const double *xb, int32_t b, double sigma, int32_t *labels_out)
{
    int k = m->k, d = m->d;
    double *N = (double *)malloc(sizeof(double) * (size_t)k);
    double *y = (double *)malloc(sizeof(double) * (size_t)d);
    double *z = (double *)malloc(sizeof(double) * (size_t)d);
    for (int j = 0; j < k; ++j) {
        const orc_center *c = &m->c[j];
        double s = 0.0;
        for (int g = 0; g < c->nterms; ++g)
            for (int a = 0; a < c->t[g].npts; ++a) {
                load_row(m, c->t[g].pts[a], y);
                for (int h = 0; h < c->nterms; ++h)
                    for (int e = 0; e < c->t[h].npts; ++e) {
                        load_row(m, c->t[h].pts[e], z);
                        s += c->t[g].coef * c->t[h].coef * gauss_sigma(y, z, d, sigma, NULL);
                    }
            }
        N[j] = s;
    }
    double f = 0.0;
    for (int r = 0; r < b; ++r) {
        const double *x = xb + (int64_t)r * d;
        int best = 0;
        double bestv = INFINITY;
        for (int j = 0; j < k; ++j) {
            const orc_center *c = &m->c[j];
            double p = 0.0;
            for (int g = 0; g < c->nterms; ++g)
                for (int a = 0; a < c->t[g].npts; ++a) {
                    load_row(m, c->t[g].pts[a], y);
                    p += c->t[g].coef * gauss_sigma(x, y, d, sigma, NULL);
                }
            double D = 1.0 - 2.0 * p + N[j];
            if (D < bestv) {
                bestv = D;
                best = j;
            }
        }
        if (labels_out)
            labels_out[r] = best;
        f += bestv;
    }
    free(N);
    free(y);
    free(z);
    return f / (double)b;
}

/* Gradient of f_B at fixed labels: with K = exp(-d2/(2 sigma^2)),
 *   dK/dx   = -K (x - y) / sigma^2,  dK/dsigma = K d2 / sigma^3,
 * so
 *   df/dx_r   = (2 / (b sigma^2)) sum_{s in S_j} w_s K(x_r,y_s) (x_r - y_s)
 *   df/dsigma = (1/b) sum_r [ -2 sum_s w_s K(x_r,y_s) d2(x_r,y_s) / sigma^3
 *                             + sum_{s,s'} w_s w_s' K(y_s,y_s') d2(y_s,y_s') / sigma^3 ]
 * where j = labels[r].  K(x,x) = 1 contributes nothing.  dX is (b x d). */
int orc_fobj_grad(orc_model *m, const double *xb, int32_t b, double sigma,
                  const int32_t *labels, double *dX, double *dsigma)
{
    int k = m->k, d = m->d;
    double s3 = sigma * sigma * sigma, s2 = sigma * sigma;
    double *dN = (double *)malloc(sizeof(double) * (size_t)k);
    double *y = (double *)malloc(sizeof(double) * (size_t)d);
    double *z = (double *)malloc(sizeof(double) * (size_t)d);
    for (int j = 0; j < k; ++j) {
        const orc_center *c = &m->c[j];
        double s = 0.0;
        for (int g = 0; g < c->nterms; ++g)
            for (int a = 0; a < c->t[g].npts; ++a) {
                load_row(m, c->t[g].pts[a], y);
                for (int h = 0; h < c->nterms; ++h)
                    for (int e = 0; e < c->t[h].npts; ++e) {
                        double dd;
                        load_row(m, c->t[h].pts[e], z);
                        double kv = gauss_sigma(y, z, d, sigma, &dd);
                        s += c->t[g].coef * c->t[h].coef * kv * dd / s3;
                    }
            }
        dN[j] = s;
    }
    double ds = 0.0;
    for (int r = 0; r < b; ++r) {
        const double *x = xb + (int64_t)r * d;
        int j = labels[r];
        if (j < 0 || j >= k) {
            free(dN);
            free(y);
            free(z);
            return -1;
        }
        double *g = dX + (int64_t)r * d;
        for (int t = 0; t < d; ++t)
            g[t] = 0.0;
        const orc_center *c = &m->c[j];
        double acc = 0.0;
        for (int h = 0; h < c->nterms; ++h)
            for (int a = 0; a < c->t[h].npts; ++a) {
                double dd;
                load_row(m, c->t[h].pts[a], y);
                double kv = gauss_sigma(x, y, d, sigma, &dd);
                double wk = c->t[h].coef * kv;
                for (int t = 0; t < d; ++t)
                    g[t] += wk * (x[t] - y[t]);
                acc += -2.0 * wk * dd / s3;
            }
        for (int t = 0; t < d; ++t)
            g[t] *= 2.0 / ((double)b * s2);
        ds += acc + dN[j];
    }
    *dsigma = ds / (double)b;
    free(dN);
    free(y);
    free(z);
    return 0;
}
