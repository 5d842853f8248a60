/*
 * hpc_oracle.c -- plain FP64 CPU oracle for the sample-based MSSC method
 * (HPClust, arXiv 2311.04517).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark load this library.  It shares no code,
 * header, table or constant generator with the HIP path, and the HIP path
 * never calls it.
 *
 * Everything here is deliberately slow and obvious: plain loops, FP64
 * arithmetic, summations in index order, no blocking and no fusion beyond
 * what the method's definition states.  Each function names the passage of
 * the paper it follows.  Where the paper is silent the reading taken is
 * stated at the function.
 *
 * Precision: the paper does not state one; the oracle computes every
 * distance, sum, centroid and objective in FP64 from the FP32 data.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* Random numbers.                                                           */
/* The paper asks for parallel random number generation (Section 5.3) but    */
/* names no generator.  Reading: Philox4x64-10, written from its definition  */
/* in Salmon, Moraes, Dror and Shaw, "Parallel Random Numbers: As Easy as    */
/* 1, 2, 3" (SC 2011).  Stream layout:                                       */
/*   key     = (seed, tag)                                                   */
/*   counter = (block, sample_id, call_id, 0); each block yields 4 words.   */
/* ------------------------------------------------------------------------ */

#define ORC_TAG_SAMPLE 0u
#define ORC_TAG_SEED 1u
#define ORC_TAG_RESEED 2u

static void mul_hi_lo(uint64_t a, uint64_t b, uint64_t *hi, uint64_t *lo) {
    unsigned __int128 p = (unsigned __int128)a * (unsigned __int128)b;
    *hi = (uint64_t)(p >> 64);
    *lo = (uint64_t)p;
}

/* Philox4x64: ten rounds of two 64x64->128 multiplications (round
 * multipliers and Weyl key increments as published for 4x64). */
void orc_philox4x64_10(const uint64_t ctr_in[4], const uint64_t key_in[2], uint64_t out[4]) {
    const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
    const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
    uint64_t x0 = ctr_in[0], x1 = ctr_in[1], x2 = ctr_in[2], x3 = ctr_in[3];
    uint64_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += W0;
            k1 += W1;
        }
        uint64_t hi0, lo0, hi1, lo1;
        mul_hi_lo(M0, x0, &hi0, &lo0);
        mul_hi_lo(M1, x2, &hi1, &lo1);
        uint64_t y0 = hi1 ^ x1 ^ k0;
        uint64_t y1 = lo1;
        uint64_t y2 = hi0 ^ x3 ^ k1;
        uint64_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

static void philox_block(uint64_t seed, uint64_t tag, uint64_t block, uint64_t sample_id,
                         uint64_t call_id, uint64_t out[4]) {
    uint64_t ctr[4] = {block, sample_id, call_id, 0};
    uint64_t key[2] = {seed, tag};
    orc_philox4x64_10(ctr, key, out);
}

/* floor(r * n / 2^64): an integer in [0, n). */
static int64_t bounded(uint64_t r, uint64_t n) {
    uint64_t hi, lo;
    mul_hi_lo(r, n, &hi, &lo);
    return (int64_t)hi;
}

/* (r >> 11) * 2^-53: a double in [0, 1). */
static double unit_double(uint64_t r) { return (double)(r >> 11) * 0x1.0p-53; }

/* ------------------------------------------------------------------------ */
/* Diagnostics: counters the paper reports (Appendix A: n_d) and the         */
/* distance of every floating-point decision from its threshold, so that a  */
/* comparison against a lower-precision implementation can tell a genuine    */
/* disagreement from a decision that sits within rounding of a boundary.     */
/* ------------------------------------------------------------------------ */
typedef struct {
    int64_t n_dist;           /* distance-function evaluations (Appendix A, n_d) */
    int64_t n_seed_calls;     /* K-means++ invocations that seeded >= 1 row      */
    int64_t n_seeded_rows;    /* rows set by K-means++                           */
    int64_t n_passes;         /* assignment passes                               */
    int64_t n_zero_weight;    /* D^2 steps that found a total weight of 0        */
    int64_t n_label_ties;     /* points whose relative top-2 gap < tie_rel       */
    double tie_rel;           /* threshold used for n_label_ties (input)         */
    double min_label_margin;  /* min relative top-2 gap (d2-d1)/d2               */
    double min_draw_margin;   /* min distance of a D^2 target to a prefix bound, / W */
    double min_cand_margin;   /* min relative gap between best and next distinct candidate potential */
    double min_stop_margin;   /* min |relative improvement - rel_tol| over stop tests */
} orc_diag;

static void diag_init(orc_diag *g) {
    double tie = g ? g->tie_rel : 0.0;
    if (!g) return;
    memset(g, 0, sizeof(*g));
    g->tie_rel = tie;
    g->min_label_margin = INFINITY;
    g->min_draw_margin = INFINITY;
    g->min_cand_margin = INFINITY;
    g->min_stop_margin = INFINITY;
}

void orc_diag_reset(orc_diag *g) { diag_init(g); }

/* ------------------------------------------------------------------------ */
/* Squared Euclidean distance, Eq. (1).                                      */
/* ------------------------------------------------------------------------ */
static double sqdist(const double *a, const double *b, int d) {
    double acc = 0.0;
    for (int t = 0; t < d; ++t) {
        double diff = a[t] - b[t];
        acc += diff * diff;
    }
    return acc;
}

/* A centroid row is degenerate when its first coordinate is NaN.  This is
 * how "set all k centroids as degenerate" (Algorithm 3, initialisation) is
 * represented. */
static int row_is_degenerate(const double *C, int j, int d) { return isnan(C[(size_t)j * d]); }

/* ------------------------------------------------------------------------ */
/* Sample draw (Section 3; Algorithm 3, "select a random sample of size s"). */
/* Reading: s indices drawn i.i.d. uniformly from [0, m) (with replacement); */
/* in the infinitely-tall setting (m = infinity) this is the only model, and */
/* at s << m it cannot be told apart from drawing without replacement.      */
/* Index j takes word j%4 of block j/4 of the stream (seed, SAMPLE, id, 0).  */
/* ------------------------------------------------------------------------ */
void orc_draw_sample(int64_t m, int32_t s, uint64_t seed, uint64_t sample_id, int64_t *idx) {
    uint64_t w[4];
    for (int32_t j = 0; j < s; ++j) {
        if (j % 4 == 0) philox_block(seed, ORC_TAG_SAMPLE, (uint64_t)(j / 4), sample_id, 0, w);
        idx[j] = bounded(w[j % 4], (uint64_t)m);
    }
}

/* Gather the sample S = X[idx] into FP64. */
static double *gather_sample(const float *X, int32_t d, const int64_t *idx, int32_t s) {
    double *S = (double *)malloc((size_t)s * d * sizeof(double));
    if (!S) return NULL;
    for (int32_t i = 0; i < s; ++i)
        for (int32_t t = 0; t < d; ++t) S[(size_t)i * d + t] = (double)X[(size_t)idx[i] * d + t];
    return S;
}

/* ------------------------------------------------------------------------ */
/* K-means++ seeding of the degenerate rows of C on the sample S.           */
/*                                                                          */
/* Paper: the first sample's centroids come from K-means++ (Section 3);     */
/* centroids of degenerate clusters are re-initialised with K-means++ on    */
/* the current sample (Section 3; Algorithm 3); three candidate points are  */
/* considered for every new centroid (Section 6.5).                         */
/*                                                                          */
/* Readings where the paper is silent:                                      */
/*  - If no row is valid, the first degenerate row takes a sample point     */
/*    chosen uniformly (the standard K-means++ first step); that costs one  */
/*    distance per point to initialise D^2.                                 */
/*  - Otherwise D^2(x) = min over the valid rows.                           */
/*  - Each further row: n_cand candidates drawn with probability D^2/W      */
/*    (inverse CDF: the smallest i whose inclusive prefix sum exceeds u*W,  */
/*    prefix summed in index order); each candidate's potential             */
/*    sum_i min(D^2_i, |x_i - cand|^2) is evaluated (s distances each) and  */
/*    the candidate of least potential is kept (ties: lowest draw).         */
/*  - If W == 0 (every point already coincides with a centre) the row takes */
/*    a uniformly chosen point (word 0 of its block).                       */
/*  - Draws: the uniform first centre uses block 0 word 0; the q-th D^2     */
/*    step (q = 1, 2, ...) uses block q, words 0..n_cand-1.                 */
/* chosen[j] receives the sample-local index given to row j, -1 otherwise.  */
/* ------------------------------------------------------------------------ */
static int kmeanspp_core(const double *S, int32_t s, int32_t d, double *C, int32_t k, int32_t n_cand,
                         uint64_t seed, uint64_t tag, uint64_t sample_id, uint64_t call_id,
                         int32_t *chosen, orc_diag *g) {
    int32_t *deg = (int32_t *)malloc((size_t)k * sizeof(int32_t));
    double *D2 = (double *)malloc((size_t)s * sizeof(double));
    if (!deg || !D2) {
        free(deg);
        free(D2);
        return -3;
    }
    int32_t n_deg = 0, n_valid = 0;
    for (int32_t j = 0; j < k; ++j) {
        if (chosen) chosen[j] = -1;
        if (row_is_degenerate(C, j, d))
            deg[n_deg++] = j;
        else
            ++n_valid;
    }
    if (n_deg == 0) {
        free(deg);
        free(D2);
        return 0;
    }
    if (g) {
        g->n_seed_calls += 1;
        g->n_seeded_rows += n_deg;
    }

    int32_t first = 0;
    if (n_valid == 0) {
        uint64_t w[4];
        philox_block(seed, tag, 0, sample_id, call_id, w);
        int64_t i0 = bounded(w[0], (uint64_t)s);
        int32_t j0 = deg[0];
        memcpy(&C[(size_t)j0 * d], &S[(size_t)i0 * d], (size_t)d * sizeof(double));
        if (chosen) chosen[j0] = (int32_t)i0;
        for (int32_t i = 0; i < s; ++i) D2[i] = sqdist(&S[(size_t)i * d], &C[(size_t)j0 * d], d);
        if (g) g->n_dist += s;
        first = 1;
    } else {
        for (int32_t i = 0; i < s; ++i) {
            double best = INFINITY;
            for (int32_t j = 0; j < k; ++j) {
                if (row_is_degenerate(C, j, d)) continue;
                double dd = sqdist(&S[(size_t)i * d], &C[(size_t)j * d], d);
                if (dd < best) best = dd;
            }
            D2[i] = best;
        }
        if (g) g->n_dist += (int64_t)s * n_valid;
    }

    for (int32_t r = first; r < n_deg; ++r) {
        uint64_t q = (uint64_t)(r + (n_valid > 0 ? 1 : 0));
        uint64_t w[4];
        philox_block(seed, tag, q, sample_id, call_id, w);
        double W = 0.0;
        for (int32_t i = 0; i < s; ++i) W += D2[i];
        int64_t pick;
        if (!(W > 0.0)) {
            pick = bounded(w[0], (uint64_t)s);
            if (g) g->n_zero_weight += 1;
        } else {
            int64_t cand[4];
            double pot[4];
            for (int32_t t = 0; t < n_cand; ++t) {
                double target = unit_double(w[t]) * W;
                double prev = 0.0, run = 0.0;
                int64_t c = -1;
                for (int32_t i = 0; i < s; ++i) {
                    prev = run;
                    run += D2[i];
                    if (run > target) {
                        c = i;
                        break;
                    }
                }
                if (c < 0) { /* u*W rounded up to W: take the last point of positive weight */
                    for (int32_t i = s - 1; i >= 0; --i)
                        if (D2[i] > 0.0) {
                            c = i;
                            break;
                        }
                    prev = target;
                    run = target;
                }
                if (g) {
                    double mg = fmin(target - prev, run - target) / W;
                    if (mg < g->min_draw_margin) g->min_draw_margin = mg;
                }
                cand[t] = c;
                double p = 0.0;
                const double *xc = &S[(size_t)c * d];
                for (int32_t i = 0; i < s; ++i) {
                    double dd = sqdist(&S[(size_t)i * d], xc, d);
                    p += (dd < D2[i]) ? dd : D2[i];
                }
                if (g) g->n_dist += s;
                pot[t] = p;
            }
            int32_t tb = 0;
            for (int32_t t = 1; t < n_cand; ++t)
                if (pot[t] < pot[tb]) tb = t;
            if (g) {
                for (int32_t t = 0; t < n_cand; ++t) {
                    if (cand[t] == cand[tb]) continue;
                    double mg = (pot[t] - pot[tb]) / (pot[tb] > 0.0 ? pot[tb] : 1.0);
                    if (mg < g->min_cand_margin) g->min_cand_margin = mg;
                }
            }
            pick = cand[tb];
        }
        int32_t j = deg[r];
        memcpy(&C[(size_t)j * d], &S[(size_t)pick * d], (size_t)d * sizeof(double));
        if (chosen) chosen[j] = (int32_t)pick;
        /* D^2 <- min(D^2, distance to the new centre); these are the chosen
         * candidate's distances already counted above. */
        for (int32_t i = 0; i < s; ++i) {
            double dd = sqdist(&S[(size_t)i * d], &C[(size_t)j * d], d);
            if (dd < D2[i]) D2[i] = dd;
        }
    }
    free(deg);
    free(D2);
    return 0;
}

/* Standalone K-means++ on the sample X[idx[0..s)] (stream tag SEED). */
int orc_kmeanspp(const float *X, int64_t m, int32_t d, const int64_t *idx, int32_t s, int32_t k,
                 int32_t n_cand, uint64_t seed, uint64_t sample_id, uint64_t call_id, double *C,
                 int32_t *chosen, orc_diag *g) {
    (void)m;
    if (n_cand < 1 || n_cand > 4 || s < 1 || k < 1 || d < 1) return -1;
    double *S = gather_sample(X, d, idx, s);
    if (!S) return -3;
    int rc = kmeanspp_core(S, s, d, C, k, n_cand, seed, ORC_TAG_SEED, sample_id, call_id, chosen, g);
    free(S);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Nearest-centroid assignment of one point (Eq. (1); Algorithm 1, assign   */
/* step).  Ties go to the lowest centroid index (reading).  Returns the     */
/* index; *dmin receives the distance and *margin the relative gap between  */
/* the two smallest distances.  Degenerate rows are skipped.                 */
/* ------------------------------------------------------------------------ */
static int32_t nearest(const double *x, const double *C, int32_t k, int32_t d, double *dmin,
                       double *margin, int32_t *n_evals) {
    double b1 = INFINITY, b2 = INFINITY;
    int32_t a = -1, ne = 0;
    for (int32_t j = 0; j < k; ++j) {
        if (row_is_degenerate(C, j, d)) continue;
        double dd = sqdist(x, &C[(size_t)j * d], d);
        ++ne;
        if (dd < b1) {
            b2 = b1;
            b1 = dd;
            a = j;
        } else if (dd < b2) {
            b2 = dd;
        }
    }
    *dmin = b1;
    if (isinf(b2))
        *margin = INFINITY;
    else if (b2 > 0.0)
        *margin = (b2 - b1) / b2;
    else
        *margin = 0.0;
    if (n_evals) *n_evals = ne;
    return a;
}

/* ------------------------------------------------------------------------ */
/* K-means (Lloyd) on the sample from the initial centroids C (k x d,       */
/* FP64, NaN rows degenerate).  Algorithm 1 (assign / update); stop rule of  */
/* Section 6.5; degenerate re-initialisation of Section 3 and Algorithm 3.  */
/*                                                                          */
/*   f_prev = inf; it = 0                                                   */
/*   repeat:                                                                */
/*     re-seed every degenerate row by K-means++ (stream RESEED, call = it) */
/*     assign every point to its nearest centroid; f = sum of the minima;   */
/*     it += 1                                                              */
/*     stop if it == max_iter, f == 0, or (f_prev - f) < rel_tol * f_prev   */
/*     f_prev = f; every centroid <- mean of its points; a centroid that    */
/*     received no point becomes degenerate                                 */
/*                                                                          */
/* Readings: "iterations exceed 300" = at most max_iter assignment passes;  */
/* "improvement less than 1e-4" is relative to the previous objective;      */
/* degenerate rows (NaN on entry or emptied by an update) are re-seeded at  */
/* the top of the next pass, so the returned C has k valid rows and f is    */
/* f(C, S) for exactly that C.                                              */
/*                                                                          */
/* labels (s, nullable) and margins (s, nullable) describe the final pass.  */
/* ------------------------------------------------------------------------ */
static int lloyd_core(const double *S, int32_t s, int32_t d, double *C, int32_t k, int32_t n_cand,
                      int32_t max_iter, double rel_tol, uint64_t seed, uint64_t sample_id,
                      int32_t *labels, double *f_out, int32_t *iters_out, double *margins,
                      orc_diag *g) {
    int32_t *a = (int32_t *)malloc((size_t)s * sizeof(int32_t));
    double *sums = (double *)malloc((size_t)k * d * sizeof(double));
    int64_t *cnt = (int64_t *)malloc((size_t)k * sizeof(int64_t));
    if (!a || !sums || !cnt) {
        free(a);
        free(sums);
        free(cnt);
        return -3;
    }
    double f_prev = INFINITY, f = INFINITY;
    int32_t it = 0;
    for (;;) {
        int rc = kmeanspp_core(S, s, d, C, k, n_cand, seed, ORC_TAG_RESEED, sample_id,
                               (uint64_t)it, NULL, g);
        if (rc) {
            free(a);
            free(sums);
            free(cnt);
            return rc;
        }
        f = 0.0;
        for (int32_t i = 0; i < s; ++i) {
            double dm, mg;
            a[i] = nearest(&S[(size_t)i * d], C, k, d, &dm, &mg, NULL);
            f += dm;
            if (margins) margins[i] = mg;
            if (g) {
                if (mg < g->min_label_margin) g->min_label_margin = mg;
                if (mg < g->tie_rel) g->n_label_ties += 1;
            }
        }
        if (g) {
            g->n_dist += (int64_t)s * k;
            g->n_passes += 1;
        }
        it += 1;
        if (g && isfinite(f_prev) && f_prev > 0.0) {
            double mg = fabs((f_prev - f) / f_prev - rel_tol);
            if (mg < g->min_stop_margin) g->min_stop_margin = mg;
        }
        if (it >= max_iter || f == 0.0 || (f_prev - f) < rel_tol * f_prev) break;
        f_prev = f;
        memset(sums, 0, (size_t)k * d * sizeof(double));
        memset(cnt, 0, (size_t)k * sizeof(int64_t));
        for (int32_t i = 0; i < s; ++i) {
            cnt[a[i]] += 1;
            for (int32_t t = 0; t < d; ++t) sums[(size_t)a[i] * d + t] += S[(size_t)i * d + t];
        }
        for (int32_t j = 0; j < k; ++j) {
            for (int32_t t = 0; t < d; ++t)
                C[(size_t)j * d + t] = cnt[j] > 0 ? sums[(size_t)j * d + t] / (double)cnt[j] : NAN;
        }
    }
    if (labels) memcpy(labels, a, (size_t)s * sizeof(int32_t));
    if (f_out) *f_out = f;
    if (iters_out) *iters_out = it;
    free(a);
    free(sums);
    free(cnt);
    return 0;
}

int orc_lloyd(const float *X, int64_t m, int32_t d, const int64_t *idx, int32_t s, int32_t k,
              int32_t n_cand, double *C, int32_t max_iter, double rel_tol, uint64_t seed,
              uint64_t sample_id, int32_t *labels, double *f_out, int32_t *iters_out,
              double *margins, orc_diag *g) {
    (void)m;
    if (s < k || k < 1 || d < 1 || max_iter < 1 || !(rel_tol >= 0.0) || n_cand < 1 || n_cand > 4)
        return -1;
    double *S = gather_sample(X, d, idx, s);
    if (!S) return -3;
    int rc = lloyd_core(S, s, d, C, k, n_cand, max_iter, rel_tol, seed, sample_id, labels, f_out,
                        iters_out, margins, g);
    free(S);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Final assignment of the whole data set (Section 3; Algorithm 3, last     */
/* step) and its objective f(C, X) of Eq. (1).  Degenerate rows of C are    */
/* skipped.  The sum of squares is accumulated with Neumaier's compensated  */
/* summation so that its own rounding is far below any tolerance used.     */
/* labels (m), counts (k) and margins (m) are nullable.                     */
/* ------------------------------------------------------------------------ */
int orc_assign_sse(const float *X, int64_t m, int32_t d, const double *C, int32_t k,
                   int32_t *labels, int64_t *counts, double *sse, double *margins, orc_diag *g) {
    if (m < 1 || d < 1 || k < 1) return -1;
    int32_t n_valid = 0;
    for (int32_t j = 0; j < k; ++j) n_valid += !row_is_degenerate(C, j, d);
    if (n_valid == 0) return -1;
    if (counts) memset(counts, 0, (size_t)k * sizeof(int64_t));
    double *x = (double *)malloc((size_t)d * sizeof(double));
    if (!x) return -3;
    double sum = 0.0, comp = 0.0;
    for (int64_t i = 0; i < m; ++i) {
        for (int32_t t = 0; t < d; ++t) x[t] = (double)X[(size_t)i * d + t];
        double dm, mg;
        int32_t a = nearest(x, C, k, d, &dm, &mg, NULL);
        double tt = sum + dm;
        if (fabs(sum) >= fabs(dm))
            comp += (sum - tt) + dm;
        else
            comp += (dm - tt) + sum;
        sum = tt;
        if (labels) labels[i] = a;
        if (counts) counts[a] += 1;
        if (margins) margins[i] = mg;
        if (g) {
            if (mg < g->min_label_margin) g->min_label_margin = mg;
            if (mg < g->tie_rel) g->n_label_ties += 1;
        }
    }
    if (g) g->n_dist += m * n_valid;
    *sse = sum + comp;
    free(x);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* One worker of Algorithm 3 (W = 1, the sequential form of Section 3):     */
/*   C_w <- all rows degenerate; f_hat <- inf                               */
/*   for t = 0 .. n_samples-1:                                              */
/*     S_t <- sample (seed, sample id t)                                    */
/*     C <- K-means on S_t from C_w (degenerate rows re-seeded first)       */
/*     if f(C, S_t) < f_hat: C_w <- C, f_hat <- f(C, S_t)   (keep the best) */
/*   final assignment of X to C_w and its objective.                        */
/* Outputs: C_w (k x d), f_hat, per-sample f (n_samples) and passes         */
/* (n_samples), and (nullable) full labels / counts / sse.                  */
/* ------------------------------------------------------------------------ */
int orc_worker_loop(const float *X, int64_t m, int32_t d, int32_t s, int32_t k, int32_t n_cand,
                    int32_t n_samples, uint64_t seed, int32_t max_iter, double rel_tol, double *C_w,
                    double *f_hat, double *f_samples, int32_t *iters_samples, int32_t *labels,
                    int64_t *counts, double *sse, orc_diag *g) {
    if (s < k || k < 1 || d < 1 || m < 1 || n_samples < 1) return -1;
    int64_t *idx = (int64_t *)malloc((size_t)s * sizeof(int64_t));
    double *C = (double *)malloc((size_t)k * d * sizeof(double));
    if (!idx || !C) {
        free(idx);
        free(C);
        return -3;
    }
    for (size_t e = 0; e < (size_t)k * d; ++e) C_w[e] = NAN;
    double best = INFINITY;
    int rc = 0;
    for (int32_t t = 0; t < n_samples && rc == 0; ++t) {
        orc_draw_sample(m, s, seed, (uint64_t)t, idx);
        memcpy(C, C_w, (size_t)k * d * sizeof(double));
        double f;
        int32_t its;
        rc = orc_lloyd(X, m, d, idx, s, k, n_cand, C, max_iter, rel_tol, seed, (uint64_t)t, NULL,
                       &f, &its, NULL, g);
        if (rc) break;
        if (f_samples) f_samples[t] = f;
        if (iters_samples) iters_samples[t] = its;
        if (f < best) {
            best = f;
            memcpy(C_w, C, (size_t)k * d * sizeof(double));
        }
    }
    if (rc == 0) {
        *f_hat = best;
        if (sse) rc = orc_assign_sse(X, m, d, C_w, k, labels, counts, sse, NULL, g);
    }
    free(idx);
    free(C);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Several independent samples, each from its own initial centroids (the    */
/* per-worker step of Algorithms 3-5 for one round).  Samples are           */
/* independent, so they may run on several threads; each sample's result    */
/* does not depend on the thread count.                                     */
/*   idx_offset[b], s[b], k[b], c_offset[b], seed[b], sample_id[b]          */
/* C is the concatenation of the k[b] x d blocks at c_offset[b].            */
/* ------------------------------------------------------------------------ */
int orc_lloyd_batch(const float *X, int64_t m, int32_t d, const int64_t *idx,
                    const int64_t *idx_offset, const int32_t *s, const int32_t *k,
                    const int64_t *c_offset, const uint64_t *seed, const uint64_t *sample_id,
                    int32_t n_samples, int32_t n_cand, double *C, int32_t max_iter, double rel_tol,
                    double *f_out, int32_t *iters_out, int32_t *labels_out, int32_t n_threads,
                    orc_diag *g_per_sample) {
    int rc_all = 0;
#ifdef _OPENMP
    if (n_threads < 1) n_threads = 1;
#pragma omp parallel for schedule(dynamic, 1) num_threads(n_threads)
#endif
    for (int32_t b = 0; b < n_samples; ++b) {
        orc_diag *g = g_per_sample ? &g_per_sample[b] : NULL;
        int rc = orc_lloyd(X, m, d, idx + idx_offset[b], s[b], k[b], n_cand, C + c_offset[b],
                           max_iter, rel_tol, seed[b], sample_id[b],
                           labels_out ? labels_out + idx_offset[b] : NULL, &f_out[b],
                           &iters_out[b], NULL, g);
        if (rc) {
#ifdef _OPENMP
#pragma omp critical
#endif
            rc_all = rc;
        }
    }
    (void)n_threads;
    return rc_all;
}

int orc_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
