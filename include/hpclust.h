/*
 * hpclust.h -- C ABI of the MI355X (gfx950) hot path of the sample-based
 * minimum sum-of-squares clustering method HPClust (arXiv 2311.04517).
 *
 * Problem (paper, Eq. (1)): data X of m points in R^d (the paper's n),
 * k centroids C; the objective is f(C, X) = sum_i min_j |x_i - c_j|^2.
 * The method (Section 3; Algorithm 3) clusters random samples S of size s
 * with K-means++ seeding and K-means (Lloyd) local search, keeps the best
 * centroids by sample objective, and finally assigns all of X.
 *
 * Conventions shared by every call
 *  - Memory.  Unless stated otherwise, every pointer is DEVICE memory owned
 *    by the caller and must stay valid until the work queued on the stream
 *    has finished.  Arrays are dense and row-major: X is m x d FP32 (row i
 *    at X + i*d), a centroid block is k x d FP32.  Host arrays are read
 *    before the call returns.
 *  - Degenerate centroids.  A centroid row whose first coordinate is NaN is
 *    "degenerate" (Algorithm 3 starts every worker with all k rows
 *    degenerate).  Seeding fills such rows; the final assignment skips them.
 *  - Streams.  hip_stream is a hipStream_t (NULL = the default stream).
 *    Calls enqueue work and return without waiting for it.
 *  - Errors.  Every call returns an hpc_status.  Arguments are validated on
 *    the host before anything is enqueued; on error nothing is launched and
 *    hpc_last_error() describes the problem.  A HIP failure while
 *    enqueueing returns HPC_ERR_HIP.  Inputs containing NaN/Inf in X give
 *    unspecified results.
 *  - Random numbers.  Philox4x64-10 (Salmon et al., SC 2011) with key
 *    (seed, tag) and counter (block, sample_id, call_id, 0); each block
 *    yields four 64-bit words.  A uniform integer in [0, n) is
 *    floor(r * n / 2^64) and a uniform double (r >> 11) * 2^-53.
 *      tag 0: sample draw; tag 1: hpc_seed_kmeanspp; tag 2: re-seeding
 *      inside hpc_lloyd_batch (call_id = assignment passes done so far).
 *  - Scratch.  The library keeps a grow-only scratch workspace per device
 *    and stream, allocated on first use (hipMalloc) and freed by
 *    hpc_release().  Calls on different streams may run concurrently.
 *  - Supported sizes: 1 <= d <= 128, 1 <= k <= 512, k <= s, m < 2^62.
 */
#ifndef HPCLUST_H
#define HPCLUST_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    HPC_OK = 0,
    HPC_ERR_INVALID_ARG = -1, /* bad pointer, size, offset or option          */
    HPC_ERR_HIP = -2,         /* a HIP runtime call failed                     */
    HPC_ERR_NO_MEMORY = -3,   /* scratch allocation failed                     */
    HPC_ERR_UNSUPPORTED = -4  /* valid request outside what this build handles */
} hpc_status;

/* Arithmetic of the point-to-centroid distance in the assignment step. */
enum {
    HPC_PREC_FP32 = 0,     /* FP32 direct differences                          */
    HPC_PREC_BF16_MFMA = 1 /* BF16 cross term on MFMA, FP32 re-check of near
                              ties (see hpc_lloyd_batch)                       */
};

/* One sample of a batch.  idx_offset: first entry of this sample in the idx
 * array (and in labels_out); s: sample size; k: number of centroids;
 * c_offset: offset, in floats, of this sample's k x d block in C;
 * seed / sample_id: its random stream (keys of the re-seeding draws). */
typedef struct {
    int64_t idx_offset;
    int64_t c_offset;
    int32_t s;
    int32_t k;
    uint64_t seed;
    uint64_t sample_id;
} hpc_sample_desc;

/* Library version string (static storage). */
const char *hpc_version(void);

/* Text of the last error on the calling thread (static, thread-local). */
const char *hpc_last_error(void);

/* Number of HIP devices visible, or a negative hpc_status. */
int hpc_device_count(void);

/* Free every scratch workspace of every device after synchronising the
 * streams that used it.  Safe to call at any time outside other calls. */
int hpc_release(void);

/* Sample draw (Section 3; Algorithm 3: "select a random sample of size s
 * from X").  Writes s i.i.d. uniform row indices in [0, m) to idx (device,
 * int64[s]): index j is word j%4 of block j/4 of the stream
 * (seed, tag 0) / (block, sample_id, 0, 0).
 * Errors: m < 1, s < 1, idx NULL. */
int hpc_draw_sample(int64_t m, int32_t s, uint64_t seed, uint64_t sample_id, int64_t *idx,
                    void *hip_stream);

/* Sample draw for every sample of a batch: for each b, writes desc[b].s
 * indices of stream (desc[b].seed, desc[b].sample_id) at idx +
 * desc[b].idx_offset.  desc is HOST memory (n_samples entries); idx_len is
 * the length of idx.  Errors: as hpc_draw_sample, or an offset + s beyond
 * idx_len. */
int hpc_draw_samples(int64_t m, const hpc_sample_desc *desc, int32_t n_samples, int64_t *idx,
                     int64_t idx_len, void *hip_stream);

/* K-means++ seeding on the sample S = X[idx[0..s)] (Section 3: the first
 * sample is seeded by K-means++; Section 6.5: n_candidates points are drawn
 * for every new centroid -- the paper uses 3 -- and the one of least
 * potential sum_i min(D^2_i, |x_i - cand|^2) is kept).
 *   C (device, k x d, in/out): NaN rows are seeded, valid rows are kept and
 *     count as existing centres.  All rows NaN = cold start: the first row
 *     gets the sample point floor(r*s/2^64) (block 0, word 0).
 *   D^2 step q = 1, 2, ... (one per further seeded row, in increasing row
 *     order) uses block q, words 0..n_candidates-1; a draw u picks the
 *     smallest i whose inclusive prefix sum of D^2 (index order) exceeds
 *     u * sum(D^2).  If sum(D^2) == 0 the row takes point floor(r*s/2^64)
 *     with r = word 0 of the block.
 *   chosen (device int32[k], nullable): sample-local index of the point given
 *     to each seeded row, -1 for kept rows.
 *   Stream: tag 1, counter (block, sample_id, call_id, 0).
 * Distances are FP32; prefix sums and potentials FP64.
 * Errors: NULL X/idx/C, s < k, n_candidates outside [1, 4], sizes out of
 * range. */
int hpc_seed_kmeanspp(const float *X, int64_t m, int32_t d, const int64_t *idx, int32_t s,
                      int32_t k, int32_t n_candidates, uint64_t seed, uint64_t sample_id,
                      uint32_t call_id, float *C, int32_t *chosen, void *hip_stream);

/* K-means (Lloyd) on every sample of a batch (Algorithm 1 assign/update;
 * Algorithm 3 per-worker step; Section 6.5 stop rule).  For sample b with
 * S = X[idx[desc[b].idx_offset ..+ s)] and centroids C + desc[b].c_offset:
 *   f_prev = inf; it = 0
 *   repeat:
 *     re-seed every degenerate row by K-means++ on S (as hpc_seed_kmeanspp,
 *       3 candidates, tag 2, call_id = it)
 *     assign each point to its nearest centroid (lowest index on ties);
 *       f = sum of the minima (FP64); it += 1
 *     stop if it == max_iter, f == 0, or (f_prev - f) < rel_tol * f_prev
 *     f_prev = f; each centroid <- mean of its points (FP64 sums); a centroid
 *       that received no point becomes degenerate
 * and writes back the centroids of the last assignment (all k rows valid),
 * f_out[b] = f, iters_out[b] = it, and (labels_out non-NULL) the labels of
 * the last pass at labels_out + desc[b].idx_offset.
 *   desc: HOST array of n_samples entries (validated against idx_len and
 *     c_len, the lengths of idx and C).
 *   precision: HPC_PREC_FP32, or HPC_PREC_BF16_MFMA (cross term in BF16 on
 *     MFMA with FP32 accumulation; a point whose two best scores are closer
 *     than the rounding bound is re-evaluated with FP32 direct differences,
 *     so labels equal those of the FP32 path).
 *   f_out (device double[n]), iters_out (device int32[n]); labels_out
 *   nullable (device int32[idx_len]).
 * Samples may be processed in any order and concurrently; each sample's
 * result depends only on its own inputs.
 * Errors: NULL required pointers, max_iter < 1, rel_tol < 0 or NaN, any
 * s < k, offsets beyond idx_len / c_len, unknown precision. */
int hpc_lloyd_batch(const float *X, int64_t m, int32_t d, const int64_t *idx, int64_t idx_len,
                    const hpc_sample_desc *desc, int32_t n_samples, float *C, int64_t c_len,
                    int32_t max_iter, double rel_tol, int32_t precision, double *f_out,
                    int32_t *iters_out, int32_t *labels_out, void *hip_stream);

/* Keep the best (Algorithm 3): for each worker w in [0, n_workers), if
 * f_new[w] < f_inc[w] (strict) then C_inc[w] <- C_new[w] (k x d floats at
 * offset w*k*d) and f_inc[w] <- f_new[w].  All pointers device; updated
 * (nullable, int32[n_workers]) receives 1 where the incumbent changed. */
int hpc_keep_best(const float *C_new, const double *f_new, float *C_inc, double *f_inc,
                  int32_t n_workers, int32_t k, int32_t d, int32_t *updated, void *hip_stream);

/* Best worker (Algorithms 3-5: "centroids of the worker with the smallest
 * f_hat"): w* = argmin_w f_inc[w] (lowest w on ties); copies C_inc[w*] to
 * C_best (k x d), f_inc[w*] to f_best (device double[1]) and w* to w_best
 * (device int32[1], nullable). */
int hpc_select_best(const float *C_inc, const double *f_inc, int32_t n_workers, int32_t k,
                    int32_t d, float *C_best, double *f_best, int32_t *w_best, void *hip_stream);

/* Final assignment of the whole data set and its objective (Section 3;
 * Algorithm 3, last step; Eq. (1)).  Degenerate rows of C are skipped.
 *   labels (device int32[m], nullable): nearest valid centroid (lowest index
 *     on ties); counts (device int64[k], nullable): points per centroid;
 *   sse (device double[1]): sum_i min_j |x_i - c_j|^2, accumulated in FP64
 *     in a fixed order (bitwise reproducible for a fixed launch shape).
 *   precision: as in hpc_lloyd_batch; the objective is always the FP32
 *     direct-difference distance to the chosen centroid summed in FP64.
 * Errors: NULL X/C/sse, m < 1, sizes out of range, every row degenerate is
 * NOT detected (sse is then +inf and labels -1). */
int hpc_assign_sse(const float *X, int64_t m, int32_t d, const float *C, int32_t k,
                   int32_t precision, int32_t *labels, int64_t *counts, double *sse,
                   void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* HPCLUST_H */
