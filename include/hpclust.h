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
 *  - Sample indices.  An index outside [0, m) is not an error: that point
 *    reads as a row of zeros (every kernel that reads rows through indices
 *    substitutes the zero row instead of reading out of bounds).
 *  - Supported sizes: 1 <= d <= 128, 1 <= k <= 512, k <= s, m < 2^62, and
 *    the k centroids (FP64, with the per-cluster sums for Lloyd) must fit a
 *    workgroup's 160 KiB of LDS.  Largest k per padded d (8, 16, 32, 64,
 *    128) for Lloyd: 512, 462, 240, 121, 60 (FP32 screening), 512, 462, 266,
 *    134, 66 (BF16), 512, 387, 240, 121, 60 (BF16x3); for hpc_assign_sse:
 *    512, 512, 400, 207, 101 (FP32 and BF16x3), 512, 512, 480, 246, 125
 *    (BF16).  Larger combinations are refused with HPC_ERR_UNSUPPORTED
 *    before anything is launched.
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
    HPC_ERR_UNSUPPORTED = -4  /* valid request outside what the library handles */
} hpc_status;

/* Arithmetic that SCREENS the nearest centroid in the assignment step.  In
 * every mode the scores |c|^2 - 2 x.c are computed on the matrix cores and
 * the winner is accepted only when its lead over the runner-up exceeds a
 * rigorous bound on the screening error; any other point is re-decided with
 * FP64 distances.  Every decided index is therefore the one FP64 distances
 * give (lowest index on exact ties); the mode changes speed only. */
enum {
    HPC_PREC_FP32 = 0,       /* FP32 operands, MFMA 16x16x4 f32                  */
    HPC_PREC_BF16_MFMA = 1,  /* BF16 operands, MFMA 16x16x32 bf16, FP32 accumulate */
    HPC_PREC_BF16X3_MFMA = 2 /* each operand split into BF16 high and low parts;
                              * three MFMA 16x16x32 bf16 products per k-chunk
                              * (hi.hi + lo.hi + hi.lo), FP32 accumulate: error
                              * bound about 10x FP32's and 60x below BF16's at
                              * d = 64, so few points need the FP64 re-decision,
                              * at under a third of FP32's matrix-core time.
                              * The centroid operand tables take twice BF16's
                              * LDS. */
};

/* The screening error bound of a precision mode: for a point x and the
 * FP64 centroids c_j of one call, every screened score s~_j satisfies
 * |s~_j - s_j| <= alpha |x| cmax + beta cmax^2 (s_j = |c_j|^2 - 2 x.c_j
 * exactly, cmax = max_j |c_j|); the winner is certified when the two best
 * keys differ by more than 2.5 times that plus the key quantisation.
 * Returns the coefficients the kernels use for dimension d (the derivation
 * is in the header of the screening code).  Host only, no GPU needed.
 * Errors: NULL outputs, d outside [1, 128], unknown precision. */
int hpc_screen_bound(int32_t d, int32_t precision, double *alpha, double *beta);

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
 * Distances, prefix sums and potentials are FP64.  A cold start is run by a
 * team of workgroups (one slice of the sample each, one exchange of slice
 * and group sums per step); a partial one by one workgroup.  The chosen
 * indices do not depend on the team size: only the order of FP64 sums does.
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
 *     c_len, the lengths of idx and C), copied to the device through one of
 *     eight pinned staging slots per stream: the call does not wait for
 *     the GPU unless eight earlier uploads on the stream are still queued.
 *   precision: HPC_PREC_FP32, HPC_PREC_BF16_MFMA or HPC_PREC_BF16X3_MFMA
 *     (screening type, see above; labels, f and centroids do not depend on
 *     it).
 *   f is evaluated in FP64 from the per-cluster sums of x - r and counts (r
 *     a reference point fixed per sample): Q + sum_j (n_j |c_j - r|^2 -
 *     2 (c_j - r).S_j), Q = sum |x - r|^2, within about 1e-12 relative of
 *     the direct sum; where f is below 1% of Q, the identity would cancel
 *     and the points' FP64 distances are summed directly.
 *   f_out (device double[n]), iters_out (device int32[n]); labels_out
 *   nullable (device int32[idx_len]).
 * Samples may be processed in any order and concurrently; each sample's
 * result depends only on its own inputs.  Cold samples (every row
 * degenerate) are first seeded by a separate kernel, each by a team of
 * workgroups sized to the free capacity (the same random stream as the
 * re-seeding above, so the result does not depend on the team).  When the
 * GPU holds at least twice as many workgroups as there are samples, a
 * sample that starts with every centroid valid (or was just seeded) and
 * whose rows of X are 16-byte aligned with d a multiple of the padded width
 * is worked by P workgroups (P <= 16, at least 1,024 points each), each on
 * every P-th tile of 16 points, which exchange their partial sums once per
 * pass (until a re-seed, the gathered copy or the direct-sum objective is
 * needed; one workgroup finishes the sample).  The results then differ from
 * one workgroup's only in the order of the FP64 sums.  A sample whose
 * partner workgroups do not all arrive within about a second (not expected:
 * the grid is sized to be resident at once) is abandoned and reports
 * f = NaN and iters_out = -1.
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
 *     in a fixed order (bitwise reproducible for a fixed launch shape; the
 *     shape follows from d, k, the precision and the device: 256-thread
 *     workgroups, or 768-thread ones for d <= 64 when the centroid tables
 *     leave more resident waves that way).
 *   precision: as in hpc_lloyd_batch; the objective is always the FP64
 *     direct-difference distance to the chosen centroid summed in FP64.
 * Errors: NULL X/C/sse, m < 1, sizes out of range, every row degenerate is
 * NOT detected (sse is then +inf and labels -1). */
int hpc_assign_sse(const float *X, int64_t m, int32_t d, const float *C, int32_t k,
                   int32_t precision, int32_t *labels, int64_t *counts, double *sse,
                   void *hip_stream);

/* The full assignment of hpc_assign_sse without any allocation, for callers
 * that cannot allocate device memory (code under HIP graph capture, serving
 * loops, harnesses that forbid hipMalloc).  Arguments, results and errors
 * are those of hpc_assign_sse.  The per-workgroup partial sums of the
 * objective go to a fixed device array of 8,192 doubles (64 KiB) that the
 * library holds on every GPU it runs on until the process ends, instead of
 * the stream's workspace; the grid is capped at 8,192 workgroups (the
 * kernel strides over the rows, so every m is accepted; on MI355X the
 * launch shape, hence the summation order and sse, is the same as
 * hpc_assign_sse's).  The device address of the array is looked up once
 * per device, on the first call with that device current.  The call itself
 * allocates nothing: no hipMalloc, no host staging.  Every call on one GPU
 * shares that GPU's array and each call writes every slot it reads, so
 * nothing needs clearing; calls that overlap on one GPU (on different
 * streams, or from several threads) race on the array and must be ordered
 * by the caller. */
int hpc_assign_sse_noalloc(const float *X, int64_t m, int32_t d, const float *C, int32_t k,
                           int32_t precision, int32_t *labels, int64_t *counts, double *sse,
                           void *hip_stream);

/* ------------------------------------------------------------------------
 * Batch plans: a fixed table of uneven samples prepared once, run many times
 * (Algorithm 3's worker loop over B workers, each sample with its own s and
 * k).  Creating a plan validates the descriptors, orders the samples longest
 * first (work ~ s*k), and allocates every device buffer a run needs (the
 * descriptor table, the gathered samples, D^2, the work queue), so running
 * it enqueues kernel launches only: no allocation, no host copy, no
 * synchronisation.  That makes a run capturable in a HIP graph; the library
 * captures one worker-loop round itself (hpc_plan_capture_round) and replays
 * it with one graph launch per round.
 * ------------------------------------------------------------------------ */
typedef struct hpc_plan_s *hpc_plan;

/* Launch configuration of the resident Lloyd kernel (one workgroup of 512
 * threads per sample at a time, persistent grid pulling samples from a
 * queue).  Every configuration computes the same labels, pass counts and
 * centroids up to FP64 summation order. */
typedef struct {
    int32_t wg_per_cu; /* resident workgroups per compute unit; 0 = as many
                          as the occupancy allows                          */
    int32_t copies;    /* private FP64 partial-sum copies per workgroup, 1..4
                          (one per wave removes LDS atomic contention
                          between waves); 0 = as many as fit in 64 KiB     */
    int32_t order;     /* 0: longest sample first; 1: descriptor order      */
    int32_t seed_team; /* workgroups per cold sample in the K-means++ seeding
                          kernel, 0..64; 0 = chosen from the free capacity:
                          every cold sample's team resident at once, at
                          most one workgroup per 256 points of the largest
                          sample                                          */
    int32_t seed_inflight; /* cold samples seeded at once at most (0 = as many
                          teams as are resident; fewer keep the samples'
                          rows and weights in the last-level cache)        */
    int32_t parts;     /* workgroups per warm sample, 0..16 (at most one per
                          1024 points of the smallest sample); 0 = automatic:
                          shared only when at least twice as many
                          workgroups are resident as there are samples.  A
                          value above resident/samples runs the samples in
                          turn, each on `parts` workgroups, which shortens
                          the tail of a batch whose samples need uneven
                          numbers of passes                                */
} hpc_tune;

/* Create a plan on the current device for n_samples samples (desc: HOST
 * array, validated as in hpc_lloyd_batch against idx_len and c_len, copied;
 * 1 <= n_samples <= 65535) of d-dimensional data, screening precision
 * `precision`.  The plan owns its device memory (about idx_len * (4*pad(d)
 * + 44) bytes, pad(d) the next of 8, 16, 32, 64, 128, plus, where samples
 * can be shared (the smallest sample has s_min >= 2048 points),
 * n_samples * 16 * (P + 1) * (kmax * (pad(d) + 1) + 8) bytes of exchange
 * slots, P = min(16, s_min / 1024)) until hpc_plan_destroy.  *out receives the
 * handle (NULL on error).  The default configuration is all zeros. */
int hpc_plan_create(int32_t d, const hpc_sample_desc *desc, int32_t n_samples, int64_t idx_len,
                    int64_t c_len, int32_t precision, hpc_plan *out);

/* Destroy a plan after synchronising the device work that uses it; frees
 * its memory and its captured graph.  NULL is a no-op. */
int hpc_plan_destroy(hpc_plan plan);

/* Set / read the launch configuration.  Errors: wg_per_cu < 0, copies
 * outside [0, 4], order outside {0, 1}, seed_team outside [0, 64],
 * seed_inflight < 0, parts outside [0, 16], or a configuration whose LDS
 * does not fit.  A parts value above the plan's limit is clamped to it.  A
 * captured round keeps the configuration it was captured with. */
int hpc_plan_set_tune(hpc_plan plan, const hpc_tune *tune);
int hpc_plan_get_tune(hpc_plan plan, hpc_tune *tune);

/* Cache key of the plan's tuning problem (device architecture, padded d,
 * precision, and power-of-two buckets of n_samples, the largest k and the
 * mean s), NUL-terminated into buf (host, len bytes). */
int hpc_plan_tune_key(hpc_plan plan, char *buf, int32_t len);

/* Autotuner: times every configuration (parts per sample automatic and
 * each power of two up to the plan's limit x copies in {1, 2, 4} x
 * wg_per_cu from 1 to the occupancy limit of that kernel form x both
 * orders when the samples are uneven; seeding knobs stay 0) on the
 * caller's inputs -- hpc_plan_lloyd from a copy of C with max_iter and
 * rel_tol (0 = exactly max_iter passes; the caller's stop rule times the
 * tail of samples that need more passes than others) -- keeps the fastest
 * (HIP-event time, best of two) as the plan's configuration and returns it
 * in *best (host) and its time in *best_ms (host, nullable).  C is not
 * modified.  SYNCHRONOUS: returns after the timing runs on hip_stream have
 * finished. */
int hpc_plan_autotune(hpc_plan plan, const float *X, int64_t m, const int64_t *idx,
                      const float *C, int32_t max_iter, double rel_tol, hpc_tune *best,
                      double *best_ms, void *hip_stream);

/* hpc_lloyd_batch on the plan's samples (same arithmetic, outputs and
 * errors).  idx holds idx_len indices and C c_len floats, as at creation.
 * Enqueues kernel launches only. */
int hpc_plan_lloyd(hpc_plan plan, const float *X, int64_t m, const int64_t *idx, float *C,
                   int32_t max_iter, double rel_tol, double *f_out, int32_t *iters_out,
                   int32_t *labels_out, void *hip_stream);

/* Draw every sample of the plan into idx (device int64[idx_len]) with the
 * plan's current sample ids (as hpc_draw_samples).  Kernel launch only. */
int hpc_plan_draw(hpc_plan plan, int64_t m, int64_t *idx, void *hip_stream);

/* sample_id += id_stride for every sample in the plan's device table (the
 * ids the next draw and the next re-seeding use).  Kernel launch only. */
int hpc_plan_advance(hpc_plan plan, uint64_t id_stride, void *hip_stream);

/* One round of the worker loop (Algorithm 3) for every sample b of the plan:
 *   draw the sample (as hpc_draw_samples, stream (seed_b, sample_id_b));
 *   C_b <- C_inc_b; Lloyd on the sample (as hpc_plan_lloyd);
 *   keep the best: if f_out[b] < f_inc[b] then C_inc_b <- C_b, f_inc[b] <-
 *     f_out[b];
 *   sample_id_b += id_stride in the plan's device table (so the next round
 *     draws fresh samples; 0 repeats the same samples).
 * idx: device int64[idx_len] (overwritten); C, C_inc: device float[c_len];
 * f_inc: device double[n_samples] (+inf = no incumbent yet; C_inc rows NaN
 * = degenerate, so the first round seeds by K-means++).  Enqueues kernel
 * launches only. */
int hpc_plan_round(hpc_plan plan, const float *X, int64_t m, int64_t *idx, float *C, float *C_inc,
                   double *f_inc, int32_t max_iter, double rel_tol, double *f_out,
                   int32_t *iters_out, uint64_t id_stride, void *hip_stream);

/* Capture hpc_plan_round with these arguments into a HIP graph held by the
 * plan (replacing any earlier one).  Nothing runs; the buffers must stay
 * valid while the graph is replayed.  The capture uses a private stream, so
 * any caller stream may replay it. */
int hpc_plan_capture_round(hpc_plan plan, const float *X, int64_t m, int64_t *idx, float *C,
                           float *C_inc, double *f_inc, int32_t max_iter, double rel_tol,
                           double *f_out, int32_t *iters_out, uint64_t id_stride);

/* Replay the captured round n_rounds times on hip_stream (one graph launch
 * each).  Errors: no captured round, n_rounds < 0. */
int hpc_plan_replay(hpc_plan plan, int32_t n_rounds, void *hip_stream);

/* Restore the plan's device descriptor table to the descriptors given at
 * creation (undoing the sample_id advances of earlier rounds).  Enqueued on
 * hip_stream from the plan's own device copy. */
int hpc_plan_reset_ids(hpc_plan plan, void *hip_stream);

/* ------------------------------------------------------------------------
 * Learned initializer.  A set encoder proposes the k starting centroids of
 * a cold sample from the sample itself, as an alternative to the K-means++
 * seeding of Section 3; the proposal is used only where its sample
 * objective (Eq. (1) on the sample) is no larger than the seeding's.
 *
 *   mu = mean of the encoder's points, sigma = sqrt(mean |x - mu|^2)
 *   x~ = (x - mu) / sigma
 *   h1 = relu(x~ W1 + b1)  (d -> 256),  h2 = relu(h1 W2 + b2)  (256 -> 256)
 *   p = mean of h2 over the points;  o = p Wh + bh  (256 -> k*d)
 *   proposal row r, column q = mu_q + sigma * o[r*d + q]
 *
 * The encoder reads the first n_b = min(s, n_enc) points of each sample
 * (the points of a sample are i.i.d., so these are a uniform subsample).
 * Parameters are FP32 masters laid out flat in the order W1 (d x 256), b1,
 * W2 (256 x 256), b2, Wh (256 x k*d), bh, matrices row-major; the kernels
 * use the weights rounded to BF16 (matrix cores, FP32 accumulation).
 * Training minimises, with Adam (lr given, betas 0.9 / 0.999, eps 1e-8),
 * the distance between o (as k rows of d) and the target centroids in
 * normalised coordinates T~ = (T - mu) / sigma after a greedy one-to-one
 * pairing pi (k times, the closest still-unpaired proposal / target rows;
 * ties to the lowest proposal, then target, index):
 *   L = mean over samples of (1/k) sum_j |o_j - T~_pi(j)|^2.
 * A model is used from one stream at a time.
 * ------------------------------------------------------------------------ */
typedef struct hpc_setenc_s *hpc_setenc;

/* Create a model for d-dimensional data (1 <= d <= 32) and k centroids
 * (1 <= k <= 64) that reads n_enc points per sample (16 <= n_enc <= 2^20)
 * and trains on at most max_batch samples per gradient call (training
 * scratch ~ 3 KiB per point: max_batch * n_enc * (3*256 + 32) floats).
 * Initial weights: uniform He initialisation from Philox (tag 4, key
 * seed).  SYNCHRONOUS. */
int hpc_setenc_create(int32_t d, int32_t k, int32_t n_enc, int32_t max_batch, uint64_t seed,
                      hpc_setenc *out);

/* Destroy a model (synchronises the device).  NULL is a no-op. */
int hpc_setenc_destroy(hpc_setenc model);

/* Number of FP32 parameters (host int64 out). */
int hpc_setenc_param_count(hpc_setenc model, int64_t *n_params);

/* Copy the parameters to / from HOST memory (param_count floats, layout
 * above).  rounded != 0 returns the weights as the kernels use them (BF16
 * round-to-nearest-even).  set_params keeps the Adam state.  SYNCHRONOUS. */
int hpc_setenc_get_params(hpc_setenc model, int32_t rounded, float *host);
int hpc_setenc_set_params(hpc_setenc model, const float *host);

/* Copy the gradient of the last hpc_setenc_grad call to HOST memory.
 * SYNCHRONOUS. */
int hpc_setenc_get_grads(hpc_setenc model, float *host);

/* Proposals for a batch: for every sample b (desc: HOST array, every
 * desc[b].k equal to the model's k), the k x d proposal is written at
 * C + desc[b].c_offset.  idx / C: device arrays of idx_len / c_len. */
int hpc_setenc_propose(hpc_setenc model, const float *X, int64_t m, const int64_t *idx,
                       int64_t idx_len, const hpc_sample_desc *desc, int32_t n_samples, float *C,
                       int64_t c_len, void *hip_stream);

/* Loss and gradient of a batch of at most max_batch samples against the
 * target centroids T (device, the k x d block of sample b at
 * T + desc[b].c_offset).  loss: device double[1], nullable. */
int hpc_setenc_grad(hpc_setenc model, const float *X, int64_t m, const int64_t *idx,
                    int64_t idx_len, const hpc_sample_desc *desc, int32_t n_samples,
                    const float *T, int64_t c_len, double *loss, void *hip_stream);

/* One Adam step with the last gradient (bias-corrected; step count kept
 * by the model). */
int hpc_setenc_adam(hpc_setenc model, float lr, void *hip_stream);

/* Seeding of a cold batch with the learned proposal where it is at least as
 * good: for every sample b,
 *   P = the model's proposal;
 *   K = the K-means++ seeding a cold start of hpc_lloyd_batch makes (all
 *       rows degenerate, re-seeding stream tag 2, call_id 0);
 *   f_prop[b] = f(P, S), f_kpp[b] = f(K, S) (one assignment pass each);
 *   C_b <- P if f_prop[b] <= f_kpp[b], else K;  accepted[b] = 1 / 0.
 * C receives the chosen seeds (all rows valid), C_kpp the K-means++
 * seeding (device float[c_len] each); f_prop / f_kpp device double[n];
 * accepted device int32[n], nullable.  Lloyd from C then continues as from
 * any start (hpc_lloyd_batch); where K is chosen, that run is the cold
 * start's run. */
int hpc_learned_seed(hpc_setenc model, const float *X, int64_t m, const int64_t *idx,
                     int64_t idx_len, const hpc_sample_desc *desc, int32_t n_samples, float *C,
                     float *C_kpp, int64_t c_len, int32_t precision, double *f_prop,
                     double *f_kpp, int32_t *accepted, void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* HPCLUST_H */
