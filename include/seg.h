/*
 * seg.h -- C ABI of the MI355X fiber-bundle segmentation library (libseg.so).
 *
 * Operation (Vazquez et al., "Parallel optimization of fiber bundle
 * segmentation for massive tractography datasets", section 2.3 and 2.4):
 * every subject fiber a (21 points, 3 float32 coordinates in mm) is compared
 * with every atlas centroid b by
 *
 *     d_ME(a, b) = min( max_i ||a_i - b_i||, max_i ||a_i - b_{20-i}|| )   (Eq. 1-2)
 *
 * A centroid is accepted when d_ME does not exceed the threshold of its
 * bundle (section 2.3).  Each fiber takes the bundle of its closest accepted
 * centroid (section 2.4, "Classification of fibers"; Algorithm 1), the lowest
 * centroid index on equal distance, or no label.
 *
 * Arithmetic contract (identical for every mode, tile and batch layout):
 *   - squared point distance in float32, evaluated exactly as
 *       dx = a.x - b.x, dy = a.y - b.y, dz = a.z - b.z   (each rounded)
 *       d2 = fma(dz, dz, fma(dy, dy, dx * dx))
 *     with round-to-nearest-even, no flushing of subnormals, no other fusion;
 *   - D = min(max_i d2 direct, max_i d2 inverse); T2 = T * T rounded to
 *     float32 for T >= 0 (a bundle with T < 0 never matches);
 *   - accepted iff D <= T2; the winner minimises (D, centroid index);
 *   - labels[f] = bundle id of the winner, dists[f] = sqrt(D) correctly
 *     rounded; a fiber with no accepted centroid gets (-1, +inf).
 *
 * Memory: every pointer argument named "device" is a device (HBM) address on
 * the current HIP device; the caller owns every input and output buffer.
 * Fibers and centroids are C-contiguous [count][21][3] float32 (array of
 * structures, 252 bytes per curve, 4-byte aligned).  The library owns its
 * scratch (prepared atlas copies, prefilter features, counters); scratch is
 * cached per (device, stream), grows on demand and is never O(N x M).
 *
 * Streams: `stream` is a hipStream_t (NULL = the default stream).  Calls are
 * asynchronous on that stream unless validation is requested.  Two calls
 * that run concurrently on different streams use different scratch.
 *
 * Errors: every int-returning function returns SEG_OK (0) or a negative
 * seg_status; seg_last_error() gives a message for the calling thread.
 */
#ifndef SEG_H
#define SEG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SEG_NPOINTS 21
#define SEG_VERSION 1

typedef enum seg_status {
  SEG_OK = 0,
  SEG_EINVAL = -1,      /* null pointer, negative size, B <= 0 with M > 0, misaligned */
  SEG_EBUNDLE = -2,     /* a centroid bundle id outside [0, B) (validate = 1) */
  SEG_ENONFINITE = -3,  /* NaN / inf coordinate or NaN threshold (validate = 1) */
  SEG_EHIP = -4,        /* a HIP runtime call failed */
  SEG_ENOMEM = -5,      /* scratch allocation failed */
  SEG_ERANGE = -6,      /* a size beyond what the kernels index (M >= 2^24;
                           N >= 2^31 for the tile-culled form) */
  SEG_EMODE = -7,       /* unknown mode or option value */
  SEG_EOFFSETS = -8,    /* an empty streamline or offsets outside the points (validate = 1) */
  SEG_ECAPACITY = -9    /* more label entries than the output holds (*total tells how many) */
} seg_status;

typedef enum seg_mode {
  /* every pair, every point, both orders: the exact stage run on all pairs */
  SEG_DENSE = 0,
  /* float32 center-point test on every pair (the paper's test1), packed
     survivors, then the paper's tests 2-4 and the full metric on them */
  SEG_PLAIN = 1,
  /* conservative mean bound on MFMA with an orientation-free feature map
     (pairs of points symmetric about the center), bf16 / fp16 / fp8 inputs,
     fp32 accumulation; exact float32 stage on survivors */
  SEG_PREFILTER_BF16 = 2,
  SEG_PREFILTER_FP16 = 3,
  SEG_PREFILTER_FP8 = 4,
  /* the same bound with one 63-wide product per point order */
  SEG_PREFILTER_BF16_ORIENTED = 5
} seg_mode;

/* Metric variants of the paper (seg_options.metric):
 *   SEG_METRIC_LENGTH_NORM  section 2.3, Eq. 3: a pair with D <= T2 is kept
 *     when d_ME + TN <= T, TN = (|l_S - l_C| / max(l_S, l_C) + 1)^2 - 1 with
 *     l the arc length of the 21-point polyline (segment lengths
 *     sqrtf(fma(dz, dz, fma(dy, dy, dx * dx))) summed in point order, TN = 0
 *     for two zero lengths, each step rounded to float32); fibers take the
 *     bundle of the smallest d_ME + TN (sqrtf(D) + TN, rounded once), which
 *     is also the reported distance;
 *   SEG_METRIC_DIRECTION  section 2.4, "Inference of fiber direction": the
 *     point order with the smaller largest end-point distance (direct on a
 *     tie) is the fiber's direction, and D is the largest point distance of
 *     that order alone (instead of the smaller of the two orders).
 * Both keep every cut of every mode exact: each accepted pair has
 * min(D_direct, D_inverse) <= T2. */
typedef enum seg_metric {
  SEG_METRIC_LENGTH_NORM = 1,
  SEG_METRIC_DIRECTION = 2
} seg_metric;

typedef struct seg_options {
  int32_t mode;          /* seg_mode; default SEG_PLAIN */
  int32_t validate;      /* 1: check inputs on the device and synchronise the
                            stream to report SEG_EBUNDLE / SEG_ENONFINITE */
  int32_t tile;          /* 0: library choice (autotuned cache if present);
                            k > 0: kernel configuration k of the mode.
                            DENSE 1-2, PLAIN 1, 2, 4; BF16 / FP16 / FP8:
                            1-7 stream every centroid tile through the
                            matrix cores (feature width 16, 32 or 48; 1, 2
                            or 4 fiber groups per wave), 8 sorts fibers and
                            centroids by the cell of their center point and
                            skips (fiber group, centroid tile) pairs whose
                            feature boxes are too far apart to match (the
                            library choice for these modes);
                            BF16_ORIENTED 1-2 */
  int32_t collect_stats; /* 1: count survivors per stage (read with
                            seg_query_stats; adds atomics, not for timing) */
  void* profile_events;  /* optional host pointer to two hipEvent_t: the
                            library records [0] right before and [1] right
                            after the launch of the mode's dominant kernel
                            (on `stream`), so a caller can time that kernel
                            alone; NULL = no events */
  int32_t metric;        /* 0 or an OR of seg_metric flags (every mode and
                            the batch path take them) */
} seg_options;

typedef struct seg_stats {
  int64_t pairs;           /* N * M of the last call */
  int64_t filter_pass;     /* pairs that passed the first cut (test1 or the
                              prefilter bound); DENSE: pairs */
  int64_t test2_pass;      /* pairs alive after the end-point test */
  int64_t test3_pass;      /* pairs alive after the four-point test */
  int64_t accepted;        /* pairs with D <= T2.  SEG_PREFILTER_BF16_ORIENTED
                              has two columns per centroid (direct and
                              reversed) and counts filter_pass .. accepted
                              per surviving column, so a pair can count twice */
  int64_t labelled;        /* -1: not collected (count labels >= 0 instead) */
  int64_t drains;          /* survivor-queue drains (wave level) */
  int64_t bound_pairs;     /* pairs the first cut evaluated one by one: N * M,
                              except for the tile-culled prefilter, which
                              skips whole (32 fibers x 32 columns) tiles */
  int64_t survivor_rows;   /* tile-culled prefilter: fibers with at least one
                              pair past the bound (the fiber records its exact
                              stage reads); -1 for the other forms */
} seg_stats;

/* Default options (mode SEG_PLAIN, no validation, library tiles, no stats,
   no profiling events). */
void seg_default_options(seg_options* opt);

/*
 * Segment one subject against one atlas.
 *   fibers             device, [n_fibers][21][3] float32
 *   centroids          device, [n_centroids][21][3] float32
 *   centroid_bundle_id device, [n_centroids] int32, each in [0, n_bundles)
 *   bundle_thresholds  device, [n_bundles] float32, mm
 *   labels, dists      device, [n_fibers] int32 / float32, written
 *   opt                host, may be NULL (defaults)
 * n_fibers = 0 returns SEG_OK without launching; n_centroids = 0 writes
 * (-1, +inf) everywhere.  A bundle id outside [0, n_bundles) never matches
 * (and is reported as SEG_EBUNDLE when opt->validate = 1).
 */
int seg_segment(const float* fibers, int64_t n_fibers, const float* centroids,
                int64_t n_centroids, const int32_t* centroid_bundle_id,
                const float* bundle_thresholds, int32_t n_bundles, int32_t* labels,
                float* dists, const seg_options* opt, void* stream);

/*
 * seg_segment for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same operation, arguments, results and errors as seg_segment in modes
 * SEG_DENSE and SEG_PLAIN (other modes return SEG_EMODE), with every byte of
 * library scratch (the prepared atlas, the validation flag, the statistics
 * counters) in one fixed device array that the library's code object holds
 * on each GPU from its first use until the process ends, about 9.4 MB.  The
 * call makes no hipMalloc / hipFree or other allocation; it only launches
 * kernels on `stream` (and, with opt->validate = 1, synchronises it to read
 * the flag back, as seg_segment does).
 *   n_centroids  at most SEG_NOALLOC_MAX_CENTROIDS, else SEG_ERANGE
 * Every call on one GPU shares that GPU's array and leaves its contents
 * behind: calls that overlap on one GPU (two streams, two threads) race and
 * must be serialised by the caller.
 */
#define SEG_NOALLOC_MAX_CENTROIDS 32768
int seg_segment_noalloc(const float* fibers, int64_t n_fibers, const float* centroids,
                        int64_t n_centroids, const int32_t* centroid_bundle_id,
                        const float* bundle_thresholds, int32_t n_bundles, int32_t* labels,
                        float* dists, const seg_options* opt, void* stream);

/* ---- prepared atlases and batches (many subjects x one or two atlases) ---- */

typedef struct seg_atlas seg_atlas;

/*
 * Copy and prepare an atlas (device inputs as in seg_segment).  The handle
 * owns device memory on the current device until seg_atlas_destroy.  The
 * inputs may be freed after the call returns (the call synchronises
 * `stream`).  Returns SEG_EBUNDLE / SEG_ENONFINITE on bad inputs.
 */
int seg_atlas_create(const float* centroids, int64_t n_centroids,
                     const int32_t* centroid_bundle_id, const float* bundle_thresholds,
                     int32_t n_bundles, void* stream, seg_atlas** out);
void seg_atlas_destroy(seg_atlas* atlas);
int64_t seg_atlas_size(const seg_atlas* atlas); /* number of centroids */

/* seg_segment against a prepared atlas. */
int seg_segment_atlas(const seg_atlas* atlas, const float* fibers, int64_t n_fibers,
                      int32_t* labels, float* dists, const seg_options* opt, void* stream);

/*
 * Segment n_subjects subjects against n_atlases prepared atlases in one call.
 * SEG_PREFILTER_BF16 / FP16 / FP8 at tile 0 (or 8) run the sorted,
 * tile-culled form on the batch in chunks of consecutive subjects of at most
 * 2^22 fibers (a larger subject is a chunk of its own): the fibers of a chunk
 * get their features once (one quantisation frame over all the atlases) and
 * are sorted together by space, then each atlas takes one culled pass over
 * the chunk.
 * SEG_PLAIN, SEG_PREFILTER_BF16_ORIENTED and the streaming tiles of the
 * symmetric prefilters run one launch of the fused kernel over a flattened
 * list of (subject, atlas, fiber block) work items, costliest atlas first.
 * Either way the launch sequence is captured once per launch shape (the
 * pointers and sizes of the call) into a HIP graph and replayed on `stream`;
 * a new shape synchronises `stream` once to upload its subject table.
 * Every route gives each pair the result of the one-subject call.
 *   atlases   host array [n_atlases] of handles
 *   fibers    host array [n_subjects] of device pointers ([n][21][3] float32)
 *   n_fibers  host array [n_subjects]
 *   labels, dists  host arrays [n_subjects * n_atlases] of device pointers;
 *                  entry s * n_atlases + a receives subject s against atlas a
 * opt->mode selects the per-pair path (SEG_PLAIN or a prefilter mode).
 */
int seg_segment_batch(const seg_atlas* const* atlases, int32_t n_atlases,
                      const float* const* fibers, const int64_t* n_fibers, int32_t n_subjects,
                      int32_t* const* labels, float* const* dists, const seg_options* opt,
                      void* stream);

/* ---- autotuning ---- */

/*
 * Time every kernel configuration ("tile") of `mode` on these inputs (device
 * fibers [n][21][3] against a prepared atlas, `reps` timed calls each after
 * one warm-up, HIP events on `stream`) and remember the fastest for calls
 * with tile = 0 whose mode and sizes fall in the same bucket (mode,
 * floor(log2 N), floor(log2 M)).  Writes the winner and its mean time (ms)
 * when the pointers are not NULL.  Allocates and frees temporary outputs;
 * synchronises `stream`.  Batches use the bucket of their largest subject.
 */
int seg_autotune(const seg_atlas* atlas, const float* fibers, int64_t n_fibers, int32_t mode,
                 int32_t reps, int32_t* best_tile, float* best_ms, void* stream);

/* Save / load the tuned choices as text lines "mode log2n log2m tile ms". */
int seg_tune_save(const char* path);
int seg_tune_load(const char* path);
/* Forget every tuned choice. */
void seg_tune_clear(void);

/* ---- diagnostics ---- */

/*
 * Survivors of the first cut of `mode` (SEG_PLAIN: the center-point test;
 * prefilter modes: the MFMA bound), written as (fiber, centroid) int32 pairs
 * into the device buffer pairs[2 * k] (at most `capacity` pairs, any order).
 * *count (host) receives the total number of survivors, which may exceed
 * capacity.  Synchronises the stream.  Used to check that a cut never drops
 * an accepted pair.
 */
int seg_filter_pairs(const float* fibers, int64_t n_fibers, const float* centroids,
                     int64_t n_centroids, const int32_t* centroid_bundle_id,
                     const float* bundle_thresholds, int32_t n_bundles, int32_t mode,
                     int32_t* pairs, int64_t capacity, int64_t* count, void* stream);

/*
 * Several labels per fiber: the classification of the algorithm's previous
 * version (section 2.4, "Classification of fibers"), where a fiber belongs to
 * every bundle whose threshold test it passes, not only the closest one.
 *
 * Fiber f is a member of bundle B when some centroid of B passes the
 * threshold rule of seg_segment under opt->metric; its distance to B is the
 * smallest over those centroids (d_ME in mm, or the complete metric with
 * SEG_METRIC_LENGTH_NORM).  The closest-bundle label of seg_segment is the
 * member of smallest distance.
 *
 * fibers         device, [n][21][3] float32.
 * max_per_fiber  slots per fiber, 1..16: a fiber passing more bundles makes
 *                the call return SEG_ERANGE (outputs then unspecified).
 * offsets        device output, [n + 1] int64, 8-byte aligned: fiber f's
 *                entries are bundles/dists[offsets[f] .. offsets[f+1]), its
 *                bundles in increasing id (a CSR table).
 * bundles, dists device outputs, [capacity] int32 / float32.
 * total          host output: the number of entries (offsets[n]); when it
 *                exceeds capacity the entries past it are not written and
 *                the call returns SEG_ECAPACITY (call again with capacity >=
 *                *total).
 * bundle_counts  device output, [n_bundles] int64, 8-byte aligned, or NULL:
 *                the number of member fibers of each bundle.
 * opt            mode SEG_PREFILTER_BF16 / FP16 / FP8 (the tile-culled form,
 *                tile 0 or 8; other modes return SEG_EMODE), metric, validate.
 * Synchronises the stream (the total is read back).  Library scratch:
 * 8 * max_per_fiber bytes per fiber.  Fewer than 2^31 fibers.
 */
int seg_segment_multi(const seg_atlas* atlas, const float* fibers, int64_t n,
                      int32_t max_per_fiber, int64_t* offsets, int32_t* bundles, float* dists,
                      int64_t capacity, int64_t* total, int64_t* bundle_counts,
                      const seg_options* opt, void* stream);

/*
 * Resampling of raw streamlines to 21 points equidistant in arc length: the
 * step before the comparison (the paper resamples every subject fiber to 21
 * equidistant points before classifying it, section 2.3; the atlas centroids
 * carry 21 equidistant points, section 2.2).
 *
 * points   device, [n_points][3] float32 (x, y, z in mm), C-contiguous,
 *          4-byte aligned.
 * offsets  device, [n + 1] int64, 8-byte aligned: streamline i is
 *          points[offsets[i]] .. points[offsets[i+1] - 1] (P_i >= 1 points).
 * fibers   device output, [n][21][3] float32 (the fiber layout of
 *          seg_segment), caller-owned.
 *
 * Arithmetic (fixed so results are reproducible bit for bit):
 *   segment j:  d = p[j+1] - p[j] and g_j = sqrtf(fma(dz, dz, fma(dy, dy,
 *   dx*dx))) in float32; q_j = g_j in units of 2^-24 mm rounded to nearest
 *   even, or 2^38 when g_j >= 2^14 mm or is not finite;
 *   S_0 = 0, S_{j+1} = S_j + q_j summed exactly in 64-bit integers, L = S_{P-1};
 *   targets t_k = floor(k L / 20), k = 1..19;
 *   point k lies on the first segment j with t_k <= S_{j+1}, at weight
 *   w = (float)(t_k - S_j) / (float)q_j clamped to [0, 1] (0 when q_j = 0):
 *   out_k = fma(w, d, p[j]) per coordinate; out_0 = p[0], out_20 = p[P-1]
 *   exactly; a single point gives 21 copies of it.
 * A streamline with no points or more than 2^24 points, or whose offsets
 * leave [0, n_points] or decrease, gets 21 NaN points and no read of
 * `points`; with validate = 1 the call synchronises the stream and returns
 * SEG_EOFFSETS for it, or SEG_ENONFINITE for a NaN / inf coordinate among
 * the n_points points.
 * n = 0 returns SEG_OK without launching.
 */
int seg_resample(const float* points, int64_t n_points, const int64_t* offsets, int64_t n,
                 float* fibers, int32_t validate, void* stream);

/*
 * Raw streamlines straight to labels: seg_resample into `fibers` (a
 * caller-owned [n][21][3] float32 device buffer, which holds the resampled
 * fibers afterwards), then seg_segment_atlas on them with `opt` (its
 * validate field applies to both steps).
 */
int seg_segment_streamlines(const seg_atlas* atlas, const float* points, int64_t n_points,
                            const int64_t* offsets, int64_t n, float* fibers, int32_t* labels,
                            float* dists, const seg_options* opt, void* stream);

/* Bytes of device memory the library holds as scratch for the current
   device and `stream` (what the calls made on that stream have grown it to;
   prepared atlases are not included): 0 when no call used the stream, -1
   when the device cannot be queried.  Host only; no synchronisation. */
int64_t seg_scratch_bytes(void* stream);

/* Counters of the last call on this thread made with collect_stats = 1
   (synchronises that call's stream). */
int seg_query_stats(seg_stats* out);

/* Message of the last error on the calling thread ("" if none). */
const char* seg_last_error(void);

int seg_version(void);

#ifdef __cplusplus
}
#endif

#endif /* SEG_H */
