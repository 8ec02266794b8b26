/*
 * sncc.h - segmented normalized cross-correlation template matching on MI355X.
 *
 * Method: Marusic, Popovic, Kalafatic, "Template Matching in Images using
 * Segmented Normalized Cross-Correlation", arXiv:2502.01286.  A template is
 * approximated by axis-aligned rectangles of constant value (Section 3,
 * Eqs. (2)-(7)); the NCC of Eq. (1) between the image and that approximation is
 * computed at every offset segment by segment through sum tables
 * (Section 4, Eqs. (8)-(18)).
 *
 * Conventions for every entry point
 *  - Return value: SNCC_OK (0) or a negative SNCC_E* code.  Nothing throws or
 *    aborts across this interface.  On error a message is kept for the
 *    calling thread and returned by sncc_last_error().
 *  - Argument checks are synchronous.  Device work is enqueued on the stream
 *    bound to the context and runs asynchronously; HIP errors of that work
 *    surface at a later call on the context or at sncc_sync().
 *  - Ownership: the caller owns every host array and every device buffer it
 *    passes (e.g. PyTorch tensors).  The library copies what it keeps (segment
 *    lists, pair lists) and owns only its handles and the scratch memory those
 *    handles hold; *_destroy frees them.  Device buffers must stay alive while
 *    work that uses them is pending.
 *  - Device pointers must be 16-byte aligned.  Pitches are in elements.
 *  - Image f is M pixels wide (x, columns) and N tall (y, rows), uint8,
 *    row-major (Section 2).  A template is W x H.  Offsets are
 *    u in [0, M-W], v in [0, N-H]; maps over offsets are row-major over v.
 */
#ifndef SNCC_H
#define SNCC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------------ status */
#define SNCC_OK 0
#define SNCC_EINVAL (-1)      /* bad argument (NULL, size, pitch, alignment)   */
#define SNCC_ENOMEM (-2)      /* host or device allocation failed               */
#define SNCC_ENOSPC (-3)      /* output capacity too small                      */
#define SNCC_ERANGE (-4)      /* exact 32-bit window sums not guaranteed        */
#define SNCC_EDEGENERATE (-5) /* uniform template approximation (Section 2)     */
#define SNCC_EDEVICE (-6)     /* HIP runtime error (text in sncc_last_error)    */

/* accumulation precision of the per-segment numerator (Eq. (12)) */
#define SNCC_FP32_KAHAN 0     /* integer box sums, FP32 compensated sum        */
#define SNCC_FP64 1           /* integer box sums, FP64 sum                    */

/* Largest template area n = W*H (2^23 - 1).  Within it every window and
 * segment sum of f is below 2^31 and exact as a difference of four entries of
 * the modulo-2^32 table, the integer terms of the FP32 path fit their 24-bit
 * multiplies, and n * (sum of f^2) fits 64 bits.  Sums of f^2 are exact for
 * boxes of up to SNCC_MAX_SQ_BOX_AREA pixels (255^2 * 66051 < 2^32); larger
 * windows are summed in bands of rows, so the template width may not exceed
 * that area. */
#define SNCC_MAX_TEMPLATE_AREA 8388607
#define SNCC_MAX_SQ_BOX_AREA 66051

/* Largest sum table of one frame, (N + 1) * sat_pitch * 4 bytes, that the
 * scoring entry points accept (2^31 - 1: they address a frame's table with
 * 32-bit byte offsets); larger frames give SNCC_EINVAL. */
#define SNCC_MAX_TABLE_BYTES 2147483647LL

/* Size of the per-device static carry scratch of sncc_build_sats_noalloc
 * (8 MiB): the call accepts B frames of M x N while
 * 8 * B * (ceil(N/64) * M + N * ceil(M/256) + ceil(N/64) * ceil(M/256))
 * does not exceed it (e.g. 25 frames 1920x1080, 55 frames 1280x720,
 * 6 frames 3840x2160). */
#define SNCC_NOALLOC_SCRATCH_BYTES 8388608

/* One rectangle of the approximation: the 5-tuple of Eq. (6) with the mean
 * k_i = sum / area kept as an exact integer ratio (Eq. (4)). */
typedef struct sncc_segment {
  int32_t x, y;      /* top-left template pixel                         */
  int32_t w, h;      /* W_i, H_i                                        */
  int64_t sum;       /* sum of template pixels over the rectangle       */
  int32_t area;      /* W_i * H_i                                       */
  int32_t reserved;  /* zero                                            */
} sncc_segment;

/* A match triplet (u, v, rho) of the algorithm's output (Section 5). */
typedef struct sncc_match {
  int32_t u, v;
  float rho;
} sncc_match;

typedef struct sncc_match64 {
  int32_t u, v;
  double rho;
} sncc_match64;

/* An entry of the two-threshold search's output (Section 5, step 7j): the
 * index of the (frame, template) pair, the offset and rho. */
typedef struct sncc_hit {
  int32_t pair;
  int32_t u, v;
  int32_t reserved;  /* zero */
  double rho;
} sncc_hit;

typedef struct sncc_ctx sncc_ctx;
typedef struct sncc_tmpl sncc_tmpl;
typedef struct sncc_batch sncc_batch;

/* --------------------------------------------------------------- utilities */
const char *sncc_status_string(int status);
/* Message of the last failing call on this thread ("" if none). */
const char *sncc_last_error(void);
/* Library version as 10000*major + 100*minor + patch. */
int sncc_version(void);

/* -------------------------------------------------- template preparation */
/*
 * precompute_template_approximation of Section 5 (host only, no device).
 *
 * Splits the template recursively (split_segment: keep a rectangle whose
 * population standard deviation is below sigma_max, Eq. (2); else halve its
 * larger side, width when w > h, first half ceil), raising sigma_max by 1 and
 * splitting again while more than K_max rectangles result (counted before
 * merging), then merges aligned neighbours with equal exact means
 * (merge_redundant_segments).  The deviation test is decided exactly.
 *
 *   t          host, H rows of W bytes, row stride t_stride >= W bytes
 *   sigma_max  threshold (> 0 to get any rectangle larger than one pixel)
 *   K_max      >= 1
 *   out        host array of cap entries; receives the K rectangles in the
 *              final (y, x) order of the merge
 *   K_out      receives K (also when SNCC_ENOSPC is returned)
 *   sigma_used receives the threshold of the accepted split (nullable)
 *   rho_max    receives the NCC between t and its approximation, steps 4-7 of
 *              the function, with the area-weighted sum of Eq. (17) (nullable)
 * Errors: SNCC_EINVAL (NULL, sizes < 1, stride < W, K_max < 1),
 *         SNCC_ENOSPC (cap < K), SNCC_EDEGENERATE (approximation uniform).
 */
int sncc_segment_template(const uint8_t *t, int W, int H, int t_stride,
                          double sigma_max, int K_max, sncc_segment *out,
                          int cap, int *K_out, double *sigma_used,
                          double *rho_max);

/*
 * Batched template preparation: sncc_segment_template for T templates at
 * once on n_threads host threads (0: one per hardware thread).  Template i
 * is t[i], W[i] x H[i] bytes with row stride t_stride[i], split with
 * sigma_max[i]; K_max is shared.  The lists are identical to the single
 * calls' and are written back to back: template i's K_i segments start at
 * out[seg_off[i]], and seg_off[T] is the total.
 *
 *   out, out_cap  host array; when the total exceeds out_cap nothing is
 *                 written to out (seg_off is still filled) and SNCC_ENOSPC
 *                 is returned
 *   seg_off       host, T + 1 entries
 *   sigma_used, rho_max, status  host, T entries each, nullable: per
 *                 template the accepted threshold, the NCC with the
 *                 approximation (NaN when uniform) and the status
 * A uniform approximation does not stop the others: every list is written
 * and the call returns SNCC_EDEGENERATE naming the first such template.
 * Errors: SNCC_EINVAL, SNCC_ENOSPC, SNCC_EDEGENERATE.
 */
int sncc_segment_templates(int T, const uint8_t *const *t, const int *W, const int *H,
                           const int *t_stride, const double *sigma_max, int K_max,
                           int n_threads, sncc_segment *out, int64_t out_cap,
                           int64_t *seg_off, double *sigma_used, double *rho_max,
                           int *status);

/* ---------------------------------------------------------------- context */
/*
 * Binds a device and a HIP stream (hipStream_t passed as an integer, e.g.
 * torch.cuda.current_stream().cuda_stream; 0 is the null stream).  All
 * device work of calls taking this context is enqueued on that stream.
 * Errors: SNCC_EINVAL, SNCC_EDEVICE, SNCC_ENOMEM.
 */
int sncc_ctx_create(int device, uintptr_t hip_stream, sncc_ctx **out);
int sncc_ctx_destroy(sncc_ctx *ctx);
/* Waits for the context's stream; reports pending HIP errors. */
int sncc_sync(sncc_ctx *ctx);
/*
 * Stage timing.  With timing enabled, calls that launch several kernels
 * record HIP events on the context's stream between their stages, and
 * sncc_ctx_stage_ms returns the device time of each stage of the last such
 * call (waiting for it): sncc_topk with SNCC_FP32_KAHAN gives {scoring,
 * selection}; sncc_threshold_match gives {fast scoring and compaction, slow
 * FP64 pass}.  *n receives the number of stages (0 when the last call
 * recorded none); at most cap values are written to ms.
 * Errors: SNCC_EINVAL, SNCC_EDEVICE.
 */
int sncc_ctx_set_timing(sncc_ctx *ctx, int enable);
int sncc_ctx_stage_ms(sncc_ctx *ctx, float *ms, int cap, int *n);

/* ------------------------------------------------------------- sum tables */
/* Minimum pitch (elements) of a sum table for images M pixels wide:
 * M + 1 rounded up to a multiple of 64. */
int sncc_sat_pitch(int M, int *pitch_elems);

/*
 * compute_sum_tables (Section 5, step 6): s of Eq. (10) and s^2 of Eq. (14)
 * for B frames, zero-padded: entry [y + 1][x + 1] is the sum over columns
 * 0..x and rows 0..y; row 0 and column 0 are zero (the values at index -1
 * in Eqs. (11), (13), (15)).  Values are stored modulo 2^32; any box sum
 * taken as a difference of four entries is exact while its true value is
 * below 2^32 (so for f^2 boxes of area <= SNCC_MAX_SQ_BOX_AREA; larger
 * windows are taken as several such boxes).
 *
 *   d_f        device, B frames of N rows x f_pitch bytes, frames contiguous
 *   d_s, d_s2  device, B frames of (N + 1) rows x sat_pitch uint32, frames
 *              contiguous; columns M+1 .. sat_pitch-1 are written with zeros
 * Errors: SNCC_EINVAL (NULL, B/M/N < 1, f_pitch < M, sat_pitch too small,
 *         misaligned), SNCC_EDEVICE, SNCC_ENOMEM (scratch).
 */
int sncc_build_sats(sncc_ctx *ctx, const uint8_t *d_f, int B, int M, int N,
                    int f_pitch, uint32_t *d_s, uint32_t *d_s2, int sat_pitch);

/*
 * sncc_build_sats without any allocation, for callers that cannot allocate
 * device memory: code being captured into a HIP graph, serving loops that
 * must not call hipMalloc, harnesses that forbid it.  Same arguments, layout
 * and results as sncc_build_sats (bit for bit); the carries between tiles go
 * to one static device array of SNCC_NOALLOC_SCRATCH_BYTES per device
 * instead of the context's scratch, so the call allocates nothing, neither
 * on the device nor on the host.  The array is looked up when a context is
 * created on the device and stays reserved until the process ends.
 * Every call on one device shares that array: calls that overlap in time on
 * one device (e.g. on two streams) race and must be ordered by the caller.
 * Errors: as sncc_build_sats; SNCC_ENOSPC when the B frames need more
 *         carry space than SNCC_NOALLOC_SCRATCH_BYTES (split them into
 *         several calls).
 */
int sncc_build_sats_noalloc(sncc_ctx *ctx, const uint8_t *d_f, int B, int M, int N,
                            int f_pitch, uint32_t *d_s, uint32_t *d_s2, int sat_pitch);

/* ------------------------------------------------------ segment lists */
/*
 * Copies T segment lists to the device together with the constants the
 * matching phase precomputes (Section 5, steps 3-4): k_bar (Eq. (7)),
 * c_i = k_i - k_bar in FP64 and FP32, and q_k = sum_i W_i H_i c_i^2
 * (area-weighted Eq. (17)).  Segments of each list must partition its
 * W x H template.
 *
 *   segs[i]    host array of K[i] segments of template i
 * Errors: SNCC_EINVAL (NULL, sizes, segments outside the template or not
 *         covering it exactly once), SNCC_ERANGE (W*H above
 *         SNCC_MAX_TEMPLATE_AREA or W above SNCC_MAX_SQ_BOX_AREA),
 *         SNCC_EDEGENERATE (q_k == 0),
 *         SNCC_ENOMEM, SNCC_EDEVICE.
 */
int sncc_upload_templates(sncc_ctx *ctx, int T, const sncc_segment *const *segs,
                          const int *K, const int *W, const int *H,
                          sncc_tmpl **out);
int sncc_tmpl_destroy(sncc_tmpl *tm);
/* W, H, K and q_k of template `index` (any pointer nullable). */
int sncc_tmpl_info(const sncc_tmpl *tm, int index, int *W, int *H, int *K,
                   double *q_k);
/* Number of templates T in the set.  Errors: SNCC_EINVAL (NULL). */
int sncc_tmpl_count(const sncc_tmpl *tm, int *T);

/* ------------------------------------------------------------- scoring */
/*
 * rho(u, v; f, k) of Eq. (18) at every offset of one frame for template
 * `index` (Section 5, step 7a-e): window sums by Eqs. (13) and (15), the
 * exact window energy n*sum f^2 - (sum f)^2 in 64-bit integers (Eq. (16)
 * times n), the numerator of Eq. (12) from integer box sums (Eq. (11)) and
 * the area-weighted denominator of Eq. (17).
 *
 *   precision  SNCC_FP32_KAHAN: d_rho is float; box sums minus (area x the
 *              window mean rounded to an integer) are accumulated in FP32
 *              with compensated summation (the context keeps the work list
 *              of its last such call and reuses it when the next has the
 *              same template set, index, sizes and pitch).  SNCC_FP64: d_rho
 *              is double; box sums are accumulated in FP64, one launch per
 *              call.
 *   d_rho      device, (N-H+1) rows x rho_pitch elements (>= M-W+1)
 *   d_degenerate  device, nullable, (N-H+1) x rho_pitch bytes: 1 where the
 *              window is uniform (rho written as 0), else 0
 * Errors: SNCC_EINVAL (NULL, template larger than image, pitches),
 *         SNCC_EDEVICE, SNCC_ENOMEM.
 */
int sncc_score(sncc_ctx *ctx, const sncc_tmpl *tm, int index,
               const uint32_t *d_s, const uint32_t *d_s2, int M, int N,
               int sat_pitch, int precision, void *d_rho, int rho_pitch,
               uint8_t *d_degenerate);

/* Forms of sncc_score_frame */
#define SNCC_FORM_AUTO 0        /* tile-local when allowed, K <= 40 and at most
                                   2^19 offsets (small frames, few segments)   */
#define SNCC_FORM_TILE_LOCAL 1  /* sum tables built per tile in LDS            */
#define SNCC_FORM_GLOBAL 2      /* the frame's tables first, then sncc_score   */

/*
 * rho of Eq. (18) at every offset of one frame for template `index`, FP32
 * compensated (as sncc_score with SNCC_FP32_KAHAN), taken straight from the
 * frame: no sum tables are passed in.  In the tile-local form each tile of
 * 64 x 16 offsets builds the sum tables (Eqs. (10), (14)) of its image region
 * (16 + H rows, 64 + W columns) in LDS and reads every window and segment box
 * sum (Eqs. (11), (13), (15)) from them; box sums are the same integers from
 * any table origin.  It applies when W * H <= SNCC_MAX_SQ_BOX_AREA, W <= 511
 * and (17 + H) x (pitch class >= 65 + W) words fit 160 KB of LDS (e.g. up to
 * 128 x 128 templates).  The global form builds the frame's tables (context
 * scratch) and runs sncc_score.
 *
 *   d_f        device, N rows x f_pitch bytes
 *   form       SNCC_FORM_AUTO, SNCC_FORM_TILE_LOCAL (SNCC_ERANGE when the
 *              template does not allow it) or SNCC_FORM_GLOBAL
 *   d_rho      device float, (N-H+1) rows x rho_pitch (>= M-W+1)
 *   d_degenerate  nullable, as in sncc_score
 *   d_energy   device, nullable, int64 at the same positions as d_rho: the
 *              exact window energy n * sum f^2 - (sum f)^2 (n times Eq. (16))
 *   form_used  host, nullable: the form that ran
 * Errors: SNCC_EINVAL, SNCC_ERANGE, SNCC_ENOMEM, SNCC_EDEVICE.
 */
int sncc_score_frame(sncc_ctx *ctx, const sncc_tmpl *tm, int index, const uint8_t *d_f,
                     int M, int N, int f_pitch, int form, float *d_rho, int rho_pitch,
                     uint8_t *d_degenerate, int64_t *d_energy, int *form_used);

/*
 * The k highest-scoring offsets of each (frame, template) pair (Section 2:
 * the match is the offset with the highest rho).  Ordering: higher rho
 * first, ties to the smaller v, then smaller u; no suppression of
 * neighbours.  The order is that of the rho the precision computes: FP32
 * values for SNCC_FP32_KAHAN, the FP64 values themselves for SNCC_FP64 (two
 * offsets whose doubles differ are never tied, even where the reported
 * float rho is the same).  SNCC_FP32_KAHAN runs every pair in one persistent launch
 * over a cost-ordered work list; SNCC_FP64 runs one launch per pair.  The
 * context keeps the FP32 form's work list of its last call on the device and
 * reuses it when the next call has the same template set, sizes, pitch, k
 * and pairs (calls on one context are ordered by its stream).
 *
 *   d_s, d_s2  sum tables of B frames (layout of sncc_build_sats)
 *   pairs      host, n_pairs x {frame, template}
 *   k          1 .. 64
 *   d_out      device, n_pairs x k matches; slots beyond the number of
 *              offsets get u = v = -1, rho = -infinity
 * Errors: SNCC_EINVAL (also a frame table above SNCC_MAX_TABLE_BYTES),
 *         SNCC_EDEVICE, SNCC_ENOMEM.
 */
int sncc_topk(sncc_ctx *ctx, const sncc_tmpl *tm, const uint32_t *d_s,
              const uint32_t *d_s2, int B, int M, int N, int sat_pitch,
              int n_pairs, const int32_t *pairs, int k, int precision,
              sncc_match *d_out);
/* sncc_topk with k = 1. */
int sncc_argmax(sncc_ctx *ctx, const sncc_tmpl *tm, const uint32_t *d_s,
                const uint32_t *d_s2, int B, int M, int N, int sat_pitch,
                int n_pairs, const int32_t *pairs, int precision,
                sncc_match *d_out);

/*
 * Fine step of the coarse-to-fine search (Section 5, steps 7f-i, with the
 * coarse threshold replaced by a candidate list): for each pair, rho with
 * the fine approximation `fine` (same template indices as the coarse set)
 * is computed in FP64 at every offset within Chebyshev distance `radius` of
 * one of the pair's candidates (clipped to valid offsets, duplicates
 * scored once), and the best of them is returned (ties: smaller v, then u).
 *
 *   d_cand     device, n_pairs x n_cand candidates (e.g. sncc_topk output);
 *              entries with u < 0 are ignored
 *   radius     0 .. 7; n_cand * (2 radius + 1)^2 <= 4096
 *   d_out      device, n_pairs results; a pair without candidates gets
 *              u = v = -1, rho = -infinity
 *   d_count    device, nullable, n_pairs int32: offsets scored per pair
 * Errors: SNCC_EINVAL, SNCC_EDEVICE.
 */
int sncc_refine(sncc_ctx *ctx, const sncc_tmpl *fine, const uint32_t *d_s,
                const uint32_t *d_s2, int B, int M, int N, int sat_pitch,
                int n_pairs, const int32_t *pairs, const sncc_match *d_cand,
                int n_cand, int radius, sncc_match64 *d_out, int32_t *d_count);

/*
 * The matching algorithm of Section 5 as printed (steps 5 and 7a-j), over
 * pairs: rho with the fast approximation at every offset (FP32 compensated,
 * one persistent launch); offsets with rho >= thr_fast[template] survive and
 * are compacted into d_cand; each survivor is scored again with the slow
 * approximation in FP64 and appended to d_out when that rho is at least
 * thr_slow[template].  The paper sets the thresholds to precision (0.9)
 * times the NCC of each approximation with its template (rho_max of
 * sncc_segment_template) and builds the approximations with sigma_max of
 * 0.99 and 0.1 times the template's standard deviation.  The fast test is
 * taken on the FP32 rho against the threshold rounded to FP32.
 *
 *   fast, slow   template sets of equal sizes (same indices)
 *   thr_fast, thr_slow  host, one finite threshold per template
 *   pairs        host, n_pairs x {frame, template}
 *   d_cand       device, cand_cap entries: survivors of the fast test with
 *                rho = the FP32 fast rho (scratch the caller owns)
 *   d_out        device, out_cap entries: matches with rho = the slow rho
 *   d_counts     device, 2 int32: survivors and matches found; either may
 *                exceed its capacity, and entries beyond it are not written
 *                (the slow pass then sees only the first cand_cap survivors)
 * Entries come in no particular order.  The context keeps the work list of
 * its last call (with the slow pass's tables) on the device and reuses it
 * when the next call has the same template sets, sizes, pitch, pairs and
 * thresholds.
 * Errors: SNCC_EINVAL (NULL, sizes, thresholds, capacities < 1, alignment,
 *         a frame table above SNCC_MAX_TABLE_BYTES), SNCC_EDEVICE,
 *         SNCC_ENOMEM.
 */
int sncc_threshold_match(sncc_ctx *ctx, const sncc_tmpl *fast, const sncc_tmpl *slow,
                         const double *thr_fast, const double *thr_slow,
                         const uint32_t *d_s, const uint32_t *d_s2, int B, int M, int N,
                         int sat_pitch, int n_pairs, const int32_t *pairs,
                         sncc_hit *d_cand, int cand_cap, sncc_hit *d_out, int out_cap,
                         int32_t *d_counts);

/* ------------------------------------------------------------ batches */
typedef struct sncc_batch_desc {
  const sncc_tmpl *coarse;   /* scored at every offset (FP32 compensated)  */
  const sncc_tmpl *fine;     /* nullable: FP64 refinement when given       */
  const uint8_t *d_f;        /* nullable: frames; sum tables built per run */
  int f_pitch;
  uint32_t *d_s, *d_s2;      /* sum tables (written when d_f is given)     */
  int sat_pitch;
  int B, M, N;
  int n_pairs;
  const int32_t *pairs;      /* host, n_pairs x {frame, template}          */
  int k;                     /* top-k per pair, 1 .. 64                    */
  int radius;                /* refinement radius (used when fine != NULL) */
  sncc_match *d_topk;        /* device, n_pairs x k                        */
  sncc_match64 *d_best;      /* device, n_pairs (when fine != NULL)        */
  int32_t *d_count;          /* device, nullable, n_pairs (refine counts)  */
  int tune;                  /* 0: default tile shape; 1: time candidates  */
  const char *tune_cache;    /* nullable: JSON file read/written by tuner  */
} sncc_batch_desc;

typedef struct sncc_batch_stats {
  int64_t coarse_evals;      /* sum over pairs of offsets x K (coarse)     */
  int64_t n_offsets;         /* sum over pairs of offsets                  */
  int64_t work_items;
  int64_t computed_evals;    /* evals incl. offsets of partial edge tiles  */
  int64_t n_passes;          /* LDS passes summed over the used templates  */
  int n_launch_classes;      /* persistent scoring launches per run        */
  int tile_u, tile_v;        /* offsets per tile (u, v)                    */
  int wg_threads;
  int lds_bytes;
  int timed;                 /* 1 when the graph records per-stage events  */
  float ms_sat;              /* last run, from events in the graph; -1 if  */
  float ms_score;            /* not recorded                                */
  float ms_select;
  float ms_refine;
  float ms_total;
} sncc_batch_stats;

/*
 * Plans a batch: builds the cost-ordered work list of (pair, offset tiles)
 * items, chooses the tile shape (default, or timed candidates when
 * desc->tune is set), and captures sum-table construction, the persistent
 * scoring launches, top-k selection and (optionally) FP64 refinement into
 * one HIP graph on the context's stream.  The descriptor's buffers are
 * bound at this point.  Errors: as for the calls it combines.
 */
int sncc_batch_create(sncc_ctx *ctx, const sncc_batch_desc *desc,
                      sncc_batch **out);
/* One launch of the captured graph on the context's stream. */
int sncc_batch_run(sncc_batch *b);
/* Statistics and, after the run has completed, per-stage device times. */
int sncc_batch_stats_get(sncc_batch *b, sncc_batch_stats *st);
int sncc_batch_destroy(sncc_batch *b);

#ifdef __cplusplus
}
#endif

#endif /* SNCC_H */
