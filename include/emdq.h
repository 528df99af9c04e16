/*
 * emdq.h -- C-ABI of the EMDQ dense deformation field + warp library for the
 * AMD MI355X (gfx950), libemdq.so.
 *
 * Method: H. Zhou and J. Jayender, "Real-time Nonrigid Mosaicking of
 * Laparoscopy Images" (arXiv 2103.07414).  The input of EMDQ is the
 * coordinates of feature matches and its output is a dense deformation field
 * (Sec. II); every pixel is then mapped between the new frame and the mosaic
 * and its colour merged (Sec. III-F).
 *
 * What the library computes (all on the GPU, FP32 unless stated):
 *   emdq_fit    per-match weighted similarity fits stored as planar dual
 *               quaternions (DQs) (Eqs. (1), (18)-(20)), with EM inlier
 *               reweighting over the N x N Gaussian match-weight matrix of
 *               Eq. (4) (Sec. II-A);
 *   emdq_field  per-pixel DQ blending of the inlier fits (Eqs. (2)-(4)), DQ
 *               normalisation, and Eq. (1): F(z) = s (R z + t);
 *   emdq_warp   emdq_field fused with a bilinear sample of the new frame at
 *               F(z) and the running-average colour merge of Eqs. (23)-(24)
 *               into an RGBA FP32 canvas (weight cap 30).
 *
 * Conventions
 *   Coordinates are pixels (x = column, y = row), pixel centres at integers,
 *   origin at the centre of the top-left pixel.  "src" points live in the
 *   reference / mosaic frame (x_0 of Eq. (1)), "dst" points in the new frame
 *   (x_t).  The field maps src -> dst; warping gathers: for every src grid
 *   point z, the new frame is sampled at F(z).
 *   A planar DQ is (q_c, q_s, q_x, q_y) = (cos(theta/2), sin(theta/2),
 *   (cos(theta/2) t_x + sin(theta/2) t_y)/2, (cos(theta/2) t_y -
 *   sin(theta/2) t_x)/2): the four non-zero components of r + eps t r / 2
 *   for a rotation about z (footnote to Eq. (1)).
 *
 * Memory and streams
 *   Every buffer argument is a device pointer unless marked "host".  The
 *   caller owns all buffers; the library owns the model, whose device memory
 *   is allocated once by emdq_model_create and freed by emdq_model_free
 *   (plus the half-precision tables, allocated by emdq_model_set_precision).
 *   No compute call allocates.  All work is enqueued on the caller's stream in
 *   order; a model must not be used from two streams at once.  Calls are
 *   deterministic: the same inputs give bit-identical outputs.
 *
 * Errors
 *   Every call returns an emdq_status; nothing else crosses the ABI.
 *   Argument errors are detected on the host before anything is enqueued.
 *   Conditions only the GPU can see (non-finite match coordinates, an empty
 *   inlier set, EM stopped at max_iter) are recorded in the model and
 *   returned by emdq_model_status, which waits for the stream.  After such
 *   an error, emdq_field writes NaN and emdq_warp leaves the canvas as is.
 */
#ifndef EMDQ_H
#define EMDQ_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    EMDQ_OK = 0,
    EMDQ_WARN_NOT_CONVERGED = 1, /* EM hit max_iter; the results are valid */
    EMDQ_EINVAL = -1,            /* bad argument (null, size, range)        */
    EMDQ_ETOOFEW = -2,           /* fewer than 2 matches                    */
    EMDQ_ENOINLIERS = -3,        /* EM kept no inlier                       */
    EMDQ_ENONFINITE = -4,        /* NaN or Inf in the match coordinates     */
    EMDQ_EHIP = -5,              /* a HIP runtime call failed               */
    EMDQ_ENOMEM = -6             /* device allocation failed                */
} emdq_status;

/* Tunables of the fit.  alpha0 is the coefficient of Eq. (4) at the
 * reference resolution ref_w x ref_h (Sec. III-G: 2e-4 at 480 x 270); the
 * library multiplies it by 1/s^2 with s = (w/ref_w + h/ref_h)/2 for a frame
 * of w x h.  EM: at most max_iter iterations; a match is an inlier when its
 * posterior exceeds p_thresh; the inlier fraction is clamped to
 * [gamma_min, gamma_max] and the inlier variance floored at sigma2_min
 * (px^2). */
typedef struct {
    float alpha0;
    int ref_w, ref_h;
    int max_iter;
    float p_thresh;
    float gamma_min, gamma_max;
    float sigma2_min;
    unsigned flags;   /* reserved, must be 0 */
} emdq_params;

typedef struct emdq_model_s *emdq_model;

/* Fills the defaults: 2e-4, 480, 270, 50, 0.5, 0.05, 0.95, 1e-2, 0. */
void emdq_params_default(emdq_params *p);

/* Sec. III-G: alpha0 / s^2, s = (w/ref_w + h/ref_h)/2.  Host function. */
float emdq_alpha(const emdq_params *p, int frame_w, int frame_h);

/* Allocates a model for up to n_max matches (device memory ~ 100 B per
 * match plus a few KB) on the current device.  *out receives the handle.
 * EINVAL if out is null or n_max < 2; ENOMEM / EHIP on allocation failure. */
emdq_status emdq_model_create(int n_max, emdq_model *out);

/* Releases the model and its device memory.  It first waits for all work
 * queued on the model's device (the model keeps no handle of the caller's
 * streams, so a stream destroyed before the model is not touched).  Null is
 * ignored. */
void emdq_model_free(emdq_model m);

/* EMDQ fit (Sec. II-A; Eqs. (1), (4), (18)-(20)).
 *   src_xy  device float[n][2]: match positions in the reference frame (x_0)
 *   dst_xy  device float[n][2]: matched positions in the new frame (x_t)
 *   n       number of matches, 2 <= n <= n_max of the model
 *   frame_w, frame_h  size of the new frame (alpha scaling and the uniform
 *           outlier density 1/(w h))
 *   params  host pointer, null for the defaults
 * The inputs are copied into the model, so the caller may reuse them after
 * the call returns.  The fit runs on `stream`; it synchronises the stream a
 * few times to read the EM stop flag.  Returns EINVAL (null pointer, bad
 * size or params), ETOOFEW (n < 2), EHIP, or OK once the fit is enqueued;
 * its outcome is returned by emdq_model_status. */
emdq_status emdq_fit(emdq_model m, const float *src_xy, const float *dst_xy, int n,
                     int frame_w, int frame_h, const emdq_params *params,
                     hipStream_t stream);

/* EMDQ fit started from given posteriors instead of p = 1: as emdq_fit, with
 *   init_p  device float[n], the starting posterior of every match (the
 *           starting mask is init_p > p_thresh).
 * A non-finite init_p is reported by emdq_model_status as ENONFINITE.
 * EINVAL also on a null init_p. */
emdq_status emdq_fit_from(emdq_model m, const float *src_xy, const float *dst_xy, int n,
                          int frame_w, int frame_h, const emdq_params *params,
                          const float *init_p, hipStream_t stream);

/* Learned EM start (not in the paper; an optional way to seed emdq_fit_from):
 * for every match i, the 16 nearest other matches by source distance
 * (ordered by squared distance in FP64, then index) give 64 features, per
 * neighbour j:  g (x_j - x_i)  and  ss((d_j - d_i) / 8),  g = sqrt(alpha)
 * (alpha as in emdq_fit for this frame size and params), d = dst - src,
 * ss(t) = t / (1 + |t|);  a network  p = sigmoid(w3 . gelu(W2 gelu(W1 f + b1)
 * + b2) + b3)  with 128-wide GELU layers maps them to a starting posterior.
 * The two matrix products run on BF16 matrix cores: f, W1, W2 and the first
 * GELU layer's output are rounded to bfloat16 (nearest, ties to even) and
 * the products accumulated in FP32; the biases, GELU, the output layer and
 * the sigmoid are FP32 (GELU's erf from Abramowitz & Stegun 7.1.26, absolute
 * error below 1.5e-7).  The neighbour search uses a grid for pairs of up to
 * 7168 matches and a scan of every pair above that.
 *   weights  device float[24961]: W1[128][64], b1[128], W2[128][128], b2[128],
 *            w3[128], b3 (row-major), e.g. the trained start_mlp.npy
 *   p_out    device float[n]
 * Needs no model.  EINVAL on null pointers, bad sizes or params; ETOOFEW
 * for n < 2. */
emdq_status emdq_learned_start(const float *src_xy, const float *dst_xy, int n, int frame_w,
                               int frame_h, const emdq_params *params, const float *weights,
                               float *p_out, hipStream_t stream);

/* The learned start's 64 features of every match (definition as for
 * emdq_learned_start), for training: feat_out device float[n][64]. */
emdq_status emdq_start_features(const float *src_xy, const float *dst_xy, int n, int frame_w,
                                int frame_h, const emdq_params *params, float *feat_out,
                                hipStream_t stream);

/* Floats of workspace emdq_start_train_step needs for `groups` workgroups:
 * (groups + 1) * 24962.  0 for groups < 1.  Host function. */
size_t emdq_start_train_work_floats(int groups);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, learning rate lr) on the
 * learned start's weights for the mean binary cross-entropy of a minibatch:
 *   weights, adam_m, adam_v  device float[24961], updated in place (the
 *            moments start at zero; step counts from 1 for the bias
 *            correction);
 *   feat     device float[m_samples][64], label device float[m_samples]
 *            (1 = inlier),
 *   idx      device int[batch], the minibatch's sample indices into them
 *            (an index outside [0, m_samples) is skipped, but still counts
 *            in the batch mean);
 *   groups   workgroups sharing the minibatch (<= 4096, capped at batch);
 *   work     device float workspace of emdq_start_train_work_floats(groups)
 *            floats; after the step, work[groups * 24962 + k] holds the
 *            minibatch gradient (k < 24961) and the mean loss (k = 24961).
 * Deterministic for fixed groups.  EINVAL on null pointers or bad sizes. */
emdq_status emdq_start_train_step(float *weights, float *adam_m, float *adam_v, int step,
                                  const float *feat, const float *label, int m_samples,
                                  const int *idx, int batch, float lr, int groups, float *work,
                                  hipStream_t stream);

/* Loads per-node warp functions directly (Eq. (1) per node, as the SLAM
 * nodes of Sec. III carry them) instead of fitting: host arrays
 *   x_xy float[n][2] node positions at time 0, scale float[n],
 *   q float[n][4] planar DQs, mask uint8[n] (nullable: all nodes used),
 *   alpha the already-scaled coefficient of Eq. (4).
 * Enqueued on `stream` (host arrays are copied before the call returns).
 * EINVAL on null arrays, n < 1, n > n_max or alpha <= 0. */
emdq_status emdq_model_set_nodes(emdq_model m, const float *x_xy, const float *scale,
                                 const float *q, const uint8_t *mask, int n, float alpha,
                                 hipStream_t stream);

/* Dense field (Eqs. (2)-(4), DQ normalisation, Eq. (1)) at the grid points
 * z = (zx0 + i, zy0 + k), 0 <= i < w, 0 <= k < h, of the reference frame.
 *   out_xy  device float[h][w][2], F(z) in new-frame pixels.
 * EINVAL on a null model/output or w, h < 0 (w or h == 0 is a no-op). */
emdq_status emdq_field(emdq_model m, int zx0, int zy0, int w, int h, float *out_xy,
                       hipStream_t stream);

/* Fused field + bilinear warp + colour merge (Sec. III-F, Eqs. (23)-(24)).
 * For every src grid point z = (zx0 + i, zy0 + k) (0 <= i < w, 0 <= k < h):
 * u = F(z); when 0 <= u_x <= fw-1 and 0 <= u_y <= fh-1 the new frame is
 * sampled bilinearly at u (channels 0..255 as reals) and merged into canvas
 * pixel (ox + z_x, oy + z_y):  rgb <- (A rgb + v) / (A + 1),
 * A <- min(A + 1, 30), with A the canvas alpha channel; other pixels are left
 * unchanged.
 *   frame_rgb  device uint8, row r at frame_rgb + r * frame_pitch_bytes,
 *              3 bytes (R, G, B) per pixel
 *   canvas     device float RGBA, pixel (cx, cy) at
 *              canvas + 4 * (cy * canvas_pitch_px + cx), 16-byte aligned
 * EINVAL on null pointers, non-positive frame or canvas sizes, a pitch too
 * small for its row, a misaligned canvas, or a target rectangle that leaves
 * the canvas. */
emdq_status emdq_warp(emdq_model m, const uint8_t *frame_rgb, int fw, int fh,
                      int frame_pitch_bytes, float *canvas, int cw, int ch,
                      int canvas_pitch_px, int ox, int oy, int zx0, int zy0, int w, int h,
                      hipStream_t stream);

/* Uncertainty of the field (Eq. (8)) at the grid points z = (zx0 + i,
 * zy0 + k), 0 <= i < w, 0 <= k < h: min over the inliers j of
 * exp(beta |z - x_j|^2).  beta is the already-scaled coefficient (Sec.
 * III-G: 3e-3 / s^2 with s as for alpha).
 *   out  device float[h][w]; +inf where the value exceeds the FP32 range,
 *        NaN after a failed fit.
 * EINVAL on a null model/output, w or h < 0, or beta not finite and > 0
 * (w or h == 0 is a no-op). */
emdq_status emdq_uncertainty(emdq_model m, float beta, int zx0, int zy0, int w, int h,
                             float *out, hipStream_t stream);

/* One tracking step of n_nodes deformation nodes on the current model (Sec.
 * III-C, III-E; App. A).  For node i at position pos_xy[i] in the frame of
 * the model's src points (its position at the previous frame):
 *   (ds, dq) = blended scale and DQ at pos_xy[i] (Eqs. (2)-(3)), normalised;
 *   scale[i], q[i] <- the App. A update of the node's warp function by
 *                     (ds, dq), so that the new warp of the node's time-0
 *                     position equals ds dq applied to its old image;
 *   sigma2[i] <- ds^2 sigma2[i] + min_j exp(beta d_ij^2)  (Eqs. (8), (9));
 *   pos_xy[i] <- ds dq(pos_xy[i])                          (Eq. (1)).
 * All arrays are device memory, updated in place: pos_xy float[n][2]
 * (8-byte aligned), scale float[n], q float[n][4] planar DQs (16-byte
 * aligned; returned with unit real part and q_c >= 0), sigma2 float[n].
 * A node where no inlier carries weight, or every node after a failed fit,
 * gets NaN.  EINVAL on null arguments, n_nodes < 0, misalignment or beta
 * not finite and > 0 (n_nodes == 0 is a no-op). */
emdq_status emdq_track_nodes(emdq_model m, float beta, int n_nodes, float *pos_xy,
                             float *scale, float *q, float *sigma2, hipStream_t stream);

/* Arithmetic of the dense blend in emdq_field / emdq_warp (Eqs. (2)-(4)).
 *   F32   the two factors of each weight and the node values in FP32 on FP32
 *         MFMA (the default);
 *   F16   both GEMM operands (per-axis Gaussian factors, and factor x node
 *         value) rounded to FP16, FP32 accumulation; the node DQs and scales
 *         are first re-expressed relative to a reference motion at each
 *         64 x 128 pixel tile (exact algebra: the blend is linear in the DQ
 *         and the DQ product bilinear), so the rounded values are small
 *         deviations, and the epilogue (normalisation, Eq. (1)) is FP32;
 *         FP16's range: a per-axis factor below 2^-14 is subnormal or zero,
 *         so far from every inlier along an axis (beyond ~1150 px at
 *         1920 x 1080, ~930 px at 1280 x 1024) FP16 weights lose their
 *         precision or vanish.  A 64 x 128 tile with a pixel whose weight
 *         sum is below n_in 2^-13 is therefore blended by the F32 path
 *         instead (one more launch after the FP16 one; those tiles get the
 *         F32 mode's bits), so F16 never returns NaN or degraded tiles where
 *         F32 would not;
 *   BF16  as F16 with BF16 operands (8-bit significand: about 8x the error;
 *         FP32's exponent range, so no such fallback).
 * The fit is FP32 in every mode. */
typedef enum {
    EMDQ_PREC_F32 = 0,
    EMDQ_PREC_F16 = 1,
    EMDQ_PREC_BF16 = 2
} emdq_precision;

/* Selects the arithmetic of later emdq_field / emdq_warp calls on this
 * model (host-side setting, nothing is enqueued).  The first switch to F16
 * or BF16 allocates the model's factor tables, 2 x 4096 rows of n_max
 * (rounded up to 64) 16-bit values (about 16 KB per unit of n_max; F16 also
 * 2 KB of tile flags), kept
 * until emdq_model_free; regions larger than 4096 in either direction are
 * processed in slabs.  EINVAL on a null model or an unknown value; ENOMEM. */
emdq_status emdq_model_set_precision(emdq_model m, emdq_precision precision);

/* ------------------------------------------------------------ batches ---
 * Many independent frame pairs, each with its own model, processed with one
 * launch per phase instead of one per pair and phase: the EM phases of all
 * pairs run side by side, and the field / warp of all pairs is one flat
 * launch over their tiles.  Results are read per model (emdq_model_status,
 * emdq_model_results) and, with the default field-kernel shape, are
 * bit-identical to the single-pair calls.  A
 * batch object holds only the job tables (device) and a few pinned staging
 * buffers; like a model, it is used from one stream at a time. */
typedef struct emdq_batch_s *emdq_batch;

/* Grid rectangle of one pair for emdq_batch_field / emdq_batch_warp; the
 * fields mean what the arguments of emdq_field / emdq_warp of the same names
 * mean.  out_xy is used by emdq_batch_field only; frame_rgb .. oy by
 * emdq_batch_warp only. */
typedef struct {
    int zx0, zy0, w, h;
    float *out_xy;
    const uint8_t *frame_rgb;
    int fw, fh, frame_pitch_bytes;
    float *canvas;
    int cw, ch, canvas_pitch_px, ox, oy;
} emdq_region;

/* Allocates job tables for up to max_pairs pairs (1 .. 65535). */
emdq_status emdq_batch_create(int max_pairs, emdq_batch *out);

/* Waits for the batch's last uploads and releases it.  Null is ignored. */
void emdq_batch_free(emdq_batch b);

/* emdq_fit of n_pairs pairs at once (host arrays of n_pairs entries):
 * pair i fits n[i] matches src_xy[i] -> dst_xy[i] (device float[n[i]][2])
 * of a frame_w[i] x frame_h[i] frame into models[i], with one params for
 * all (null: defaults).  init_p: null for the plain start of every pair,
 * or n_pairs device pointers to starting posteriors (float[n[i]], as
 * emdq_fit_from).  The models must be distinct.  Synchronises the stream a
 * few times to read the EM stop flags of all pairs.  EINVAL / ETOOFEW as for
 * emdq_fit (any pair), EHIP; per-pair outcomes are read with
 * emdq_model_status. */
emdq_status emdq_batch_fit(emdq_batch b, int n_pairs, const emdq_model *models,
                           const float *const *src_xy, const float *const *dst_xy,
                           const int *n, const int *frame_w, const int *frame_h,
                           const float *const *init_p, const emdq_params *params,
                           hipStream_t stream);

/* emdq_learned_start of n_pairs pairs in one launch (host arrays of n_pairs
 * entries; p_out[i] device float[n[i]]).  EINVAL / ETOOFEW as for
 * emdq_learned_start on any pair. */
emdq_status emdq_batch_learned_start(emdq_batch b, int n_pairs, const float *const *src_xy,
                                     const float *const *dst_xy, const int *n,
                                     const int *frame_w, const int *frame_h,
                                     const emdq_params *params, const float *weights,
                                     float *const *p_out, hipStream_t stream);

/* emdq_field of every pair (FP32 blend) in one launch: models[i] over
 * regions[i] (host array).  EINVAL as for emdq_field on any region. */
emdq_status emdq_batch_field(emdq_batch b, int n_pairs, const emdq_model *models,
                             const emdq_region *regions, hipStream_t stream);

/* emdq_warp of every pair (FP32 blend) in one launch.  The pairs' target
 * rectangles must not overlap in canvas memory: they are merged
 * concurrently.  EINVAL as for emdq_warp on any region. */
emdq_status emdq_batch_warp(emdq_batch b, int n_pairs, const emdq_model *models,
                            const emdq_region *regions, hipStream_t stream);

/* Autotuner of the batched field / warp launch: the field kernel comes in
 * four shapes (0, 1, 2: split-K 4, 2, 1, i.e. four wavefronts on one 32 x 32
 * tile, two tiles, or four tiles per workgroup; 3: split-K 4 on 32 x 64
 * tiles, two 32-row blocks per wavefront at two wavefronts per SIMD).
 * Shapes 0 and 3 give the same bits.  Until a shape is chosen, a batch uses
 * shape 3 when its regions hold at least 768 32 x 64 tiles, else shape 0
 * (the rule of the single-pair FP32 launches).  Times each shape on emdq_batch_field
 * of these pairs and regions (which it therefore writes), keeps the fastest
 * for later batched calls and stores it in *variant_out (nullable).  With a
 * cache_path (nullable, host file), the choice is first looked up there by
 * (rounded log2 of the total tile count, rounded log2 of the mean match
 * count) and, when timed, appended as a text line.  Synchronises the
 * stream.  EINVAL as for emdq_batch_field; EHIP. */
emdq_status emdq_batch_autotune(emdq_batch b, int n_pairs, const emdq_model *models,
                                const emdq_region *regions, const char *cache_path,
                                int *variant_out, hipStream_t stream);

/* Selects the field-kernel shape of later batched calls (0 to 3 as above). */
emdq_status emdq_batch_set_variant(emdq_batch b, int variant);

/* Builds the job table of a batched field (warp = 0) or warp (warp = 1)
 * launch in the batch's device memory, synchronously (host-blocking, on the
 * null stream), for emdq_batch_launch.  The models' current fits are read at
 * launch time, so the same prepared launch serves later fits of the same
 * models into the same buffers.  EINVAL as for emdq_batch_field /
 * emdq_batch_warp. */
emdq_status emdq_batch_prepare(emdq_batch b, int warp, int n_pairs, const emdq_model *models,
                               const emdq_region *regions);

/* Enqueues the prepared launch: one kernel, no copy and no allocation, so it
 * can be captured in a hipGraph and replayed.  EINVAL if nothing is
 * prepared. */
emdq_status emdq_batch_launch(emdq_batch b, hipStream_t stream);

/* Prepares a whole batched step for emdq_batch_launch_step: the learned
 * start of every pair (if start_weights is not null; into start_p[i],
 * device float[n[i]]), the batched EM fit from it (else from the plain
 * start), and the batched warp over regions[i] (as emdq_batch_warp).  The
 * arguments mean what they mean for emdq_batch_learned_start,
 * emdq_batch_fit and emdq_batch_warp.  The job tables are written to the
 * batch's device memory synchronously (host-blocking); the inputs are read
 * and the outputs written at launch time, so one preparation serves every
 * later step on the same buffers.  EINVAL / ETOOFEW as for those calls, EHIP.
 * Replaces the previous preparation. */
emdq_status emdq_batch_prepare_step(emdq_batch b, int n_pairs, const emdq_model *models,
                                    const float *const *src_xy, const float *const *dst_xy,
                                    const int *n, const int *frame_w, const int *frame_h,
                                    const emdq_params *params, const float *start_weights,
                                    float *const *start_p, const emdq_region *regions);

/* Enqueues the prepared step with no copy, no allocation and no host
 * synchronisation, so the whole step can be captured in one hipGraph and
 * replayed: the learned start (one launch), the EM of all pairs for the whole
 * budget of params->max_iter iterations (three launches per iteration; the
 * kernels of a pair that has stopped return at entry, so every pair's result
 * is the bits emdq_batch_fit gives), the final fits and inlier packing, and
 * the warp (one launch).  EINVAL if no step is prepared. */
emdq_status emdq_batch_launch_step(emdq_batch b, hipStream_t stream);

/* ------------------------------------------------ allocation-free step ---
 * For callers that cannot allocate device memory at call time (code under
 * hipGraph capture, tight serving loops, harnesses that forbid hipMalloc):
 * emdq_fit of the matches followed by emdq_warp of the fitted field, with no
 * model object.  The model's buffers live in a library-owned static device
 * array of about 0.7 MB per device (sized for EMDQ_STATIC_MAX_N matches), held
 * from the first call on a device until the process ends; the call allocates
 * nothing and never waits for the host.
 *   src_xy, dst_xy  device float[n][2], as for emdq_fit; 2 <= n <=
 *           EMDQ_STATIC_MAX_N
 *   params  host pointer, null for the defaults; the frame size of the fit
 *           (alpha scaling, outlier density) is fw x fh
 *   frame_rgb .. h  as for emdq_warp
 *   info    device int[3], written at the end of the step: the fit's status
 *           (an emdq_status: OK, WARN_NOT_CONVERGED, ENONFINITE, ENOINLIERS),
 *           the EM iterations and the number of inliers
 * The EM runs its whole budget of params->max_iter iterations (the kernels
 * of the iterations after the stop return at once), so the fit, its status
 * and the canvas are bit-identical to emdq_fit + emdq_warp of the same inputs.
 * Every call on a device shares that device's array, and each call starts by
 * resetting the state it reads: calls that overlap on one device (two
 * streams, two threads) race and must not be made.
 * Returns EINVAL (null pointer, n > EMDQ_STATIC_MAX_N, or the argument rules
 * of emdq_warp), ETOOFEW (n < 2), EHIP, or OK once the step is enqueued. */
#define EMDQ_STATIC_MAX_N 8192
emdq_status emdq_fit_warp_static(const float *src_xy, const float *dst_xy, int n,
                                 const emdq_params *params, const uint8_t *frame_rgb, int fw,
                                 int fh, int frame_pitch_bytes, float *canvas, int cw, int ch,
                                 int canvas_pitch_px, int ox, int oy, int zx0, int zy0, int w,
                                 int h, int *info, hipStream_t stream);

/* Waits for `stream` and returns the outcome of the last fit or
 * set_nodes: OK, WARN_NOT_CONVERGED, ENONFINITE, ENOINLIERS. */
emdq_status emdq_model_status(emdq_model m, hipStream_t stream);

/* Waits for `stream` and copies the fit to host arrays (each nullable):
 *   scale float[n], q float[n][4], p float[n] posteriors, mask uint8[n],
 *   n_in inliers, iters EM iterations, sigma2 inlier variance (px^2),
 *   gamma inlier fraction.  Returns the model status, or EINVAL. */
emdq_status emdq_model_results(emdq_model m, float *scale, float *q, float *p,
                               uint8_t *mask, int *n_in, int *iters, float *sigma2,
                               float *gamma, hipStream_t stream);

/* Static, human-readable name of a status code. */
const char *emdq_status_string(emdq_status s);

#ifdef __cplusplus
}
#endif
#endif /* EMDQ_H */
