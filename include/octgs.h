/*
 * octgs.h - C ABI of the Octree-GS render path for AMD MI355X (gfx950).
 *
 * The library renders one view of an anchor-based, octree-structured set of
 * neural Gaussians (Octree-GS, arXiv 2403.17898) in five stages, each a
 * hand-written HIP kernel sequence:
 *   1. octgs_select_lod     - visible anchors at the level set by Eq. 7;
 *   2. octgs_decode         - k neural Gaussians per selected anchor (Eq. 3, Eq. 4);
 *   3-5. octgs_rasterize_fwd - EWA projection, 16x16 tile binning with depth
 *                             order, front-to-back alpha blending (Eq. 2);
 * plus the backward passes used for training and the anchor-skip predictor.
 *
 * Conventions for every entry point:
 *  - Pointers named d_* or documented "device" are device memory owned by the
 *    caller; the library never allocates, frees or retains them after return.
 *    Host structs (octgs_camera, octgs_anchors, ...) are read during the call
 *    only.
 *  - Every call only enqueues work on `stream` (a hipStream_t passed as
 *    void*, NULL = the null stream) and returns without synchronising.
 *  - Calls on different streams may run at the same time when they write
 *    disjoint memory (each its own workspace and outputs): several frames in
 *    flight, each with its own buffers, is the intended use.  Calls that
 *    accumulate into the same arrays (octgs_decode_bwd into one set of
 *    gradients, octgs_densify_accumulate into one set of statistics, the
 *    loss scalars) must be ordered by the caller, e.g. with events.
 *    Element counts produced on the device (selected anchors, Gaussians,
 *    pairs) stay on the device; kernels read them from device scalars.
 *  - Return value: OCTGS_OK, or a negative octgs_status when host-side
 *    argument validation fails (nothing is enqueued then), or OCTGS_EHIP if a
 *    launch reports an error.  Device-detected conditions (pair-list
 *    overflow, a look-back wait that exceeded its bound, decode truncation
 *    at the Gaussian capacity) are ORed into the caller's status word
 *    (octgs_gaussians.status), and the rasterizer's also appear in
 *    octgs_raster_stats; both are readable once the stream has passed the
 *    call.
 *  - Layouts are structure-of-arrays unless stated; "planar [F][cap]" means
 *    field f of slot i at index f * cap + i.
 */
#ifndef OCTGS_H
#define OCTGS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#if defined(__GNUC__)
#define OCTGS_API __attribute__((visibility("default")))
#else
#define OCTGS_API
#endif

typedef void *octgs_stream; /* hipStream_t */

typedef enum {
  OCTGS_OK = 0,
  OCTGS_EINVAL = -1,      /* bad argument (null pointer, size, range) */
  OCTGS_ENOSPC = -2,      /* workspace smaller than octgs_*_workspace_bytes */
  OCTGS_EHIP = -3,        /* a HIP launch or runtime call failed */
  OCTGS_EUNSUPPORTED = -4 /* shape outside what the kernels implement */
} octgs_status;

typedef enum {
  OCTGS_FP32 = 0, /* plain path: FP32 inputs, FP32 MFMA, FP32 activations */
  OCTGS_BF16 = 1  /* fast path: BF16 features and weights on MFMA, FP32 accumulation */
} octgs_precision;

/* Pinhole camera.  Camera-space point = R (p - C); x right, y down, z forward.
 * Pixel (i, j) is sampled at (i + 0.5, j + 0.5).  lod_scale2 is s^2, the
 * squared focal scale factor s of Eq. 7 (Sec. IV-A, "Anchor Selection").
 * lod_blend = 1 renders with LOD transition blending (Sec. IV-A, the last
 * paragraph of "Anchor Selection"): selection also takes anchors of level
 * L_hat + 1, and decode scales every opacity by min(1, max(0, L* - L + 1))
 * with L* the clamped fractional level, i.e. by L* - L_hat for those
 * anchors and by 1 for the others.  0 = the cumulative rule alone. */
typedef struct {
  float R[9];  /* row-major world->camera rotation */
  float C[3];  /* camera centre, world */
  float fx, fy, cx, cy;
  int32_t width, height;
  float z_near;
  float lod_scale2;
  int32_t lod_blend;
} octgs_camera;

/* Anchor set (Sec. IV-A): anchors of all octree levels in one flat array.
 * All pointers are device memory. */
typedef struct {
  int64_t n;                 /* anchor count, < 2^31 */
  int32_t k;                 /* neural Gaussians per anchor, 1..16 */
  int32_t feat_dim;          /* anchor feature width; must be 32 */
  int32_t n_levels;          /* octree depth K; level values are 0..K-1 */
  float d_max;               /* the distance quantile d_max of Eq. 5 / Eq. 7 */
  const float *pos;          /* [n][3] anchor position x_v */
  const uint8_t *level;      /* [n] octree level L_v */
  const float *lod_bias;     /* [n] learnable LOD bias Delta L_v */
  const float *feat;         /* [n][feat_dim] FP32 feature (plain path) */
  const uint16_t *feat_bf16; /* [n][feat_dim] BF16 bit patterns (BF16 path; written by
                                octgs_prepare_anchors), may be NULL otherwise */
  const float *offsets;      /* [n][k][3] offsets O_i of Eq. 3 */
  const float *offset_scale; /* [n][3] scaling l_v of Eq. 3 */
  const float *base_scale;   /* [n][3] upper bound of each decoded Gaussian scale */
  const float *thr2;         /* [n] from octgs_prepare_anchors */
  const float *bound_r;      /* [n] from octgs_prepare_anchors */
} octgs_anchors;

/* The three decoding MLPs of Eq. 4 (Sec. III-B): head 0 opacity (k outputs),
 * head 1 colour (3k), head 2 covariance (7k: per Gaussian 3 scale logits then
 * a quaternion w, x, y, z).  Each head is Linear(in, width) -> ReLU ->
 * Linear(width, out) with in = feat_dim + 4 (feature, relative distance,
 * viewing direction).  w1 is [in][width], w2 is [width][out], row-major,
 * FP32, device memory; the BF16 path rounds them to BF16 itself. */
typedef struct {
  int32_t width; /* hidden width, 16..64, multiple of 16 */
  const float *w1[3], *b1[3], *w2[3], *b2[3];
} octgs_mlp;

/* Decoded neural Gaussians, planar [14][capacity] FP32 in the field order
 * mean(3), scale(3), quat(w, x, y, z), opacity, rgb(3).  Slot s*k + i holds
 * Gaussian i of the s-th listed anchor.  *count (device) is the number of
 * slots written by octgs_decode and read by octgs_rasterize_fwd.  status
 * (device, nullable): a caller-owned word the calls that write these
 * Gaussians, and the rasterizer that reads them, OR their device-detected
 * conditions into (OCTGS_STATUS_* bits), so a caller can render many frames
 * and check once; the library never clears it. */
typedef struct {
  int64_t capacity;
  float *data;
  uint32_t *count;
  uint32_t *status;
} octgs_gaussians;

/* Status bits OR-ed into octgs_gaussians.status. */
#define OCTGS_STATUS_PAIR_OVERFLOW 1u /* octgs_rasterize_fwd: the pair list overflowed (image incomplete) */
#define OCTGS_STATUS_SYNC_ERROR 2u    /* octgs_rasterize_fwd: a look-back wait hit its bound (invalid) */
#define OCTGS_STATUS_TRUNCATED 4u     /* octgs_decode*: more listed anchors than capacity / k (the rest dropped) */

/* Rasterizer constants.  alpha_max clamps each per-pixel alpha; entries with
 * alpha below alpha_min are skipped; a pixel stops after the Gaussian that
 * takes its transmittance below t_min; dilation (px^2) is added to the
 * diagonal of every 2D covariance; jac_clamp limits |x/z| and |y/z| in the
 * projection Jacobian to jac_clamp times the half-image tangent; bg is the
 * background added with the final transmittance. */
typedef struct {
  float alpha_max, alpha_min, t_min, dilation, jac_clamp;
  float bg[3];
  uint32_t flags; /* OCTGS_RASTER_* bits */
} octgs_raster_params;

/* flags: the forward keeps what octgs_rasterize_bwd needs (each emitted
 * pair's slot, and each sorted pair's emission index, carried through the
 * tile sort); required for a later backward of the same frame, off for
 * rendering only (two fewer 4-byte writes per pair and a lighter sort). */
#define OCTGS_RASTER_TRAIN 1u
/* flags: before compositing, order each XCD's tiles by list length, longest
 * first (one small extra kernel), so the last blocks to run are short ones;
 * the backward of the same frame then uses the same order.  It shortens the
 * compositing kernels when the frame runs alone on the GPU (a training step,
 * a single view); with several frames in flight their kernels already fill
 * each other's tails, and the extra kernel costs more than it saves.  The
 * image is the same bit for bit either way. */
#define OCTGS_RASTER_TILE_ORDER 2u

#define OCTGS_RASTER_STAGES 5

/* Counters the rasterizer leaves at byte 0 of its workspace. */
typedef struct {
  uint32_t n_slots;       /* Gaussian slots read (min(*count, capacity)) */
  uint32_t n_visible;     /* slots that survived the projection culls */
  uint32_t n_pairs;       /* (tile, Gaussian) pairs listed: tiles the 3-sigma ellipse meets
                             (0 on overflow) */
  uint32_t pair_overflow; /* 1 if n_candidates exceeded the pair capacity (image incomplete) */
  uint32_t sync_error;    /* 1 if a look-back wait (scans, sorts) hit its bound (output
                             invalid); partitions are taken in the order blocks start, so
                             every wait is on a running block and this is not expected */
  uint32_t n_candidates;  /* tiles of the survivors' 3-sigma rectangles, tested against the
                             ellipse; the pair capacity must hold this many (saturates) */
  uint32_t reserved[10];
} octgs_raster_stats;

/* ---------------------------------------------------------------------- */

/* Per-scene preparation for Eq. 7 (Sec. IV-A, "Anchor Selection").
 * thr2[j] = (d_max * 2^(lod_bias[j] - level[j]))^2 rounded once to FP32
 * (evaluated in double), +inf for level 0: the anchor passes the LOD rule
 * iff |x_v - C|^2 s^2 <= thr2 (the clamp of Eq. 7 applied to the sum of the
 * log term and Delta L).  bound_r[j] = max_i |O_i * l_v| + 3 max(base_scale),
 * a sphere around x_v that holds the 3-sigma extent of every Gaussian the
 * anchor can decode.  feat_bf16 (nullable, device [n][feat_dim]): the BF16
 * copy of a->feat that the OCTGS_BF16 decode reads, each value rounded to
 * nearest even.  Reads pos-independent fields of `a` (level, lod_bias,
 * offsets, offset_scale, base_scale, d_max; feat with feat_bf16);
 * a->thr2 / a->bound_r are ignored.  Outputs: device [n] each.  All three
 * depend on trained arrays: call again after every update of offsets,
 * offset_scale, base_scale, feat or lod_bias, before the next selection or
 * decode reads them. */
OCTGS_API int octgs_prepare_anchors(const octgs_anchors *a, float *thr2, float *bound_r,
                                    uint16_t *feat_bf16, octgs_stream stream);

/* Workspace bytes octgs_select_lod needs for n anchors. */
OCTGS_API size_t octgs_select_workspace_bytes(int64_t n);

/* Anchor selection (Eq. 7 and the cumulative rule L_v <= L_hat, Sec. IV-A):
 * anchor j is selected iff |x_v - C|^2 s^2 <= thr2[j] and its bound sphere
 * is visible; with cam->lod_blend the threshold is that of level L_v - 1,
 * 4 thr2[j] (exact in FP32): level L_hat + 1 is taken too, except level-1
 * anchors farther than where L* reaches 0 (their opacity factor would be 0).
 * Visibility ("visible anchors", Sec. IV-A) is conservative for a render
 * with the raster parameters p: the sphere is dropped only if it lies in
 * front of the near plane or beyond a side plane by enough that none of its
 * Gaussians' dilated 3-sigma EWA ellipses (Jacobian clamped by
 * p->jac_clamp) reaches a pixel centre; each side plane is moved out by
 * 3 sqrt(p->dilation) pixels and the sphere's radius is weighted by the
 * plane normal's length plus the clamped Jacobian's largest slope change.
 * Every decision is taken in FP32 by a fixed operation order.  Outputs:
 * sel_idx (device, capacity n) receives the selected indices in ascending
 * order; *sel_count (device) their number.  ws: device, >= the size above.
 * OCTGS_EINVAL also for cam->z_near <= 0, p->dilation < 0 or
 * p->jac_clamp <= 0. */
OCTGS_API int octgs_select_lod(const octgs_anchors *a, const octgs_camera *cam,
                               const octgs_raster_params *p, uint32_t *sel_idx,
                               uint32_t *sel_count, void *ws, size_t ws_bytes,
                               octgs_stream stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * selection as octgs_select_lod, with the same outputs, but its ballots and
 * block counts live in a buffer the library holds in static device memory
 * (about 1 MiB per GPU, kept until the process ends) instead of a workspace
 * argument.  It allocates nothing.  At most OCTGS_SELECT_NOALLOC_MAX_ANCHORS
 * anchors: a larger a->n returns OCTGS_ENOSPC and enqueues nothing.  The
 * first call on a device looks up that device's buffer address (the device
 * must be current, and `stream`, when not NULL, must belong to it;
 * OCTGS_EINVAL otherwise).  Every call on one GPU shares that GPU's buffer:
 * calls that may overlap on one GPU (different streams, several host
 * threads) race and must be ordered by the caller. */
#define OCTGS_SELECT_NOALLOC_MAX_ANCHORS 8388608 /* 2^23 */
OCTGS_API int octgs_select_lod_noalloc(const octgs_anchors *a, const octgs_camera *cam,
                                       const octgs_raster_params *p, uint32_t *sel_idx,
                                       uint32_t *sel_count, octgs_stream stream);

/* Workspace bytes of octgs_decode for a precision (OCTGS_FP32 or
 * OCTGS_BF16; 0 for any other value).  It does not depend on the scene or
 * the MLP size. */
OCTGS_API size_t octgs_decode_workspace_bytes(int32_t precision);

/* Neural-Gaussian decode (Eq. 3 and Eq. 4, Sec. III-B) of the first
 * min(*count, out->capacity / k) anchors listed in idx (device).  Network
 * input x = [feature, |x_v - C| / d_max, (x_v - C) / |x_v - C|]; outputs
 * opacity = tanh, rgb = sigmoid, scale = base_scale * sigmoid, quaternion
 * normalised (identity when its norm is 0), mean = x_v + O_i * l_v; with
 * cam->lod_blend the opacity is scaled by the transition factor above
 * (needs a->level and a->lod_bias; FP32, log2 of the distance ratio).  A
 * Gaussian with opacity <= 0 is written and later culled by the rasterizer.
 * precision selects the FP32 or the BF16 (needs a->feat_bf16) MFMA path.
 * ws: device, 16-byte aligned, >= octgs_decode_workspace_bytes(precision);
 * each call first writes the MLP weights there in the operand layout of its
 * matrix instructions (rounded to BF16 on that path), so a call always uses
 * the weights as they are when it runs.  Calls that may run at the same time
 * (different streams) need separate workspaces.  Writes out->data and
 * *out->count (device). */
OCTGS_API int octgs_decode(const octgs_anchors *a, const octgs_mlp *mlp, const octgs_camera *cam,
                 const uint32_t *idx, const uint32_t *count, int precision,
                 const octgs_gaussians *out, void *ws, size_t ws_bytes, octgs_stream stream);

/* Workspace bytes of octgs_rasterize_fwd / _bwd for a Gaussian-slot capacity,
 * a (tile, Gaussian) pair capacity and an image size; 0 for a negative
 * capacity or an image outside the rasterizer's range (at most 2^24 16x16
 * tiles, about 4.3 gigapixels; the two calls reject such images with
 * OCTGS_EINVAL). */
OCTGS_API size_t octgs_raster_workspace_bytes(int64_t gauss_capacity, int64_t pair_capacity,
                                    int32_t width, int32_t height);

/* Forward rasterization of *g->count Gaussians (Sec. III-A: EWA projection,
 * tile-based front-to-back depth order, Eq. 2 blending):
 *  - cull: opacity <= 0, camera z <= z_near, 2D covariance not positive
 *    definite, or a 3-sigma rectangle outside the image;
 *  - bin into 16x16 tiles: candidates are the tiles of the rectangle around
 *    the 3-sigma circle; a candidate is kept iff the 3-sigma ellipse
 *    {q(x) <= 9} meets the box spanned by the tile's pixel centres inside
 *    the image (canonical FP32 test); order each tile's list by camera-space
 *    depth of the Gaussian centre, ties by slot index;
 *  - per pixel: a_i = min(alpha_max, opacity_i * G'_i(x')), C = sum T_i a_i c_i,
 *    T_i = prod_{j<i} (1 - a_j), stop after T < t_min, add T * bg.
 * Outputs (device): rgb planar [3][H][W]; T_final [H][W]; last [H][W] = list
 * entries the pixel consumed (needed by the backward pass; nullable for a
 * render that no backward follows, which then skips counting); gauss_w (nullable,
 * [g->capacity]) = per-slot sum over pixels of a_i T_i (blend-weight log).
 * The workspace keeps the sorted lists for octgs_rasterize_bwd and starts
 * with octgs_raster_stats.  stage_events (nullable): 2 * OCTGS_RASTER_STAGES
 * hipEvent_t created by the caller; events 2s and 2s+1 are recorded on
 * `stream` around stage s (0 project + compaction, 1 depth sort, 2 pair
 * emission, 3 tile sort + ranges, 4 composite) for per-stage timing.
 * OCTGS_EINVAL also for cam->z_near <= 0 (depth keys are the float bits of
 * positive depths), p->dilation < 0 or p->jac_clamp <= 0. */
OCTGS_API int octgs_rasterize_fwd(const octgs_gaussians *g, const octgs_camera *cam,
                        const octgs_raster_params *p, int64_t pair_capacity, float *rgb,
                        float *T_final, uint32_t *last, float *gauss_w, void *ws,
                        size_t ws_bytes, void *const *stage_events, octgs_stream stream);

/* Backward rasterization (training, Sec. V: losses on rendered images):
 * given dL/drgb (planar [3][H][W], device) for the image the forward call
 * produced, writes dL/dGaussian planar [14][g->capacity] (same field order
 * as octgs_gaussians; zero for culled slots) into d_gauss.  Each pixel walks
 * its tile list in reverse from the entry count `last` the forward stored and
 * recovers transmittance as T_i = T_{i+1} / (1 - a_i) from T_final, so no
 * per-pixel list is kept.  g, cam, p, the capacities and the workspace must be
 * those of the forward call, unchanged since; p->flags must include
 * OCTGS_RASTER_TRAIN (OCTGS_EINVAL otherwise).  stage_events (nullable):
 * 2 * OCTGS_RASTER_BWD_STAGES hipEvent_t; events 2s and 2s+1 are recorded on
 * `stream` around stage s (0 the compositing backward, 1 the per-Gaussian
 * reduction and the projection backward). */
#define OCTGS_RASTER_BWD_STAGES 2
OCTGS_API int octgs_rasterize_bwd(const octgs_gaussians *g, const octgs_camera *cam,
                                  const octgs_raster_params *p, int64_t pair_capacity,
                                  const float *T_final, const uint32_t *last,
                                  const float *dL_drgb, float *d_gauss, void *ws,
                                  size_t ws_bytes, void *const *stage_events,
                                  octgs_stream stream);

/* Gradients of the anchor arrays (device, same shapes as octgs_anchors'
 * pos, feat, offsets, offset_scale, base_scale).  Accumulated (+=). */
typedef struct {
  float *pos, *feat, *offsets, *offset_scale, *base_scale;
} octgs_anchor_grads;

/* Gradients of the three heads' weights and biases (device, same shapes as
 * octgs_mlp).  Accumulated (+=). */
typedef struct {
  float *w1[3], *b1[3], *w2[3], *b2[3];
} octgs_mlp_grads;

/* Workspace bytes of octgs_decode_bwd for up to max_anchors listed anchors. */
OCTGS_API size_t octgs_decode_bwd_workspace_bytes(int64_t max_anchors, int32_t k, int32_t width);

/* Backward of the decode (Eq. 3 and Eq. 4, FP32): from dL/dGaussian planar
 * [14][gauss_capacity] of the slots octgs_decode wrote for the first
 * min(*count, gauss_capacity / k) anchors of idx, accumulates the gradients
 * of the listed anchors' arrays (each listed anchor at most once per call)
 * and of the MLP weights.  The forward activations are recomputed. */
OCTGS_API int octgs_decode_bwd(const octgs_anchors *a, const octgs_mlp *mlp,
                               const octgs_camera *cam, const uint32_t *idx,
                               const uint32_t *count, const float *d_gauss,
                               int64_t gauss_capacity, const octgs_anchor_grads *ga,
                               const octgs_mlp_grads *gm, void *ws, size_t ws_bytes,
                               octgs_stream stream);

/* octgs_decode_bwd in two halves (Sec. III-B, Eq. 3 and Eq. 4), for several
 * views whose gradients go into one set of arrays.  octgs_decode_bwd_rows
 * computes every listed anchor's gradient row and the MLP weight-gradient
 * partial sums into ws and touches no gradient array, so the rows of
 * different views (separate workspaces) may run at the same time.
 * octgs_decode_bwd_apply adds a workspace's rows into ga (each listed anchor
 * once) and its partial sums into gm; applies that share ga and gm must be
 * ordered by the caller.  octgs_decode_bwd is the two in sequence, and the
 * arguments mean the same as there; apply takes the idx, count, capacity
 * and workspace of its rows call, unchanged since. */
OCTGS_API int octgs_decode_bwd_rows(const octgs_anchors *a, const octgs_mlp *mlp,
                                    const octgs_camera *cam, const uint32_t *idx,
                                    const uint32_t *count, const float *d_gauss,
                                    int64_t gauss_capacity, void *ws, size_t ws_bytes,
                                    octgs_stream stream);
OCTGS_API int octgs_decode_bwd_apply(const octgs_anchors *a, const octgs_mlp *mlp,
                                     const uint32_t *idx, const uint32_t *count,
                                     int64_t gauss_capacity, const octgs_anchor_grads *ga,
                                     const octgs_mlp_grads *gm, const void *ws, size_t ws_bytes,
                                     octgs_stream stream);

/* Mean-L1 image loss of the training step: dimg = scale * sign(img - target)
 * and *loss += scale * sum |img - target| (device scalar, accumulated), over n
 * elements.  scale is 1 / (elements averaged over). */
OCTGS_API int octgs_l1_loss_grad(const float *img, const float *target, int64_t n, float scale,
                                 float *dimg, float *loss, octgs_stream stream);

/* Workspace bytes of octgs_photometric_loss_grad for n_images planes of
 * height x width. */
OCTGS_API size_t octgs_photometric_workspace_bytes(int64_t n_images, int32_t height,
                                                   int32_t width);

/* Photometric training loss of the 3D-GS model (Sec. V, implementation
 * details: L1 and SSIM weighted 0.8 and 0.2):
 *   *loss += w_l1 mean|img - target| + w_ssim (1 - mean SSIM(img, target)),
 * and dimg (overwritten) = its gradient with respect to img.  img, target,
 * dimg: device, n_images planes of [height][width] FP32 (views x 3 colour
 * channels, each plane an image of its own).  SSIM is the standard form of
 * Wang et al. (2004): 11 x 11 Gaussian window with sigma 1.5, C1 = 0.01^2,
 * C2 = 0.03^2 (data range 1), windowed statistics over a zero-padded
 * same-size correlation, averaged over every pixel of every plane.  With
 * w_ssim = 0 the call is the L1 term alone and needs no workspace.  ws:
 * device, >= octgs_photometric_workspace_bytes (three derivative maps).
 * n_images <= 65535. */
OCTGS_API int octgs_photometric_loss_grad(const float *img, const float *target,
                                          int64_t n_images, int32_t height, int32_t width,
                                          float w_l1, float w_ssim, float *dimg, float *loss,
                                          void *ws, size_t ws_bytes, octgs_stream stream);

/* Volume regularisation of the Scaffold-GS model (Sec. V, implementation
 * details: L_vol = sum_i Prod(s_i), weight 0.01): over the first
 * min(*g->count, g->capacity) decoded slots with opacity > 0 (those the
 * rasterizer draws), *loss += weight * sum s_x s_y s_z, and the scale rows
 * (fields 3..5) of d_gauss (planar [14][g->capacity], device) receive
 * += weight * the product of the other two scales. */
OCTGS_API int octgs_volume_loss_grad(const octgs_gaussians *g, float weight, float *d_gauss,
                                     float *loss, octgs_stream stream);

/* One Adam update of n parameters (bias-corrected, step >= 1):
 * m = b1 m + (1 - b1) g; v = b2 v + (1 - b2) g^2;
 * p -= lr (m / (1 - b1^step)) / (sqrt(v / (1 - b2^step)) + eps). */
OCTGS_API int octgs_adam_step(float *param, const float *grad, float *m, float *v, int64_t n,
                              float lr, float beta1, float beta2, float eps, int32_t step,
                              octgs_stream stream);

/* The same update for count arrays at once (one launch per 32 arrays):
 * params[i], grads[i], m[i], v[i] are device arrays of n[i] floats; the
 * pointer tables and n are host arrays read during the call. */
OCTGS_API int octgs_adam_step_many(int32_t count, float *const *params, const float *const *grads,
                                   float *const *m, float *const *v, const int64_t *n, float lr,
                                   float beta1, float beta2, float eps, int32_t step,
                                   octgs_stream stream);

/* ---- learned anchor skip ---------------------------------------------
 * A per-anchor contribution predictor extending the view-dependent anchor
 * selection of Sec. IV-A: input z = [feature (32), unit direction camera ->
 * anchor in camera coordinates R (x_v - C) / |x_v - C| (3),
 * log2(|x_v - C| / d_max), level] (37 values); network 37 -> 64
 * -> ReLU -> 64 -> ReLU -> 1 (logit).  Weights FP32, row-major [in][out],
 * device memory. */
typedef struct {
  const float *w1, *b1, *w2, *b2, *w3, *b3; /* [37][64], [64], [64][64], [64], [64][1], [1] */
} octgs_skip_net;

typedef struct {
  float *w1, *b1, *w2, *b2, *w3, *b3;
} octgs_skip_net_grads;

/* Per listed anchor, the sum of its k Gaussians' logged blend weights:
 * w_out[m] = sum_i gauss_w[m * k + i] for m < min(*count, cap_anchors)
 * (gauss_w from octgs_rasterize_fwd; count = listed anchors). */
OCTGS_API int octgs_anchor_weights(const float *gauss_w, const uint32_t *count, int32_t k,
                                   int64_t cap_anchors, float *w_out, octgs_stream stream);

/* Predictor inputs z [cap][37] (FP32) of the first min(*count, cap) anchors of idx. */
OCTGS_API int octgs_skip_features(const octgs_anchors *a, const octgs_camera *cam,
                                  const uint32_t *idx, const uint32_t *count, int64_t cap,
                                  float *z, octgs_stream stream);

/* Workspace bytes of octgs_skip_predict for lists of up to cap anchors. */
OCTGS_API size_t octgs_skip_predict_workspace_bytes(int64_t cap);

/* Skip prediction over the selected anchors (BF16 MFMA, FP32 accumulation):
 * keeps anchor sel_idx[p] iff its logit >= logit_threshold.  keep_idx (device,
 * capacity cap) receives the kept indices in ascending order, *keep_count
 * their number; logits (nullable, [cap]) the logit per list position. */
OCTGS_API int octgs_skip_predict(const octgs_anchors *a, const octgs_camera *cam,
                                 const octgs_skip_net *net, float logit_threshold,
                                 const uint32_t *sel_idx, const uint32_t *sel_count, int64_t cap,
                                 uint32_t *keep_idx, uint32_t *keep_count, float *logits,
                                 void *ws, size_t ws_bytes, octgs_stream stream);

/* Workspace bytes of octgs_skip_train_grad for a batch size. */
OCTGS_API size_t octgs_skip_train_workspace_bytes(int32_t batch);

/* Gradient of the mean weighted binary cross-entropy of the predictor on a
 * batch: row b of the batch is z[r][0..36], label y[r] in {0, 1}, with
 * r = rows[b] (device, nullable: r = b); positives are weighted by
 * pos_weight.  Inputs whose bit in input_mask is clear read as zero, so their
 * rows of the w1 gradient are zero (all 37 inputs: (1 << 37) - 1).  Forward
 * and backward run on BF16 MFMA (16x16x16, FP32 accumulation) with BF16
 * copies of the FP32 weights; layer 3, the loss and the bias gradients are
 * FP32.  Gradients are overwritten; *loss (device) is incremented by the
 * batch loss.  The result does not depend on scheduling: each block sums its
 * rows in a fixed order and the block sums are added in block order.
 * Every rows[b] must index a row of z and y (not checked).  Pair with
 * octgs_adam_step for the update. */
OCTGS_API int octgs_skip_train_grad(const octgs_skip_net *net, const float *z, const float *y,
                                    const uint32_t *rows, int32_t batch, uint64_t input_mask,
                                    float pos_weight, const octgs_skip_net_grads *grads,
                                    float *loss, void *ws, size_t ws_bytes, octgs_stream stream);

/* ---- explicit Gaussians on the anchors --------------------------------
 * The 3D-GS instance of the anchor framework (Sec. V, "Our-3D-GS"): every
 * anchor carries k explicit 3D Gaussians (Sec. III-A) instead of a feature
 * decoded by MLPs.  Selection (octgs_select_lod, Eq. 7) and rasterization
 * are shared with the neural path; only the per-scene preparation and the
 * decode differ.  Arrays are indexed by Gaussian g = anchor * k + i, device
 * memory, FP32 unless stated. */
typedef struct {
  int32_t sh_degree;       /* D, 0..3: (D+1)^2 colour coefficients per channel */
  const float *mean;       /* [n][k][3] world position */
  const float *log_scale;  /* [n][k][3] scale = exp(log_scale) */
  const float *rot;        /* [n][k][4] quaternion w, x, y, z (normalised on use), 16-byte aligned */
  const float *opacity;    /* [n][k] logit; opacity = sigmoid(logit) */
  const float *sh;         /* [n][k][(D+1)^2][3] real SH coefficients, 16-byte aligned */
  const uint16_t *sh_bf16; /* same layout as BF16 bit patterns (OCTGS_BF16; D = 1 or 3), 16-byte
                              aligned; may be NULL otherwise */
} octgs_explicit;

/* Gradients of the explicit arrays (same shapes; rot and sh 16-byte
 * aligned).  Accumulated (+=). */
typedef struct {
  float *mean, *log_scale, *rot, *opacity, *sh;
} octgs_explicit_grads;

/* Per-scene preparation for Eq. 7 with explicit Gaussians: thr2 as in
 * octgs_prepare_anchors; bound_r[j] = max_i |mean_i - x_v| + 3 exp(max log_scale)
 * over the anchor's Gaussians (canonical FP32; the exponential of the
 * largest log-scale is taken in double and rounded once), a sphere holding
 * every Gaussian's 3-sigma extent.  sh_bf16 (nullable, device, the layout
 * of e->sh): the BF16 copy of e->sh that the OCTGS_BF16 decode reads, each
 * value rounded to nearest even.  Reads a->n, k, d_max, pos, level,
 * lod_bias and e->mean, e->log_scale (e->sh with sh_bf16).  Outputs: device
 * [n] each.  Call again after any update of those arrays. */
OCTGS_API int octgs_prepare_explicit(const octgs_anchors *a, const octgs_explicit *e,
                                     float *thr2, float *bound_r, uint16_t *sh_bf16,
                                     octgs_stream stream);

/* Decode of the explicit Gaussians of the first min(*count, out->capacity / k)
 * anchors listed in idx (device): slot p*k + i receives Gaussian i of the
 * p-th listed anchor as mean, exp(log_scale), the normalised quaternion
 * (identity when its norm is 0), sigmoid(logit) and the colour
 * max(0, sum_lm sh_lm Y_lm(d) + 0.5), d the unit vector from the camera
 * centre to the mean and Y_lm the real spherical harmonics with the
 * Condon-Shortley phase kept, ordered l^2 + l + m (the 3D-GS colour model).
 * With cam->lod_blend the opacity is scaled by the transition factor of
 * octgs_camera (needs a->pos, level, lod_bias).  precision OCTGS_BF16 reads
 * e->sh_bf16 (other attributes stay FP32; arithmetic is FP32).  Writes
 * out->data and *out->count like octgs_decode.  Returns OCTGS_EUNSUPPORTED for
 * D > 3, or BF16 with D other than 1 and 3; OCTGS_EINVAL for misaligned rot or
 * sh. */
OCTGS_API int octgs_decode_explicit(const octgs_anchors *a, const octgs_explicit *e,
                                    const octgs_camera *cam, const uint32_t *idx,
                                    const uint32_t *count, int precision,
                                    const octgs_gaussians *out, octgs_stream stream);

/* Backward of octgs_decode_explicit (FP32 coefficients; lod_blend returns
 * OCTGS_EUNSUPPORTED): from dL/dGaussian planar [14][gauss_capacity] of the
 * slots written for the first min(*count, gauss_capacity / k) anchors of idx,
 * accumulates the gradients of their explicit arrays, the mean also through
 * the view direction of the colour.  Each listed anchor at most once per
 * call (no atomics). */
OCTGS_API int octgs_decode_explicit_bwd(const octgs_anchors *a, const octgs_explicit *e,
                                        const octgs_camera *cam, const uint32_t *idx,
                                        const uint32_t *count, const float *d_gauss,
                                        int64_t gauss_capacity, const octgs_explicit_grads *g,
                                        octgs_stream stream);

/* ---- densification statistics (Sec. IV-B, adaptive anchor control) ----
 * Accumulated over the training views of an interval of T iterations, then
 * turned into growth, LOD-bias and pruning decisions.  Arrays are device
 * memory indexed by anchor j or Gaussian g = j * k + i; the caller zeroes
 * them at the start of an interval. */
typedef struct {
  float *grad_sum;       /* [n][k] sum over views of |dL/d(projected centre)|, NDC units */
  uint32_t *grad_count;  /* [n][k] views in which the Gaussian was rasterized */
  float *opacity_sum;    /* [n] sum over selecting views of sum_i max(opacity_i, 0) */
  uint32_t *view_count;  /* [n] views that selected the anchor */
} octgs_densify_stats;

/* Thresholds of the decisions: tau_g and beta of the level threshold
 * tau_g 2^(beta L) (paper defaults 0.0002 and 0.2), the LOD-bias step
 * epsilon (0.01), the minimum average opacity tau_opacity, the minimum view
 * frequency tau_v (0.7, 0.01 or 0.2 by dataset in the paper), and the number
 * of training views the statistics cover. */
typedef struct {
  float tau_g, beta, epsilon, tau_opacity, tau_v;
  int32_t n_views;
} octgs_densify_params;

/* Statistics of one training view, after its octgs_rasterize_bwd (g, cam,
 * pair_capacity and raster_ws as in that call, unchanged since; g decoded
 * from the anchors idx / count with k Gaussians each): every slot the view
 * rasterized (survived the projection culls) adds the norm of its
 * projected-centre gradient in normalised device coordinates (the pixel
 * gradient scaled by (W/2, H/2)) to grad_sum and 1 to grad_count of its
 * Gaussian; every listed anchor adds the sum of its Gaussians' opacities
 * (negative taken as 0) to opacity_sum and 1 to view_count.  Each anchor at
 * most once per call. */
OCTGS_API int octgs_densify_accumulate(const octgs_gaussians *g, const octgs_camera *cam,
                                       int64_t pair_capacity, const void *raster_ws,
                                       size_t ws_bytes, const uint32_t *idx,
                                       const uint32_t *count, int32_t k,
                                       const octgs_densify_stats *st, octgs_stream stream);

/* Decisions of an interval, in FP32 with the level thresholds
 * tau_L = tau_g 2^(beta L) rounded once from double:
 *  - grow_level[g] (device [n][k]): -1, or the level of the new anchor the
 *    Gaussian seeds: with grad = grad_sum / grad_count (0 if never
 *    rasterized) and L its anchor's level, L if grad > tau_L, L + 1 if also
 *    grad > tau_(L+1) and L + 1 < K ("next-level growing", Sec. IV-B);
 *  - lod_bias[j] (device, in/out) += epsilon where the mean grad of the
 *    anchor's rasterized Gaussians exceeds tau_L / 4;
 *  - prune[j] (device [n]) = 1 if view_count / n_views < tau_v, or if the
 *    anchor was selected and opacity_sum / (k view_count) < tau_opacity;
 *  - counts (device [4], overwritten): Gaussians that grow, of them
 *    promoted, bias updates, pruned anchors.
 * Reads a->n, k, n_levels (<= 64), level.  Thresholds of Eq. 7 depend on
 * lod_bias: run octgs_prepare_anchors again after the update.  Placing the
 * grown anchors (empty-voxel test) and removing the pruned ones are left to
 * the caller. */
OCTGS_API int octgs_densify_decide(const octgs_anchors *a, const octgs_densify_stats *st,
                                   const octgs_densify_params *p, float *lod_bias,
                                   int8_t *grow_level, uint8_t *prune, uint32_t *counts,
                                   octgs_stream stream);

/* Device pointers into a rasterizer workspace (as laid out for these
 * capacities and image size) to the state octgs_rasterize_fwd leaves there:
 * the stats header, the sorted pair list (tile id and slot per entry, length
 * n_pairs when pair_overflow is 0) and the per-tile ranges [tiles][2] =
 * [start, end).  Read-only views; valid until the workspace is reused.
 * Needs no HIP call. */
OCTGS_API int octgs_raster_views(const void *ws, int64_t gauss_capacity, int64_t pair_capacity,
                       int32_t width, int32_t height, const octgs_raster_stats **stats,
                       const uint32_t **pair_tile, const uint32_t **pair_slot,
                       const uint32_t **tile_ranges);

/* Error string of a status code (static storage). */
OCTGS_API const char *octgs_strerror(int status);

/* Library version, for load checks. */
OCTGS_API int octgs_version(void);

#ifdef __cplusplus
}
#endif

#endif /* OCTGS_H */
