/*
 * gsr.h - C ABI of an MI355X (gfx950) differentiable 3D Gaussian-splatting
 * rasterizer: Gaussians plus cameras in; colour, depth and alpha images out;
 * gradients back.
 *
 * What it computes.  MAGS-SLAM optimises each agent's Gaussian submap by
 * gradient descent on an L1 photometric plus depth loss over a window of
 * keyframes (Sec. III-A, Eq. (map_loss)) and refines the fused map on the
 * differentiably rendered RGB and depth with per-keyframe pose deltas
 * (Sec. III-C, Eq. (refine_loss)); both call a 3D Gaussian-splatting
 * rasterizer (cited in Sec. I and II-A) on every iteration.  A Gaussian has a
 * mean, a scale vector, a rotation, an opacity and a colour (Sec. III-C,
 * Eq. (gauss_update)); a keyframe has a world-to-camera pose (Sec. III-B)
 * and pinhole intrinsics (Appendix A).  This library implements:
 *
 *   forward : EWA projection of every (view, Gaussian) pair, opacity-aware
 *             tile binning, a (tile, depth)-key radix sort, and per-pixel
 *             front-to-back alpha compositing of colour, depth and opacity
 *             (alpha = min(0.99, sigma*G); entries with alpha < 1/255 are
 *             skipped; compositing stops before transmittance would drop
 *             below 1e-4).
 *   backward: the exact gradient of a loss with respect to the Gaussian
 *             parameters and each view's SE(3) pose, by reverse compositing
 *             with transmittance recomputed by division.
 *
 * Conventions.  Camera space is x right, y down, z forward.  Pixel (i, j) is
 * sampled at (i + 0.5, j + 0.5).  A view matrix is the row-major 3x4
 * world-to-camera [R | t].  Quaternions are (w, x, y, z) and need not be
 * unit length (they are normalised inside).  Scales are given as natural
 * logarithms, opacities as logits (opacity = sigmoid(logit)).  Colours are
 * raw RGB for sh_degree 0, or real spherical-harmonic coefficients
 * (Condon-Shortley phase, index l*l + l + m) evaluated as
 * max(0, 0.5 + sum Y_lm(d) k_lm) along the unit direction d from the camera
 * centre to the mean for sh_degree 1..3.  Depth is the unnormalised sum of
 * z * alpha * T; alpha is 1 - final transmittance; colour includes
 * T_final * bg.  The pose gradient is with respect to a left perturbation
 * [R|t] <- Exp(xi) [R|t] at xi = 0, xi = (rho, phi), translation first.
 *
 * Memory.  Every float pointer in gsr_scene, gsr_views, gsr_images,
 * gsr_grads and the state buffer is DEVICE memory of the context's GPU,
 * caller-owned, FP32, C-contiguous.  set_offsets, view_set and needs_grad
 * (the call's structure, not its values) are HOST arrays read during the
 * call and turned into kernel arguments: changing a set's size or a view's
 * set therefore needs a new call (and a new capture of a graph that holds
 * the old one), while the Gaussians' values and the cameras may change in
 * place between replays.  The context owns its workspace (allocated by
 * gsr_plan).  Each forward writes its saved state into a caller-owned
 * device buffer of gsr_state_bytes() bytes, which the matching backward
 * reads; several forwards may be alive at once.
 *
 * Limits.  One call renders at most GSR_MAX_VIEWS (64) views of at most
 * GSR_MAX_SETS (64) Gaussian sets: the per-view tables travel as kernel
 * arguments and the backward's view mask is one 64-bit word.  Larger batches
 * are split into several calls (the gradients of the calls add).
 *
 * Streams.  `stream` is a hipStream_t passed as void* (NULL = default
 * stream).  gsr_forward and gsr_backward only enqueue work: they do not
 * allocate, free, synchronise or copy to the host, so they may be captured
 * in a HIP graph.  Work-dependent sizes (visible pairs, row entries) stay
 * on the device.
 *
 * Errors.  Every call returns a gsr_status and never aborts; the context's
 * last error message gives details.  One context is used by one host
 * thread at a time.  A forward whose binning entries exceed the planned
 * capacity sets a device flag, renders nothing useful, and gsr_poll then
 * reports GSR_E_OVERFLOW with the needed capacity.
 */
#ifndef GSR_H
#define GSR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GSR_MAX_VIEWS 64 /* views per forward/backward call */
#define GSR_MAX_SETS 64  /* Gaussian sets (submaps) per call */
/* grid points (ceil(W / stride) x ceil(H / stride)) of one gsr_seed_noalloc
 * call: its library-held block counts take 4 B per 256 points (256 KiB) */
#define GSR_SEED_NOALLOC_MAX_POINTS (1 << 24)

typedef enum gsr_status {
  GSR_OK = 0,
  GSR_E_INVALID_ARG = 1,   /* null pointer, bad size, unsupported option */
  GSR_E_NOT_PLANNED = 2,   /* forward/backward before gsr_plan */
  GSR_E_CAPACITY = 3,      /* a host-known size exceeds the plan */
  GSR_E_OVERFLOW = 4,      /* a device-side count exceeded the plan (gsr_poll) */
  GSR_E_DEVICE = 5,        /* HIP error or no usable gfx950 device */
  GSR_E_OOM = 6,           /* device allocation failed */
  GSR_E_UNIMPLEMENTED = 7
} gsr_status;

typedef struct gsr_ctx gsr_ctx;

/* Capacities.  All workspace is sized from these at gsr_plan time. */
typedef struct gsr_plan_desc {
  int64_t max_pairs;     /* >= sum over views of the size of the view's set */
  int64_t max_instances; /* >= (Gaussian, tile row) entries per forward call:
                            the binning stores each visible pair once per
                            tile row its rect spans, and every tile's list
                            is that row's list filtered by column, so a
                            bound on the (Gaussian, tile) copies is also
                            enough */
  int32_t max_views;     /* 1..GSR_MAX_VIEWS */
  int32_t width;         /* image size every call of this plan uses */
  int32_t height;
  int32_t tile_w;        /* tile shape: 8, 16 or 32 each, tile_w*tile_h in [64, 512] */
  int32_t tile_h;
  int32_t chunk;         /* depth-sorted pairs per binning chunk, at most 256
                            (0 = automatic) */
  int32_t fwd_batch;     /* list entries staged per lane per round in the
                            forward compositing: 1 or 2 (0 = 1) */
  int32_t bwd_batch;     /* list entries staged per lane per round in the
                            backward compositing: 1, 2 or 4 (0 = 1) */
  int32_t persistent;    /* 1: compositing kernels run a grid of resident
                            workgroups whose waves take tiles from a queue
                            ordered by decreasing list length; 0: one wave per
                            tile */
  int32_t bwd_cols;      /* tiles of a tile row per backward wave: 1 or 2
                            (0 = 1); 2 needs tile_w <= 16 and
                            2 tile_w tile_h <= 512, and its backward always
                            runs one wave per pair of tiles (no queue) */
} gsr_plan_desc;

/* Gaussians, concatenated over sets; set s owns [set_offsets[s], set_offsets[s+1]). */
typedef struct gsr_scene {
  const float* means;          /* device [N,3] */
  const float* log_scales;     /* device [N,3] */
  const float* quats;          /* device [N,4] (w,x,y,z) */
  const float* opacity_logits; /* device [N] */
  const float* colors;         /* device [N,3] (sh_degree 0) or [N,sh_stride,3] */
  const int64_t* set_offsets;  /* HOST [n_sets+1], non-decreasing, set_offsets[0] == 0 */
  int32_t n_sets;              /* 1..GSR_MAX_SETS */
  int32_t sh_degree;           /* 0 (raw RGB) or 1..3 */
  int32_t sh_stride;           /* coefficient rows per Gaussian (>= (D+1)^2; ignored for D=0) */
  int32_t reserved;
} gsr_scene;

typedef struct gsr_views {
  const float* viewmats;     /* device [V,3,4] world->camera */
  const float* intrinsics;   /* device [V,4] fx, fy, cx, cy (pixels) */
  const int32_t* view_set;   /* HOST [V] set rendered by each view */
  const uint8_t* needs_grad; /* HOST [V] or NULL (all 1): backward skips views with 0 */
  int32_t n_views;           /* 1..max_views */
  int32_t width;             /* must equal the plan's */
  int32_t height;
  int32_t reserved;
} gsr_views;

typedef struct gsr_settings {
  float z_near; /* Gaussians with camera depth <= z_near are culled (default 0.2) */
  float bg[3];  /* background colour composited with the final transmittance */
} gsr_settings;

typedef struct gsr_images {
  float* color;      /* device [V,3,H,W] */
  float* depth;      /* device [V,H,W] */
  float* alpha;      /* device [V,H,W] */
  int32_t* n_eval;   /* device [V,H,W] list entries examined per pixel, or NULL */
} gsr_images;

typedef struct gsr_grad_images {
  const float* color; /* device [V,3,H,W] dL/dcolor, or NULL (= 0) */
  const float* depth; /* device [V,H,W] dL/ddepth, or NULL */
  const float* alpha; /* device [V,H,W] dL/dalpha, or NULL */
} gsr_grad_images;

/* Gradients are overwritten (not accumulated).  Gaussians of sets that no
 * grad-needing view renders get zeros.  d_pose rows of views with
 * needs_grad == 0 get zeros. */
typedef struct gsr_grads {
  float* d_means;          /* device [N,3] */
  float* d_log_scales;     /* device [N,3] */
  float* d_quats;          /* device [N,4] */
  float* d_opacity_logits; /* device [N] */
  float* d_colors;         /* device, same shape as colors */
  float* d_pose;           /* device [V,6] (rho, phi) */
} gsr_grads;

typedef struct gsr_counts {
  int64_t visible_pairs; /* pairs that survived culling, summed over views */
  int64_t instances;     /* (Gaussian, tile) copies of the last forward (the
                            tile lists' total length; never stored) */
  int64_t row_entries;   /* (Gaussian, tile row) entries of the last forward */
  int64_t capacity;      /* max_instances of the plan */
  int32_t overflow;      /* 1 if row_entries > capacity */
  int32_t n_views;
} gsr_counts;

/* Create a context on HIP device `device`.  GSR_E_DEVICE (with *out = NULL)
 * when no such device exists or it is not gfx950. */
gsr_status gsr_create(gsr_ctx** out, int device);
void gsr_destroy(gsr_ctx* ctx);

/* Allocate the context's workspace for the given capacities (replacing any
 * previous plan).  Must not be called while work of this context is queued
 * on a stream that has not finished. */
gsr_status gsr_plan(gsr_ctx* ctx, const gsr_plan_desc* plan);

/* Bytes of the per-forward saved-state buffer for this plan (host only;
 * needs no device).  The buffer must be 256-byte aligned. */
gsr_status gsr_state_bytes(const gsr_plan_desc* plan, size_t* out_bytes);

/* Forward render of every view (Sec. III-A Eq. (map_loss) and Sec. III-C
 * Eq. (refine_loss) consume its colour and depth).  Writes `out` and the
 * saved state into `state`. */
gsr_status gsr_forward(gsr_ctx* ctx, const gsr_scene* scene, const gsr_views* views,
                       const gsr_settings* settings, void* state, const gsr_images* out,
                       void* stream);

/* Backward of the forward that wrote `state` (same scene, views, settings,
 * unchanged device contents). */
gsr_status gsr_backward(gsr_ctx* ctx, const gsr_scene* scene, const gsr_views* views,
                        const gsr_settings* settings, const void* state,
                        const gsr_grad_images* grad_in, const gsr_grads* out, void* stream);

/* Synchronise `stream` and read the device counters of the forward that
 * wrote `state`.  Returns GSR_E_OVERFLOW if its row entries exceeded the
 * plan (re-plan with max_instances >= row_entries). */
gsr_status gsr_poll(gsr_ctx* ctx, const void* state, gsr_counts* out, void* stream);

/* Test/debug export of a forward's binning (synchronises `stream`; the tile
 * lists and the blend counts are formed by debug kernels in temporary device
 * buffers).  Host buffers, each may be NULL:
 *   zkeys   uint32 [P]  FP32 bits of camera depth per pair, 0xFFFFFFFF = culled
 *   rects   uint16 [P,4] tile rect x0,y0,x1,y1 (zeros when culled)
 *   order   uint32 [P]  pair ids of each view's visible pairs in (depth, id)
 *                       order, views concatenated
 *   vis_off int64 [V+1] offsets of each view's part of `order`
 *   inst    uint32 [I]  pair id of every tile instance, tile-major, depth order
 *   ranges  uint32 [V*TX*TY,2] [first, last+1) per tile, (0,0) when empty
 *   t_final float [V,H,W], last uint32 [V,H,W] (last blended list position + 1)
 *   n_blend int32 [V,H,W] list entries blended per pixel (counted by a debug
 *                       kernel with the forward's skip arithmetic)
 * P is the call's pair count (sum of set sizes over views; order and inst
 * map visible-list positions back to pair ids through the first n_pairs
 * pairs, so n_pairs must be P for them); I from gsr_poll. */
typedef struct gsr_debug {
  uint32_t* zkeys;
  uint16_t* rects;
  uint32_t* order;
  int64_t* vis_off;
  uint32_t* inst;
  uint32_t* ranges;
  float* t_final;
  uint32_t* last;
  int32_t* n_blend;
  int64_t n_pairs;     /* in: capacity of zkeys/rects/order (elements) */
  int64_t n_inst;      /* in: capacity of inst (elements) */
} gsr_debug;
gsr_status gsr_debug_export(gsr_ctx* ctx, const void* state, int32_t n_views,
                            gsr_debug* dbg, void* stream);

/* viewmats_out[v] = Exp(delta[v]) * viewmats_in[v] for v < n_views (the
 * per-keyframe pose delta of Sec. III-C); in-place allowed.  Device arrays
 * [V,3,4], [V,6], [V,3,4]. */
gsr_status gsr_apply_pose_delta(const float* viewmats_in, const float* delta,
                                float* viewmats_out, int32_t n_views, void* stream);

/* Sim(3) correction of Gaussian sets (Sec. III-C, Eq. (gauss_update)).  The
 * Gaussians [set_offsets[k], set_offsets[k+1]) of set k move by
 * sims[k] = (s, qw, qx, qy, qz, tx, ty, tz) (s > 0; the quaternion is
 * normalised here): means -> s R means + t, log_scales -> log_scales + ln s,
 * quats -> q_R * quats (Hamilton product, the norm of quats kept).  Opacity
 * and colours, SH coefficients of every degree included, are not touched.
 * Device arrays means [N,3], log_scales [N,3], quats [N,4] (out may alias
 * in) and sims [n_sets,8]; set_offsets is a HOST array of n_sets+1
 * non-decreasing offsets starting at 0, n_sets in 1..GSR_MAX_SETS.
 * Enqueues one kernel on `stream`; GSR_E_INVALID_ARG for null pointers or
 * bad offsets, GSR_E_DEVICE if the launch fails. */
gsr_status gsr_sim3_gaussians(const float* means_in, const float* log_scales_in,
                              const float* quats_in, const int64_t* set_offsets, int32_t n_sets,
                              const float* sims, float* means_out, float* log_scales_out,
                              float* quats_out, void* stream);

/* Lift of keyframe poses into the global frame (Sec. III-B, Eq. (mapgba_lift)):
 * view v of set view_set[v], with sims[view_set[v]] = (s, q, t) and R = R(q),
 * gets viewmats_out[v] = [Rv R^T | s tv - Rv R^T t].  This is the rigid form
 * of Tv o C^{-1}: the same camera with its length unit scaled by s, so pixels
 * are unchanged and camera depths (and the near plane) scale by s.  Device
 * viewmats [n_views,3,4] (out may alias in) and sims [n_sets,8]; view_set is
 * a HOST array [n_views] of set indices < n_sets.  Enqueues one kernel;
 * GSR_E_INVALID_ARG for null pointers or out-of-range sizes. */
gsr_status gsr_sim3_views(const float* viewmats_in, const float* sims, const int32_t* view_set,
                          int32_t n_views, int32_t n_sets, float* viewmats_out, void* stream);

/* Gradient of the L1 terms of the refinement loss (Sec. III-C, Eq.
 * (refine_loss)) on the exposure-compensated render I~ = exp(a_v) I^ + b_v:
 *   L = w_color mean|I~ - I| + w_depth mean|D^ - D|
 * (means over every channel and pixel of the n_views views; the subgradient
 * of |.| at 0 is 0).  With exposure == NULL (a = b = 0) and w_color = 0.95,
 * w_depth = 0.25 it is the L1 part of the mapping loss, Eq. (map_loss).
 * Device arrays, C-contiguous: color and target_color [V,3,H,W], depth and
 * target_depth [V,H,W], exposure [V,2] = (a, b) or NULL; outputs (overwritten)
 * d_color [V,3,H,W], d_depth [V,H,W] or NULL (no depth term: depth inputs
 * may then be NULL), d_exposure [V,2] = (dL/da, dL/db) or NULL.  Enqueues
 * two kernels on `stream` (graph-capturable); GSR_E_INVALID_ARG for null
 * required pointers or bad sizes. */
gsr_status gsr_l1_loss_grad(const float* color, const float* depth, const float* target_color,
                            const float* target_depth, const float* exposure, int32_t n_views,
                            int32_t width, int32_t height, float w_color, float w_depth,
                            float* d_color, float* d_depth, float* d_exposure, void* stream);

/* Workspace bytes gsr_ssim_grad needs for n_views x 3 x height x width
 * images (host only). */
gsr_status gsr_ssim_workspace_bytes(int32_t n_views, int32_t width, int32_t height,
                                    size_t* out_bytes);

/* SSIM term of the refinement loss (Sec. III-C, Eq. (refine_loss)),
 * L = weight (1 - mean SSIM(I~, I)) with I~ = exp(a_v) I^ + b_v (weight = 0.2
 * in the paper).  SSIM per colour channel under an 11 x 11 Gaussian window
 * (sigma 1.5, zero outside the image), C1 = 0.01^2, C2 = 0.03^2, the mean
 * taken over every pixel, channel and view.  ADDS dL/dI^ into d_color
 * [V,3,H,W] and, if d_exposure != NULL, dL/d(a, b) into d_exposure [V,2], so
 * it composes with gsr_l1_loss_grad (which overwrites them); writes the mean
 * SSIM to ssim_out (one device float) if not NULL.  color, target_color
 * [V,3,H,W] and exposure [V,2] (or NULL: a = b = 0) are device arrays;
 * workspace is a 256-byte aligned device buffer of at least
 * gsr_ssim_workspace_bytes bytes, overwritten.  Enqueues up to three kernels on
 * `stream`, allocates nothing and does not synchronise (graph-capturable).
 * GSR_E_INVALID_ARG for null pointers, a misaligned workspace or sizes out of
 * range. */
gsr_status gsr_ssim_grad(const float* color, const float* target_color, const float* exposure,
                         int32_t n_views, int32_t width, int32_t height, float weight,
                         void* workspace, float* d_color, float* d_exposure, float* ssim_out,
                         void* stream);

/* Occupancy-aware deduplication of borrowed Gaussians (Sec. III-C, Eqs.
 * (envelope), (free_carve), (dedup)).  With voxel index floor(x / voxel)
 * per axis (FP64 from the FP32 inputs): occupied voxels are every voxel
 * meeting a target Gaussian's box [mu - k_env s, mu + k_env s],
 * s = exp(log_scales); free voxels are every voxel met by the segment from a
 * keyframe's camera centre to the back-projected depth of one of its pixels
 * (pixel centres, parameters t in [0, 1); depth <= 0 carves nothing); a
 * borrowed Gaussian is kept (keep[i] = 1) only if the voxel of its mean is
 * in neither set.  The paper gives neither voxel nor k_env. */
typedef struct gsr_dedup_params {
  double voxel;          /* v > 0, in the map's length unit */
  double k_env;          /* >= 0 */
  int64_t table_slots;   /* hash-set slots, a power of two; size it at about
                            twice the distinct voxels expected */
} gsr_dedup_params;

/* Workspace bytes of a hash set of table_slots slots (host only). */
gsr_status gsr_dedup_workspace_bytes(int64_t table_slots, size_t* out_bytes);

/* Device arrays: tgt_means, tgt_log_scales [n_tgt,3]; depth [K,H,W] (camera
 * depth per pixel), viewmats [K,3,4] world->camera, intrinsics [K,4] for the
 * target's keyframes; src_means [n_src,3]; keep uint8 [n_src] (out);
 * workspace 256-byte aligned, >= gsr_dedup_workspace_bytes(table_slots),
 * overwritten.  Synchronises `stream`; n_voxels (HOST, may be NULL) gets the
 * number of distinct voxels inserted.  GSR_E_OVERFLOW (keep not valid) when
 * the hash set ran out of slots; GSR_E_INVALID_ARG for bad parameters, or
 * (found on the device; keep not valid) a voxel index outside +-2^20 per
 * axis, a non-finite input, or one box or segment of more than 2^22 voxels. */
gsr_status gsr_dedup(const gsr_dedup_params* params, const float* tgt_means,
                     const float* tgt_log_scales, int64_t n_tgt, const float* depth,
                     const float* viewmats, const float* intrinsics, int32_t n_keyframes,
                     int32_t width, int32_t height, const float* src_means, int64_t n_src,
                     uint8_t* keep, void* workspace, int64_t* n_voxels, void* stream);

/* Opacity pruning of the refinement (Sec. III-C): keeps the Gaussians with
 * sigmoid(opacity_logit) >= min_opacity (0.005 in the paper), in their
 * order, set by set.  `scene` gives the device input arrays and the HOST
 * set_offsets (n = set_offsets[n_sets] Gaussians; colors rows of 3 floats,
 * or 3*sh_stride for sh_degree > 0).  Outputs are device arrays with room
 * for n rows each, not aliasing the inputs: the kept rows of means,
 * log_scales, quats, opacity logits and colours; set_offsets_out is a HOST
 * array [n_sets+1] of the pruned set offsets (its last entry = rows kept).
 * Allocates a small temporary device buffer and synchronises `stream` (set-up
 * work, not capturable).  GSR_E_INVALID_ARG for null pointers, bad offsets or
 * min_opacity outside (0, 1). */
gsr_status gsr_prune(const gsr_scene* scene, float min_opacity, float* means_out,
                     float* log_scales_out, float* quats_out, float* opacity_out,
                     float* colors_out, int64_t* set_offsets_out, void* stream);

/* Isotropy term of the mapping loss (Sec. III-A, Eq. (map_loss)):
 * L_iso = sum_i sum_c |s_ic - mean_c s_ic| with s = exp(log_scales) (the
 * paper weights it by lambda_s = 10).  ADDS weight * dL_iso/d log_scales into
 * d_log_scales [n,3] (the subgradient of |.| at 0 is 0).  log_scales,
 * d_log_scales: device arrays.  One kernel on `stream`, no allocation or
 * synchronisation (graph-capturable).  GSR_E_INVALID_ARG for n < 0 or null
 * pointers with n > 0. */
gsr_status gsr_iso_grad(const float* log_scales, int64_t n, float weight, float* d_log_scales,
                        void* stream);

/* Depth-normal term of the mapping loss (Sec. III-A, Eq. (map_loss), weight
 * lambda_n = 1e-2 in the paper): for camera points P(i, j) = D(i, j)
 * ((i + 0.5 - cx)/fx, (j + 0.5 - cy)/fy, 1), the normal at an interior pixel
 * is N = normalize((P(i, j+1) - P(i, j-1)) x (P(i+1, j) - P(i-1, j))), which
 * faces the camera; L = sum over interior pixels with the four neighbour
 * depths > 0 and a non-zero cross product of (1 - N . prior), divided by
 * V (H-2) (W-2).  ADDS weight * dL/dD into d_depth [V,H,W].  depth [V,H,W]
 * (rendered depth), normal_prior [V,3,H,W] (channel planes, not required to
 * be unit length), intrinsics [V,4] (fx, fy, cx, cy): device arrays.  One
 * kernel on `stream`, no allocation or synchronisation (graph-capturable);
 * images narrower or lower than 3 pixels have no interior and leave d_depth
 * unchanged.  GSR_E_INVALID_ARG for null pointers or bad sizes. */
gsr_status gsr_normal_loss_grad(const float* depth, const float* normal_prior,
                                const float* intrinsics, int32_t n_views, int32_t width,
                                int32_t height, float weight, float* d_depth, void* stream);

/* Seeding of a new keyframe's Gaussians (Sec. III-A: means back-projected
 * through the keyframe's pose, mu = T^-1 pi^-1(u, d)).  One Gaussian per
 * pixel (stride*gi, stride*gj) of the stride grid with depth > 0, in
 * row-major grid order: mean = R^T (p - t) for the camera point p of the
 * pixel centre at its depth; isotropic log-scale = log of the mean distance
 * from p to the points of its up to four grid neighbours (at +-stride) with
 * depth > 0, or log(d stride / fx) without one; quaternion (1, 0, 0, 0);
 * opacity logit = opacity_logit; colour = the pixel's RGB.  depth [H,W],
 * color [3,H,W] (channel planes), viewmat [3,4] world->camera, intrinsics
 * [4]: device arrays.  Outputs (device, capacity max_out rows): means_out,
 * log_scales_out, colors_out [max_out,3], quats_out [max_out,4],
 * opacity_out [max_out].  Allocates a small temporary and synchronises
 * `stream`; *n_out (HOST) gets the number of seeded Gaussians.
 * GSR_E_OVERFLOW when that exceeds max_out (the first max_out rows are
 * written); GSR_E_INVALID_ARG for null pointers or bad sizes. */
gsr_status gsr_seed(const float* depth, const float* color, const float* viewmat,
                    const float* intrinsics, int32_t width, int32_t height, int32_t stride,
                    float opacity_logit, int64_t max_out, float* means_out,
                    float* log_scales_out, float* quats_out, float* opacity_out,
                    float* colors_out, int64_t* n_out, void* stream);

/* One Adam step (Kingma & Ba 2015) over up to GSR_ADAM_MAX_GROUPS arrays
 * in one launch: the optimiser of the mapping loss (Sec. III-A, Eq.
 * (map_loss)) and of the refinement (Sec. III-C, Eq. (refine_loss)), which
 * the paper minimises by gradient steps with per-parameter learning rates.
 * With t = *step + 1 and per element
 *   m <- beta1 m + (1 - beta1) g,   v <- beta2 v + (1 - beta2) g^2,
 *   p <- p - lr (m / (1 - beta1^t)) / (sqrt(v / (1 - beta2^t)) + eps),
 * then *step <- t.  All arrays are device FP32 of length n (param, exp_avg
 * and exp_avg_sq updated in place; exp_avg and exp_avg_sq start at zero and
 * *step at 0); `step` is a device int32.  The betas are FP64 so that
 * 1 - beta and the bias corrections 1 - beta^t (which cancel) keep their
 * digits; the moment updates run in FP32.  Enqueues two kernels on `stream`
 * (no allocation, no synchronisation: graph-capturable).  GSR_E_INVALID_ARG
 * for null pointers, n < 0, betas outside [0, 1), eps < 0, n_groups outside
 * 1..GSR_ADAM_MAX_GROUPS or more than 2^31 - 8 chunks of 1024 elements. */
#define GSR_ADAM_MAX_GROUPS 8
typedef struct gsr_adam_group {
  float* param;
  const float* grad;
  float* exp_avg;
  float* exp_avg_sq;
  int64_t n;
  float lr;
  int32_t reserved;
} gsr_adam_group;
gsr_status gsr_adam(const gsr_adam_group* groups, int32_t n_groups, double beta1, double beta2,
                    double eps, int32_t* step, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): gsr_seed
 * with its per-block counts in a buffer the library holds (a file-scope
 * device array, one per GPU, kept until the process ends) instead of a
 * temporary allocation.  Same inputs, outputs and kernels as gsr_seed,
 * except that the number of seeded Gaussians goes to *n_out_dev, a DEVICE
 * int64 written on `stream` (no host synchronisation; the caller compares
 * it with max_out: only the first max_out rows are written).  At most
 * GSR_SEED_NOALLOC_MAX_POINTS grid points per call (GSR_E_CAPACITY above).
 * Calls no allocating routine.  Every call on a GPU shares that GPU's
 * buffer: calls that overlap on one GPU (other streams or host threads)
 * race and must be serialised by the caller.  GSR_E_INVALID_ARG for null
 * pointers or bad sizes; GSR_E_DEVICE for a HIP error (including a current
 * device beyond the library's device table). */
gsr_status gsr_seed_noalloc(const float* depth, const float* color, const float* viewmat,
                            const float* intrinsics, int32_t width, int32_t height,
                            int32_t stride, float opacity_logit, int64_t max_out,
                            float* means_out, float* log_scales_out, float* quats_out,
                            float* opacity_out, float* colors_out, int64_t* n_out_dev,
                            void* stream);

/* Time forward+backward of the given call for each candidate plan and
 * report the fastest in `best`, by coordinate search: every tile shape with
 * one and, where allowed, two tiles per backward wave (binning chunk
 * automatic, one entry per lane in the forward and in the backward, grid
 * launch), then for the fastest plan so far each
 * binning chunk of 64, 128 and 256 pairs, the forward's 1 or 2 entries per
 * lane, the backward's 1, 2 or 4 entries per lane, and the grid or
 * persistent tile queue.  `best` holds tile_w, tile_h, chunk, fwd_batch,
 * bwd_batch, persistent and bwd_cols; other fields are copied from `base` (the
 * entry capacity raised if a candidate overflowed).  Synchronises;
 * allocates its own temporary contexts and buffers. */
gsr_status gsr_autotune(int device, const gsr_plan_desc* base, const gsr_scene* scene,
                        const gsr_views* views, const gsr_settings* settings,
                        gsr_plan_desc* best, float* best_ms, void* stream);

/* Stage timing.  When enabled, gsr_forward and gsr_backward record a pair
 * of HIP events around each stage on the call's stream (not while the
 * stream is being captured into a graph); gsr_profile_read synchronises on
 * them and writes the elapsed milliseconds of each stage of the most recent
 * calls into ms[0..n) (0 for stages not run), indexed by gsr_stage. */
typedef enum gsr_stage {
  GSR_STAGE_PROJECT = 0,     /* key path of every (view, Gaussian) pair */
  GSR_STAGE_COMPACT = 1,     /* ordered compaction of visible pairs */
  GSR_STAGE_DEPTH_SORT = 2,  /* depth digits of the (tile, depth) key sort */
  GSR_STAGE_BINNING = 3,     /* tile digit: counts, scans, scatter */
  GSR_STAGE_RENDER_FWD = 4,  /* per-tile compositing */
  GSR_STAGE_ZERO = 5,        /* clearing of the backward accumulators */
  GSR_STAGE_RENDER_BWD = 6,  /* reverse compositing, splat gradients */
  GSR_STAGE_PROJECT_BWD = 7, /* chain rule to parameters and poses */
  GSR_STAGE_RECORD = 8,      /* screen-space records of the visible pairs */
  GSR_NUM_STAGES = 9
} gsr_stage;
gsr_status gsr_profile_enable(gsr_ctx* ctx, int enable);
gsr_status gsr_profile_read(gsr_ctx* ctx, float* ms, int32_t n);

const char* gsr_status_string(gsr_status s);
const char* gsr_last_error(const gsr_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* GSR_H */
