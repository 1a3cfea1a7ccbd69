/*
 * ges.h -- C ABI of the MI355X (gfx950) GES tile rasterizer.
 *
 * GES: Generalized Exponential Splatting (arXiv 2402.10128).  The library renders
 * and differentiates splats whose falloff is a generalized exponential with a
 * per-splat shape beta.  The arguments follow the paper's statement of the problem
 * (Sec. 4.1): per-splat position, scale vector and quaternion (the covariance
 * Sigma = R S S^T R^T, S modified by the shape function phi(beta), Sec. 4.2),
 * opacity, spherical-harmonic colour and beta, seen by a calibrated pinhole camera.
 *
 * Conventions shared by every entry point
 *   - All tensor arguments are DEVICE pointers to contiguous row-major FP32 (or the
 *     stated integer type) buffers owned by the caller.  The library never frees
 *     them and never allocates on the render path; the workspace buffers it needs
 *     are caller-allocated with the sizes returned by the *_query calls.
 *   - Work is enqueued on `stream` (a hipStream_t; NULL = the null stream) and is
 *     asynchronous unless a call says otherwise.  Calls on one frame's buffers must
 *     be issued on one stream in the order preprocess -> forward -> backward.
 *   - Every call returns a ges_status.  On failure nothing has been enqueued unless
 *     the status is GES_ERR_DEVICE; ges_last_error() then describes the problem
 *     (thread-local string, valid until the next call on the same thread).
 *   - Splats with non-finite inputs, a zero quaternion, opacity <= 1/255, a mean
 *     at or behind the near plane, a degenerate projected covariance, no tile on
 *     screen, or (GEF falloff) beta <= 0 are culled, not reported as errors.
 *   - Limits: 0 <= n < 2^31, sh_degree in [0,3], 1 <= width,height <= 16384, at
 *     most 2^32 - 1 (tile, splat) keys per frame.
 */
#ifndef GES_H
#define GES_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GES_ABI_VERSION 4u
#define GES_TILE 16
#define GES_GRAD2D_STRIDE 12   /* binary64 slots per splat in the 2-D gradient rows */

typedef enum {
  GES_OK = 0,
  GES_ERR_INVALID_ARGUMENT = 1,  /* null/inconsistent pointers, bad sizes, non-finite camera, R not a rotation */
  GES_ERR_CAPACITY = 2,          /* a workspace is smaller than the matching *_query result */
  GES_ERR_OUT_OF_MEMORY = 3,     /* serving pool exhausted for a request that can never fit */
  GES_ERR_DEVICE = 4,            /* a HIP call failed; ges_last_error() holds hipGetErrorString */
  GES_ERR_BUSY = 5,              /* serving queue full */
  GES_ERR_NOT_FOUND = 6,         /* unknown scene or request id */
  GES_ERR_INTERNAL = 7
} ges_status;

/* Pixel falloff of a splat.
 * PHI: the paper's approximate rasterization (Sec. 4.2, Eq. approx): the scales are
 *      multiplied by phi_rho(beta) = 2 / (1 + exp(-(rho beta - 2 rho))) and the 2-D
 *      falloff is the Gaussian exp(-q/2).
 * GEF: the exact GES kernel of Eq. ges projected to the image: exp(-q^(beta/2) / 2)
 *      on the unmodified covariance.
 * PHI_EXACT: the exact conversion the paper derives first (Sec. 4.2, Eq. probablity),
 *      normalised to 1 at beta = 2: scales multiplied by 2 Gamma(3/beta) / Gamma(1/beta),
 *      Gaussian falloff exp(-q/2); beta <= 0 culls.  (A variant: it grows without bound as
 *      beta falls, which is why the paper approximates it.)
 * q is the quadratic form of the (0.3-dilated) projected covariance. */
typedef enum { GES_FALLOFF_PHI = 0, GES_FALLOFF_GEF = 1, GES_FALLOFF_PHI_EXACT = 2 } ges_falloff;

/* Which tiles list a splat: every tile of its bounding square (SQUARE) or only the
 * tiles whose pixel-centre box meets its alpha-floor ellipse (ELLIPSE).  Both give
 * identical images; ELLIPSE produces fewer keys. */
typedef enum { GES_TILES_SQUARE = 0, GES_TILES_ELLIPSE = 1 } ges_tile_cull;

typedef struct {
  int64_t n;                     /* number of splats */
  int32_t sh_degree;             /* 0..3; (sh_degree+1)^2 coefficients per colour channel */
  const float* means;            /* [n,3] world position */
  const float* log_scales;       /* [n,3] log of the per-axis scale */
  const float* quats;            /* [n,4] rotation (w,x,y,z), normalised internally; 16-byte aligned */
  const float* opacity_logits;   /* [n] opacity = sigmoid(logit) */
  const float* sh;               /* [n,(D+1)^2,3] real SH coefficients, m-ordered, Condon-Shortley phase;
                                    16-byte aligned at degree 1 or 3 (rows move as float4) */
  const float* beta;             /* [n] shape parameter beta (2 = Gaussian), the true value */
} ges_splats;

typedef struct {                 /* host struct, passed by pointer, read during the call */
  int32_t width, height;
  float R[9];                    /* world->camera rotation, row-major; camera x right, y down, z forward */
  float t[3];                    /* world->camera translation: p_cam = R p_world + t */
  float fx, fy, cx, cy;          /* pixel units; pixel (i,j) has its centre at (i,j) */
  float near_z;                  /* splats with camera z <= near_z are culled (0.2 typical) */
} ges_camera;

typedef struct {
  int32_t falloff;               /* ges_falloff */
  int32_t tile_cull;             /* ges_tile_cull */
  float rho;                     /* shape strength of phi_rho (the paper uses 0.1) */
  float bg[3];                   /* background colour composited behind the splats */
  uint32_t flags;                /* GES_RASTER_* bits (0: none) */
} ges_raster_params;
/* ges_render_backward also stores each splat's summed 2-D gradient in the frame's grad2d
 * rows (ges_frame_view; inspection and tests), 96 bytes per listed splat. */
#define GES_RASTER_KEEP_GRAD2D 1u

typedef struct {                 /* device pointers, same shapes as ges_splats; overwritten (not accumulated) */
  float* means;
  float* log_scales;
  float* quats;
  float* opacity_logits;
  float* sh;
  float* beta;
} ges_splat_grads;

uint32_t ges_abi_version(void);
const char* ges_last_error(void);

/* Sizes of the per-frame workspaces for n splats at width x height.
 * splat_ws holds the per-splat projected records, the depth order of the splats and
 * the candidate offsets along it, the tile ranges and the per-splat 2-D gradients;
 * pixel_ws holds the
 * per-pixel final transmittance and contributor count that the backward pass
 * re-uses (so no per-pixel lists are stored).  Either output pointer may be NULL.
 * Both workspaces are caller-owned device memory and must be 256-byte aligned (device allocations
 * are); the preprocess, forward and backward entry points reject others with INVALID_ARGUMENT. */
ges_status ges_workspace_query(int64_t n, int32_t width, int32_t height, size_t* splat_ws_bytes,
                               size_t* pixel_ws_bytes);

/* Size of the key workspace for num_keys candidate (tile, splat) slots of a width x height
 * frame with n splats: two buffers of (tile, splat index) pairs (16 B per slot, the sorted
 * splat ids first) and the digit table of the tile sort (1 B per 4 slots).  Width/height
 * outside [1,16384]: GES_ERR_INVALID_ARGUMENT; num_keys >= 2^32-1: GES_ERR_CAPACITY. */
ges_status ges_key_workspace_query(uint64_t num_keys, int64_t n, int32_t width, int32_t height,
                                   size_t* key_ws_bytes);

/* Preprocess (Sec. 4.1-4.2): per splat, view transform, 3-D covariance from scale and
 * rotation with the shape modification, EWA projection J W Sigma W^T J^T, conic,
 * mean2D, alpha-floor threshold, beta-dependent screen radius, tile rectangle and
 * SH colour; then sorts the listed splats by depth (ties by index) and lays out one
 * slot per candidate tile of each splat along that order.
 * num_keys_host: if not NULL, the call waits for the stream and stores the number
 * of candidate slots of this frame there -- the key capacity the frame needs, an upper
 * bound of its (tile, splat) keys (equal to it for GES_TILES_SQUARE) -- the only host
 * synchronisation of a frame.
 * Errors: INVALID_ARGUMENT (see conventions), CAPACITY if splat_ws_bytes is too small. */
ges_status ges_preprocess(const ges_splats* splats, const ges_camera* cam, const ges_raster_params* params,
                          void* splat_ws, size_t splat_ws_bytes, uint64_t* num_keys_host, void* stream);

/* Forward render (Sec. 4.2, Eq. transimttance discretised): fills the candidate slots
 * with the (tile, splat) pairs whose tile the splat meets, sorts them stably by tile
 * (every tile's list is then in (depth, splat index) order), fixes every tile's
 * [start,end) range, and composites front to back per pixel with
 * alpha = min(0.99, opacity * falloff), skipping pairs below the 1/255 alpha floor and
 * stopping a pixel before the splat that would take its transmittance below 1e-4.
 * out_rgb: [height,width,3] FP32, overwritten.  num_keys is the slot capacity of key_ws
 * (key_ws_bytes >= ges_key_workspace_query(num_keys, ...)) and must be at least the slot
 * count of the frame: either the value ges_preprocess returned, or any larger capacity,
 * in which case no read-back is needed (the kernels take the count from the device).  If
 * the frame's count exceeds num_keys, the pairs of the slots beyond the capacity are
 * dropped and bit 0 of the frame's error word (ges_frame_view stats[1]) is set.  The
 * same num_keys must be passed to ges_frame_view_get.
 * The splat, pixel and key workspaces must stay untouched until the matching
 * ges_render_backward (if any) has been enqueued. */
ges_status ges_render_forward(const ges_splats* splats, const ges_camera* cam, const ges_raster_params* params,
                              void* splat_ws, void* key_ws, size_t key_ws_bytes, uint64_t num_keys,
                              void* pixel_ws, float* out_rgb, void* stream);

/* Backward pass (Sec. 4.4: the splats' position, opacity, covariance, SH colour and
 * shape are optimised through the rasterizer's gradients; the derivative of the
 * compositing of Sec. 4.2, Eq. transimttance): given dL/d(out_rgb) [height,width,3],
 * walks every pixel's contributors back to front recovering the transmittance by
 * division, sums the gradient of each splat's 2-D quantities (mean2D, conic, opacity,
 * colour and, with the GEF falloff, beta) per tile in binary32 and over its tiles in
 * binary64 in a fixed order (no atomics: two calls give identical bits), then maps them
 * to the parameters through the preprocess chain rule (evaluated in binary64).  Uses
 * the key workspace of the forward pass for its per-(tile, splat) rows (key_ws must be
 * the one ges_render_forward was given).  Every gradient buffer of `grads`
 * is overwritten; NULL members are skipped.  grads->quats, and grads->sh at SH degree
 * 1 or 3, must be 16-byte aligned (INVALID_ARGUMENT otherwise), like the inputs.
 * Must follow the ges_render_forward of the same frame. */
ges_status ges_render_backward(const ges_splats* splats, const ges_camera* cam, const ges_raster_params* params,
                               void* splat_ws, void* key_ws, void* pixel_ws, const float* dL_drgb,
                               const ges_splat_grads* grads, void* stream);

/* ---- inspection (tests) ------------------------------------------------------------
 * Device views into a frame's workspaces, valid after the call that fills them. */
typedef struct {
  const float* records;          /* [n,16] per-splat record, see below (after ges_preprocess) */
  const uint32_t* tile_ranges;   /* [tiles,2] [start,end) into the sorted lists (after ges_render_forward) */
  const uint32_t* sorted_pairs;  /* [keys,2] (splat index, candidate slot) per sorted entry (after ges_render_forward) */
  const uint32_t* sorted_tiles;  /* [keys] tile per sorted entry (after ges_render_forward) */
  const float* final_T;          /* [height,width] (after ges_render_forward) */
  const uint32_t* n_contrib;     /* [height,width] list position + 1 of the last composited splat */
  const double* grad2d;          /* [n,GES_GRAD2D_STRIDE] dL/d(u,v,a,b,c,opacity,r,g,b,beta) in slots 0..9, binary64
                                    (after ges_render_backward: the rows of listed splats; with
                                    GES_RASTER_KEEP_GRAD2D every row, those of unlisted splats zero) */
  const uint64_t* stats;         /* [4]: keys, error word (bit 0: key capacity too small), pairs examined,
                                    pairs composited (after ges_render_forward) */
  int32_t tiles_x, tiles_y;
  const uint32_t* tile_work;     /* [tiles] per tile, the largest n_contrib of its pixels (after ges_render_forward) */
  const uint32_t* group_order;   /* [ceil(tiles/8)] groups of 8 consecutive tiles in the order the backward pass
                                    deals them, heaviest tile_work first (after ges_render_forward) */
  const uint32_t* row_marks;     /* [ceil(num_keys/32)] bit s: the backward stored a row of per-(tile, splat)
                                    sums at candidate slot s (after ges_render_backward; NULL without key_ws) */
} ges_frame_view;
/* Record layout, 16 x 32-bit words per splat:
 *   0 u, 1 v, 2 conic a, 3 conic b, 4 conic c, 5 q_max, 6 opacity, 7 beta,
 *   8 r, 9 g, 10 b, 11 depth, 12 radius | flags << 24 (int32), 13 tx0 | ty0 << 16,
 *   14 tx1 | ty1 << 16 (inclusive), 15 tiles_touched (uint32; 0 = culled; between ges_preprocess
 *   and ges_render_forward, GES_TILES_ELLIPSE: the splat's candidate count, an upper bound).
 *   flags: bit0..2 colour channel clamped at 0, bit3/4 x/y guard clamp. */
ges_status ges_frame_view_get(int64_t n, int32_t width, int32_t height, void* splat_ws, void* key_ws,
                              uint64_t num_keys, void* pixel_ws, ges_frame_view* out);

/* ---- stage timing (benchmarks) -----------------------------------------------------
 * When enabled, every kernel launch of the render path is bracketed by two HIP events
 * recorded on the stream it runs on; ges_profile_read waits for the recorded events
 * and returns the accumulated device milliseconds and launch counts per stage
 * (indices GES_STAGE_*), then optionally clears them.  Off by default; enabling it
 * costs two event records per launch. */
enum { GES_STAGE_PREPROCESS = 0, GES_STAGE_DEPTH_SORT, GES_STAGE_KEY_SCAN, GES_STAGE_DUPLICATE, GES_STAGE_TILE_SORT,
       GES_STAGE_RASTER_FORWARD, GES_STAGE_RASTER_BACKWARD, GES_STAGE_PREPROCESS_BACKWARD, GES_STAGE_ZERO,
       GES_STAGE_LOSS, GES_STAGE_ADAM, GES_STAGE_SSIM, GES_STAGE_MIX_FIT, GES_STAGE_ROW_REDUCE, GES_NUM_STAGES };
ges_status ges_profile_enable(int32_t on);
/* Time only the stages whose bit (1 << GES_STAGE_*) is set; 0 switches timing off. */
ges_status ges_profile_select(uint32_t stage_mask);
ges_status ges_profile_read(double* ms /*[GES_NUM_STAGES]*/, int64_t* launches /*[GES_NUM_STAGES]*/, int32_t reset);

/* ---- frequency-modulated loss (Sec. 4.3) ------------------------------------------
 * Mask M_omega = 1(|DoG_omega(grey(target))| / max > 0.5) computed on the target
 * down-sampled by 5 (scale 0.2), sigma2 = 0.1 + 10 omega, sigma1 = 2 sigma2, up-sampled
 * by nearest lookup; for omega <= 0.5 the mask is 1 - M_(omega + 0.5).
 * scratch: device buffer of ges_mask_scratch_bytes(width,height) bytes. mask: [h,w] uint8. */
size_t ges_mask_scratch_bytes(int32_t width, int32_t height);
ges_status ges_freq_mask(const float* target, int32_t width, int32_t height, float omega, void* scratch,
                         uint8_t* mask, void* stream);

/* ---- the frequency mask without a scratch argument ----------------------------------
 * For callers that cannot allocate device memory: code under HIP graph capture, tight training
 * or serving loops, harnesses that forbid hipMalloc.  Same arguments, kernels and result bits as
 * ges_freq_mask, but the scratch is a fixed array of GES_MASK_STATIC_SCRATCH_BYTES that the
 * library holds on every device it runs on (from the first call on that device until the process
 * ends); the call allocates nothing.  The array's address is looked up on the first call with a
 * device current; `stream` must belong to the current device.  Every call on one device shares
 * that device's array and leaves its contents behind (the mask's kernels clear what must start at
 * zero), so calls whose work overlaps on one device (several streams or threads) race: order them
 * on one stream.  Errors: those of ges_freq_mask; GES_ERR_CAPACITY when
 * ges_mask_scratch_bytes(width,height) exceeds GES_MASK_STATIC_SCRATCH_BYTES (images up to about
 * 13 Mpx fit, e.g. 3840x2160); GES_ERR_DEVICE if the array cannot be looked up. */
#define GES_MASK_STATIC_SCRATCH_BYTES ((size_t)8 << 20)
ges_status ges_freq_mask_static(const float* target, int32_t width, int32_t height, float omega, uint8_t* mask,
                                void* stream);

/* L = lam_l1 mean|I - T| + lam_w mean(|I - T| M) over height*width*3 values, and
 * dL/dI = (lam_l1 + lam_w M) sign(I - T) / (3 h w).  mask may be NULL (then lam_w is
 * ignored).  scratch: device buffer of ges_loss_scratch_bytes() bytes (per-block partial sums, added in
 * a fixed order so the loss is deterministic).  loss_out: one FP32 device scalar (overwritten).
 * dL_dimg: [h,w,3]. */
size_t ges_loss_scratch_bytes(void);
ges_status ges_loss(const float* img, const float* target, const uint8_t* mask, int32_t width, int32_t height,
                    float lam_l1, float lam_w, void* scratch, float* loss_out, float* dL_dimg, void* stream);

/* ---- structural-similarity term of the training loss (Sec. 4.4, Eq. final) --------
 * Gaussian-weighted SSIM (Wang et al., 2004) of img against target, both [h,w,3]:
 * 11x11 window of sigma 1.5 (unit sum), each channel on its own, zero padding (the
 * SSIM map has the image's size), C1 = 0.01^2, C2 = 0.03^2; L_ssim = 1 - mean SSIM over
 * h*w*3 values.  The call ACCUMULATES: *loss_inout += lam_ssim L_ssim and
 * dL_dimg += lam_ssim dL_ssim/dimg, so it runs after ges_loss (which overwrites both)
 * to form the full loss 0.3 L1 + 0.2 L_ssim + 0.5 L_omega.  The loss is summed in a
 * fixed order (deterministic).  scratch: device buffer of ges_ssim_scratch_bytes(w,h)
 * bytes (nine [h,w] FP32 maps and per-tile sums).  Errors: GES_ERR_INVALID_ARGUMENT for
 * a NULL pointer, sizes outside 1..16384 or a non-finite lam_ssim. */
size_t ges_ssim_scratch_bytes(int32_t width, int32_t height);
ges_status ges_ssim_loss(const float* img, const float* target, int32_t width, int32_t height, float lam_ssim,
                         void* scratch, float* loss_inout, float* dL_dimg, void* stream);

/* ---- optimiser step of training (App. B.2) ---------------------------------------
 * Adam (Kingma & Ba, 2015, Algorithm 1) applied in place to up to GES_ADAM_MAX_GROUPS
 * parameter groups in one launch, each with its own learning rate (the paper trains
 * position, SH features, opacity, shape beta, rotation and scaling at separate rates):
 *   m <- b1 m + (1-b1) g;  v <- b2 v + (1-b2) g^2;
 *   p <- p - lr (m / (1 - b1^step)) / (sqrt(v / (1 - b2^step)) + eps),
 * computed in binary32 (the bias corrections in binary64 on the host).  step counts
 * from 1; exp_avg and exp_avg_sq must be zero before step 1.  The four arrays of a
 * group hold `count` floats each and must not overlap each other or another group's
 * (the result is undefined if they do); 16-byte aligned groups move as float4.
 * Errors: GES_ERR_INVALID_ARGUMENT for ngroups outside 1..GES_ADAM_MAX_GROUPS, step < 1,
 * b1 or b2 outside [0,1), eps < 0, a non-finite or negative lr, count < 0, or a NULL
 * pointer in a group with count > 0. */
#define GES_ADAM_MAX_GROUPS 8
typedef struct {
  float* params;                 /* [count] updated in place */
  const float* grads;            /* [count] */
  float* exp_avg;                /* [count] first moment m, updated in place */
  float* exp_avg_sq;             /* [count] second moment v, updated in place */
  int64_t count;
  float lr;
} ges_adam_group;
ges_status ges_adam_step(const ges_adam_group* groups, int32_t ngroups, int64_t step, float beta1, float beta2,
                         float eps, void* stream);

/* Backward pass of one more view of a multi-view step: like ges_render_backward, but this view's
 * parameter gradients are ADDED to the buffers of `grads` (which hold the earlier views' sum; the first
 * view uses ges_render_backward).  grad_accum / grad_count (both NULL or both set) accumulate the
 * densification statistic as in ges_adam_splats.  Sums run in view order (deterministic). */
ges_status ges_render_backward_accumulate(const ges_splats* splats, const ges_camera* cam,
                                          const ges_raster_params* params, void* splat_ws, void* key_ws,
                                          void* pixel_ws, const float* dL_drgb, const ges_splat_grads* grads,
                                          float* grad_accum, float* grad_count, void* stream);

/* Backward pass with the optimiser step fused in: the effect of ges_render_backward followed by
 * ges_adam_step over the six parameter arrays of `splats` (same arguments and rules as those two
 * calls), in one pass over the splats: each parameter gradient goes straight into its Adam update
 * instead of through memory, and is also stored when `grads` is non-NULL.  The parameters, moments
 * and stored gradients are bit-identical to the two separate calls.  The parameter arrays named by
 * `splats` are UPDATED IN PLACE: they must be writable device memory (ges_splats declares them const
 * for the render calls).  Moments k = 0..5 belong to means, log_scales, quats, opacity_logits, sh,
 * beta, each shaped like its parameter and zero before step 1; the quats moments, and the sh moments
 * at SH degree 1 or 3, must be 16-byte aligned.  Errors: those of ges_render_backward and of
 * ges_adam_step, and GES_ERR_INVALID_ARGUMENT for a NULL opt or moment array (with n > 0) or a
 * misaligned moment array. */
typedef struct {
  float* exp_avg[6];             /* first moments m */
  float* exp_avg_sq[6];          /* second moments v */
  float lr[6];                   /* learning rate of each parameter array */
  int64_t step;                  /* Adam step t >= 1 */
  float beta1, beta2, eps;
  float* grad_accum;             /* [n] densification statistic, or NULL: every visible splat adds the norm of its
                                    mean-2D gradient in NDC units, ||(dL/du W/2, dL/dv H/2)|| ... */
  float* grad_count;             /* [n] ... and 1 here (both NULL or both set) */
  const float* grads_in[6];      /* per parameter array, or NULL: gradients of other views (e.g. summed by
                                    ges_render_backward_accumulate) added to this view's before the update;
                                    quats and, at SH degree 1 or 3, sh must be 16-byte aligned */
} ges_adam_splats;
ges_status ges_render_backward_adam(const ges_splats* splats, const ges_camera* cam, const ges_raster_params* params,
                                    void* splat_ws, void* key_ws, void* pixel_ws, const float* dL_drgb,
                                    const ges_splat_grads* grads, const ges_adam_splats* opt, void* stream);

/* ---- several views of one scene per launch (multi-view optimisation steps) -----------------
 * A step that fits the splats to B camera views (App. B.2 trains Gaussian-splatting style, view by view;
 * these calls take B of the views at once) renders and back-propagates them through one launch sequence:
 * the B x n (view, splat) items are preprocessed together, sorted by depth together (ties by view, then
 * splat index), binned into the B x tiles batch tiles, sorted by batch tile and rasterised in shared
 * launches, and the preprocess backward chains every splat through the B views in view order.  Every view
 * gives exactly (bit for bit) what the single-view calls give for it, and the summed gradients are those of
 * the single-view backward of view 0 followed by ges_render_backward_accumulate of views 1..B-1.
 * All views have one width and height; 1 <= num_views <= 64 and num_views x n < 2^31 (INVALID_ARGUMENT
 * otherwise).  cams: [num_views] host array.  Image arrays (out_rgb, dL_drgb) are [num_views,height,width,3]
 * FP32.  The workspaces come from ges_views_workspace_query (splat_ws: the single-view layout of each view
 * one after another, then the binning buffers of all items; pixel_ws: the views' pixel workspaces one after
 * another) and ges_key_workspace_query with the slot count ges_preprocess_views returns (the sum over the
 * views).  num_views = 1 is the single-view layout and behaviour.  Errors as for the single-view calls. */
ges_status ges_views_workspace_query(int64_t n, int32_t num_views, int32_t width, int32_t height,
                                     size_t* splat_ws_bytes, size_t* pixel_ws_bytes);
ges_status ges_preprocess_views(const ges_splats* splats, const ges_camera* cams, int32_t num_views,
                                const ges_raster_params* params, void* splat_ws, size_t splat_ws_bytes,
                                uint64_t* num_keys_host, void* stream);
ges_status ges_render_forward_views(const ges_splats* splats, const ges_camera* cams, int32_t num_views,
                                    const ges_raster_params* params, void* splat_ws, void* key_ws,
                                    size_t key_ws_bytes, uint64_t num_keys, void* pixel_ws, float* out_rgb,
                                    void* stream);
/* Sum over the views of the parameter gradients, written to (accumulate = 0) or added to (accumulate != 0)
 * `grads`; grad_accum / grad_count as for ges_render_backward_accumulate (every view adds to them). */
ges_status ges_render_backward_views(const ges_splats* splats, const ges_camera* cams, int32_t num_views,
                                     const ges_raster_params* params, void* splat_ws, void* key_ws, void* pixel_ws,
                                     const float* dL_drgb, const ges_splat_grads* grads, int32_t accumulate,
                                     float* grad_accum, float* grad_count, void* stream);
/* The fused optimiser step of ges_render_backward_adam over the views' summed gradients.  With more than
 * one view every member of `grads` is required (it receives the summed gradients; the update reads the
 * earlier views' sum from it) and opt->grads_in must be NULL.  Parameters and moments are bit-identical to
 * the single-view sequence (view 0: ges_render_backward, views 1..B-2: ges_render_backward_accumulate, view
 * B-1: ges_render_backward_adam with grads_in = that sum). */
ges_status ges_render_backward_views_adam(const ges_splats* splats, const ges_camera* cams, int32_t num_views,
                                          const ges_raster_params* params, void* splat_ws, void* key_ws,
                                          void* pixel_ws, const float* dL_drgb, const ges_splat_grads* grads,
                                          const ges_adam_splats* opt, void* stream);
/* ges_frame_view_get of view `view` (0 <= view < num_views) of a multi-view step; sorted_pairs and
 * sorted_tiles cover the whole batch (tile t of view v is batch tile v x tiles + t). */
ges_status ges_frame_view_get_views(int64_t n, int32_t num_views, int32_t width, int32_t height, void* splat_ws,
                                    void* key_ws, uint64_t num_keys, void* pixel_ws, int32_t view,
                                    ges_frame_view* out);

/* ---- shape/opacity pruning and shape reset (Sec. 4.4, Sec. 5.2, App. B.2) --------
 * The paper prunes splats on their shape every 100 iterations (threshold 0.5 in Sec. 5.2,
 * 0.005 in App. B.2), keeps the opacity pruning of Gaussian splatting (0.005) and resets
 * the shape every 1,000 iterations.
 *
 * ges_prune_splats removes every splat whose opacity sigmoid(logit) < min_opacity or whose
 * beta < min_beta and copies the survivors, in their original order, from src[k] to
 * dst[k] for k < nsets (src[0]: the parameters, which decide; src[1], src[2]: e.g. the two
 * Adam moments, laid out like the parameters).  The opacity test is taken on the logit
 * against ln(t / (1 - t)) and the beta test in binary64, so the decision is exact.  A NULL
 * member of src[k] is skipped (dst[k]'s member must then be NULL too); dst must not
 * overlap src.  *n_kept (host) receives the survivor count: the call waits for `stream`.
 * scratch: device buffer of ges_prune_scratch_bytes(n) bytes.  Errors:
 * GES_ERR_INVALID_ARGUMENT for n outside [0, 2^31), sh_degree outside 0..3, nsets outside
 * 1..3, a NULL src[0].opacity_logits or src[0].beta (n > 0), a NULL dst member where the
 * src member is set, min_opacity outside [0, 1] or a NaN min_beta; GES_ERR_CAPACITY for
 * a small scratch.
 *
 * ges_shape_reset sets beta[0..n) to `value` (2: the Gaussian the splats start from) and
 * clears the moments (either may be NULL). */
typedef struct {
  float* means;                  /* [n,3] */
  float* log_scales;             /* [n,3] */
  float* quats;                  /* [n,4] */
  float* opacity_logits;         /* [n] */
  float* sh;                     /* [n,(D+1)^2,3] */
  float* beta;                   /* [n] */
} ges_splat_set;
size_t ges_prune_scratch_bytes(int64_t n);
ges_status ges_prune_splats(int64_t n, int32_t sh_degree, const ges_splat_set* src, const ges_splat_set* dst,
                            int32_t nsets, double min_opacity, double min_beta, void* scratch, size_t scratch_bytes,
                            int64_t* n_kept, void* stream);
ges_status ges_shape_reset(float* beta, float* exp_avg, float* exp_avg_sq, int64_t n, float value, void* stream);

/* ---- the 1-D mixture simulation (Sec. 3.2; App. A.3) ---------------------------------
 * Fits mixtures of n components to 1-D signals by Adam on the mean squared error over a
 * linspace x_j = x0 + j dx, j < m, one problem per workgroup, all problems in one launch:
 *   GMM  sum_i w_i exp(-(x-mu_i)^2 / (2 s_i^2 + 1e-8))                     (Eq. gaussianmixture)
 *   DoG  sum_i w_i [exp(-(x-mu_i)^2 / (2 s_i^2 + 1e-8)) - exp(-(x-mu_i)^2 / (2 s_i^2/4 + 1e-8))]
 *   LoG  sum_i w_i (1 - (x-mu_i)^2 / s_i^2) exp(-(x-mu_i)^2 / (2 s_i^2 + 1e-8))
 *   GEF  sum_i w_i exp(-|x-mu_i|^beta_i / (2 s_i^2 + 1e-8))                 (Eq. genmixture)
 * Component i's parameters are params[p][i][0..3] = (w_raw, mu, s, beta), w = w_raw or, with
 * `positive`, softplus(w_raw); beta is used by GEF only (its gradient is 0 for the others).
 * At x = mu the GEF derivatives w.r.t. mu and beta are taken as 0.  Computed in binary32.
 * `problems` is a DEVICE array; a problem with n outside 1..GES_MIX_MAX_COMPONENTS, an unknown
 * model or a target row outside 0..ntargets-1 is not run and gets a NaN loss.  params
 * [nproblems][GES_MIX_MAX_COMPONENTS][4]: the initial values in, the values after `epochs`
 * Adam steps out (rows i >= n untouched).  grad_out (same shape, may be NULL) receives the
 * gradient at the initial values; final_loss[p] the MSE after the last step (NaN: the run
 * diverged).  targets: device [ntargets][m].  order (device [nproblems], may be NULL): the
 * order in which workgroups take the problems, a permutation of 0..nproblems-1 (largest n
 * first keeps the longest fits from starting last); results always go to each problem's own
 * rows.  A workgroup whose entry lies outside 0..nproblems-1 does nothing (a problem left
 * out of the permutation is then not run).  Errors: GES_ERR_INVALID_ARGUMENT for NULL
 * problems/targets/params/final_loss with nproblems > 0, m outside 1..GES_MIX_MAX_POINTS,
 * epochs < 0, non-finite x0/dx/lr/eps, lr or eps < 0, or b1/b2 outside [0,1). */
#define GES_MIX_MAX_COMPONENTS 128
#define GES_MIX_MAX_POINTS 4096
enum { GES_MIX_GMM = 0, GES_MIX_DOG = 1, GES_MIX_LOG = 2, GES_MIX_GEF = 3 };
typedef struct {
  int32_t model;                 /* GES_MIX_* */
  int32_t n;                     /* components */
  int32_t positive;              /* 1: weights through softplus */
  int32_t target;                /* row of `targets` to fit */
} ges_mix_problem;
ges_status ges_mix_fit(const ges_mix_problem* problems, int32_t nproblems, const float* targets, int32_t ntargets,
                       int32_t m, float x0, float dx, float* params, float* grad_out, float* final_loss,
                       const int32_t* order, int32_t epochs, float lr, float beta1, float beta2, float eps,
                       void* stream);

/* ---- densification kept from Gaussian splatting (Sec. 5.2; App. B.2) ---------------
 * ges_densify classifies each splat from its statistic (ges_adam_splats.grad_accum /
 * grad_count): selected when accum/count (0 if never visible) >= grad_threshold (0.0003),
 * then cloned when its largest log-scale <= ln(scale_threshold) (percent_dense 0.01 times
 * the scene extent) and split otherwise (tests in binary64).  dst[k] receives, for every
 * set k < nsets, the unsplit splats in order, then one clone per cloned splat, then two
 * children per split splat: means mu + R(q)(s * z_c) with z = normals[i][c][0..2] (given
 * standard normal draws, [n][2][3]), log-scales reduced by ln 1.6, the other parameters
 * copied.  Set 0 is the parameters (all six arrays required); sets 1, 2 are moments, copied
 * for the unsplit splats and zero for clones and children.  *n_out (host) receives the new
 * count (the call waits for `stream` after counting); when it exceeds dst_capacity nothing
 * is written and GES_ERR_CAPACITY is returned (n_out still set).  scratch:
 * ges_densify_scratch_bytes(n) bytes.  dst must not overlap src.
 *
 * ges_opacity_reset lowers every opacity above max_opacity (0.01) to it, on the logit
 * (compared in binary64), and clears the moments (either may be NULL). */
size_t ges_densify_scratch_bytes(int64_t n);
ges_status ges_densify(int64_t n, int32_t sh_degree, const ges_splat_set* src, const ges_splat_set* dst,
                       int32_t nsets, int64_t dst_capacity, const float* grad_accum, const float* grad_count,
                       const float* normals, double grad_threshold, double scale_threshold, void* scratch,
                       size_t scratch_bytes, int64_t* n_out, void* stream);
ges_status ges_opacity_reset(float* opacity_logits, float* exp_avg, float* exp_avg_sq, int64_t n, double max_opacity,
                             void* stream);

/* Learning rate at `step` of a log-linear decay from lr_init (step 0) to lr_final (step
 * max_steps, constant afterwards), times a delay factor that rises from delay_mult to 1
 * along a quarter sine over delay_steps (none when delay_steps <= 0).  The paper decays
 * the position rate this way (App. B.2).  Host function; returns NaN for lr_init or
 * lr_final <= 0 or max_steps < 1. */
double ges_expon_lr(int64_t step, double lr_init, double lr_final, int64_t max_steps, int64_t delay_steps,
                    double delay_mult);

/* Loss schedule of an iteration (host function): the frequency-mask strength omega grows linearly with
 * training progress, omega = iteration / total_iterations clamped to [0, 1] (Sec. 4.3), and the L1 weight
 * is what the SSIM and masked-L1 weights leave, lam_l1 = 1 - lam_ssim - lam_omega (Sec. 4.4, Eq. final;
 * the paper uses lam_ssim = 0.2, lam_omega = 0.5).  Both in binary64, rounded once to binary32.  Either
 * output may be NULL.  INVALID_ARGUMENT for total_iterations < 1 or non-finite weights. */
ges_status ges_loss_schedule(int64_t iteration, int64_t total_iterations, float lam_ssim, float lam_omega,
                             float* omega, float* lam_l1);

/* ---- serving: continuous batching of render requests -----------------------------
 * Forward renders (Sec. 4.2, Eq. transimttance, the same kernels as ges_render_forward)
 * of scenes resident in device memory, for many cameras and resolutions at once: the
 * real-time rendering the method is built for (Sec. 1; Sec. 5.2 reports render speed).
 * Requests arriving while a batch runs are admitted into the next batch as slots and
 * pool memory free up; every batch runs one preprocess, one scatter/sort and one raster
 * launch over all of its views, on one of two streams. */
typedef struct ges_server ges_server;

typedef struct {
  int32_t max_slots;             /* requests rendered together in one batched launch (1..32) */
  int32_t queue_capacity;        /* pending requests accepted before submit returns BUSY */
  int32_t falloff, tile_cull;    /* raster mode for every request */
  float rho;
  float bg[3];
  int32_t sequential;            /* 1: one request per launch (the baseline policy) */
} ges_serve_config;

typedef enum { GES_REQ_QUEUED = 0, GES_REQ_RUNNING = 1, GES_REQ_DONE = 2, GES_REQ_FAILED = 3,
               GES_REQ_REJECTED = 4, GES_REQ_CANCELLED = 5 } ges_request_state;

typedef struct {
  int32_t state;                 /* ges_request_state */
  int32_t status;                /* ges_status of the request (DONE -> GES_OK) */
  uint64_t t_submit_ns;          /* steady clock, submit */
  uint64_t t_start_ns;           /* admitted into a batch */
  uint64_t t_done_ns;            /* completion observed on the device */
  uint64_t num_keys;
  int32_t batch_size;            /* slots in the batch that rendered it */
} ges_request_info;

/* pool: caller-owned device buffer the server sub-allocates all per-request
 * workspaces from (the admission budget). */
ges_status ges_serve_create(const ges_serve_config* cfg, void* pool, size_t pool_bytes, ges_server** out);
/* Host-only variant for testing the scheduler without a GPU: the executor never touches device
 * memory; every view of a batch produces keys_per_view keys, a batch takes batch_ns + per_view_ns
 * per view, and batches holding a request for scene fail_scene fail with GES_ERR_DEVICE.  The pool
 * of pool_bytes is accounted but never dereferenced. */
ges_status ges_serve_create_simulated(const ges_serve_config* cfg, size_t pool_bytes, uint64_t keys_per_view,
                                      uint64_t batch_ns, uint64_t per_view_ns, int32_t fail_scene,
                                      ges_server** out);
/* The scene's device buffers must stay alive and unchanged until ges_serve_destroy. */
ges_status ges_serve_add_scene(ges_server* s, const ges_splats* scene, int32_t* scene_id);
/* Queue a render of scene_id from cam into out_rgb_device [h,w,3] FP32.  Returns BUSY when
 * the queue is full, NOT_FOUND for an unknown scene, INVALID_ARGUMENT for a bad camera. */
ges_status ges_serve_submit(ges_server* s, int32_t scene_id, const ges_camera* cam, float* out_rgb_device,
                            uint64_t* request_id);
ges_status ges_serve_poll(ges_server* s, uint64_t request_id, ges_request_info* info);
/* As ges_serve_submit, and (tests) the finished request also leaves copies of its frame
 * arrays in inspect_device, a 256-byte-aligned device buffer of inspect_bytes bytes laid
 * out as (each part starting on a 256-byte boundary, in this order):
 *   records   [n,16] FP32, the per-splat record of ges_frame_view (64 B per splat);
 *   ranges    [tiles,2] u32, each tile's [start,end) in the batch's sorted ids;
 *   n_contrib [height,width] u32 (written there by the raster itself);
 *   header    4 x u64: this view's keys, error word, pairs examined, pairs composited
 *             (the part is 256 bytes);
 *   ids       [batch keys,2] u32, the batch's sorted (splat index, slot) pairs (every view),
 *             copied only if inspect_bytes >= ges_serve_inspect_bytes(n, w, h, batch keys);
 *             ges_serve_poll's num_keys gives the batch's key count.
 * inspect_bytes below ges_serve_inspect_bytes(n, w, h, 0): CAPACITY; a misaligned
 * buffer: INVALID_ARGUMENT.  The buffer must stay alive until the request finishes. */
ges_status ges_serve_submit_inspect(ges_server* s, int32_t scene_id, const ges_camera* cam, float* out_rgb_device,
                                    void* inspect_device, size_t inspect_bytes, uint64_t* request_id);
/* Size of that layout for a scene of n splats, a width x height view and a batch of
 * batch_keys keys (0 for invalid sizes). */
size_t ges_serve_inspect_bytes(int64_t n, int32_t width, int32_t height, uint64_t batch_keys);
/* Block until every request submitted so far has finished (done, failed or rejected). */
ges_status ges_serve_drain(ges_server* s);
/* Stops the server; requests still queued are cancelled, running ones are completed. */
ges_status ges_serve_destroy(ges_server* s);

#ifdef __cplusplus
}
#endif
#endif
