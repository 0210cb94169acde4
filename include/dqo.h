/*
 * libdqo — MI355X (gfx950) kernels for the GPU-side optimization of DQO-MAP
 * (object-aware 3D Gaussian Splatting): differentiable rasterization of colour,
 * depth and per-Gaussian object id, the object loss it feeds, the Adam step, and
 * the per-object dual-quadric fit from 2D boxes.
 *
 * Paper passages the calls follow:
 *   - Gaussians share the quadric's shape: mean, rotation, axis scales
 *     (Sec. III-A, Eq. (2)-(3)); each Gaussian carries an object id
 *     (Sec. III-C, the text after Eq. (7)-(8)).
 *   - Colour and depth are rendered by alpha blending, and the instance
 *     channel ins of Eq. (12) bounds an object's outline (Sec. III-D).
 *   - The object loss is Eq. (10)-(14): colour, depth and instance terms,
 *     weighted by lambda.
 *   - Rasterization and its backward run as GPU kernels (Sec. IV,
 *     implementation detail).
 *   - The object quadric Q*_k satisfies pi^T Q* pi = 0 for the planes
 *     back-projected from box edges (Eq. (1)); cameras are P = K [R|t]
 *     (text after Eq. (4)).
 *
 * Conventions shared by every call
 *   - Every data pointer is DEVICE memory owned by the caller (e.g. torch
 *     tensors).  The library never allocates, frees or synchronises in the
 *     compute calls; every compute call only enqueues kernels on `stream`
 *     (a hipStream_t, NULL = default stream), so a sequence of calls can be
 *     captured in a HIP graph.  Host pointers are marked "host".
 *   - `dtype` selects the arithmetic: DQO_F32 (float) or DQO_F64 (double).
 *     Every floating-point buffer of a call is of that type.
 *   - Gaussian parameters are structure-of-arrays params[14][n], row r holds
 *     component r of every Gaussian: rows 0-2 mean (world), 3-5 log-scale,
 *     6-9 quaternion (w,x,y,z; need not be normalised), 10 opacity logit,
 *     11-13 colour.  ids[n] are int32 object ids.
 *   - Images are [V][C][H][W] row-major, V = number of views.
 *   - Return value: DQO_OK (0) or a negative DQO_E* code; on error the
 *     context's dqo_last_error() holds a message and nothing was enqueued.
 *     Argument validation happens on the host before any launch.
 *   - Errors found on the device (pair-list overflow, non-finite inputs) set
 *     bits in a status word inside the state buffer; read it with
 *     dqo_read_status() at a point of the caller's choosing.
 *   - A context is not thread-safe; use one per host thread.
 */
#ifndef DQO_H
#define DQO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DQO_MAX_VIEWS 16
#define DQO_MAX_K 64
#define DQO_NUM_PARAMS 14

enum dqo_status {
    DQO_OK = 0,
    DQO_EINVAL = -1,      /* bad argument: NULL, size, dtype, K, view count, tile shape */
    DQO_ECAPACITY = -2,   /* pair list needs more than pair_capacity entries */
    DQO_ENONFINITE = -3,  /* a parameter was NaN/Inf (those Gaussians were culled) */
    DQO_EDEGENERATE = -4, /* not enough independent constraints */
    DQO_EHIP = -5,        /* a HIP runtime call failed; message in dqo_last_error */
    DQO_EINTERNAL = -6    /* a device-side wait exceeded its bound (library bug) */
};

enum dqo_dtype { DQO_F32 = 0, DQO_F64 = 1 };

/* How the pairs of a tile come to be in depth order (dqo_config.depth_order).
 * Both give the same order: by the item's depth key (the FP32 bits of its
 * camera depth), ties by item index.
 * GLOBAL: every item is radix-sorted by depth, the pairs are emitted in that
 *   order and stably sorted by tile.
 * TILE: the pairs are emitted in item order and stably sorted by tile, then
 *   each tile's pairs are sorted by depth on their own (one workgroup per
 *   tile, in LDS up to 4096 pairs).  Cheaper when tiles hold few pairs.
 * AUTO: GLOBAL (measured faster: at 200k Gaussians, 640x480, 8x8 tiles the
 *   four depth passes take 50 us, the per-tile sorts 107 us). */
enum dqo_depth_order { DQO_DEPTH_ORDER_AUTO = 0, DQO_DEPTH_ORDER_GLOBAL = 1, DQO_DEPTH_ORDER_TILE = 2 };

/* Bits of the device status word (dqo_read_status). */
enum dqo_status_bits {
    DQO_STATUS_OVERFLOW = 1,   /* more pairs than pair_capacity: outputs undefined */
    DQO_STATUS_NONFINITE = 2,  /* non-finite parameters met (Gaussians culled) */
    DQO_STATUS_TIMEOUT = 4     /* a bounded device wait gave up: outputs undefined */
};

/* Rasterizer constants.  The paper does not state them; these are the readings
 * used throughout (defaults from dqo_config_default). */
typedef struct dqo_config {
    int32_t tile_w, tile_h;  /* pixel tile: 16x16 default; 8x8, 16x8, 32x8, 8x32 also accepted */
    double z_near;           /* 0.2: cull if camera depth <= z_near */
    double dilation;         /* 0.3 px^2 added to the 2D covariance diagonal */
    double q_max;            /* 9: contribute only where the Mahalanobis form Q <= q_max */
    double alpha_min;        /* 1/255: contribute only if alpha >= alpha_min */
    double alpha_max;        /* 0.99: alpha = min(alpha_max, o * exp(-Q/2)) */
    double t_min;            /* 1e-4: stop before transmittance would drop below t_min */
    double bg[3];            /* background colour added with weight T_final */
    int32_t depth_order;     /* dqo_depth_order: DQO_DEPTH_ORDER_AUTO default */
    int32_t tile_sort_lds;   /* TILE order: pairs of a tile sorted in LDS, 1..4096 (0 = 4096); longer
                                tiles take a slower global-memory path */
} dqo_config;

/* Pinhole camera: world -> camera x_c = R x_w + t; pixel = (fx x/z + cx, fy y/z + cy).
 * Pixel (u, v) is sampled at (u + 1/2, v + 1/2).  Host struct. */
typedef struct dqo_camera {
    double R[9]; /* row-major */
    double t[3];
    double fx, fy, cx, cy;
    int32_t width, height;
} dqo_camera;

/* Size of one frame of work.  All views must share width and height.
 * The per-view arrays below are host memory, read at every call that takes
 * the descriptor; each may be NULL.
 * segments: NULL, in which case every view sees all n Gaussians, or
 *   [n_views][2] = (first, count): view v sees Gaussians [first, first + count)
 *   only.  Segments let one launch render independent Gaussian sets (object
 *   crops, per-object jobs) each in its own view; they may overlap.
 * windows: NULL (whole images) or [n_views][4] = (x0, y0, x1, y1): view v
 *   renders only pixels x0 <= u < x1, y0 <= v < y1 (within the image; empty
 *   when x1 <= x0 or y1 <= y0).  Pixels outside the window are written as if
 *   no Gaussian covered them (colour = background, depth 0, T_final 1, last
 *   -1, p_target as for an empty pixel), carry no loss, and the pairs of tiles
 *   outside it are never made.
 * jobs: NULL (every view whole-scene) or [n_views]: -1 for a whole-scene
 *   view, k in [0, K) for a per-object job of object k (the objects are
 *   optimised in parallel, Sec. III-D): the view's Gaussians (its segment)
 *   are object k's, its instance channel ins_k of Eq. (12) is then
 *   1 - T_final, and Eq. (13) compares it with the observed mask of k.  In
 *   the forward, the loss and the backward, the target id t of a job's pixel
 *   is read as k where t == k and -1 ("not this object": probability
 *   T_final) elsewhere, and its colour and depth terms count only the pixels
 *   observed as k. */
typedef struct dqo_frame_desc {
    int64_t n;             /* Gaussians, >= 0 */
    int32_t n_views;       /* 1..DQO_MAX_VIEWS */
    int32_t K;             /* object classes for the instance channels, 0..DQO_MAX_K */
    int64_t pair_capacity; /* max (tile, Gaussian) pairs over all views, <= 2^30 */
    int32_t dtype;         /* DQO_F32 or DQO_F64 */
    int32_t reserved;
    const int64_t* segments; /* NULL or [n_views][2] (first, count), within [0, n] */
    const int32_t* windows;  /* NULL or [n_views][4] pixel windows (x0, y0, x1, y1) */
    const int32_t* jobs;     /* NULL or [n_views] object of a per-object job, -1 = whole scene */
} dqo_frame_desc;

/* Sub-buffers of the caller-allocated state buffer (dqo_state_layout). */
enum dqo_buf {
    DQO_BUF_SPLATS = 0,  /* [V*n] records of 16 values: mx,my,A,B,C,opacity,z,id,r,g,b,0, first pair slot,
                            tile rectangle x0 | y0 << 16, rectangle width, 0 (integers as FP32 bit patterns,
                            FP64 values) */
    DQO_BUF_RECTS,       /* [V*n] int16x4 tile rectangle x0,y0,x1,y1 (inclusive), empty = x1<x0 */
    DQO_BUF_COUNTS,      /* [V*n] uint32 tiles covered */
    DQO_BUF_OFFSETS,     /* [V*n] uint32 first slot of the item's pairs in emission order */
    DQO_BUF_DEPTH_KEYS,  /* [V*n] uint32 sorted depth keys (float bits of z; culled = 0xffffffff) */
    DQO_BUF_DEPTH_ORDER, /* [V*n] uint32 item index (view*n + g) in depth order (GLOBAL depth order only) */
    DQO_BUF_PAIR_KEYS,   /* [cap] uint32 sorted global tile id (view*tiles + tile) */
    DQO_BUF_PAIR_VALS,   /* [cap] uint32 item index, in (tile, depth, index) order; after a render
                            forward, bit 31 is set on the pairs whose Gaussian cannot contribute at
                            any pixel of their tile (the render backward skips them) */
    DQO_BUF_RANGES,      /* [V*tiles][2] uint32 [start, end) of each tile in the sorted pairs */
    DQO_BUF_PARTIALS,    /* [cap][10] per-pair gradient partials (render backward; valid only for the pairs
                            it marks written, the others are left as they were and count as zero) */
    DQO_BUF_CONTROL,     /* status word, pair count, counters, histograms, loss partials */
    DQO_BUF_SCRATCH,     /* sort double buffers and wait state */
    DQO_BUF_COUNT
};

typedef struct dqo_layout {
    int64_t offset[DQO_BUF_COUNT]; /* byte offset of each sub-buffer, 256-byte aligned */
    int64_t bytes[DQO_BUF_COUNT];
    int64_t total;                 /* bytes the caller must allocate */
    int32_t tiles_x, tiles_y;      /* tile grid per view */
    int32_t pair_key_bits;         /* significant bits of the pair keys */
    int32_t reserved;
} dqo_layout;

/* Rendered images (device, caller-owned).  Optional pointers may be NULL. */
typedef struct dqo_images {
    void* color;           /* [V][3][H][W] colour incl. T_final * bg */
    void* depth;           /* [V][H][W] sum of w_i z_i (camera depth, not normalised) */
    void* t_final;         /* [V][H][W] transmittance after the last blended Gaussian */
    int32_t* last;         /* [V][H][W] position in the sorted pair list of the last
                              blended Gaussian, -1 if none */
    void* probs;           /* optional [V][K][H][W] instance channels P_k = ins_k */
    int32_t* id_map;       /* optional [V][H][W] argmax over (P_0..P_{K-1}, T_final), -1 = none;
                              needs probs */
    const int32_t* target; /* optional [V][H][W] target object id per pixel, -1 = none */
    void* p_target;        /* optional [V][H][W] probability of the target: P_t, or
                              T_final where target = -1; needs target */
    int32_t* n_blend;      /* optional [V][H][W] number of Gaussians blended at the pixel */
} dqo_images;

/* Upstream gradients of the images (device).  Optional pointers may be NULL. */
typedef struct dqo_image_grads {
    void* d_color;     /* [V][3][H][W] */
    void* d_depth;     /* [V][H][W] */
    void* d_t_final;   /* optional [V][H][W] */
    void* d_probs;     /* optional [V][K][H][W] */
    void* d_p_target;  /* optional [V][H][W], interpreted through dqo_images.target */
} dqo_image_grads;

typedef struct dqo_targets {
    const void* color;   /* [V][3][H][W] */
    const void* depth;   /* [V][H][W]; pixels with depth <= 0 carry no depth term */
    const int32_t* id;   /* [V][H][W] target object id, -1 = none */
} dqo_targets;

/* Loss weights: L = w_rgb * L_rgb + w_depth * L_depth + lambda * L_obj (Eq. (14)).
 * ce_eps clamps the probability inside the log of the cross-entropy. */
typedef struct dqo_loss_weights {
    double w_rgb, w_depth, lambda, ce_eps;
} dqo_loss_weights;

/* Adam hyper-parameters, one learning rate per parameter row. */
typedef struct dqo_adam {
    double lr[DQO_NUM_PARAMS];
    double beta1, beta2, eps;
} dqo_adam;

typedef struct dqo_ctx dqo_ctx;

/* ---- context ------------------------------------------------------------ */
void dqo_config_default(dqo_config* cfg /* host, out */);
/* Creates a context (host memory only).  cfg may be NULL for the defaults. */
int dqo_ctx_create(dqo_ctx** out, const dqo_config* cfg);
int dqo_ctx_destroy(dqo_ctx* ctx);
/* Message of the last failing call on this context ("" if none). */
const char* dqo_last_error(const dqo_ctx* ctx);
const char* dqo_status_string(int code);
/* Library version string. */
const char* dqo_version(void);

/* ---- state buffer ------------------------------------------------------- */
/* Layout of the state buffer for a frame (host computation only).  The caller
 * allocates `total` bytes of device memory (256-byte aligned) and passes it to
 * every call of that frame. */
int dqo_state_layout(const dqo_ctx* ctx, const dqo_frame_desc* desc, const dqo_camera* cams /* host [V] */,
                     dqo_layout* out /* host */);
/* Clears the control block (status word, counters) of a fresh state buffer. */
int dqo_state_init(const dqo_ctx* ctx, const dqo_frame_desc* desc, const dqo_camera* cams, void* state,
                   void* stream);
/* Synchronises `stream` and copies the status word and the pair count to the
 * host.  Returns DQO_ECAPACITY / DQO_ENONFINITE / DQO_EINTERNAL when the
 * matching status bit is set, else DQO_OK. */
int dqo_read_status(const dqo_ctx* ctx, const dqo_frame_desc* desc, const dqo_camera* cams, void* state,
                    uint32_t* status /* host, out */, int64_t* num_pairs /* host, out */, void* stream);
/* Clears the status word (enqueued on stream). */
int dqo_clear_status(const dqo_ctx* ctx, const dqo_frame_desc* desc, const dqo_camera* cams, void* state,
                     void* stream);

/* ---- hot path ----------------------------------------------------------- */
/* Projection, culling and binning (EWA projection of the Gaussian shape of
 * Eq. (2) into every view).  Per (view, Gaussian) item: 2D mean, conic,
 * opacity, depth, tile rectangle of the 3-sigma box; then the items are sorted
 * by depth (float bits of camera z, stable, so ties keep index order), and the
 * (tile, item) pairs are emitted in that order into the pair list.  The pair
 * count stays on the device; if it exceeds pair_capacity the OVERFLOW status
 * bit is set.  params: [14][n] of dtype; ids: [n]. */
int dqo_project_cull_bin(const dqo_ctx* ctx, const dqo_frame_desc* desc, const dqo_camera* cams,
                         const void* params, const int32_t* ids, void* state, void* stream);

/* The blending order of the alpha blending of Sec. III-D (front to back,
 * by camera depth; the rasterization kernel of Sec. IV): stable radix sort
 * of the pair list by global tile id (the list is already in depth order, so
 * the result is ordered by (tile, depth, item index)), then the [start, end)
 * range of every tile, the launch order of the render workgroups (heaviest
 * tiles first), and cleared written-marks of the per-pair gradient partials
 * for dqo_render_backward.  Needs dqo_project_cull_bin on the same state;
 * the pair count is read on the device (no host synchronisation). */
int dqo_sort(const dqo_ctx* ctx, const dqo_frame_desc* desc, const dqo_camera* cams, void* state,
             void* stream);

/* Front-to-back alpha blending of colour, depth and the instance channels of
 * Eq. (12) for every pixel of every view (Sec. III-D): Gaussian i contributes
 * at pixel sample s iff Q_i(s) <= q_max and alpha_i = min(alpha_max,
 * o_i exp(-Q_i/2)) >= alpha_min; w_i = alpha_i T_i; blending stops before a
 * Gaussian that would take T below t_min.  P_k = sum of w_i over Gaussians with
 * id k, so sum_k P_k + T_final = 1.  Needs dqo_project_cull_bin and dqo_sort
 * on the same state.  probs requires K >= 1.  Also marks, in the pair list
 * (DQO_BUF_PAIR_VALS bit 31), the pairs whose Gaussian cannot contribute at
 * any pixel of their tile; marking is idempotent and changes no result. */
int dqo_render_forward(const dqo_ctx* ctx, const dqo_frame_desc* desc, const dqo_camera* cams,
                       const void* state, const dqo_images* img, void* stream);

/* Object loss of Eq. (10)-(14), read as: L_rgb = mean |C - C^| over the
 * colour pixels (3 channels each), L_depth = mean |D - D^| over the colour
 * pixels with D^ > 0, L_obj = mean over the window pixels of
 * -log max(p_t, ce_eps) with p_t = img->p_target; total = w_rgb L_rgb +
 * w_depth L_depth + lambda L_obj.  Window pixels: every pixel of every view
 * unless the descriptor gives windows.  Colour pixels: the window pixels of
 * whole-scene views and, of a per-object job of object k, those observed as
 * k (tgt->id, then required).  Each mean is taken over all views together.
 * Writes loss[4] = {total, L_rgb, L_depth, L_obj} (device double) and the
 * upstream gradients d_color, d_depth and d_p_target of `g` (zero outside
 * the counted pixels; sign(0) = 0; no CE gradient where p_t < ce_eps).  The
 * reduction order is fixed, so the result is bitwise reproducible. */
int dqo_object_loss(const dqo_ctx* ctx, const dqo_frame_desc* desc, const dqo_camera* cams,
                    const dqo_images* img, const dqo_targets* tgt, const dqo_loss_weights* w,
                    double* loss /* device [4] */, const dqo_image_grads* g, void* state, void* stream);

/* dqo_object_loss for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): the same loss, gradients and reduction order (bitwise the
 * same results), but no state buffer: the per-workgroup partial sums and
 * the valid-depth count live in a scratch array of the library, one 32 KiB
 * copy per device (held until the process ends), whose address is looked
 * up once per device on the first call there.  The call allocates nothing.
 * Every call on one device shares that scratch, and nothing in it needs to
 * start at zero (each call overwrites what it reads): calls that overlap on
 * one device (other streams, other host threads) race and must be ordered
 * by the caller.  The scratch holds 511 rows of partial sums, the most the
 * loss pass uses for any frame (one row per reduction workgroup); a size
 * check rejects with DQO_EINVAL a call that would need more, which no valid
 * frame does.  desc->n, pair_capacity and segments are not used (n may be
 * 0); windows and jobs are honoured as by dqo_object_loss.  At most 64
 * devices. */
int dqo_object_loss_noalloc(const dqo_ctx* ctx, const dqo_frame_desc* desc, const dqo_camera* cams,
                            const dqo_images* img, const dqo_targets* tgt, const dqo_loss_weights* w,
                            double* loss /* device [4] */, const dqo_image_grads* g, void* stream);

/* Adjoint of dqo_render_forward with the blended set held fixed: the
 * back-propagation of the rendering losses through the alpha blending of
 * colour, depth and the instance channels of Eq. (12) (Sec. III-D; the
 * back-propagation kernel of Sec. IV).  Walks each pixel back to front from
 * its last blended Gaussian, recomputing the transmittance
 * T_i = T_{i+1} / (1 - alpha_i) instead of storing it, and writes one
 * gradient record per (tile, Gaussian) pair into the state (partials of
 * mean2d, conic, opacity, colour, depth).  No atomics: the per-Gaussian sums
 * are taken in dqo_project_backward in a fixed order.
 * img must hold the outputs of a dqo_render_forward on this state since its
 * last dqo_project_cull_bin (the positions in img->last index that pair
 * list); g the upstream gradients of those images (d_color required).
 * With 8x8 tiles and at most 8192 tiles over all views, and when neither img
 * holds instance channels nor g their gradients, each tile's pair range is
 * walked in 64-pair segments by separate wavefronts, each restarting from
 * the state the forward stored at the segment's end.  Those states belong
 * to the last such forward; the device checks that it is this binning and
 * these images (img->last and img->target), and otherwise walks every tile
 * whole, which gives the same gradients up to rounding order. */
int dqo_render_backward(const dqo_ctx* ctx, const dqo_frame_desc* desc, const dqo_camera* cams,
                        void* state, const dqo_images* img, const dqo_image_grads* g, void* stream);

/* Back-propagation through the projection of the Gaussian shape of
 * Eq. (2)-(3) (the Gaussian's mean, rotation and axis scales, Sec. III-A)
 * into every view, which completes the gradient of the rendering losses of
 * Sec. III-D with respect to the Gaussian parameters: sums each Gaussian's
 * pair partials over tiles and views in a fixed order and applies the chain
 * rule through the projection to grads[14][n] (same layout as params;
 * overwritten; zero for Gaussians culled in every view).  params must be the
 * parameters the state was projected with; needs dqo_render_backward on the
 * same state. */
int dqo_project_backward(const dqo_ctx* ctx, const dqo_frame_desc* desc, const dqo_camera* cams,
                         const void* params, const void* state, void* grads, void* stream);

/* One Adam step (bias-corrected, PyTorch semantics) over params[14][n] with
 * per-row learning rates; m and v are the moment buffers (same layout).
 * step >= 1 is the 1-based step count. */
int dqo_adam_step(const dqo_ctx* ctx, int32_t dtype, void* params, const void* grads, void* m, void* v,
                  int64_t n, const dqo_adam* hp /* host */, int64_t step, void* stream);

/* Same update as dqo_adam_step, with the step count kept in device memory so
 * that the call can be captured once in a HIP graph and replayed: the update
 * uses step = *d_step + 1 and then stores it back into *d_step (int64, device,
 * caller-owned, start at 0). */
int dqo_adam_step_counted(const dqo_ctx* ctx, int32_t dtype, void* params, const void* grads, void* m, void* v,
                          int64_t n, const dqo_adam* hp /* host */, int64_t* d_step, void* stream);

/* Camera-pose gradient of every view, for tracking with the rasterizer (the
 * paper tracks the camera through the same differentiable rendering, Sec. IV).
 * The pose of view v is x_c = R x_w + t, perturbed on the left in the camera
 * frame: R' = exp([w]x) R, t' = exp([w]x) t + tau.  pose_grads (device
 * double [V][6], overwritten) = (dL/dw, dL/dtau) at w = tau = 0, for the loss
 * whose image gradients the preceding dqo_render_backward took.  Reduction
 * order is fixed (bitwise reproducible). */
int dqo_pose_backward(const dqo_ctx* ctx, const dqo_frame_desc* desc, const dqo_camera* cams, const void* params,
                      const void* state, double* pose_grads, void* stream);

/* dqo_project_backward and dqo_adam_step_counted in one pass: each
 * Gaussian's gradient is applied at once by the same Adam update to params
 * (in place), m and v (device, [14][n], the frame's dtype); the update uses
 * step = *d_step + 1 and the call advances *d_step by one.  grads (optional,
 * NULL to skip) receives the gradient.  Results are bitwise those of the two
 * separate calls.  params must be the parameters the frame was projected
 * with (they are read before being overwritten, per Gaussian). */
int dqo_project_backward_adam(const dqo_ctx* ctx, const dqo_frame_desc* desc, const dqo_camera* cams, void* params,
                              const void* state, void* m, void* v, const dqo_adam* hp /* host */, int64_t* d_step,
                              void* grads, void* stream);

/* ---- incremental update ---------------------------------------------------- */

/* Thresholds of Eq. (7) and the opacities of the Gaussians added where they
 * fire (opaque OG for geometry, transparent TG for colour; Sec. IV).
 * Defaults: theta_alpha 0.5 (unstated in the paper), theta_d = theta_c = 0.1
 * (stated), OG 0.9, TG 0.1. */
typedef struct dqo_increment_cfg {
    double theta_alpha; /* ins below it: the object's geometry is missing */
    double theta_d;     /* |rendered depth - observed depth| above it: incomplete */
    double theta_c;     /* mean |rendered colour - observed colour| over r, g, b above it */
    double og_opacity, tg_opacity;
} dqo_increment_cfg;

/* Unstable-pixel masks of Eq. (7), per object as in Eq. (8), from the images
 * of a loss-mode forward (img->color, depth and p_target, rendered with
 * img->target = tgt->id, so that p_target = ins of the observed object) and
 * the observed frame tgt (colour, depth, id).  masks[V][H][W] uint8 (device,
 * written): bit 0 Mask_geo (ins < theta_alpha, or observed depth > 0 and
 * |D - observed| > theta_d), bit 1 Mask_rgb (mean colour error > theta_c);
 * pixels observed as no object (id -1) or with id >= K are 0.  obj_counts
 * (device int32 [K][2], overwritten): per object, its Mask_geo and Mask_rgb
 * pixel counts.  All floating-point buffers are of the frame's dtype. */
int dqo_incremental_masks(const dqo_ctx* ctx, const dqo_frame_desc* d, const dqo_camera* cams,
                          const dqo_images* img, const dqo_targets* tgt, const dqo_increment_cfg* cfg /* host */,
                          uint8_t* masks, int32_t* obj_counts, void* stream);

/* Gaussians added at the unstable pixels with observed depth d > 0: an OG
 * Gaussian at Mask_geo pixels, else a TG Gaussian at Mask_rgb pixels, in view
 * order then raster order; the mean is the pixel centre (u + 1/2, v + 1/2)
 * back-projected at depth d through view v's camera, log-scales log(d / fx),
 * identity quaternion, opacity logit of og/tg_opacity, the observed colour,
 * id = the observed id.  They are written to columns [n_old, n_cap) of
 * params[14][n_cap] (frame dtype) and ids[n_cap]; counts (device int64
 * [V + 1], written): [0] the number to add (columns beyond n_cap are not
 * written: compare with n_cap - n_old), [1 + v] per view. */
int dqo_densify(const dqo_ctx* ctx, const dqo_frame_desc* d, const dqo_camera* cams, const dqo_targets* tgt,
                const uint8_t* masks, const dqo_increment_cfg* cfg /* host */, int64_t n_old, int64_t n_cap,
                void* params, int32_t* ids, int64_t* counts, void* stream);

/* ---- quadric -------------------------------------------------------------- */

/* 2D boxes of every object in rendered id maps (the observed boxes from which
 * the quadric of Eq. (1) is fitted): for view v and object k, the pixel-edge
 * box (x0, y0, x1, y1) = (min u, min v, max u + 1, max v + 1) over pixels with
 * id_map == k.  Outputs (device): boxes[V*K][4] double, box_obj[V*K] (k, or -1
 * when the object covers no pixel of the view) and box_view[V*K] (v), in the
 * input format of dqo_fit_dual_quadric.  id_map: [V][H][W] int32. */
int dqo_id_boxes(const dqo_ctx* ctx, const int32_t* id_map, int32_t n_views, int32_t width, int32_t height,
                 int32_t K, double* boxes, int32_t* box_obj, int32_t* box_view, void* stream);
enum dqo_quadric_status { DQO_QUADRIC_OK = 0, DQO_QUADRIC_DEGENERATE = 1, DQO_QUADRIC_NOT_ELLIPSOID = 2 };

/* Per-object dual quadric from 2D boxes (Eq. (1)): every box edge line l of
 * object k seen by camera P_v (3x4, P = K [R|t]) gives the plane pi = P_v^T l
 * (normalised), and pi^T Q* pi = 0 is one linear equation in the 10 unique
 * entries of the symmetric Q*.  Q* is the right singular vector of the
 * smallest singular value of the stacked equations (FP64 one-sided Jacobi
 * SVD), scaled so Q*_44 = -1, then decoupled as Eq. (2)-(3): mu = -Q*[0:3,3],
 * Q*[0:3,0:3] + mu mu^T = R diag(a^2,b^2,c^2) R^T (axes ascending, det R = +1).
 * Edges within `border` px of the image border are dropped when img_wh is
 * given.  Inputs (device): boxes[n_boxes][4] (x0,y0,x1,y1), box_obj[n_boxes],
 * box_view[n_boxes], P[n_views][12] row-major, img_wh[n_views][2] or NULL.
 * Outputs (device): Q[n_obj][16], mu[n_obj][3], R[n_obj][9], axes[n_obj][3],
 * status[n_obj] (dqo_quadric_status; DEGENERATE when fewer than 9 equations
 * or a null space of dimension > 1).  At most 256 equations per object. */
int dqo_fit_dual_quadric(const dqo_ctx* ctx, int32_t n_obj, int64_t n_boxes, const double* boxes,
                         const int32_t* box_obj, const int32_t* box_view, int32_t n_views, const double* P,
                         const int32_t* img_wh, double border, double* Q, double* mu, double* R, double* axes,
                         int32_t* status, void* stream);

/* ---- quadric refinement ---------------------------------------------------- */

/* Object pose training by the IoU loss of Eq. (9).  An object's quadric is
 * theta[10] = (mu[3], q[4] = (w, x, y, z), log-axes[3]): Q* = Z diag(a^2, b^2,
 * c^2, -1) Z^T with Z = [[R(q / |q|), mu], [0, 1]] (Eq. (2)-(3)).  For each
 * box of the object (box_obj == k, 0 <= box_view < n_views), the dual conic
 * C* = P Q* P^T of camera P[box_view] (Eq. (4)) gives the tangent box
 * (x0, y0, x1, y1), clipped to [0, W] x [0, H] when img_wh is given; the
 * object's loss is J_k = sum over its boxes of 1 - IoU(predicted, observed).
 * A box whose conic is not an ellipse in front of the camera counts 1 with no
 * gradient.  Inputs use the format of dqo_fit_dual_quadric; at most 256 boxes
 * per object (an object with more gets NaN losses and is left unchanged).
 * All buffers are device FP64 / int32. */
typedef struct dqo_refine_cfg {
    int32_t iterations;               /* Adam steps, >= 0 */
    double lr_mu, lr_rot, lr_axes;    /* learning rates of mu, q and the log-axes */
    double beta1, beta2, eps;         /* Adam (PyTorch's update with bias correction) */
} dqo_refine_cfg;

/* J_k and dJ_k/dtheta_k for every object at the given theta[n_obj][10]:
 * loss[n_obj], grad[n_obj][10]; box_iou[n_boxes] (optional) receives the IoU
 * of every box of an object (entries of other boxes are not written). */
int dqo_quadric_iou_grad(const dqo_ctx* ctx, int32_t n_obj, int64_t n_boxes, const double* boxes,
                         const int32_t* box_obj, const int32_t* box_view, int32_t n_views, const double* P,
                         const int32_t* img_wh, const double* theta, double* loss, double* grad, double* box_iou,
                         void* stream);

/* Refines every object whose status is DQO_QUADRIC_OK (status may be NULL:
 * all objects) in one launch: theta is formed from mu[n_obj][3], R[n_obj][9]
 * (row-major rotation) and axes[n_obj][3], `iterations` Adam steps on J_k are
 * taken, and mu, R = R(q / |q|) and axes = exp(log-axes) are overwritten;
 * Q[n_obj][16] (optional) receives the refined Q*.  loss[n_obj][2] = (J_k
 * before, J_k after); NaN for objects that are skipped.  box_iou[n_boxes]
 * (optional): final IoU of each box of a refined object. */
int dqo_refine_quadrics(const dqo_ctx* ctx, int32_t n_obj, int64_t n_boxes, const double* boxes,
                        const int32_t* box_obj, const int32_t* box_view, int32_t n_views, const double* P,
                        const int32_t* img_wh, const int32_t* status, const dqo_refine_cfg* cfg /* host */,
                        double* mu, double* R, double* axes, double* Q, double* loss, double* box_iou, void* stream);

/* ---- object association ---------------------------------------------------- */

/* Association scores of a batch of detections (Sec. III-B, Eq. (4)-(6)), FP64.
 * Objects: mu[n_obj][3], R[n_obj][9] (row-major rotation), axes[n_obj][3].
 * Detections: boxes[n_det][4] (x0, y0, x1, y1) of frames det_frame[n_det] in
 * [0, n_frames), whose cameras are P[n_frames][12] (P = K [R|t]) and image
 * sizes img_wh[n_frames][2].  Outputs (device, overwritten):
 *   iou[n_obj][n_det]  IoU of object k's projected box (the tangent box of
 *                      C* = P Q* P^T, clipped to the image; 0 when the
 *                      projection is not an ellipse in front of the camera)
 *                      with detection j, in detection j's frame;
 *   match[n_det]       the object of largest IoU (lowest index among equals)
 *                      when that IoU >= iou_min, else -1 (a new object);
 *   occ[n_det][n_det]  (optional, NULL to skip) Eq. (6)'s overlap ratio
 *                      |B_i n B_j| / |B_j| for detections of the same frame
 *                      with |B_j| < |B_i|, else 0.
 * All inputs are device memory. */
int dqo_associate(const dqo_ctx* ctx, int32_t n_obj, const double* mu, const double* R, const double* axes,
                  int64_t n_det, const double* boxes, const int32_t* det_frame, int32_t n_frames, const double* P,
                  const int32_t* img_wh, double iou_min, double* iou, int32_t* match, double* occ, void* stream);

/* Quadric distance of Eq. (5) between two sets of quadrics:
 * qd[a][b] = exp(-tau (||mu_a - mu_b|| + ||S_a - S_b||_F)) with the shape
 * matrix S = R diag(axes^2) R^T (device FP64 in and out; qd[na][nb]). */
int dqo_quadric_distance(const dqo_ctx* ctx, int32_t na, const double* mu_a, const double* R_a, const double* axes_a,
                         int32_t nb, const double* mu_b, const double* R_b, const double* axes_b, double tau,
                         double* qd, void* stream);

/* The decisions taken from the association scores (Sec. III-B, Eq. (5)-(6)).
 * Inputs (device): match[n_det] from dqo_associate; qd_obs[n_det][n_obj] the
 * QD between each detection's observed quadric and each object (NULL when
 * n_obj == 0); occ[n_det][n_det] the overlap ratios from dqo_associate;
 * qd_det[n_det][n_det] the QD between the detections' observed quadrics;
 * label[n_det] the detector's class of each detection.  Outputs (device,
 * overwritten):
 *   fine[n_det]    match[j] when QD(observation j, object match[j]) >= qd_min,
 *                  else -1 (a wrong match is dropped);
 *   parent[n_det]  the detection i of the same label with occ[i][j] > t_occ
 *                  and qd_det[i][j] > qd_occ (j is a piece of i's object and
 *                  is popped), the largest ratio winning, then the lowest
 *                  index; -1 when there is none;
 *   root[n_det]    the end of j's chain of parents (j when not absorbed);
 *   obj[n_det]     fine[root[j]]: the object j's observation updates, -1 for
 *                  a new object seeded by detection root[j].
 * Integer decisions on FP64 inputs, no rounding: equal inputs give equal
 * outputs on any device.  DQO_EINVAL for negative sizes, n_det > 32768,
 * non-finite thresholds or missing buffers. */
int dqo_associate_decide(const dqo_ctx* ctx, int64_t n_det, int32_t n_obj, const int32_t* match, const double* qd_obs,
                         const double* occ, const double* qd_det, const int32_t* label, double qd_min, double t_occ,
                         double qd_occ, int32_t* fine, int32_t* parent, int32_t* root, int32_t* obj, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* DQO_H */
