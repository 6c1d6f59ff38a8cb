/*
 * gslic.h - C ABI of the MI355X (gfx950) mapping step of a 3D Gaussian map.
 *
 * Method: Gaussian-LIC (arXiv 2404.06926). A map of anisotropic 3D Gaussians (Sec. III-A)
 * is optimised online from posed keyframes (Sec. III-C): every step projects the
 * Gaussians (Eq. 1-3), bins them into 16x16 tiles with a depth-ordered key sort, blends
 * front to back (Eq. 4-5) with a per-keyframe 3x4 exposure affine (Sec. III-C.3), takes
 * the L1 + D-SSIM loss (Eq. 9), back-propagates, and applies sparse Adam to the Gaussians
 * seen in the step (Sec. III-D.2). New points become Gaussians by the rule of
 * Sec. III-C.1.
 *
 * Conventions shared by every call
 *   - All pointers named "device" are HIP device pointers; all other pointers are host.
 *     Nothing is copied between host and device implicitly except the small per-view
 *     parameters carried in gs_view (passed by value to the kernels).
 *   - Every call that takes a `stream` (a hipStream_t, NULL = default stream) only
 *     enqueues work and returns; results are ready when the stream reaches that point.
 *   - Return value: GS_OK (0) or a negative gs_status. On a validation error nothing is
 *     enqueued and the map is unchanged; gs_last_error() describes the failure
 *     (thread-local, valid until the next call on the same thread).
 *   - A map is used from one host thread and one stream at a time. Different maps are
 *     independent. No C++ exception crosses this ABI.
 *   - Gaussian parameters are stored as planes (structure of arrays) of FP32:
 *       plane 0..2   mean (world frame)
 *       plane 3..5   log-scale            (scale = exp)
 *       plane 6..9   quaternion w, x, y, z (normalised when used)
 *       plane 10     opacity logit        (opacity = sigmoid)
 *       plane 11+3k+c  SH coefficient k (k < (deg+1)^2) of colour channel c
 *     Plane f of a buffer starts at base + f * capacity.
 */
#ifndef GSLIC_H
#define GSLIC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gs_map gs_map; /* opaque */
typedef int32_t gs_status;

enum {
  GS_OK = 0,
  GS_ERR_INVALID = -1,       /* bad argument; nothing enqueued */
  GS_ERR_OOM = -2,           /* an allocation failed; map unchanged */
  GS_ERR_HIP = -3,           /* a HIP runtime call failed */
  GS_ERR_CAPACITY = -4,      /* a fixed capacity (views per call, instances, 2^30 Gaussians) is exceeded */
  GS_ERR_STATE = -6,         /* call order violated (e.g. backward without a render) */
  GS_ERR_UNIMPLEMENTED = -7
};

enum { GS_MAX_VIEWS = 16, GS_TILE = 16, GS_EXPOSURE_STATE_FLOATS = 48 };

/* Optional device-memory provider. alloc returns a device pointer of at least `bytes`
 * bytes (256-byte aligned) usable on `stream`, or NULL; free releases it. When the
 * allocator passed to gs_create_map is NULL, the library calls hipMalloc / hipFree. */
typedef struct {
  void* (*alloc)(size_t bytes, void* stream, void* ctx);
  void (*free)(void* ptr, void* stream, void* ctx);
  void* ctx;
} gs_allocator;

/* Map hyper-parameters. Learning rates are per parameter group (Sec. IV-A.1: vanilla
 * 3DGS rates, not decayed). */
typedef struct {
  int32_t sh_degree;         /* 0..3 (the paper uses 3, Sec. III-A) */
  int64_t initial_capacity;  /* Gaussians; grows by doubling */
  float near_z;              /* cull depth <= near_z (camera frame); 0.2 */
  float lr_mean, lr_log_scale, lr_quat, lr_opacity, lr_sh_dc, lr_sh_rest, lr_exposure;
  float beta1, beta2, eps;   /* Adam */
  float expand_tau;          /* keyframe expansion threshold tau of Eq. 8 (0.99, Sec. IV-A.1);
                                <= 0 appends every point of a keyframe */
} gs_map_desc;

/* One camera of a step. The pose maps world points into the camera frame
 * (x_c = R_cw x_w + t_cw; camera x right, y down, z forward), Sec. III-A Eq. 2.
 * Pixel (u, v) is sampled at its centre (u + 0.5, v + 0.5). */
typedef struct {
  float R_cw[9];             /* row-major */
  float t_cw[3];
  float fx, fy, cx, cy;      /* pinhole intrinsics in pixels */
  int32_t width, height;     /* pixels, 1..16384 each */
  float bg[3];               /* background colour added behind the Gaussians */
  const float* exposure;     /* device float[12]: 3x4 [A | b] row-major; out = A c + b
                                (Sec. III-C.3). NULL = identity. Read by gs_render and by
                                the gs_render_backward that follows: keep it valid until then. */
} gs_view;

/* Per-view outputs of gs_render (all device, caller-owned, H*W pixels).
 *   rgb       float[3][H][W]  exposed colour, required
 *   final_T   float[H][W]     transmittance after the last contributor (1 - opacity map,
 *                             Eq. 7); NULL = kept inside the map's workspace
 *   n_contrib uint32[H][W]    list position after the last contributing Gaussian of the
 *                             pixel's tile list; NULL = kept inside the workspace
 *   depth     float[H][W]     depth map D = sum_i d_i a_i T_i, d_i the Gaussian's
 *                             camera-frame depth (Sec. III-A Eq. 6); NULL = not computed
 *   opacity   float[H][W]     opacity map O = sum_i a_i T_i = 1 - final_T (Eq. 7);
 *                             NULL = not computed
 * When given, final_T and n_contrib must stay alive until gs_render_backward. */
typedef struct {
  float* rgb;
  float* final_T;
  uint32_t* n_contrib;
  float* depth;
  float* opacity;
} gs_frame;

/* Defaults: SH 3, near 0.2, 3DGS learning rates, Adam (0.9, 0.999, 1e-15). */
void gs_default_desc(gs_map_desc* desc);

/* Create an empty map. `allocator` may be NULL (hipMalloc); it is copied. */
gs_status gs_create_map(const gs_map_desc* desc, const gs_allocator* allocator, gs_map** out);

/* Release every buffer of the map (synchronises the device first). NULL is a no-op. */
gs_status gs_destroy_map(gs_map* map);

/* Append n Gaussians (Sec. III-C.1 parameters, already in parameter space).
 * Inputs are device arrays in rows: means n x 3, log_scales n x 3, quats n x 4 (w,x,y,z),
 * opacity_logits n, sh n x K x 3 (K = (deg+1)^2, coefficient-major). Gradients and Adam
 * moments of the new rows start at zero. Capacity doubles as needed (device copy on
 * `stream`), up to 2^30 Gaussians (GS_ERR_CAPACITY beyond). n = 0 is a no-op. */
gs_status gs_add_gaussians(gs_map* map, int64_t n, const float* means, const float* log_scales,
                           const float* quats, const float* opacity_logits, const float* sh,
                           void* stream);

/* Initialise Gaussians from coloured points as in Sec. III-C.1: centre = point, SH DC
 * chosen so the colour renders as `rgb`, other SH 0, opacity o_init, rotation identity,
 * isotropic scale d / f where d is the point's depth in `view` and f = view.fx.
 * xyz, rgb: device n x 3. Points with depth <= near_z get scale near_z / f. */
gs_status gs_add_points(gs_map* map, int64_t n, const float* xyz, const float* rgb,
                        const gs_view* view, float o_init, void* stream);

/* Map expansion (Sec. III-C.2, Eq. 8): render the opacity map O of the current map at
 * `view`, keep the points (device xyz, rgb: n_points x 3) whose projection falls inside
 * the image on a pixel with O < tau, and append them in input order as Gaussians by the
 * Sec. III-C.1 rule (as gs_add_points). The pixel of a point is decided in FP32:
 * x_c = ((R00 x + R01 y) + R02 z) + t0 (likewise y_c, z_c), u = f_x (x_c / z_c) + c_x,
 * v likewise; inside when z_c > near_z, 0 <= u < width, 0 <= v < height; pixel =
 * (floor u, floor v). *n_added (host, may be NULL) receives the number appended; the call
 * waits for the stream to read it. The render replaces the map's last render (a
 * gs_render_backward cannot follow). GS_ERR_INVALID for tau <= 0 or o_init outside (0, 1). */
gs_status gs_expand(gs_map* map, const gs_view* view, int64_t n_points, const float* xyz, const float* rgb,
                    float tau, float o_init, int64_t* n_added, void* stream);

/* Sky Gaussians (Sec. III-C.1): one Gaussian at each of the n >= 2 device positions xyz
 * (n x 3; the caller draws them, e.g. on the upper hemisphere of radius R), white SH DC,
 * opacity o_sky, identity rotation, isotropic scale = distance to the closest other of
 * these positions (brute force on the device). */
gs_status gs_add_sky(gs_map* map, int64_t n, const float* xyz, float o_sky, void* stream);

/* Forward pass over n_views views of the same map in one batch (Sec. III-A Eq. 1-5,
 * Sec. III-C.3 exposure, Sec. III-D.2 tile culling). Tiles of all views are numbered
 * consecutively and processed by the same launches. Saves what gs_render_backward needs. */
gs_status gs_render(gs_map* map, int32_t n_views, const gs_view* views, const gs_frame* frames,
                    void* stream);

/* Reverse pass of the immediately preceding gs_render on this map (same n_views).
 * dL_drgb[v]: device float[3][H][W]. dL_ddepth[v], dL_dopacity[v]: device float[H][W]
 * gradients of the depth and opacity maps (Eq. 6-7); the arrays or any entry may be NULL
 * (no gradient through that map). dL_dexposure[v]: device float[12] that receives
 * (+=) dL/d[A|b]; the array or any entry may be NULL. Parameter gradients are added to
 * the map's gradient planes (they accumulate until gs_adam_step) and the Gaussians seen
 * by any view are marked for the next sparse Adam step. GS_ERR_STATE without a render. */
gs_status gs_render_backward(gs_map* map, int32_t n_views, const float* const* dL_drgb,
                             const float* const* dL_ddepth, const float* const* dL_dopacity,
                             float* const* dL_dexposure, void* stream);

/* One sparse Adam step (Sec. III-D.2, Sec. IV-A.1): rows marked since the last step move,
 * other rows keep parameters and moments bit-identical; gradients of moved rows are
 * cleared. The step count t is kept on the device (bias correction 1 - beta^t).
 * exposure_states[e]: device float[48] = exposure [A|b] (12), its gradient (12), Adam m
 * (12), Adam v (12); each is updated with lr_exposure and its gradient cleared. */
gs_status gs_adam_step(gs_map* map, int32_t n_exposures, float* const* exposure_states,
                       void* stream);

/* Eq. 9 loss between out and gt (device float[3][H][W] each):
 *   L = (1 - lambda) mean|out - gt| + lambda (1 - mean SSIM(out, gt)),
 * SSIM per channel with an 11x11 Gaussian window (sigma 1.5), C1 = 1e-4, C2 = 9e-4 and
 * zero padding. Writes L to loss_dev (device float[1]) and dL/dout to dL_dout (device,
 * same shape; may alias nothing). Uses the map's workspace. */
gs_status gs_loss(gs_map* map, const float* out, const float* gt, int32_t height, int32_t width,
                  float lambda, float* loss_dev, float* dL_dout, void* stream);

/* gs_loss for callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): the same kernels and the same
 * results as gs_loss, with no map and no allocation. Its per-tile partial sums live in a
 * fixed device array of GS_LOSS_NOALLOC_SCRATCH_FLOATS floats (about 128 KiB, one copy per
 * GPU, held until the process ends), enough for images of up to 16384 output tiles of
 * 32x32 pixels (e.g. 4096 x 4096); larger images return GS_ERR_CAPACITY and enqueue
 * nothing. Arguments, layout and results are those of gs_loss. Every call on one GPU
 * shares that GPU's array: calls that overlap on one GPU (different streams, or threads
 * without ordering) race and may return wrong values; calls ordered on one stream are
 * safe. The first call on a device looks the array's address up (no allocation). */
#define GS_LOSS_NOALLOC_SCRATCH_FLOATS 32832
gs_status gs_loss_noalloc(const float* out, const float* gt, int32_t height, int32_t width,
                          float lambda, float* loss_dev, float* dL_dout, void* stream);

/* One mapping job on a keyframe (Sec. III-C): append Gaussians from the keyframe's points
 * (gs_expand with the map's expand_tau, Eq. 8, or gs_add_points when expand_tau <= 0; with
 * o_init), store the keyframe (pose, a copy of `image`, an identity
 * exposure with fresh Adam state) in a window of the `window` most recent keyframes
 * (window <= GS_MAX_VIEWS), then run `iters` steps, each = one batched gs_render over
 * the window, Eq. 9 loss per keyframe, gs_render_backward, gs_adam_step (Gaussians and
 * window exposures). image: device float[3][H][W]; xyz, rgb: device n_points x 3.
 * The steps run without host waits (fused steps): the instance buffers are sized from the
 * map's previous job, scaled to this window with a quarter to spare (a map's first job
 * plans its first render with a wait); a step whose render needs more is skipped on the
 * device and run again after the others with planning, so a job always applies `iters`
 * steps. The call waits once, at the job's end, for the overflow counters (it clears the
 * map's overflow flag). done_event (a hipEvent_t, may be NULL) is recorded on `stream`
 * after the last step. */
gs_status gs_submit_keyframe(gs_map* map, const gs_view* view, const float* image,
                             int64_t n_points, const float* xyz, const float* rgb,
                             int32_t iters, int32_t window, float lambda, float o_init,
                             void* done_event, void* stream);

/* The paper's keyframe schedule (Sec. III-C.3): every keyframe is kept for the session.
 * gs_add_keyframe expands the map with the keyframe's points (as gs_submit_keyframe) and
 * keeps the keyframe (pose, a copy of `image`, an identity exposure with fresh Adam state)
 * under the id written to *keyframe_id (0, 1, 2, ... in call order).
 * gs_optimize_keyframes runs one mapping step (gs_step over that single keyframe: render,
 * Eq. 9 loss, backward, Adam over the Gaussians and that keyframe's exposure) per entry of
 * ids, sequentially in the given order. The selection of K keyframes and their shuffle
 * are the caller's random draws, passed in as ids. done_event (hipEvent_t, may be NULL) is
 * recorded after the last step. gs_keyframe_count reports how many are kept. */
gs_status gs_add_keyframe(gs_map* map, const gs_view* view, const float* image, int64_t n_points,
                          const float* xyz, const float* rgb, float o_init, int32_t* keyframe_id,
                          void* stream);
/* Frame intake of Sec. III-C.2. Every frame brings a pose, its image and its coloured
 * points (device xyz, rgb: n_points x 3). The first frame bootstraps the map with all of
 * its points (Sec. III-C.1 initialisation, as gs_add_points). Frames 0, 5, 10, ... are
 * keyframes: at each keyframe after the first, the points of the five frames since the
 * previous keyframe (the four before it and its own), merged in arrival order, go through
 * the opacity mask of the keyframe's view (Eq. 8, tau = the map's expand_tau; as
 * gs_expand), and the keyframe is kept as by gs_add_keyframe. Points of other frames are
 * held on the device until then (their image may be NULL and is not kept).
 * *keyframe_id (may be NULL) receives the keyframe's id, or -1 for other frames.
 * GS_ERR_INVALID for a keyframe without an image or o_init outside (0, 1). */
gs_status gs_add_frame(gs_map* map, const gs_view* view, const float* image, int64_t n_points,
                       const float* xyz, const float* rgb, float o_init, int32_t* keyframe_id,
                       void* stream);
gs_status gs_optimize_keyframes(gs_map* map, int32_t n, const int32_t* ids, float lambda,
                                void* done_event, void* stream);
gs_status gs_keyframe_count(gs_map* map, int32_t* count);
/* Device pointer to kept keyframe `id`'s exposure state float[48] = exposure [A|b] (12),
 * its gradient (12), Adam m (12), Adam v (12) (Sec. III-C.3), owned by the map and valid
 * until it is destroyed. GS_ERR_INVALID for an unknown id. */
gs_status gs_keyframe_state(gs_map* map, int32_t id, float** state);

/* One mapping step over n_views keyframes of one map (Sec. III-C.3): one batched
 * gs_render, the Eq. 9 loss of every view against targets[v] (device float[3][H][W]),
 * gs_render_backward, and gs_adam_step over the Gaussians and the views' exposures.
 * exposure_states[v] (device float[48], see gs_adam_step) supplies the exposure of view v
 * (it replaces views[v].exposure) and receives its gradient; frames[v] receive the
 * renders; dl_drgb[v] (device float[3][H][W]) holds the image gradient; loss_dev (device
 * float[n_views]) receives each view's loss. */
gs_status gs_step(gs_map* map, int32_t n_views, const gs_view* views, const gs_frame* frames,
                  const float* const* targets, float lambda, float* const* exposure_states,
                  float* const* dl_drgb, float* loss_dev, void* stream);

/* gs_step runs the projection backward and the Adam update of each Gaussian row in one
 * kernel (enable = 1, the default): the step's gradient is complete after its backward,
 * so the gradient planes are neither written nor read back; gradients accumulated by
 * earlier gs_render_backward calls are included and cleared as gs_adam_step would.
 * enable = 0 runs gs_render_backward then gs_adam_step. Both give the same update. */
gs_status gs_set_fused_step(gs_map* map, int32_t enable);

/* A captured mapping step (HIP graph). gs_capture_step records the kernels gs_step would
 * enqueue, with the same arguments, into a graph without running them. Requirements: the
 * map's instance policy has sync_plan = 0 (no host wait inside the step), and an eager
 * gs_step with the same views has sized the workspace (capture never allocates; it fails
 * with GS_ERR_STATE otherwise). Every pointer passed is baked into the graph and must stay
 * valid while it is used; the map must not grow. gs_launch_step returns GS_ERR_STATE, and
 * launches nothing, once the map's row count or capacity has changed or any of its device
 * buffers has been reallocated since the capture (capture again then). Each gs_launch_step
 * performs one more step (the Adam step count lives on the device). A step captured while the gradient
 * planes were known to be zero skips reading them; gs_launch_step then returns
 * GS_ERR_STATE if they may hold values again (gs_render_backward or gs_map_params since). */
typedef struct gs_step_graph gs_step_graph;
gs_status gs_capture_step(gs_map* map, int32_t n_views, const gs_view* views, const gs_frame* frames,
                          const float* const* targets, float lambda, float* const* exposure_states,
                          float* const* dl_drgb, float* loss_dev, void* stream, gs_step_graph** out);
gs_status gs_launch_step(gs_step_graph* graph, void* stream);
gs_status gs_destroy_step(gs_step_graph* graph);

/* Thread-local description of the last failure on this thread ("" if none). */
const char* gs_last_error(void);

/* Size and memory: live Gaussians, capacity, bytes the map holds (parameters, gradients,
 * moments, workspace). Host-side values; never synchronises. */
gs_status gs_map_info(const gs_map* map, int64_t* n, int64_t* capacity, int64_t* resident_bytes);

/* Device pointers to plane 0 of the parameter, gradient and Adam m / v buffers, and the
 * plane stride (= capacity). Valid until the map grows or is destroyed. Any may be NULL.
 * Asking for the gradient pointer tells the map its gradient planes may be written: the
 * next fused step reads them (otherwise it skips that read while they are known zero). */
gs_status gs_map_params(gs_map* map, float** params, float** grads, float** adam_m, float** adam_v,
                        int64_t* plane_stride);

/* Device pointer to the per-Gaussian "seen since the last Adam step" flags (uint8[n]). */
gs_status gs_map_visibility(gs_map* map, uint8_t** vis);

/* Number of renders of this map so far: gs_render calls, including those inside gs_step,
 * keyframe jobs, expansion and replays of a captured step. A caller that keeps a render's
 * outputs for a later gs_render_backward (an autograd graph) compares it before the
 * backward: the backward always pairs with the most recent render. Host-side value. */
gs_status gs_map_render_generation(const gs_map* map, int64_t* generation);

/* Number of Adam steps taken (host mirror of the device counter). */
gs_status gs_map_step_count(const gs_map* map, int64_t* t);

/* Sets the Adam step counter t (Sec. III-D.2: the bias corrections 1 - beta^t of the next
 * step use t + 1), on `stream`, as a checkpoint restore of parameters and moments needs.
 * t < 0 or a NULL map: GS_ERR_INVALID. Ordered on `stream` like the steps around it. */
gs_status gs_map_set_step_count(gs_map* map, int64_t t, void* stream);

/* Device views of the last gs_render's intermediate results, valid until the next render:
 *   tiles     uint32[n_inst]  global tile id of each instance, in blend order (tile, then
 *                             depth, then Gaussian index); the sort key of instance k is
 *                             tiles[k] << 32 | float bits of its Gaussian's depth
 *   vals      uint32[n_inst]  Gaussian index of each instance
 *   ranges    uint32[2 * n_tiles] [start, end) of each global tile in the sorted list
 *   proj      float[16 * n_views * n]  per (view, Gaussian) record, view-major:
 *             mean2d x, y, conic A, B, C, opacity, colour r, g, b, depth, unused,
 *             2 ln(255 opacity), tile rectangle x0 | y0 << 16 and x1 | y1 << 16 (uint32
 *             bits), 2 unused; written only where the tile count is > 0
 *   counts    uint32[n_views * n]  tiles reached by each (view, Gaussian), view-major
 * n_inst is read back from the device (this call synchronises `stream`). */
gs_status gs_debug_last_render(gs_map* map, void* stream, const uint32_t** tiles,
                               const uint32_t** vals, int64_t* n_inst, const uint32_t** ranges,
                               int64_t* n_tiles, const float** proj, const uint32_t** counts);

/* Instance-buffer policy. sync_plan = 1 (default): gs_render reads the instance count back
 * after binning and grows the buffers to fit (one host wait per render). sync_plan = 0:
 * no host wait inside gs_render (a graph-capturable sequence); a render that needs more
 * than `capacity` instances drops them all (its images hold only the background, and its
 * gs_render_backward adds no gradient) and is flagged, to be checked with
 * gs_check_overflow. A fused step (gs_step, gs_launch_step)
 * whose render dropped instances is skipped: the parameters, their Adam moments, the
 * exposures and the Adam step count are left as they were (its loss value is not
 * meaningful). */
gs_status gs_set_instance_policy(gs_map* map, int32_t sync_plan, int64_t capacity);

/* Synchronise `stream` and report whether any render since the last check dropped
 * instances (1) or not (0); clears the flag. After skipped fused steps the map's step
 * count (gs_map_step_count) follows the device's again. */
gs_status gs_check_overflow(gs_map* map, void* stream, int32_t* overflow);

/* Per-stage GPU timing. With timing enabled, every stage of the calls below records a
 * pair of HIP events on the call's stream around its kernels. gs_stage_times synchronises
 * `stream`, writes the summed milliseconds and the number of timed launches of each stage
 * since the previous query into ms[GS_NUM_STAGES] and count[GS_NUM_STAGES], and resets.
 * Stage order: GS_STAGE_* below. */
enum {
  GS_STAGE_PROJECT = 0,       /* per-Gaussian projection and tile count */
  GS_STAGE_SCAN = 1,          /* exclusive scan of tile counts in depth order */
  GS_STAGE_DUPLICATE = 2,     /* tile id of every instance, emitted in depth order */
  GS_STAGE_SORT = 3,          /* stable radix sort of the instances by tile */
  GS_STAGE_RANGES = 4,        /* per-tile [start, end) */
  GS_STAGE_BLEND = 5,         /* forward blend */
  GS_STAGE_LOSS = 6,          /* L1 + D-SSIM and its gradient */
  GS_STAGE_BLEND_BACKWARD = 7,
  GS_STAGE_PROJECT_BACKWARD = 8,
  GS_STAGE_ADAM = 9,
  GS_STAGE_DEPTH_SORT = 10,   /* radix sort of (view, Gaussian) pairs by depth */
  GS_NUM_STAGES = 11
};
gs_status gs_set_stage_timing(gs_map* map, int32_t enable);
gs_status gs_stage_times(gs_map* map, void* stream, double* ms, int64_t* count);

/* Deterministic backward (enable = 1): the backward blend writes every instance's
 * gradient to its own record with a fixed-order reduction over the tile's waves, and the
 * projection backward adds a Gaussian's records in emission order; the exposure gradient
 * is reduced over tiles in tile order. Results then do not depend on scheduling (bit-equal
 * across runs and concurrent work), at the cost of 48 B per instance and extra traffic.
 * Default 0: wave-reduced float atomics. Takes effect from the next gs_render. */
gs_status gs_set_deterministic(gs_map* map, int32_t enable);

/* Parallelisation of the backward blend. mode 0 (default): pixel order, lanes own pixels
 * and walk their lists back to front, per-Gaussian terms summed across the wave. mode 1:
 * per Gaussian (Sec. III-D.1), lanes own a tile's list entries and walk its pixels, with
 * suffix products and sums across lanes for the transmittance in front of each entry and
 * the colour behind it. Gradients of the depth and opacity maps always use mode 0. Takes
 * effect from the next gs_render. */
gs_status gs_set_backward_mode(gs_map* map, int32_t mode);

/* Launch configuration of the blend kernels: pixels per lane in the forward and backward
 * (1, 2 or 4; default 1 and 1). With p pixels per lane a tile is processed by 256 / p
 * lanes and each list entry's LDS reads and gradient reductions are shared by p pixels.
 * Results do not depend on it beyond FP32 summation order. */
gs_status gs_set_blend_config(gs_map* map, int32_t fwd_px_per_lane, int32_t bwd_px_per_lane);

/* Long tile lists (Sec. III-A: every tile blends its depth-sorted list front to back).
 * A tile whose list holds more than `balance` times the mean list length and more than
 * L = max(min_chunk, ceil(instances / parallel)) entries (L rounded up to a multiple of
 * 64) is blended by ceil(n / L) workgroups, each over one of as many near-equal chunks
 * of the list, and the chunks are composited in depth order; the backward walks the same
 * chunks in parallel.
 * With that L at most `parallel` tiles are split and the extra workgroups number at most
 * `parallel`. parallel = 0 blends every tile in one workgroup; balance = 0 drops the
 * comparison with the mean. Default: parallel 4096, min_chunk 128, balance 1.25. Results
 * differ from the unsplit blend by FP32 summation order only (and, where a pixel's
 * transmittance meets the stop threshold within rounding, by where it stops). Device
 * memory: about 14 KiB per unit of `parallel`. The next gs_render_backward needs a
 * gs_render after this call.
 * Errors: GS_ERR_INVALID for parallel outside [0, 65536], min_chunk outside [1, 2^24] or
 * balance outside [0, 1e6]; GS_ERR_STATE while capturing. */
gs_status gs_set_tile_split(gs_map* map, int32_t parallel, int32_t min_chunk, float balance);

#ifdef __cplusplus
}
#endif
#endif /* GSLIC_H */
