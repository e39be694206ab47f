/*
 * isogs — differentiable tile rasterizer of 3-D Gaussians for isosurface
 * visualization, native to AMD Instinct MI355X (gfx950).
 *
 * The paper ("Toward Distributed 3D Gaussian Splatting for High-Resolution
 * Isosurface Visualization", Sec. III) initialises 3D-GS primitives from
 * isosurface points, generates synthetic views on a structured orbit and
 * trains the 3D-GS model to match them.  This C ABI exposes that training
 * path as calls on plain pointers and sizes: orbit cameras, initialisation
 * from points, render (forward), loss gradient, render backward and the Adam
 * step, plus a batched hipGraph step, an autotuner and a render server.
 *
 * Conventions shared by every call
 *  - Pointers documented as "device" point to HIP device memory on the
 *    context's device; "host" pointers to ordinary host memory.
 *  - Parameter, gradient and optimiser-state arrays are structure-of-arrays,
 *    float32, owned by the caller:
 *        means[3][n], log_scales[3][n], quats[4][n] (w, x, y, z),
 *        opacity_logits[n], sh[(d+1)^2 * 3][n] with row index j*3 + c.
 *  - Images are planar float32 [3][height][width], owned by the caller.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Device work is enqueued on it asynchronously unless stated otherwise.
 *  - Every call returns a gs_status; none throws.  On failure the calling
 *    thread's gs_last_error() describes the cause.  HIP runtime failures map
 *    to GS_ERR_HIP, capacity overruns to GS_ERR_CAPACITY.
 *  - Objects created by the library (contexts, frames, graphs, servers) are
 *    owned by it and freed by their *_destroy / *_release call.
 *  - Some calls keep scratch in the context (noted at each: the loss
 *    workspace, the densify and extraction block totals and read-backs, the
 *    host-point copy); such calls on one context must not overlap.  A frame
 *    is used by one call at a time.
 */
#ifndef ISOGS_H
#define ISOGS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  GS_OK = 0,
  GS_ERR_INVALID = -1,     /* bad argument (null pointer, size out of range) */
  GS_ERR_NOMEM = -2,       /* device memory or the context budget exhausted */
  GS_ERR_HIP = -3,         /* a HIP runtime call failed */
  GS_ERR_CAPACITY = -4,    /* more (Gaussian, tile) records than fit: a frame holds at
                              most 2^32 - 2^20 records and as many (view, Gaussian)
                              entries */
  GS_ERR_UNSUPPORTED = -5, /* device is not gfx950, or option not supported */
  GS_ERR_BUSY = -6         /* object in use (server queue full, ...) */
} gs_status;

typedef struct gs_ctx gs_ctx;
typedef struct gs_frame gs_frame;
typedef struct gs_graph gs_graph;
typedef struct gs_server gs_server;

/* Gaussian parameters (or gradients, or Adam moments) of one scene: device
 * pointers into caller-owned SoA float32 arrays (layout above).  n >= 1,
 * sh_degree in 0..3. */
typedef struct {
  float* means;
  float* log_scales;
  float* quats;
  float* opacity_logits;
  float* sh;
  int64_t n;
  int32_t sh_degree;
  int32_t reserved;
} gs_params;

/* Pinhole camera.  R is the row-major world->camera rotation and t the
 * translation (p_cam = R p + t); camera axes x right, y down, z forward.
 * fx, fy, cx, cy in pixels; pixel (x, y) is sampled at (x + 0.5, y + 0.5).
 * Gaussians with camera depth <= z_near are culled.  width, height in
 * [1, 16384]. */
typedef struct {
  float R[9];
  float t[3];
  float fx, fy, cx, cy;
  float z_near;
  int32_t width, height;
  int32_t reserved;
} gs_camera;

/* Render options.  tile in {8, 16, 32} (pixels per tile side); lds_depth in
 * {32, 64, 128, 256} (Gaussians staged in LDS per batch; 0 = default 256,
 * clipped to the tile's pixel count for tile 8); bg = background colour;
 * flags: GS_RENDER_PERSISTENT blends all views' tiles with one persistent
 * launch (a resident grid draining a work queue), GS_RENDER_LONGEST_FIRST
 * orders that queue by descending tile list length (to within 1/16 of an
 * octave).  Results do not depend on the flags.  GS_RENDER_RADII also keeps
 * every (view, Gaussian)'s integer pixel radius in the frame (0 where the
 * Gaussian touches no tile), which gs_density_accumulate reads. */
enum { GS_RENDER_PERSISTENT = 1, GS_RENDER_LONGEST_FIRST = 2, GS_RENDER_RADII = 4 };
typedef struct {
  int32_t tile;
  int32_t lds_depth;
  float bg[3];
  int32_t flags;
} gs_render_opts;

/* Adam hyper-parameters; learning rate per parameter group. */
typedef struct {
  float lr_means, lr_log_scales, lr_quats, lr_opacity, lr_sh_dc, lr_sh_rest;
  float beta1, beta2, eps;
  int32_t zero_grads; /* nonzero: gradients are cleared after use */
} gs_adam_opts;

/* Initialisation from isosurface points (Sec. III: the point cloud
 * initialises the Gaussian primitives).  Log-scales are log_scale +
 * U(-log_scale_jitter, +log_scale_jitter) per axis when log_scale_lo >=
 * log_scale_hi, else U(log_scale_lo, log_scale_hi); quaternions are the
 * identity or uniformly random; opacity logits constant; SH coefficients
 * N(0, sh_std) (0 = all zero).  Random draws use Philox4x32-10 keyed by the
 * seed with counter (Gaussian index, stream id, 0, 0). */
typedef struct {
  float log_scale;
  float log_scale_jitter;
  float log_scale_lo, log_scale_hi;
  int32_t random_quats;
  float opacity_logit;
  float sh_std;
  int32_t reserved;
} gs_init_opts;

/* Per-frame figures, read back to the host. */
typedef struct {
  int32_t n_views;
  int32_t tile;
  int64_t n_gaussians;
  int64_t n_records;        /* K: (Gaussian, tile) records over all views */
  int64_t n_visible;        /* (view, Gaussian) pairs touching >= 1 tile (after a step
                               graph replay: that replay's, once gs_step_graph_sync ran) */
  int64_t n_tiles;          /* tiles over all views */
  int64_t n_pixels;         /* pixels over all views */
  int64_t device_bytes;     /* device memory held by the frame */
} gs_frame_stats;

/* What gs_frame_export copies out (device -> caller's device buffer). */
typedef enum {
  GS_EXPORT_KEYS = 0,       /* uint64[K]: (global tile << 32) | float32 depth bits, sorted */
  GS_EXPORT_VALUES = 1,     /* uint32[K]: view * n + Gaussian index, same order */
  GS_EXPORT_RANGES = 2,     /* uint32[n_tiles][2]: [start, end) per global tile */
  GS_EXPORT_FINAL_T = 3,    /* float[n_pixels]: transmittance left after blending */
  GS_EXPORT_N_CONTRIB = 4,  /* uint32[n_pixels]: position + 1 of the last contributor */
  GS_EXPORT_SCREEN_GRADS = 5, /* float[n_views][n][12]: dL/d(m_x, m_y, A, B, C, opacity, r, g, b), 3 pad */
  GS_EXPORT_SPLATS = 6,     /* float[n_views][n][12]: conic A, B, C, opacity; floor(mean x),
                               floor(mean y) as int32 bits, 0.5 - frac(mean x), 0.5 - frac(mean y);
                               r, g, b; half-widths of the conservative alpha >= 1/255 box as two
                               fp16 (x in the low 16 bits, y in the high; negative when the splat
                               can never pass the alpha test).  Only touched entries are defined. */
  GS_EXPORT_RECTS = 7,      /* uint32[n_views][n][2]: tile x0 | y0 << 16, x1 | y1 << 16
                               (x1 < x0 when the Gaussian touches no tile) */
  GS_EXPORT_DEPTHS = 8      /* uint32[n_views][n]: float32 camera depth bits of touched entries,
                               0xffffffff for untouched */
} gs_export;

/* ------------------------------------------------------------------ core */

/* Description of the calling thread's last failure (library-owned string,
 * valid until the thread's next failing call). */
const char* gs_last_error(void);

/* Library version string, e.g. "isogs 0.1 gfx950". */
const char* gs_version(void);

/* Create a context on HIP device `device`.  mem_budget caps the device
 * memory the library allocates for its own scratch (0 = no cap).  Fails with
 * GS_ERR_UNSUPPORTED on a device that is not gfx950. */
gs_status gs_ctx_create(int device, size_t mem_budget, gs_ctx** out);
/* Destroy a context.  Frames, step graphs and render servers created on it hold
 * it: while any of them is alive the call only marks the context, and its last
 * release (gs_frame_release, gs_step_graph_destroy, gs_server_destroy) frees it.
 * No other call may use the context after this one. */
void gs_ctx_destroy(gs_ctx* ctx);
/* Bytes of device scratch currently held by the context and its frames. */
gs_status gs_ctx_memory(gs_ctx* ctx, size_t* in_use, size_t* peak);

/* Stage timing.  When enabled, every pipeline stage the context launches is
 * bracketed by HIP events on its stream (the events add no work to the
 * kernels).  Enabling or disabling resets the totals.  gs_ctx_stage_time
 * waits for the recorded events and returns the summed duration (ms) and the
 * number of timed launches of one stage; gs_stage_name gives the stage's name
 * ("project", "depth_sort", "scan", "emit", "tile_sort", "ranges",
 * "blend_fwd", "loss", "blend_bwd", "project_bwd", "adam", "init", "probe") or NULL
 * past the last stage. */
gs_status gs_ctx_set_timing(gs_ctx* ctx, int32_t enable);
gs_status gs_ctx_stage_time(gs_ctx* ctx, int32_t stage, double* total_ms, int64_t* launches);
const char* gs_stage_name(int32_t stage);

/* Structured orbit of look-at views (Sec. III: synthetic views "in a
 * structured orbit"; Sec. IV: 448 views per dataset).  View i of n sits on a
 * Fibonacci sphere of the given radius at height y = 1 - 2 (i + 0.5) / n and
 * azimuth i * pi * (3 - sqrt 5), looking at the origin, world up +y (+z when
 * |y| > 0.99); focal length from the vertical field of view, square pixels,
 * principal point at the image centre, z_near 0.2.  Host only; `out` is a
 * caller-owned host array of n_views cameras. */
gs_status gs_orbit_cameras(int32_t n_views, float radius, float fov_y_deg,
                           int32_t width, int32_t height, gs_camera* out);

/* Gaussians from isosurface points (Sec. III).  xyz: float32 [3][n] point
 * coordinates in device or host memory; host points are copied to a context
 * buffer and the call then synchronises `stream` (the array may be reused on
 * return), device points are read by the kernel (asynchronous).  Writes every
 * array of `out` (device, caller-owned, sized for n and out.sh_degree):
 * means = points, the rest per `opts`.  Calls that share a context and pass
 * host points must not overlap. */
gs_status gs_init_from_points(gs_ctx* ctx, const float* xyz, int64_t n,
                              const gs_init_opts* opts, uint64_t seed,
                              gs_params out, void* stream);

/* Forward render of n_views views (1..16) of one scene: EWA projection and
 * SH colour, tile binning and sort, front-to-back compositing.  This is the
 * differentiable renderer of the 3D-GS model that Sec. III (Method Overview)
 * trains to match the orbit views; the paper adopts it by citation (Sec. I,
 * III) without restating it, so the readings of the projection, colour and
 * compositing conventions are those of the standard 3D-GS rasterizer.  images[v]
 * (device, [3][H_v][W_v]) receives view v.  `*state` receives the frame that
 * the backward pass needs; pass a previous frame to reuse its memory, or
 * NULL to create one (release with gs_frame_release).  The record count is
 * read back to size the sort, so this call synchronises `stream` once. */
gs_status gs_render_fwd(gs_ctx* ctx, gs_params params, const gs_camera* cams,
                        int32_t n_views, float* const* images,
                        const gs_render_opts* opts, gs_frame** state,
                        void* stream);

/* Forward render of n_views views (1..16) each of its own scene: params[v]
 * (device SoA, caller-owned) is the scene of view v; views of the same scene
 * (same parameter pointers) share one projection launch, and all views share
 * one depth sort, one tile sort and one compositing launch.  Every view's
 * image is bit-identical to rendering it alone (a view's tiles hold only its
 * own records, in the same order).  For serving several resident scenes:
 * forward only (gs_render_bwd, gs_density_accumulate and the per-(view,
 * Gaussian) exports of such a frame return GS_ERR_UNSUPPORTED).  Inside the
 * frame the views are grouped by scene (scenes in order of first
 * appearance); the per-pixel exports follow that order.  opts->flags: only
 * GS_RENDER_PERSISTENT and GS_RENDER_LONGEST_FIRST.  Synchronises `stream`
 * once, as gs_render_fwd. */
gs_status gs_render_fwd_multi(gs_ctx* ctx, const gs_params* params, const gs_camera* cams,
                              int32_t n_views, float* const* images,
                              const gs_render_opts* opts, gs_frame** state, void* stream);

/* Training loss of n_views rendered images against targets and its image
 * gradient: mean over views of (1 - lambda) L1 + lambda (1 - SSIM), SSIM with
 * an 11x11 Gaussian window (sigma 1.5), C1 = 1e-4, C2 = 9e-4, zero padding.
 * The objective with which the splatting model "is trained to match these
 * views" (Sec. III); its form is the 3D-GS training loss, which the paper
 * uses without stating it (SSIM is also one of its quality metrics, Sec. IV).
 * loss_out: device float (may be NULL); dl_dimg[v]: device [3][H_v][W_v]
 * (NULL: the loss value only).  The context's loss workspace grows to the
 * largest view seen; calls on one context must not overlap on different
 * streams (they share that workspace). */
gs_status gs_loss_grad(gs_ctx* ctx, const float* const* rendered,
                       const float* const* target, const gs_camera* cams,
                       int32_t n_views, float lambda_dssim, float* loss_out,
                       float* const* dl_dimg, void* stream);

/* gs_loss_grad without allocation, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, kernels and results as gs_loss_grad,
 * but the workspace is a fixed device array of 39,346,176 bytes per GPU,
 * held from the first context created on that GPU until the process ends:
 * each view may hold at most 1,048,576 (2^20) pixels, e.g. 1024 x 1024; larger
 * views return GS_ERR_CAPACITY before anything is launched.  The call
 * allocates nothing (no hipMalloc, hipFree or event creation) and records no
 * stage timing.  Every call on one GPU shares that array (its contents are
 * whatever the last call left; nothing in it needs clearing between calls):
 * calls that overlap on one GPU, on different streams or from different
 * threads, race and give wrong results. */
gs_status gs_loss_grad_noalloc(gs_ctx* ctx, const float* const* rendered,
                               const float* const* target, const gs_camera* cams,
                               int32_t n_views, float lambda_dssim, float* loss_out,
                               float* const* dl_dimg, void* stream);

/* Image-quality metrics of n_views rendered images against references, the
 * quality measures the paper reports for its trained models (PSNR and SSIM,
 * Sec. IV, Tables II-III): out (device float[n_views][4]) receives per view
 * the mean squared error over pixels and channels, PSNR = 10 log10(1 / MSE)
 * (values in [0, 1]; +inf when MSE is 0), the mean absolute error and the
 * mean SSIM (the loss's window and constants).  Sums in float64 in a fixed
 * order (deterministic).  Uses the context's loss workspace, like
 * gs_loss_grad. */
gs_status gs_image_metrics(gs_ctx* ctx, const float* const* rendered,
                           const float* const* reference, const gs_camera* cams,
                           int32_t n_views, float* out, void* stream);

/* Backward of gs_render_fwd for the frame's views (the gradient step of the
 * 3D-GS training adopted in Sec. III): reverse front-to-back traversal that
 * recomputes transmittance (no per-pixel lists are stored), then the chain
 * rule to every parameter.  dl_dimg[v] as above.  grads (device,
 * caller-owned, same shapes as params) receive the gradient summed over the
 * views; flags:
 *   GS_BWD_ACCUMULATE    add to the contents of grads instead of writing them;
 *   GS_BWD_KEEP_SCREEN   leave the per-(view, Gaussian) screen-space sums of
 *                        the traversal in the frame (gs_frame_export
 *                        GS_EXPORT_SCREEN_GRADS); the next gs_render_fwd on
 *                        the frame clears them, and a second backward before it
 *                        fails with GS_ERR_INVALID.
 * Without GS_BWD_KEEP_SCREEN the sums are consumed and cleared, so one
 * forward supports one backward. */
enum { GS_BWD_ACCUMULATE = 1, GS_BWD_KEEP_SCREEN = 2 };
gs_status gs_render_bwd(gs_ctx* ctx, gs_frame* frame, gs_params params,
                        const float* const* dl_dimg, gs_params grads,
                        int32_t flags, void* stream);

/* One fused, bias-corrected Adam step over every parameter group (step
 * counts from 1): the optimiser of the 3D-GS training the paper adopts
 * (Sec. III), applied once per step to the gradient of all views of the step,
 * as after the paper's gradient all-reduce.  p, m, v updated in place; g read
 * (and cleared if opts->zero_grads). */
gs_status gs_adam_step(gs_ctx* ctx, gs_params p, gs_params g, gs_params m,
                       gs_params v, const gs_adam_opts* opts, int64_t step,
                       void* stream);

/* Achievable-bandwidth probe: copy `bytes` (multiple of 16) from src to dst,
 * both device, 16-byte aligned, with a plain grid-stride kernel.  Timed as
 * stage "probe" when timing is enabled.  Not part of the method: it gives the
 * HBM roofline denominator and calibrates traffic counters. */
gs_status gs_bw_probe(gs_ctx* ctx, const void* src, void* dst, size_t bytes, void* stream);

gs_status gs_frame_stats_get(gs_frame* frame, gs_frame_stats* out);
/* Copy a frame buffer (see gs_export) for view `view` (-1 = all views) into
 * the caller's device buffer dst of `bytes` bytes (must be large enough;
 * GS_EXPORT_SCREEN_GRADS also needs dst 16-byte aligned).  Errors:
 * GS_ERR_INVALID for a null frame or dst, a view out of range, an unknown
 * export, a short or misaligned dst. */
gs_status gs_frame_export(gs_frame* frame, int32_t what, int32_t view, void* dst,
                          size_t bytes, void* stream);
void gs_frame_release(gs_frame* frame);

/* ------------------------------------------------------- batched step graph
 * One training step over n_views views (mixed sizes allowed) captured as a
 * hipGraph: projection, sort, compositing, loss gradient, backward and (if
 * with_adam) Adam, with no host synchronisation inside.  The paper trains on
 * many views of one scene (Sec. III-IV); on one GPU the views of a step are
 * rendered together instead of being spread over devices.
 * All pointers are caller-owned device memory that must stay valid while the
 * graph exists; the views' cameras are copied.  The record capacity is
 * capacity_slack (>= 1.05, default 1.25) times the record count of a
 * measuring pass run by gs_step_graph_create (which also writes the images,
 * dl_dimg, loss and grads once, without Adam).  A replay whose records exceed
 * the capacity sets an overflow flag and applies no Adam update;
 * gs_step_graph_sync then reports it, grows the capacity and recaptures, and
 * the step should be replayed (gs_step_graph_run does all of this). */
typedef struct {
  gs_params params;              /* read */
  gs_params grads;               /* written (not accumulated) every step */
  gs_params adam_m, adam_v;      /* Adam moments, updated in place */
  const gs_camera* cams;         /* host array of n_views cameras (copied) */
  int32_t n_views;               /* 1..16 */
  float* const* images;          /* device [3][H][W] per view: rendered images */
  const float* const* targets;   /* device [3][H][W] per view: training targets */
  float* const* dl_dimg;         /* device [3][H][W] per view: image gradients */
  float* loss;                   /* device float: the step's loss */
  gs_render_opts render;
  gs_adam_opts adam;
  int32_t with_adam;
  float lambda_dssim;
  int64_t first_step;            /* Adam step number of the first replay (>= 1) */
  double capacity_slack;
} gs_step_desc;

gs_status gs_step_graph_create(gs_ctx* ctx, const gs_step_desc* desc, gs_graph** out,
                               void* stream);
/* gs_step_graph_create with the measuring pass on the null stream. */
gs_status gs_step_graph_capture(gs_ctx* ctx, const gs_step_desc* desc, gs_graph** out);
/* Enqueue one replay on `stream` (asynchronous). */
gs_status gs_step_graph_launch(gs_graph* graph, void* stream);
/* Wait for the last replay; report the record count and whether it overflowed
 * (then the capacity has been grown and the graph recaptured). */
gs_status gs_step_graph_sync(gs_graph* graph, int32_t* overflowed, int64_t* records,
                             void* stream);
/* Launch + sync, replaying after an overflow; synchronous. */
gs_status gs_step_graph_run(gs_graph* graph, int64_t* records, void* stream);
/* Capacity, last record count and the graph's frame (owned by the graph). */
gs_status gs_step_graph_info(gs_graph* graph, int64_t* capacity, int64_t* records,
                             gs_frame** frame);
void gs_step_graph_destroy(gs_graph* graph);

/* ----------------------------------------------------------- render server
 * Serving of trained scenes (the paper's aim of real-time post hoc and in situ
 * visualization, Sec. I and V): scenes stay resident on the device and novel
 * views are rendered on request.  n_slots worker threads (1..8) each own a
 * HIP stream; a free worker takes the scene of the oldest pending request and
 * up to max_batch_views of that scene's pending requests (any resolutions)
 * and renders them as one multi-view forward.  A batch is admitted when its
 * estimated scratch plus the scratch held by the other slots fits mem_budget
 * (0 = no limit; an idle device always admits one batch); otherwise it waits
 * for a running batch to finish.  Latency = submission to completion of the
 * request's batch.  Stage timing (gs_ctx_set_timing) must be off while a
 * server runs.  A request's image is the same in any batch. */
typedef struct {
  int32_t n_slots;
  int32_t max_batch_views;
  size_t mem_budget;
  gs_render_opts render;
  int32_t max_queue;         /* pending requests before submit returns GS_ERR_BUSY */
  int32_t reserved;
} gs_server_opts;

typedef struct {
  int64_t submitted, completed, batches, deferred;
  double mean_batch_views;
  double p50_ms, p99_ms, mean_ms, max_ms;
  double mpix_per_s;         /* completed pixels / (last completion - first submission) */
  int64_t peak_bytes;        /* high-water mark of the admission ledger */
} gs_serve_stats;

gs_status gs_server_create(gs_ctx* ctx, const gs_server_opts* opts, gs_server** out);
/* Register a resident scene (device parameters stay caller-owned and must
 * outlive the server); *scene_id receives its id. */
gs_status gs_server_add_scene(gs_server* server, gs_params scene, int32_t* scene_id);
/* Queue a render of `scene` seen from *cam into out_image (device [3][H][W],
 * caller-owned, untouched until the request completes). */
gs_status gs_server_submit(gs_server* server, int32_t scene, const gs_camera* cam,
                           float* out_image, uint64_t* ticket);
/* Non-blocking completion check (a completed ticket is forgotten after it is
 * reported), or a blocking wait; latency in ms. */
gs_status gs_server_poll(gs_server* server, uint64_t ticket, int32_t* done, double* latency_ms);
gs_status gs_server_wait(gs_server* server, uint64_t ticket, double* latency_ms);
/* Wait until every submitted request has completed. */
gs_status gs_server_drain(gs_server* server);
gs_status gs_server_stats(gs_server* server, gs_serve_stats* out);
gs_status gs_server_reset_stats(gs_server* server);
void gs_server_destroy(gs_server* server);

/* ------------------------------------------------- adaptive density control
 * Clone, split and prune of the 3D-GS training that Sec. III (Method
 * Overview) adopts by citation; the paper restates none of it, so the
 * statistics, thresholds and output order below are the readings this library
 * takes of that model's density control.
 *
 * Statistics (caller-owned device arrays of n entries, zeroed by the caller
 * at the start of an interval): grad = sum over views of scale * |dL/dmean2D|
 * in normalised device coordinates ((dL/dm_x W/2, dL/dm_y H/2), W x H the
 * view's size), count = number of views in which the Gaussian touched a
 * tile, max_radius = its largest pixel radius over those views. */
typedef struct {
  float* grad;
  int32_t* count;
  int32_t* max_radius;
  int64_t n;
} gs_density_stats;

/* Adds the views of `frame` to the statistics.  The frame must have been
 * rendered with GS_RENDER_RADII and its backward run with
 * GS_BWD_KEEP_SCREEN (GS_ERR_INVALID otherwise); stats.n must equal the
 * frame's Gaussian count.  scale multiplies each view's norm (the number of
 * views of a batch whose loss is their mean makes every view count as in
 * one-view training).  Asynchronous on `stream`. */
gs_status gs_density_accumulate(gs_ctx* ctx, gs_frame* frame, gs_density_stats stats,
                                float scale, void* stream);

/* Densification thresholds (3D-GS defaults in brackets). */
typedef struct {
  double grad_threshold;  /* mean NDC gradient that selects a Gaussian [0.0002] */
  double percent_dense;   /* selected with largest scale <= percent_dense * extent are
                             cloned, larger ones split [0.01] */
  double min_opacity;     /* opacity below it is pruned [0.005] */
  double max_screen;      /* > 0: also prune max_radius > max_screen or largest scale >
                             max_world * extent (<= 0: no size prune) [20 after the
                             first opacity reset] */
  double max_world;       /* [0.1] */
  double extent;          /* scene extent (radius of the camera set) */
  double split_div;       /* children's scales = parent's / split_div [1.6] */
  int32_t n_split;        /* children per split Gaussian, 1..8 [2] */
  int32_t reserved;
  uint64_t seed;          /* key of the children's Philox draws */
} gs_density_opts;

typedef struct {
  int64_t n_in, n_out;    /* Gaussians before and after */
  int64_t kept;           /* originals kept */
  int64_t cloned;         /* clones made (and kept) */
  int64_t split;          /* Gaussians split (the parent is removed) */
  int64_t children;       /* children kept */
  int64_t pruned;         /* originals removed other than by a split */
} gs_density_info;

/* One densification of params p with Adam moments m, v (device SoA, n
 * entries) from the statistics:
 *  - mean gradient g = grad / count (0 where count is 0), in float64; g >=
 *    grad_threshold selects a Gaussian; a selected one is cloned (an exact
 *    copy) when its largest scale exp(log_scale) <= percent_dense * extent,
 *    split otherwise into n_split children at mean + R(q) (s * z), z three
 *    standard normals (Philox4x32-10 keyed by the seed's two words, counter
 *    (parent index, 16 + child, 0, 0), Box-Muller of its two pairs, first
 *    three values), log-scales minus log(split_div), the parent's rotation,
 *    opacity and colour; the parent is removed;
 *  - prune: opacity < min_opacity, and with max_screen > 0 also max_radius >
 *    max_screen or largest scale > max_world * extent (clones: opacity and
 *    scale; children: opacity and their own scale);
 *  - output order: kept originals in index order, then clones in the order of
 *    their sources, then children source by source (child 0 first); Adam
 *    moments are copied for originals and zero for new Gaussians.
 * p_out, m_out, v_out (device, caller-owned, must not overlap the inputs)
 * receive the new set and must have n equal to info->n_out; pass p_out.means
 * = NULL to only count (info filled, nothing written).  src_index (optional,
 * device int32[n_out]) receives the source index of every output.  The
 * statistics and inputs are read, not changed.  Synchronises `stream` once
 * (the counts are read back through context scratch: calls on one context
 * must not overlap).  GS_ERR_CAPACITY when p_out.n < n_out, GS_ERR_INVALID
 * when larger. */
gs_status gs_densify(gs_ctx* ctx, gs_params p, gs_params m, gs_params v,
                     gs_density_stats stats, const gs_density_opts* opts, gs_params p_out,
                     gs_params m_out, gs_params v_out, int32_t* src_index,
                     gs_density_info* info, void* stream);

/* Opacity reset of the same training: opacity = min(opacity, max_opacity)
 * (in logit form, max_opacity in (0, 1), 0.01 in 3D-GS) and the opacity's
 * Adam moments set to zero.  In place, asynchronous. */
gs_status gs_opacity_reset(gs_ctx* ctx, gs_params p, gs_params m, gs_params v,
                           double max_opacity, void* stream);

/* ------------------------------------------- isosurface points and targets
 * The extraction and target rendering that Sec. III (Method Overview) does
 * with ParaView, on a volume already in device memory (the in-situ direction
 * of Sec. V).  volume: values[k][j][i] (device float32, caller-owned) at the
 * vertices of an nx x ny x nz grid over the box [lo, hi] (vertex (i, j, k) at
 * lo + (i, j, k) h, h = (hi - lo) / (n - 1)); each side 2 .. 2^20. */
typedef struct {
  const float* values;
  int64_t nx, ny, nz;
  float lo[3], hi[3];
} gs_volume;

/* Isosurface points: every grid edge whose end values lie strictly on both
 * sides of iso gives the point p0 + t (p1 - p0), t = (v0 - iso) / (v0 - v1)
 * (the vertex rule of marching cubes), in canonical order (vertices
 * row-major in (k, j, i), per vertex its +x, +y, +z edges).  A crossing on
 * edge e = 3 vertex + axis is kept when the Philox4x32-10 uniform
 * (x0 >> 8) 2^-24 of counter (e low, e high, 3, 0), key (seed low, seed
 * high), is below keep_prob (1: all).  *n_points receives the number kept;
 * with xyz (device float32 [3][capacity]) non-NULL they are written there
 * (GS_ERR_CAPACITY, nothing written, if they do not fit).  Synchronises
 * `stream` once (the count is read back through context scratch: calls on one
 * context must not overlap). */
gs_status gs_iso_extract(gs_ctx* ctx, gs_volume volume, float iso, float keep_prob,
                         uint64_t seed, float* xyz, int64_t capacity, int64_t* n_points,
                         void* stream);

/* Ray-cast target views of the isosurface: per pixel the ray from the camera
 * centre through the pixel centre, clipped to the box, sampled every `step`
 * (world units) with the trilinear interpolant; the first rise from below iso
 * to at least iso is refined by ten bisections and shaded albedo(p) (0.2 +
 * 0.8 |n . d|), n the interpolant's normalised gradient, albedo = (0.85,
 * 0.45 + 0.25 z, 0.30 + 0.25 (x + 1)); misses are black.  images[v]: device
 * float32 [3][H][W].  step > 0 and >= 1e-5 of the box diagonal.  Float64
 * arithmetic.  Asynchronous. */
gs_status gs_raycast(gs_ctx* ctx, gs_volume volume, float iso, const gs_camera* cams,
                     int32_t n_views, float step, float* const* images, void* stream);

/* -------------------------------------------------------------- autotuner
 * Times forward + backward of the given views for tile sizes {8, 16, 32},
 * LDS depths {32, 64, 128, 256} and the grid or persistent longest-first
 * forms, `reps` timed repetitions each after a warm-up, and returns the
 * fastest options in *best.  table (optional, host) receives up to table_cap
 * entries; *table_n their number.  Synchronous. */
typedef struct {
  int32_t tile, lds_depth, flags;
  float ms;
} gs_tune_entry;

gs_status gs_autotune(gs_ctx* ctx, gs_params params, const gs_camera* cams, int32_t n_views,
                      int32_t reps, gs_render_opts* best, gs_tune_entry* table,
                      int32_t table_cap, int32_t* table_n, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* ISOGS_H */
