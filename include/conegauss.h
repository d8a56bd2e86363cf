/*
 * conegauss.h -- C ABI of the MI355X (gfx950) ConeGaussian renderer.
 *
 * Per-pixel anti-aliased Gaussian ray rendering for generic central cameras
 * (ConeGaussian, arXiv 2609.13397).  A camera is its inverse mapping Pi^{-1} plus an
 * optical centre (Sec. 3); every pixel is a bundle of rays (Sec. 4.1, Eq. 5) whose
 * centre ray and two half-pixel edge rays define an anisotropic footprint covariance
 * (Eq. 6, 8).  Each Gaussian's closed-form filtered response (Eq. 9), with the
 * per-Gaussian frequency floor (Eq. 10) and marginal composition (Eq. 12), is
 * alpha-composited front to back (Eq. 4).
 *
 * Conventions shared by every entry point
 *   - Pointers are DEVICE pointers unless marked (host).  Floating point is float32.
 *   - Arrays are component-major: a "[C][N]" array holds component c of item i at
 *     index c*N + i, contiguous.
 *   - The caller owns every input and output buffer.  Scratch memory is taken from
 *     the cg_allocator passed in, or, when that is NULL, from the library's own
 *     stream-ordered caching pool (device memory that stays cached until
 *     cg_release_cached_memory is called).
 *   - All device work is enqueued on `stream` and is asynchronous unless stated.
 *   - Every call returns a cg_status and never throws; on failure cg_last_error()
 *     gives a message (thread-local).  Arguments are validated on the host (sizes,
 *     enums, camera intrinsics, crop windows, Kannala-Brandt monotonicity).  Values
 *     inside device arrays are not scanned: NaN in gives NaN out.
 *   - Calls are thread-safe when different threads use different streams.
 */
#ifndef CONEGAUSS_H
#define CONEGAUSS_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CG_VERSION 1

typedef enum {
  CG_OK = 0,
  CG_ERR_INVALID_ARG = -1,
  CG_ERR_UNSUPPORTED = -2,
  CG_ERR_OUT_OF_MEMORY = -3,
  CG_ERR_HIP = -4,
  CG_ERR_STATE = -5,
  CG_ERR_TIMEOUT = -6  /* a server request not admitted within its time limit */
} cg_status;

/* Camera models.  The paper names pinhole and fisheye cameras only (Sec. 5); the
 * equations below are this library's readings.  Camera axes follow OpenCV (x right,
 * y down, z forward); d_world = R_c2w d_cam.  For pinhole and fisheye,
 * m = ((x - cx)/fx, (y - cy)/fy) with (x, y) continuous coordinates of the full image.
 *   CG_PINHOLE:    d_cam = (m_x, m_y, 1) / |.|
 *   CG_FISHEYE_KB: equidistant Kannala-Brandt, theta_d = |m| solves
 *                  theta (1 + k1 theta^2 + k2 theta^4 + k3 theta^6 + k4 theta^8) = theta_d
 *                  on [0, theta_max]; d_cam = (sin(theta) m / theta_d, cos(theta)).
 *                  Pixels with theta_d beyond theta_d(theta_max) are invalid.
 *   CG_EQUIRECT:   phi = 2 pi (x / full_w - 1/2), lambda = pi (1/2 - y / full_h),
 *                  d_cam = (cos(lambda) sin(phi), -sin(lambda), cos(lambda) cos(phi)). */
typedef enum { CG_PINHOLE = 0, CG_FISHEYE_KB = 1, CG_EQUIRECT = 2 } cg_camera_model;

/* One view (host struct, passed by pointer, read during the call only).
 * Pixel (i, j) of the crop window has centre (crop_x0 + i + 1/2, crop_y0 + j + 1/2)
 * in the full virtual image of full_w x full_h pixels.  A zoomed view (the paper's
 * scale convention, Sec. 5: calibration scaled with resolution) is a crop of a large
 * virtual image.  The crop must lie inside the full image. */
typedef struct {
  int32_t model;                            /* cg_camera_model                          */
  int32_t full_w, full_h;                   /* virtual image size                       */
  int32_t crop_x0, crop_y0, crop_w, crop_h; /* rendered window                          */
  float fx, fy, cx, cy;                     /* pixels (pinhole, fisheye); unused equirect */
  float k[4];                               /* fisheye k1..k4; 0 otherwise              */
  float R_c2w[9];                           /* row-major camera-to-world rotation       */
  float origin[3];                          /* optical centre o (world)                 */
  float theta_max;                          /* fisheye valid half field of view (rad)   */
} cg_camera;

/* Gaussians (Sec. 3): raw parameters, SoA [C][n] float32 device arrays.
 *   means [3][n]; log_scales [3][n] (s = exp); quats [4][n] (w, x, y, z; normalised
 *   inside); opacity_logits [n] (sigma = sigmoid); color: color_mode 0 -> rgb [3][n],
 *   color_mode 3 -> degree-3 real SH [48][n] with index 3*coef + channel, coefficients
 *   in (l, m) order, m = -l..l, Condon-Shortley phase; colour = max(sum + 1/2, 0);
 *   rho2 [n] floor variance of Eq. 10 (NULL = 0). */
typedef struct {
  int64_t n;
  int32_t color_mode;
  const float* means;
  const float* log_scales;
  const float* quats;
  const float* opacity_logits;
  const float* color;
  const float* rho2;
} cg_gaussians;

enum { CG_FILTER_CENTER_RAY = 0, CG_FILTER_ANISOTROPIC = 1, CG_FILTER_ISOTROPIC = 2 };
enum { CG_COMPOSE_MARGINAL = 0, CG_COMPOSE_ADDITIVE = 1 };
enum { CG_ORDER_KEY = 0, CG_ORDER_RAY = 1 };
enum { CG_BACKBONE_MAX_RESPONSE = 0, CG_BACKBONE_RAY_INTEGRAL = 1 };

/* Render options.  cg_default_opts fills the defaults given in brackets.
 *   filter_mode     CG_FILTER_* [ANISOTROPIC]: centre ray = Eq. 3 with C = 1;
 *                   anisotropic = Eq. 9; isotropic = Eq. 9 with the footprint replaced
 *                   by the in-plane isotropic covariance of equal trace.
 *   use_floor       [0] apply Eq. 10 with rho2; the render footprint is then composed
 *                   with the floor by `composition`.
 *   composition     CG_COMPOSE_* [MARGINAL]: Eq. 12, or the plain sum (ablation).
 *   alpha_min       [1/255] pairs with alpha = min(T, alpha_max) below it are skipped.
 *   alpha_max       [0.99]
 *   T_min           [1e-4]  a pixel stops before the pair that would take its
 *                   transmittance below T_min.
 *   t_near          [0.2]   pairs with max-response depth t* <= t_near give T = 0.
 *   bg[3]           [0]     background, added as T_final * bg.
 *   footprint_scale [1]     multiplies the neighbour-ray differentials (0 = centre ray).
 *   count_pairs     [0]     when set, cg_fwd_stats also receives the pair counts below
 *                   (a counting variant of the render kernel; results are identical).
 *   order_mode      CG_ORDER_* [KEY]: the front-to-back order of Eq. 4.  KEY: one key
 *                   per view and Gaussian, |mu - o| (ties by Gaussian index).  RAY: each
 *                   pixel's pairs by their own max-response depth t* along its ray
 *                   (Sec. 3), ties by list position.  RAY holds up to 16 pending pairs
 *                   per pixel and composites one as soon as no later Gaussian of the
 *                   tile's list can have a smaller t* (every record bounds its t* from
 *                   below).  A full buffer defers the pair with the largest t* to a
 *                   further walk of the tile list over the deferred depth range, so the
 *                   order is exact however many pairs a pixel has; deferrals are
 *                   counted in cg_fwd_stats.n_order_overflow.  RAY is forward-only:
 *                   state_out must be NULL (CG_ERR_UNSUPPORTED otherwise).
 *   backbone        CG_BACKBONE_* [MAX_RESPONSE]: the longitudinal factor C[w] of the
 *                   weighted ray response (Sec. 3) that multiplies Eq. 9.  MAX_RESPONSE:
 *                   w = delta(t - t*), C = 1.  RAY_INTEGRAL: w = 1, C = sqrt(2 pi) /
 *                   (Z_G sqrt(det Sigma_eff) |W d|); the paper leaves Z_G open, and the
 *                   value taken is sqrt(2 pi) det(Sigma_eff)^(-1/3), for which an
 *                   isotropic Gaussian gets C = 1; then C = 1 / (g |W d|) with g the
 *                   geometric mean of s'. */
typedef struct {
  int32_t filter_mode;
  int32_t use_floor;
  int32_t composition;
  float alpha_min, alpha_max, T_min, t_near;
  float bg[3];
  float footprint_scale;
  int32_t count_pairs;
  int32_t order_mode;
  int32_t backbone;
} cg_render_opts;

/* Scratch allocator.  alloc returns device memory usable in stream order on `stream`
 * (NULL on failure -> CG_ERR_OUT_OF_MEMORY); free releases it in stream order.
 * cg_render_forward makes two allocations (the buffers whose sizes are known up front,
 * then those sized by the pair count), cg_render_backward one.  On a failure the call
 * frees every block it already holds before it returns; the blocks of a training
 * state are freed by cg_fwd_state_release, with the allocator the forward was given. */
typedef struct {
  void* ctx;
  void* (*alloc)(void* ctx, size_t bytes, hipStream_t stream);
  void (*free)(void* ctx, void* ptr, hipStream_t stream);
} cg_allocator;

/* Opaque forward state kept for cg_render_backward (the sorted per-tile lists, the
 * per-view Gaussian records and the per-pixel stopping points).  It refers to the
 * Gaussian arrays passed to cg_render_forward, which must stay alive and unchanged
 * until the backward call.  Owned by the caller; release with cg_fwd_state_release. */
typedef struct cg_fwd_state cg_fwd_state;

/* Counters of one forward call (host struct). */
typedef struct {
  int64_t n_pairs;          /* (tile, Gaussian) pairs after binning                  */
  int64_t n_tiles;          /* tiles over all views                                  */
  int64_t n_pixels;         /* pixels over all views                                 */
  int64_t n_gaussian_views; /* n * n_views                                           */
  int32_t sort_bits;        /* radix-sort key width                                  */
  int32_t n_segments;       /* work items of the split tile render (see
                               cg_set_tile_split); 0: one workgroup per tile         */
  /* filled only with opts.count_pairs (else -1):                                    */
  int64_t n_evaluated;      /* (pixel, Gaussian) pairs a pixel walked through        */
  int64_t n_full;           /* ... that passed the cheap rejection (full Eq. 9 work) */
  int64_t n_contrib;        /* ... that were composited (alpha >= alpha_min, before
                               termination): the method's unit of work              */
  int64_t n_order_overflow; /* order_mode RAY: pairs deferred to a further walk of
                               their tile list because a pixel's pending buffer was
                               full; the order stays exact (else -1)                */
  int64_t max_tile_pairs;   /* longest tile list, when the call considered the split
                               tile render (see cg_set_tile_split; else -1)         */
} cg_fwd_stats;

int cg_version(void);
const char* cg_last_error(void);
void cg_default_opts(cg_render_opts* opts /* host */);

/* Forward render of n_views views of one set of Gaussians (Eq. 4-12).
 *   cams       host array [n_views].
 *   out_rgba   device [sum_v crop_h_v * crop_w_v][4], view-major, row-major within a
 *              view: premultiplied RGB plus the background term, and alpha = 1 - T_final.
 *   state_out  NULL for inference; otherwise receives a state for cg_render_backward.
 *   stats_out  host, may be NULL.
 * The call waits once for the work queued on `stream`, to read back the number of
 * pairs.  A call shaped like the calling thread's previous one (same Gaussian count,
 * views, tiles and pixels, and both with or both without state_out) sizes its pair
 * buffers from that call's pair count and queues the pair emission before it waits;
 * if its own count is larger, it emits again into buffers of the right size.  Images,
 * counts and states do not depend on this. */
cg_status cg_render_forward(const cg_gaussians* g /* host struct, device arrays */, const cg_camera* cams,
                            int32_t n_views, const cg_render_opts* opts /* host */, const cg_allocator* alloc,
                            float* out_rgba, cg_fwd_state** state_out, cg_fwd_stats* stats_out,
                            hipStream_t stream);

/* cg_render_forward for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * inference forward, same kernels and same result, with every scratch buffer carved
 * from a 64 MiB file-scope device array instead of an allocator.  The call allocates
 * nothing (no hipMalloc, hipFree or allocating library routine); the caller still
 * passes its inputs and out_rgba.  Each GPU holds its own copy of the array from the
 * library's load until the process ends; its device address is looked up on the first
 * call on that device.
 *   A call whose scratch would exceed 64 MiB returns CG_ERR_INVALID_ARG (found before
 *   anything is written for the buffers sized up front; after the pair count for the
 *   pair lists), and the next call is unaffected.  As a guide, a call needs about
 *   190 B per (view, Gaussian), 64 B per pixel (rounded up to 16x16 tiles) and 16 B per
 *   (tile, Gaussian) pair, plus sort buffers.
 *   Every call on one GPU uses that GPU's one array, which keeps the last call's
 *   contents (every buffer that must start at zero is cleared by the call): calls that
 *   overlap on one GPU, for instance on two streams, race and give wrong images.
 *   Calls in stream order on one stream are safe.  No training state (no state_out). */
cg_status cg_render_forward_noalloc(const cg_gaussians* g /* host struct, device arrays */,
                                    const cg_camera* cams /* host */, int32_t n_views,
                                    const cg_render_opts* opts /* host */, float* out_rgba,
                                    cg_fwd_stats* stats_out /* host, may be NULL */, hipStream_t stream);

/* Gradients of L = sum(grad_rgba * out_rgba) with respect to the raw Gaussian
 * parameters of the forward call that produced `st` (summed over its views).  The
 * outputs have the shapes of the inputs and are OVERWRITTEN; rho2 gets no gradient.
 * Pairs are reduced per tile and then per Gaussian without atomics, so the result is
 * deterministic.  grad_rgba has the layout of out_rgba.  The call is asynchronous
 * on `stream` (no host synchronisation unless scratch guard bands are enabled). */
cg_status cg_render_backward(cg_fwd_state* st, const float* grad_rgba, float* d_means, float* d_log_scales,
                             float* d_quats, float* d_opacity_logits, float* d_color, hipStream_t stream);

/* Releases a forward state: its blocks go back to the allocator in the order of the
 * forward's stream, after waiting for the last backward on it if that ran on another
 * stream.  NULL is a no-op. */
void cg_fwd_state_release(cg_fwd_state* st);

/* Diagnostic of the last cg_render_backward on `st`: the number of pixels whose
 * replayed front-to-back walk did not end at the transmittance the forward stored
 * (0 when the replay is exact); -1 before any backward call or on a HIP error.  The
 * count stays on the device until this call, which waits for the backward's stream. */
int64_t cg_bwd_replay_mismatches(const cg_fwd_state* st);

/* Inverse mapping Pi^{-1} (Sec. 3) of n continuous full-image pixel coordinates.
 *   pix_xy [2][n] device; dirs [3][n] unit world directions (0 where invalid);
 *   valid [n] 1/0. */
cg_status cg_camera_unproject(const cg_camera* cam /* host */, int64_t n, const float* pix_xy, float* dirs,
                              uint8_t* valid, hipStream_t stream);

/* Per-Gaussian floor variance of Eq. 11: the minimum over the views in which a
 * Gaussian is visible of half the trace of the world-space footprint covariance at
 * the pixel its mean projects to (half-pixel neighbour rays from Pi^{-1}, projected
 * orthogonally to the ray through the mean, at the mean's distance).  Visible: the
 * projection is valid and inside the full image, and the distance exceeds t_near.
 * A Gaussian visible in no view gets 0.  rho2_out [n] device. */
cg_status cg_bake_rho2(const cg_gaussians* g /* host struct, device arrays */, const cg_camera* cams /* host */,
                       int32_t n_views, float t_near, float* rho2_out, hipStream_t stream);

/* ---------------------------------------------------------------------------- serving
 * A render server with continuous batching (extension of the paper's renderer to a
 * serving loop).  Scenes are registered once and stay device-resident (the server
 * keeps the device pointers; the caller keeps the arrays alive).  Requests (scene,
 * camera, caller-owned device output [crop_h][crop_w][4]) queue in arrival order.
 * Each of n_workers threads owns a HIP stream; a free worker takes the oldest
 * request when its estimated scratch memory fits hbm_budget_bytes next to the
 * requests already running (or when nothing runs), and fuses further queued
 * requests for the same scene into the same multi-view render call, up to
 * max_batch_views views, max_batch_pixels pixels and max_batch_pairs estimated pairs
 * (a + b * pixels per view, a and b fitted per scene to the calls completed so far; a
 * request above the cap runs alone), while they fit the budget.  The pair cap bounds a fused
 * call's duration, which every request in it waits for.
 * A fused call renders each view bit for bit as a call with that view alone.
 * With n_workers = 1 and max_batch_views = 1 the server is the plain one-view-per-
 * launch renderer.  With request_timeout_ms > 0, a request still queued that long
 * after its submission is not rendered: it completes with CG_ERR_TIMEOUT and its
 * output buffer is left untouched (checked whenever a worker looks for work, at
 * least every request_timeout_ms while one waits, and by every poll and drain).  fake_executor = 1 replaces rendering by a sleep of
 * fake_ns_per_call + fake_ns_per_pixel * pixels (scheduler tests without a GPU). */
typedef struct cg_server cg_server;

typedef struct {
  size_t hbm_budget_bytes;     /* [24 GiB] scratch that admitted requests may hold together */
  int32_t max_batch_views;     /* [8]      views fused into one render call                 */
  int32_t n_workers;           /* [3]      concurrent render calls, one HIP stream each     */
  int64_t max_batch_pixels;    /* [16 Mi]  pixel cap of one fused call                      */
  int32_t fake_executor;       /* [0]                                                       */
  int32_t device;              /* [0]      HIP device of the worker streams                 */
  double fake_ns_per_pixel;    /* [1]                                                       */
  double fake_ns_per_call;     /* [50000]                                                   */
  double request_timeout_ms;   /* [0]      time limit from submission to admission (0: none) */
  double max_batch_pairs;      /* [12e6]   estimated (tile, Gaussian) pairs of one fused call  */
} cg_server_config;

/* One finished (or cancelled: status CG_ERR_STATE; timed out: CG_ERR_TIMEOUT) request.  Times are seconds on the
 * clock of cg_server_now(): submission, admission, start and end of its render call. */
typedef struct {
  int64_t request_id;
  int32_t status;
  int32_t scene;
  int32_t batch_views;
  int32_t reserved;
  double t_submit, t_admit, t_start, t_done;
  int64_t n_pairs;             /* pairs of the fused call that rendered it */
} cg_server_completion;

typedef struct {
  int64_t queued, in_flight, completed, batches, views, max_batch_views;
  int64_t reserved_bytes, peak_reserved_bytes;
  int64_t timed_out;           /* requests completed with CG_ERR_TIMEOUT */
} cg_server_stats;

void cg_server_default_config(cg_server_config* cfg /* host */);
cg_status cg_server_create(const cg_server_config* cfg, cg_server** out);
/* g: host struct of device arrays (kept by pointer); opts: render options of the scene. */
cg_status cg_server_add_scene(cg_server* s, const cg_gaussians* g, const cg_render_opts* opts, int32_t* scene_id);
/* Validates the camera on the host and queues the request; returns at once. */
cg_status cg_server_submit(cg_server* s, int32_t scene, const cg_camera* cam, float* out_rgba, int64_t* request_id);
/* Removes a request that has not been admitted yet; *cancelled = 1 if it was found. */
cg_status cg_server_cancel(cg_server* s, int64_t request_id, int32_t* cancelled);
/* Moves up to `capacity` completions into out (waiting up to wait_ms for the first). */
cg_status cg_server_poll(cg_server* s, cg_server_completion* out, int32_t capacity, int32_t* n_out, int32_t wait_ms);
/* Blocks until the queue is empty and no render call is running. */
cg_status cg_server_drain(cg_server* s);
cg_status cg_server_get_stats(cg_server* s, cg_server_stats* out);
/* Drops queued requests, waits for running calls, stops the workers. */
void cg_server_destroy(cg_server* s);
double cg_server_now(void);

/* Per-stage GPU timing.  When enabled, every kernel launch of the library is
 * bracketed with HIP events on its stream.  cg_profile_collect synchronises on the
 * recorded events and adds their durations to per-stage totals; cg_profile_read
 * copies the totals (host arrays of length cg_profile_num_stages()) and resets them.
 * cg_profile_enable(on) enables every stage (on != 0) or none; cg_profile_enable_stages
 * enables the stages whose bit (1 << stage) is set in mask, so that a timed region can
 * bracket only the kernels it reports (each bracket costs an event record on the
 * stream). */
int cg_profile_num_stages(void);
const char* cg_profile_stage_name(int stage);
void cg_profile_enable(int on);
void cg_profile_enable_stages(uint32_t mask);
cg_status cg_profile_collect(void);
void cg_profile_read(double* total_ms /* host */, int64_t* launches /* host */);

/* Calibration kernel for the VALU rate (profiling only; not part of rendering): n_blocks
 * workgroups of 256 threads, each thread running `iters` rounds of 8 independent
 * float32 FMA chains, so it issues exactly 8 * iters v_fma_f32 per wave (plus loop
 * control) and touches no memory; out (device, one float) is never written in
 * practice.  Timed with the stage profiler ("valu_probe") and read by rocprofv3's SQ
 * counters, it gives the FP32 issue rate the hardware sustains and what the counters
 * read at that rate.  Enqueued on `stream`. */
cg_status cg_profile_valu_probe(int32_t n_blocks, int32_t iters, float* out, hipStream_t stream);

/* Split tile render.  One workgroup per tile takes at least as long as the longest tile
 * list, walked by one workgroup while the rest of the chip may be idle (a small view of
 * a large scene, or a low resolution where a few tiles hold most pairs).  In a forward
 * call without training state, pair counting or per-ray order, every view with fewer
 * than max_tiles tiles has its longest list and its pair count P_v read back after the
 * tile sort (one more host synchronisation), and is split when its longest list
 * exceeds both min_longest and P_v / 1024 (about half the pairs each of the chip's
 * ~2048 resident workgroups would get were the view's work spread evenly, since the
 * split render makes about two passes over every pair).  The decision and the segment
 * length depend on the view alone, so a view renders the same in any call.  Each
 * tile's depth-ordered list of a split view is cut into segments of seg_len pairs
 * (0: max(384, P_v / 16384)), each rendered by its own workgroup: one pass composites
 * every segment on its own from T = 1 (its colour and its transmittance product, Eq. 4's
 * factors 1 - alpha, ending with the one that takes it below T_min); where a pixel's
 * walk ends inside a segment (the product of the segments in front is at least T_min,
 * times this one's below it), a second pass composites that segment again from the
 * product in front; a last step adds the segments' colours, each scaled by the product
 * in front, up to the one where the pixel terminated.  The image equals the
 * one-workgroup-per-tile render up to the rounding order of those products and sums.  The other views of the call render in whole
 * tiles.  Arguments <= 0 restore the defaults (2048 tiles, 2048 pairs, seg_len 0).
 * Process-wide; calls already enqueued keep the values they were issued with. */
void cg_set_tile_split(int64_t max_tiles, int64_t min_longest, int64_t seg_len);

/* Scratch guard bands (a debugging aid, off by default; extension of the renderer, not
 * part of the paper's method).  mode 1: every scratch buffer of the forward and
 * backward calls is followed by a 256-byte band of a fixed 32-bit pattern, written
 * before the call's kernels and compared after them (one more host synchronisation
 * per call); a changed word makes the call return CG_ERR_STATE, naming the number of
 * changed words, and adds it to cg_debug_guard_violations().  mode 2: as 1, and the
 * host overwrites one word of the call's first band before the comparison, so that a
 * test can see the check fire without a kernel writing out of bounds.  mode 0 (or any
 * other value): off.  Process-wide; takes effect for calls issued afterwards.  Images
 * and gradients do not depend on the mode. */
void cg_debug_set_scratch_guards(int32_t mode);
/* Total number of changed guard words found since the library was loaded. */
int64_t cg_debug_guard_violations(void);

/* Returns the library's cached scratch memory to the device (waits for the device to
 * be idle). */
cg_status cg_release_cached_memory(void);

#ifdef __cplusplus
}
#endif

#endif /* CONEGAUSS_H */
