/*
 * drk.h -- C ABI of libdrk, a tile-based differentiable rasterizer for Deformable Radial Kernel
 * (DRK) primitives on AMD Instinct MI355X (gfx950).
 *
 * Method: "Deformable Radial Kernel Splatting" (arXiv 2412.11752).  A DRK is a planar primitive
 * with centre mu, rotation q, K radial bases (lengths s_k, polar angles theta_k), an L1/L2 blend
 * weight eta, a sharpness tau, an opacity o and a colour (Sec. 4).  A pixel's colour is the
 * front-to-back alpha blend of the kernels its ray hits (Eq. 1, Sec. 3.1), evaluated at the
 * ray-plane intersection (Sec. 3.3).
 *
 * Conventions shared by every entry point
 *  - Every call returns a drk_status.  DRK_OK is 0.  drk_last_error() returns a thread-local
 *    message for the last failure on the calling thread.  Nothing throws across the ABI.
 *  - Array arguments are DEVICE pointers (hipMalloc'd or torch tensors on the GPU) unless marked
 *    "host".  They are borrowed: the caller keeps them alive until the work enqueued on the given
 *    stream has completed.  Outputs are caller-allocated.
 *  - Layout: structure-of-arrays, float32, contiguous, primitive index fastest ([rows][n]).
 *  - The only calls that allocate device memory are drk_ws_create and drk_serve_create /
 *    drk_serve_add_scene; free with drk_ws_destroy / drk_serve_destroy.
 *  - Asynchronous errors (pair-buffer overflow) are recorded in a device status word and reported
 *    by drk_ws_status, which synchronises the stream it is given.
 *  - `stream` is a hipStream_t passed as void* (0 = the null stream).
 */
#ifndef DRK_H
#define DRK_H

#include <stdint.h>
#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  DRK_OK = 0,
  DRK_EINVAL = 1,     /* invalid argument or (validate mode) invalid primitive */
  DRK_ENOMEM = 2,     /* device allocation failed, or a request can never fit the HBM budget */
  DRK_EOVERFLOW = 3,  /* tile-pair buffer too small; drk_ws_status reports the size needed */
  DRK_EAGAIN = 4,     /* try again: request queue full / request still running */
  DRK_ENOTFOUND = 5,  /* unknown request or scene id */
  DRK_EDEVICE = 6     /* HIP runtime error */
} drk_status;

/* Scene: N primitives with K bases (Sec. 4, parameter set Theta).
 *   mu      [3][n]  centres (world)
 *   q       [4][n]  rotation quaternion (w, x, y, z); need not be unit length.  The columns of
 *                   R(q) are the local u axis, v axis and plane normal (3D-GS rotation, Sec. 3.1).
 *   scale   [K][n]  radial basis lengths s_k > 0 (Sec. 4.1)
 *   theta   [K][n]  basis polar angles, ascending in [0, 2*pi), every gap (wrap included) < pi
 *   eta     [n]     L1/L2 blend weight in [0, 1] (Sec. 4.2)
 *   tau     [n]     sharpness in (-1, 1) (Sec. 4.3)
 *   opacity [n]     o in (0, 1]
 *   color   [3][n] (color_mode 0, RGB) or [3*(sh_degree+1)^2][n] (color_mode 1, real SH, row
 *           3*coef + channel, coefficient index l*l + l + m).  Colour = SH(view dir) + 0.5,
 *           clamped at 0, view dir = normalize(mu - camera centre).                          */
typedef struct drk_scene {
  int64_t n;
  int32_t K;            /* 3 <= K <= 16 */
  int32_t color_mode;   /* 0 = RGB, 1 = spherical harmonics */
  int32_t sh_degree;    /* 0..3 when color_mode == 1 */
  int32_t reserved;
  const float* mu;
  const float* q;
  const float* scale;
  const float* theta;
  const float* eta;
  const float* tau;
  const float* opacity;
  const float* color;
} drk_scene;

/* Writable scene arrays (device, caller-allocated), the layout of drk_scene with RGB colour
 * [3][n]: the output of drk_mesh_to_drk.                                                      */
typedef struct drk_scene_out {
  float* mu;
  float* q;
  float* scale;
  float* theta;
  float* eta;
  float* tau;
  float* opacity;
  float* color;
} drk_scene_out;

/* Gradient buffers: same shapes as drk_scene's arrays (device, caller-allocated, overwritten). */
typedef struct drk_scene_grad {
  float* mu;
  float* q;
  float* scale;
  float* theta;
  float* eta;
  float* tau;
  float* opacity;
  float* color;
} drk_scene_grad;

/* Pinhole camera (OpenCV: x right, y down, z forward).  Pixel (x, y) has its centre at
 * (x + 0.5, y + 0.5).  R (row-major) and t map world to camera: X_c = R X_w + t.            */
typedef struct drk_camera {
  int32_t width, height;
  float fx, fy, cx, cy;
  float R[9];
  float t[3];
  float bg[3];          /* background, added with the final transmittance */
} drk_camera;

/* Rasterization options.  Defaults (drk_opts_default): alpha_min 1/255, alpha_max 0.99,
 * T_min 1e-4, near 0.2, lowpass_sl sqrt(2)/2 px (Sec. 4.4 low-pass; 0 disables it),
 * cache_len 8 (Sec. 4.4 cache sorting; 1..8, 1 = pre-sort order only; any value >= 2^30 = the
 * exact per-pixel order: every contribution composited by its hit depth, ties by index, the
 * ideal the cache approximates; drk_render_fwd only, several list passes per frame),
 * cull_mode 0 (0 = conservative support polygon, 1 = the paper's endpoint polygon (lossy),
 * 2 = every tile), validate 0 (1 = return DRK_EINVAL for invalid primitives),
 * key_mode 0: the pre-sort key of the tile lists (supplement, cache-sorting evaluation):
 *   0 = view depth of the primitive's centre (one key per primitive),
 *   1 = "most centric": per (tile, primitive), the depth at which the ray through the centre of
 *       the tile's pixel-centre rectangle, cut to the primitive's projected support box, meets
 *       the primitive's plane (the centre depth when that ray meets it at or behind the near plane),
 *   2 = "nearest": per (tile, primitive), the smallest such depth over the four corner rays of that
 *       rectangle (the support's nearest depth when none meets the plane in front);
 *   keys 1 and 2 are held to the depth range of the support disc (radius sqrt(2) c max_k s_k),
 *   computed in float64 in a fixed order and rounded to float32; ties go to the lower index.    */
typedef struct drk_opts {
  float alpha_min, alpha_max, T_min, near_plane, lowpass_sl;
  int32_t cache_len, cull_mode, validate, key_mode;
  int32_t launch_order;   /* raster launch order of the tiles: 0 (default) longest lists first, so
                             the launch does not end on a few long tiles; 1 row-major, which leaves
                             that tail to kernels of other streams (frames rendered concurrently
                             overlap better).  Images are identical either way.                   */
  int32_t counters;       /* 1: drk_render_fwd also writes the per-pixel work counters that
                             drk_ws_export 5-9 read (instrumentation); 0 (default): it writes only
                             the image and the transmittance.                                       */
} drk_opts;

typedef struct drk_ws drk_ws;

drk_opts drk_opts_default(void);
const char* drk_last_error(void);
const char* drk_version(void);

/* Workspace for up to max_views views of up to max_n primitives with K bases at up to
 * max_w x max_h pixels, with pair_capacity tile-primitive pairs per view.  Allocates device
 * memory on the current device.  Returns DRK_ENOMEM / DRK_EINVAL / DRK_EDEVICE on failure.
 * The preprocess stores each primitive's tile-row spans in a buffer of 16 * max_n + 65536 rows per
 * view; the environment variable DRK_SPAN_ROWS (a non-negative integer, read here and by
 * drk_ws_size_query) sets another size.  Primitives whose rows do not fit have their spans
 * re-derived during drk_bin_sort, which is slower but gives the same pairs. */
drk_status drk_ws_create(int64_t max_n, int32_t K, int32_t max_views, int32_t max_w, int32_t max_h,
                         int64_t pair_capacity, drk_ws** out);
drk_status drk_ws_destroy(drk_ws* ws);
/* Bytes drk_ws_create would allocate for the same arguments (host-only query). */
drk_status drk_ws_size_query(int64_t max_n, int32_t K, int32_t max_views, int32_t max_w, int32_t max_h,
                             int64_t pair_capacity, size_t* bytes);

/* Step 1 (Sec. 4.4 Kernel Culling; Sec. 3.3; SH colour as in 3D-GS).  Per (view, primitive):
 * rotation, view-space centre depth (the global pre-sort key), near/opacity culling, colour,
 * calibrated support radius, conservative support polygon projected and clipped to the near
 * plane, the 16x16 tiles it touches, and the per-primitive record the raster kernels read.
 * cams: HOST array of n_views cameras (copied into the launch).  The scene must stay alive until
 * drk_render_fwd / drk_render_bwd of this frame have been enqueued and completed.
 * Every call ends the workspace's previous frame: after a refused call drk_bin_sort and the
 * renders return DRK_EINVAL until a drk_preprocess succeeds.
 * Returns DRK_EINVAL, before any device work, for options outside these ranges: alpha_min,
 * alpha_max and T_min in (0, 1), near_plane > 0, lowpass_sl >= 0, cache_len in [1, 8] or
 * >= 2^30, cull_mode and key_mode in [0, 2], launch_order and counters 0 or 1.  Likewise for
 * n_views outside [1, max_views], a camera larger than the workspace's max_w x max_h, with a
 * focal length that is not positive or a non-finite or singular R, and for a scene with more
 * than max_n primitives, another K, an sh_degree outside [0, 3] with SH colour, or a null array
 * when n > 0. */
drk_status drk_preprocess(drk_ws* ws, const drk_scene* scene, const drk_camera* cams, int32_t n_views,
                          const drk_opts* opts, void* stream);

/* Step 2 (Sec. 4.4 Kernel Culling + Cache Sorting pre-sort).  Per view, key_mode 0: stable
 * radix sort of primitives by centre depth, duplication into (tile, primitive) pairs in that
 * order, stable radix sort of the pairs by tile id.  key_mode 1 or 2: duplication in primitive
 * order with the per-pair key, stable radix sort of the pairs by key, then by tile id.  Then
 * per-tile [start, end) ranges, and (launch_order 0) the raster's launch order: tiles by
 * decreasing list length (the longest lists start first).  The
 * resulting per-tile lists are ordered by (tile, key, primitive index).  If a view needs more pairs than pair_capacity the overflow is recorded
 * (see drk_ws_status) and that view renders nothing.                                         */
drk_status drk_bin_sort(drk_ws* ws, void* stream);

/* Step 3 (Eq. 1; Sec. 3.3; Sec. 4.1-4.4; Algorithm 1).  Per pixel: ray-plane hit through each
 * listed primitive, DRK kernel, low-pass, cutoffs, cache sorting (cache_len slots) and
 * front-to-back compositing with early termination.
 *   rgb     [V][3][H][W] float32 output (H, W of each view's camera; views packed back to back)
 *   T_final [V][H][W]    float32 output: final transmittance (may be NULL)                   */
drk_status drk_render_fwd(drk_ws* ws, float* rgb, float* T_final, void* stream);

/* drk_render_fwd that also records, per pixel, the composited contributions in front-to-back
 * order (supplement, cache-sorting evaluation: the depths processed front to back):
 *   trace_n   [V][H][W]       int32 output: contributions composited at the pixel (not capped)
 *   trace_idx [V][H][W][cap]  int32 output: primitive index of the first min(n, cap) of them
 *   trace_z   [V][H][W][cap]  float32 output: view depth of their hit (the cache key)
 * Entries past min(n, cap) are left untouched.  1 <= cap <= 1024, else DRK_EINVAL.            */
drk_status drk_render_trace(drk_ws* ws, float* rgb, float* T_final, int32_t cap, int32_t* trace_n,
                            int32_t* trace_idx, float* trace_z, void* stream);

/* Sorting-accuracy measures of recorded traces (device arrays as written by drk_render_trace,
 * npx pixels, the first m = min(trace_n, cap) depths of each; cap <= 64).  out: 6 doubles
 * (device), overwritten: [0] sum of m, [1] positions holding the depth the sorted sequence holds
 * there, [2] sum over pixels with m >= 2 of Kendall's tau between composite order and depth
 * (ties count as neither concordant nor discordant), [3] pixels with m >= 2, [4] sum of
 * |depth - sorted depth| per position, [5] pixels with trace_n > cap.  Accuracy = [1]/[0],
 * mean tau = [2]/[3], MAE = [4]/[0].  The sums use float atomics (the order of additions, and
 * so the last bits, may vary between calls).                                                  */
drk_status drk_trace_metrics(const int32_t* trace_n, const float* trace_z, int64_t npx, int32_t cap, double* out,
                             void* stream);

/* drk_render_fwd that also writes the depth and normal channels (supplement, mesh conversion:
 * rendered depth and normal images), blended with the colour's weights T_i alpha_i (Eq. 1):
 *   depth  [V][H][W]     float32 output: sum of T_i alpha_i * view depth of the hit
 *   normal [V][3][H][W]  float32 output: sum of T_i alpha_i * unit camera-frame normal of the
 *                        primitive's plane, turned toward the camera
 * Divide by 1 - T_final for the expected depth and normal of the covered part.                */
drk_status drk_render_depth_normal(drk_ws* ws, float* rgb, float* T_final, float* depth, float* normal,
                                   void* stream);

/* Parametrization (supplement S4): raw, unconstrained parameters -> the renderer's parameters.
 *   raw  a drk_scene whose arrays hold raw values (same shapes; q need not be unit length)
 *   out  the activated arrays (same shapes), written:
 *        mu, colour copied; q / |q|; s_k = exp(raw); eta, o = sigmoid(raw);
 *        tau = -0.1 + 1.09 sigmoid(raw), in (-0.1, 0.99);
 *        theta: sector gaps proportional to sigmoid(raw_k) + 1/(K - 2), summing to 2 pi,
 *        theta_k = the gaps before k (theta_0 = 0); every gap is below pi unless the sigmoids
 *        saturate in float32 (|raw| above about 17), where a gap of pi makes the primitive invalid.
 * Float32, one thread per primitive.                                                            */
drk_status drk_activate(const drk_scene* raw, const drk_scene_out* out, void* stream);

/* Vector-Jacobian product of drk_activate: from dL/d(activated) (g_act, read) and the raw
 * parameters, writes dL/d(raw) into g_raw (same shapes).                                        */
drk_status drk_activate_bwd(const drk_scene* raw, const drk_scene_grad* g_act, const drk_scene_out* g_raw,
                            void* stream);

/* One Adam step (bias-corrected; the supplement's training follows 3D-GS's Adam) on n float32
 * elements in place: m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
 * p -= lr (m / (1 - b1^step)) / (sqrt(v / (1 - b2^step)) + eps).  step >= 1.                    */
drk_status drk_adam_step(float* param, float* m, float* v, const float* grad, int64_t n, float lr, float beta1,
                         float beta2, float eps, int32_t step, void* stream);

/* Mesh to DRK (section "Converting Mesh to DRK" and its supplement): one DRK per planar convex
 * face, with the basis endpoints at the face's vertices, without any optimisation.
 *   vertices [3][nv] float32 (device)      faces [nf][m] int32 vertex indices (device), -1 pads
 *   face_rgb [3][nf] float32 (device)      K: bases per DRK, 3 <= K <= 16, m <= K
 * Per face (float64): centre = mean of the vertices; t_u toward the first vertex; normal from the
 * face's winding; theta_k = the vertex directions in the listed order (theta_0 = 0); faces with
 * fewer than K vertices get endpoints evenly spaced along their edges (edge i takes
 * floor((K-m')/m') of them, one more when i < (K-m') mod m'); s_k = distance / sqrt(2 ln 2), so the
 * face outline is the alpha = o/2 contour; eta = 1 (straight L1 edges), the given tau and opacity,
 * the face's RGB colour.  A face that is degenerate, not convex, has an index outside [0, nv) or
 * a sector of pi or more gets opacity 0 (never rendered) and is counted in *rejected (device
 * uint32, may be NULL; overwritten).                                                           */
drk_status drk_mesh_to_drk(const float* vertices, int64_t nv, const int32_t* faces, int64_t nf, int32_t m,
                           const float* face_rgb, int32_t K, float tau, float opacity, const drk_scene_out* out,
                           uint32_t* rejected, void* stream);

/* Step 4 (supplement S4: backward front to back, consistent with cache sorting).  Recomputes
 * each pixel's emission sequence and accumulates dL/dparameter for every primitive:
 *   rgb      [V][3][H][W]  the forward output (read)
 *   dL_drgb  [V][3][H][W]  upstream gradient (read)
 *   grads    same shapes as the scene arrays; zeroed and written by the call.
 * Gradients of all views are summed into one set of buffers.
 * Currently switched off: returns DRK_EDEVICE (with a message in drk_last_error) without
 * touching the device, because its kernels took an unexplained illegal memory access on gfx950. */
drk_status drk_render_bwd(drk_ws* ws, const drk_scene* scene, const float* rgb, const float* dL_drgb,
                          const drk_scene_grad* grads, void* stream);

/* Number of drk_preprocess calls made on the workspace so far (host-side, no synchronisation).
 * The lists, records and per-pixel state drk_render_bwd replays belong to the latest one, so a
 * caller that keeps a forward output for a later backward records this value with it and checks
 * that it is unchanged before calling drk_render_bwd.                                          */
drk_status drk_ws_generation(drk_ws* ws, uint64_t* generation);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): drk_preprocess -> drk_bin_sort -> drk_render_fwd of ONE
 * view without a workspace.  Every intermediate lives in a fixed device array of the library
 * (128 MiB per GPU, reserved from the first call on that GPU until the process ends); the pair
 * capacity is whatever that array holds beyond the scene- and image-sized parts.
 *   scene, cam, opts  as for drk_preprocess (one camera; opts->counters must be 0)
 *   rgb [3][H][W], T_final [H][W] (may be NULL): device, caller-owned, written
 * The call synchronises `stream` and returns the frame's final status: DRK_ENOMEM (nothing
 * enqueued) when the scene and image alone do not fit the array, DRK_EOVERFLOW when the frame's
 * tile pairs do not (the image is then incomplete), DRK_EINVAL for invalid arguments or (validate
 * mode) invalid primitives.  Allocates no memory of any kind.  Calls on one GPU share its array
 * and keep its last contents: calls that overlap on the same GPU (several host threads or
 * streams) race and must be serialised by the caller.                                          */
drk_status drk_render_fwd_noalloc(const drk_scene* scene, const drk_camera* cam, const drk_opts* opts, float* rgb,
                                  float* T_final, void* stream);

/* Synchronises `stream` and reports the status word: DRK_OK, or DRK_EOVERFLOW with
 * *pairs_needed set to the largest pair count any view of the last drk_bin_sort needed.      */
drk_status drk_ws_status(drk_ws* ws, void* stream, int64_t* pairs_needed);

/* Inspection (tests and tools): copy an internal array of view `view` into `dst` (device),
 * at most `bytes` bytes, enqueued on `stream`.  *out_count (host) receives the element count.
 * Synchronises `stream` to read counts.  what:
 *   0 depth keys   uint32 [n]   (float32 bits of the centre depth; 0xFFFFFFFF when culled)
 *   1 tile counts  uint32 [n]   (tiles touched per primitive, primitive order)
 *   2 pair tiles   uint32 [P]   (sorted)
 *   3 pair prims   uint32 [P]   (sorted)
 *   4 ranges       uint32 [2*tiles] (start, end per tile)
 * Exports 5-9 need a forward rendered with drk_opts.counters = 1 (else DRK_EINVAL):
 *   5 emitted      int32  [H*W] (contributions composited per pixel, from the last forward)
 *   6 consumed     int32  [H*W] (list entries read per pixel before it terminated)
 *   7 contributors int32  [H*W] (entries with alpha >= alpha_min that entered the cache)
 *   8 hits         int32  [H*W] (entries whose ray-plane hit was evaluated)
 *   9 kernels      int32  [H*W] (entries that went through the full kernel evaluation)
 *  10 pair keys    uint32 [P]   (pre-sort key of each sorted pair: float32 bits)               */
drk_status drk_ws_export(drk_ws* ws, int32_t view, int32_t what, void* dst, int64_t bytes, int64_t* out_count,
                         void* stream);

/* ---------------------------------------------------------------------------------------------
 * Serving: a continuous-batching request loop.  Scenes are copied into resident device memory
 * once; requests (scene, camera) arrive at any time and are admitted while the HBM budget and
 * the in-flight limit allow; admitted requests run concurrently on separate streams with
 * per-(scene, resolution) workspaces whose launches are captured in HIP graphs.            */
typedef struct drk_server drk_server;

typedef struct drk_serve_cfg {
  int64_t hbm_budget_bytes;   /* device memory the server may use for workspaces (0 = 50% of free) */
  int32_t max_inflight;       /* requests on the GPU at once (streams) */
  int32_t queue_capacity;     /* pending requests before submit returns DRK_EAGAIN */
  int32_t use_graphs;         /* 1 = capture per-workspace launch sequences in HIP graphs */
  int32_t initial_pairs;      /* first pair capacity of a new workspace (0 = from scene and image size);
                                 a request that overflows is rerun with a larger workspace */
  drk_opts opts;
} drk_serve_cfg;

typedef struct drk_req_stats {
  double submit_us, start_us, done_us;   /* host monotonic clock, microseconds */
  int64_t pairs;                          /* tile pairs the request needed */
  int32_t status;                         /* drk_status of the request */
  int32_t width, height;
} drk_req_stats;

drk_status drk_serve_create(const drk_serve_cfg* cfg, drk_server** out);
drk_status drk_serve_destroy(drk_server* srv);
/* Copies the scene's arrays (device pointers) into memory owned by the server. */
drk_status drk_serve_add_scene(drk_server* srv, const drk_scene* scene, int32_t* scene_id);
/* Enqueue a render of scene_id from *cam into out_rgb ([3][H][W] float32, device, caller-owned,
 * must stay alive until the request completes).  DRK_EAGAIN if the queue is full, DRK_ENOMEM if
 * the request could never fit the budget, DRK_ENOTFOUND for an unknown scene.               */
drk_status drk_serve_submit(drk_server* srv, int32_t scene_id, const drk_camera* cam, float* out_rgb,
                            uint64_t* request_id);
/* DRK_OK when done (stats filled, the request is then forgotten), DRK_EAGAIN while pending
 * (after waiting up to wait_us microseconds), DRK_ENOTFOUND for an unknown id.               */
drk_status drk_serve_poll(drk_server* srv, uint64_t request_id, int32_t wait_us, drk_req_stats* out);

#ifdef __cplusplus
}
#endif

#endif /* DRK_H */
