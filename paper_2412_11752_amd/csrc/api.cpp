// Host side of libdrk: workspace management and the C ABI entry points of include/drk.h.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <cstdlib>
#include <string>
#include <vector>

#include "drk_internal.hpp"

namespace drk {

// last error message of this thread (fixed storage: reporting an error allocates nothing)
static thread_local char g_err[512];

void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}

// kernels in other translation units
hipError_t set_views(Views*, const Views&, hipStream_t);
hipError_t launch_preprocess(const SceneDev&, const Views*, int, const OptsDev&, float*, uint32_t*, uint32_t*,
                             uint32_t*, uint32_t*, uint32_t*, uint32_t*, uint2*, uint32_t*, uint32_t*, int64_t,
                             uint32_t*, int64_t, double*, hipStream_t);
hipError_t launch_duplicate(const SceneDev&, const Views*, const OptsDev&, int, const uint32_t*, const uint32_t*,
                            const uint32_t*, const uint2*, const uint32_t*, uint32_t*, uint32_t*, const uint64_t*,
                            int64_t, const uint64_t*, uint32_t*, uint32_t*, const double*, uint32_t*, hipStream_t);
hipError_t launch_pair_keys(const Views*, const OptsDev&, int, const uint32_t*, const uint32_t*, int64_t,
                            const uint32_t*, const double*, uint32_t*, hipStream_t);
hipError_t gather_pairs(const uint32_t*, const uint32_t*, const uint32_t*, const uint64_t*, uint32_t*, uint32_t*,
                        hipStream_t);
hipError_t launch_trace_metrics(const int32_t*, const float*, int64_t, int, double*, hipStream_t);
hipError_t radix_sort(int, const uint64_t*, uint32_t* const*, uint32_t* const*, int, uint32_t*, uint32_t*, hipStream_t);
hipError_t scan_counts(const uint32_t*, const uint32_t*, const uint64_t*, int64_t, uint32_t*, uint64_t*, uint64_t*,
                       uint64_t*, int64_t, uint32_t*, hipStream_t);
hipError_t compact_visible(const uint32_t*, const uint32_t*, int64_t, uint32_t*, uint64_t*, uint64_t*, uint64_t*,
                           uint32_t*, uint32_t*, uint32_t*, hipStream_t);
hipError_t tile_ranges(const uint32_t*, const uint64_t*, uint32_t*, int, hipStream_t);
hipError_t tile_length_keys(const uint32_t*, int, uint32_t*, uint32_t*, hipStream_t);
hipError_t set_u64(uint64_t*, uint64_t, hipStream_t);
hipError_t fill_u32(uint32_t*, uint32_t, int64_t, hipStream_t);
hipError_t launch_render_fwd(int, const float*, const uint32_t*, const uint32_t*, const CamDev*, int, const uint32_t*,
                             const OptsDev&,
                             float*, float*, int32_t*, int32_t*, int32_t*, int32_t*, int, void*, int32_t*, float*, int,
                             hipStream_t);
hipError_t launch_activate(const drk_scene&, const drk_scene_out&, int, hipStream_t);
hipError_t launch_activate_bwd(const drk_scene&, const drk_scene_grad&, const drk_scene_out&, int, hipStream_t);
hipError_t launch_adam(float*, float*, float*, const float*, int64_t, float, float, float, float, int, hipStream_t);
hipError_t launch_mesh_to_drk(const float*, int64_t, const int32_t*, int64_t, int, const float*, int, float, float,
                              const drk_scene_out&, uint32_t*, hipStream_t);
hipError_t launch_render_bwd(int, const float*, const uint32_t*, const uint32_t*, const CamDev*, int, const OptsDev&,
                             const float*, const float*, float*, int64_t, hipStream_t);
hipError_t launch_preprocess_bwd(const SceneDev&, const Views*, const OptsDev&, const uint32_t*, const float*, int64_t,
                                 const drk_scene_grad&, hipStream_t);

}  // namespace drk

using namespace drk;

struct drk_ws {
  int device = 0;
  int64_t max_n = 0;
  int K = 0, RF = 0, max_views = 0, max_w = 0, max_h = 0, max_tiles = 0;
  int64_t cap = 0;
  size_t bytes = 0;
  std::vector<void*> allocs;

  float* records = nullptr;
  uint32_t* depth_keys = nullptr;
  uint32_t* tile_counts = nullptr;
  uint32_t *dk_a = nullptr, *dv_a = nullptr, *dk_b = nullptr, *dv_b = nullptr;
  uint32_t* offsets = nullptr;
  uint64_t* block_tot = nullptr;
  uint32_t *pk_tmp = nullptr, *pv_tmp = nullptr, *pk_tmp2 = nullptr, *pv_tmp2 = nullptr;
  uint32_t *pair_tiles = nullptr, *pair_prims = nullptr;
  uint32_t* ranges = nullptr;
  uint64_t* totals = nullptr;
  uint64_t* n_eff = nullptr;
  uint64_t* n_prims = nullptr;      // [0] visible primitives of the view being binned, [1] scratch
  uint32_t *ck = nullptr, *cv = nullptr;   // compacted visible (key, index)
  uint32_t* status = nullptr;
  int32_t *n_emit = nullptr, *consumed = nullptr, *contrib = nullptr, *work_px = nullptr;
  uint32_t *hist = nullptr, *tot = nullptr;
  float* grad_rec = nullptr;
  Views* views_dev = nullptr;     // cameras read by every kernel (set by a one-thread kernel)
  uint32_t* work = nullptr;       // per view: primitives that may touch the view (small list), then per view the big list
  uint32_t* counters = nullptr;   // small and big list counts per view, then kSpanPools span-row pool fills per view
  uint2* span_meta = nullptr;     // per view and primitive: row-span offset, first row | rows << 16
  uint32_t* span_rows = nullptr;  // per view: tile columns i0 | i1 << 16 of each spanned row
  int64_t row_cap = 0;
  float* out_rgb = nullptr;       // internal output image [3][max_h][max_w] (graph-captured renders)
  uint32_t* dup_big = nullptr;    // sorted slots of the primitives duplicated a workgroup at a time
  uint32_t* dup_count = nullptr;  // their count
  double* keygeo = nullptr;       // per view and primitive: float64 data of the per-tile keys (KG_N)
  uint32_t* tile_order = nullptr; // per view: tiles by decreasing list length (the raster's launch order)
  uint32_t* tk = nullptr;         // tile-order sort scratch: 4 x max_tiles

  SceneDev scene{};
  Views views{};
  OptsDev opts{};
  bool have_pre = false, have_bins = false;
  bool counted = false;           // the last forward wrote the per-pixel counters (exports 5-9)
  bool lean = false;              // forward-only layout: no backward, counter or serving arrays
  bool lean_keys = false;         // (lean layout) keep the per-tile key data (key_mode 1, 2)
  uint64_t generation = 0;        // preprocess calls so far: identifies the frame the lists belong to
};

namespace {

// The backward raster and per-primitive backward kernels took an illegal memory access on gfx950
// that a CPU build of the same kernels (ASan, per-slot allocations, garbage-filled memory, index
// asserts) does not reproduce; until the cause is shown, drk_render_bwd returns DRK_EDEVICE.
constexpr bool kBackwardEnabled = false;

struct Plan {
  size_t off = 0;
  template <class T>
  size_t add(size_t count) {
    size_t o = (off + 255) & ~(size_t)255;
    off = o + count * sizeof(T);
    return o;
  }
};

size_t layout(drk_ws* ws, bool assign, char* base) {
  Plan p;
  const size_t N = (size_t)ws->max_n, V = (size_t)ws->max_views, cap = (size_t)ws->cap;
  const size_t px = (size_t)ws->max_w * ws->max_h;
#define SLOT(field, T, count)                       \
  {                                                 \
    size_t o = p.add<T>(count);                     \
    if (assign) ws->field = reinterpret_cast<T*>(base + o); \
  }
  SLOT(records, float, V * N * ws->RF)
  SLOT(depth_keys, uint32_t, V * N)
  SLOT(tile_counts, uint32_t, V * N)
  SLOT(dk_a, uint32_t, N)
  SLOT(dv_a, uint32_t, N)
  SLOT(dk_b, uint32_t, N)
  SLOT(dv_b, uint32_t, N)
  SLOT(offsets, uint32_t, N)
  SLOT(block_tot, uint64_t, N / 1024 + 2)
  SLOT(pk_tmp, uint32_t, cap)
  SLOT(pv_tmp, uint32_t, cap)
  SLOT(pk_tmp2, uint32_t, cap)
  SLOT(pv_tmp2, uint32_t, cap)
  SLOT(pair_tiles, uint32_t, V * cap)
  SLOT(pair_prims, uint32_t, V * cap)
  SLOT(ranges, uint32_t, V * 2 * ws->max_tiles)
  SLOT(totals, uint64_t, V)
  SLOT(n_eff, uint64_t, V)
  SLOT(n_prims, uint64_t, 2)
  SLOT(ck, uint32_t, N)
  SLOT(cv, uint32_t, N)
  SLOT(status, uint32_t, V)
  SLOT(n_emit, int32_t, ws->lean ? 0 : V * px)
  SLOT(consumed, int32_t, ws->lean ? 0 : V * px)
  SLOT(contrib, int32_t, ws->lean ? 0 : V * px)
  SLOT(work_px, int32_t, ws->lean ? 0 : 2 * V * px)
  SLOT(hist, uint32_t, 256 * 1024)
  SLOT(tot, uint32_t, 256)
  SLOT(grad_rec, float, ws->lean ? 0 : V * N * grad_fields(ws->K))
  SLOT(views_dev, Views, 1)
  SLOT(work, uint32_t, 2 * V * N)
  SLOT(counters, uint32_t, (2 + kSpanPools) * V)
  SLOT(span_meta, uint2, V * N)
  SLOT(span_rows, uint32_t, V * (size_t)ws->row_cap)
  SLOT(out_rgb, float, ws->lean ? 0 : 3 * px)
  SLOT(dup_big, uint32_t, N)
  SLOT(dup_count, uint32_t, 4)
  SLOT(keygeo, double, (ws->lean && !ws->lean_keys) ? 0 : V * N * KG_N)
  SLOT(tile_order, uint32_t, V * (size_t)ws->max_tiles)
  SLOT(tk, uint32_t, 4 * (size_t)ws->max_tiles)
#undef SLOT
  return p.off;
}

drk_status check_hip(hipError_t e, const char* what) {
  if (e == hipSuccess) return DRK_OK;
  set_error("%s: %s", what, hipGetErrorString(e));
  return DRK_EDEVICE;
}

bool valid_ws_args(int64_t max_n, int32_t K, int32_t max_views, int32_t max_w, int32_t max_h, int64_t cap) {
  if (max_n < 0 || max_n > (int64_t)0xFFFFFFF0) { set_error("max_n out of range"); return false; }
  if (K < 3 || K > kMaxK) { set_error("K must be in [3, %d]", kMaxK); return false; }
  if (max_views < 1 || max_views > kMaxViews) { set_error("max_views must be in [1, %d]", kMaxViews); return false; }
  if (max_w < 1 || max_h < 1 || max_h > kMaxTileRows * kTile || max_w > 8192) {
    set_error("image size must be within 8192 x %d", kMaxTileRows * kTile);
    return false;
  }
  if (cap < 1 || cap > (int64_t)0xFFFFFF00) { set_error("pair_capacity out of range"); return false; }
  return true;
}

}  // namespace

namespace drk {

hipError_t fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t s);

}  // namespace drk

namespace drk {

drk_status ws_set_cameras(drk_ws* ws, const drk_camera* cams, int32_t n_views, hipStream_t s) {
  if (!ws || !cams) { set_error("null argument"); return DRK_EINVAL; }
  if (n_views < 1 || n_views > ws->max_views) { set_error("n_views %d outside [1, %d]", n_views, ws->max_views); return DRK_EINVAL; }
  Views views{};
  views.nv = n_views;
  for (int v = 0; v < n_views; ++v) {
    const drk_camera& c = cams[v];
    if (c.width < 1 || c.height < 1 || c.width > ws->max_w || c.height > ws->max_h) {
      set_error("camera %d size %dx%d exceeds workspace %dx%d", v, c.width, c.height, ws->max_w, ws->max_h);
      return DRK_EINVAL;
    }
    if (!(c.fx > 0.0f) || !(c.fy > 0.0f)) { set_error("camera %d focal length must be positive", v); return DRK_EINVAL; }
    for (int i = 0; i < 9; ++i)
      if (!isfinite(c.R[i])) { set_error("camera %d rotation is not finite", v); return DRK_EINVAL; }
    CamDev& d = views.cam[v];
    d.W = c.width; d.H = c.height;
    d.tiles_x = (c.width + kTile - 1) / kTile; d.tiles_y = (c.height + kTile - 1) / kTile;
    d.fx = c.fx; d.fy = c.fy; d.cx = c.cx; d.cy = c.cy;
    for (int i = 0; i < 9; ++i) d.R[i] = c.R[i];
    for (int i = 0; i < 3; ++i) { d.t[i] = c.t[i]; d.bg[i] = c.bg[i]; }
    // camera centre: the exact inverse of the float32 R (its transpose is only approximately it)
    {
      double m[9];
      for (int i = 0; i < 9; ++i) m[i] = (double)c.R[i];
      const double c0 = m[4] * m[8] - m[5] * m[7], c1 = m[5] * m[6] - m[3] * m[8], c2 = m[3] * m[7] - m[4] * m[6];
      const double det = m[0] * c0 + m[1] * c1 + m[2] * c2;
      if (!(fabs(det) > 1e-6)) { set_error("camera %d rotation is singular", v); return DRK_EINVAL; }
      const double inv[9] = {c0 / det, (m[2] * m[7] - m[1] * m[8]) / det, (m[1] * m[5] - m[2] * m[4]) / det,
                             c1 / det, (m[0] * m[8] - m[2] * m[6]) / det, (m[2] * m[3] - m[0] * m[5]) / det,
                             c2 / det, (m[1] * m[6] - m[0] * m[7]) / det, (m[0] * m[4] - m[1] * m[3]) / det};
      for (int i = 0; i < 3; ++i)
        d.campos[i] = -(inv[3 * i] * (double)c.t[0] + inv[3 * i + 1] * (double)c.t[1] + inv[3 * i + 2] * (double)c.t[2]);
    }
  }
  drk_status st = check_hip(set_views(ws->views_dev, views, s), "set cameras");
  if (st) return st;
  ws->views = views;
  return DRK_OK;
}

// Integer from the environment variable `name`, or `def` when it is unset, malformed or out of
// [lo, hi].
static int64_t env_int(const char* name, int64_t def, int64_t lo, int64_t hi) {
  const char* e = std::getenv(name);
  if (!e) return def;
  char* end = nullptr;
  const long long v = std::strtoll(e, &end, 10);
  return (end != e && *end == '\0' && v >= lo && v <= hi) ? (int64_t)v : def;
}

// Host-side checks of a frame's scene and options against the workspace (no device work).
bool valid_frame_args(const drk_ws* ws, const drk_scene* scene, const drk_opts* opts) {
  if (!ws || !scene || !opts) { set_error("null argument"); return false; }
  if (scene->n < 0 || scene->n > ws->max_n) { set_error("scene n %lld exceeds workspace max_n %lld", (long long)scene->n, (long long)ws->max_n); return false; }
  if (scene->K != ws->K) { set_error("scene K %d != workspace K %d", scene->K, ws->K); return false; }
  if (scene->color_mode != 0 && scene->color_mode != 1) { set_error("color_mode must be 0 or 1"); return false; }
  if (scene->color_mode == 1 && (scene->sh_degree < 0 || scene->sh_degree > 3)) { set_error("sh_degree must be in [0, 3]"); return false; }
  if (scene->n > 0 && (!scene->mu || !scene->q || !scene->scale || !scene->theta || !scene->eta || !scene->tau ||
                       !scene->opacity || !scene->color)) {
    set_error("scene array is null");
    return false;
  }
  if (!(opts->alpha_min > 0.0f && opts->alpha_min < 1.0f) || !(opts->alpha_max > 0.0f && opts->alpha_max < 1.0f) ||
      !(opts->T_min > 0.0f && opts->T_min < 1.0f) || !(opts->near_plane > 0.0f) || !(opts->lowpass_sl >= 0.0f) ||
      opts->cache_len < 1 || (opts->cache_len > kMaxCache && opts->cache_len < kExactOrder) || opts->cull_mode < 0 ||
      opts->cull_mode > 2 ||
      opts->key_mode < 0 || opts->key_mode > 2 || opts->launch_order < 0 || opts->launch_order > 1 ||
      opts->counters < 0 || opts->counters > 1) {
    set_error("invalid drk_opts (cache_len must be in [1, %d] or at least 2^30 for the exact order, key_mode in "
              "[0, 2], launch_order and counters 0 or 1)", kMaxCache);
    return false;
  }
  return true;
}

drk_status ws_preprocess_core(drk_ws* ws, const drk_scene* scene, const drk_opts* opts, hipStream_t s) {
  if (!valid_frame_args(ws, scene, opts)) return DRK_EINVAL;
  if (ws->views.nv < 1) { set_error("no cameras set"); return DRK_EINVAL; }
  SceneDev sc;
  sc.n = scene->n; sc.K = scene->K; sc.color_mode = scene->color_mode;
  sc.sh_degree = scene->color_mode == 1 ? scene->sh_degree : 0;
  sc.ncol = scene->color_mode == 1 ? 3 * (sc.sh_degree + 1) * (sc.sh_degree + 1) : 3;
  sc.mu = scene->mu; sc.q = scene->q; sc.scale = scene->scale; sc.theta = scene->theta;
  sc.eta = scene->eta; sc.tau = scene->tau; sc.opacity = scene->opacity; sc.color = scene->color;
  OptsDev od;
  od.alpha_min = opts->alpha_min; od.alpha_max = opts->alpha_max; od.T_min = opts->T_min;
  od.near_plane = opts->near_plane; od.lowpass_sl = opts->lowpass_sl; od.cache_len = opts->cache_len;
  od.cull_mode = opts->cull_mode; od.validate = opts->validate; od.key_mode = opts->key_mode;
  od.launch_order = opts->launch_order;
  od.counters = opts->counters;
  // the thread-per-primitive polygon walk runs from 131072 small primitives on (enough threads for
  // 2 waves per SIMD of it); DRK_SMALL_MIN and DRK_WINDOW_ADMIT change that choice for tests
  od.small_min = (int32_t)env_int("DRK_SMALL_MIN", 131072, 0, 1 << 30);
  od.win_admit = (int32_t)env_int("DRK_WINDOW_ADMIT", 4, 1, 64);
  drk_status st = check_hip(fill_u32(ws->status, 0u, ws->max_views, s), "clear status");
  if (st) return st;
  if ((st = check_hip(fill_u32(ws->counters, 0u, (2 + kSpanPools) * ws->max_views, s), "clear counters"))) return st;
  const int V = ws->max_views;
  st = check_hip(launch_preprocess(sc, ws->views_dev, ws->views.nv, od, ws->records, ws->depth_keys, ws->tile_counts,
                                   ws->work, ws->counters, ws->work + (size_t)V * ws->max_n, ws->counters + V,
                                   ws->span_meta, ws->span_rows, ws->counters + 2 * V, ws->row_cap, ws->status,
                                   ws->max_n, ws->keygeo, s),
                 "preprocess launch");
  if (st) return st;
  ws->scene = sc;
  ws->opts = od;
  ws->have_pre = true;
  ws->have_bins = false;
  ++ws->generation;
  return DRK_OK;
}

float* ws_out_rgb(drk_ws* ws) { return ws->out_rgb; }
void ws_status_ptrs(drk_ws* ws, uint32_t** status, uint64_t** totals) {
  *status = ws->status;
  *totals = ws->totals;
}
size_t ws_bytes(drk_ws* ws) { return ws->bytes; }
int64_t ws_capacity(drk_ws* ws) { return ws->cap; }

// Reads the status words (the caller has synchronised the stream).
drk_status ws_read_status(drk_ws* ws, int64_t* pairs_needed) {
  std::vector<uint32_t> status(ws->max_views);
  std::vector<uint64_t> totals(ws->max_views);
  drk_status st;
  if ((st = check_hip(hipMemcpy(status.data(), ws->status, sizeof(uint32_t) * ws->max_views, hipMemcpyDeviceToHost),
                      "read status")))
    return st;
  if ((st = check_hip(hipMemcpy(totals.data(), ws->totals, sizeof(uint64_t) * ws->max_views, hipMemcpyDeviceToHost),
                      "read totals")))
    return st;
  uint32_t all = 0;
  uint64_t need = 0;
  const int nv = ws->have_pre ? ws->views.nv : 0;
  for (int v = 0; v < nv; ++v) {
    all |= status[v];
    need = std::max(need, totals[v]);
  }
  if (pairs_needed) *pairs_needed = (int64_t)need;
  if (all & ST_INVALID) { set_error("invalid primitive parameters (validate mode)"); return DRK_EINVAL; }
  if (all & ST_OVERFLOW) {
    set_error("tile-pair buffer overflow: need %llu pairs, capacity %lld", (unsigned long long)need, (long long)ws->cap);
    return DRK_EOVERFLOW;
  }
  return DRK_OK;
}

}  // namespace drk

extern "C" {

drk_opts drk_opts_default(void) {
  drk_opts o;
  o.alpha_min = 1.0f / 255.0f;
  o.alpha_max = 0.99f;
  o.T_min = 1e-4f;
  o.near_plane = 0.2f;
  o.lowpass_sl = 0.70710678118654752f;
  o.cache_len = 8;
  o.cull_mode = 0;
  o.validate = 0;
  o.key_mode = 0;
  o.launch_order = 0;
  o.counters = 0;
  return o;
}

const char* drk_last_error(void) { return g_err; }

const char* drk_version(void) { return "libdrk 0.1 (gfx950)"; }

// Rows of stored tile-row spans per view: 16 per primitive plus 65536 unless DRK_SPAN_ROWS gives
// another count (primitives whose rows do not fit are re-derived during duplication).
static int64_t span_row_capacity(int64_t max_n) {
  if (const char* e = std::getenv("DRK_SPAN_ROWS")) {
    char* end = nullptr;
    const long long v = std::strtoll(e, &end, 10);
    if (end != e && *end == '\0' && v >= 0) return (int64_t)v;
  }
  return 16 * max_n + 65536;
}

drk_status drk_ws_size_query(int64_t max_n, int32_t K, int32_t max_views, int32_t max_w, int32_t max_h,
                             int64_t pair_capacity, size_t* bytes) {
  if (!bytes) { set_error("bytes is null"); return DRK_EINVAL; }
  if (!valid_ws_args(max_n, K, max_views, max_w, max_h, pair_capacity)) return DRK_EINVAL;
  drk_ws tmp;
  tmp.max_n = max_n; tmp.K = K; tmp.RF = rec_floats(K); tmp.max_views = max_views;
  tmp.max_w = max_w; tmp.max_h = max_h; tmp.cap = pair_capacity;
  tmp.max_tiles = ((max_w + kTile - 1) / kTile) * ((max_h + kTile - 1) / kTile);
  tmp.row_cap = span_row_capacity(max_n);
  *bytes = layout(&tmp, false, nullptr);
  return DRK_OK;
}

drk_status drk_ws_create(int64_t max_n, int32_t K, int32_t max_views, int32_t max_w, int32_t max_h,
                         int64_t pair_capacity, drk_ws** out) {
  if (!out) { set_error("out is null"); return DRK_EINVAL; }
  *out = nullptr;
  if (!valid_ws_args(max_n, K, max_views, max_w, max_h, pair_capacity)) return DRK_EINVAL;
  drk_ws* ws = new drk_ws();
  ws->max_n = max_n; ws->K = K; ws->RF = rec_floats(K); ws->max_views = max_views;
  ws->max_w = max_w; ws->max_h = max_h; ws->cap = pair_capacity;
  ws->max_tiles = ((max_w + kTile - 1) / kTile) * ((max_h + kTile - 1) / kTile);
  ws->row_cap = span_row_capacity(max_n);
  if (hipGetDevice(&ws->device) != hipSuccess) { delete ws; set_error("hipGetDevice failed"); return DRK_EDEVICE; }
  size_t bytes = layout(ws, false, nullptr);
  void* base = nullptr;
  hipError_t e = hipMalloc(&base, bytes);
  if (e != hipSuccess) {
    delete ws;
    set_error("hipMalloc(%zu bytes) failed: %s", bytes, hipGetErrorString(e));
    return DRK_ENOMEM;
  }
  ws->allocs.push_back(base);
  ws->bytes = bytes;
  layout(ws, true, reinterpret_cast<char*>(base));
  *out = ws;
  return DRK_OK;
}

drk_status drk_ws_destroy(drk_ws* ws) {
  if (!ws) return DRK_OK;
  for (void* p : ws->allocs) hipFree(p);
  delete ws;
  return DRK_OK;
}

drk_status drk_preprocess(drk_ws* ws, const drk_scene* scene, const drk_camera* cams, int32_t n_views,
                          const drk_opts* opts, void* stream) {
  if (!ws) { set_error("null workspace"); return DRK_EINVAL; }
  // the earlier frame is given up whatever the outcome: past the checks its cameras are replaced
  ws->have_pre = ws->have_bins = false;
  if (!drk::valid_frame_args(ws, scene, opts)) return DRK_EINVAL;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  drk_status st = drk::ws_set_cameras(ws, cams, n_views, s);
  if (st) return st;
  return drk::ws_preprocess_core(ws, scene, opts, s);
}

drk_status drk_bin_sort(drk_ws* ws, void* stream) {
  if (!ws) { set_error("null workspace"); return DRK_EINVAL; }
  if (!ws->have_pre) { set_error("drk_bin_sort before drk_preprocess"); return DRK_EINVAL; }
  ws->have_bins = false;   // until every view's lists are enqueued again
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const int64_t N = ws->scene.n;
  drk_status st = DRK_OK;
  for (int v = 0; v < ws->views.nv; ++v) {
    const CamDev& cam = ws->views.cam[v];
    const int ntiles = cam.tiles_x * cam.tiles_y;
    const uint32_t* counts = ws->tile_counts + (size_t)v * ws->max_n;
    // 1. stable compaction of visible primitives (index order), then stable radix sort by centre
    //    depth: equal keys keep index order
    if ((st = check_hip(compact_visible(counts, ws->depth_keys + (size_t)v * ws->max_n, N, ws->offsets, ws->block_tot,
                                        ws->n_prims, ws->n_prims + 1, ws->ck, ws->cv, ws->status + v, s),
                        "compact")))
      return st;
    const bool tile_keys = ws->opts.key_mode != 0;
    const uint32_t* order = ws->cv;      // visible primitives in index order
    if (!tile_keys) {
      uint32_t* kb[5] = {ws->ck, ws->dk_a, ws->dk_b, ws->dk_a, ws->dk_b};
      uint32_t* vb[5] = {ws->cv, ws->dv_a, ws->dv_b, ws->dv_a, ws->dv_b};
      if ((st = check_hip(radix_sort(32, ws->n_prims, kb, vb, 5, ws->hist, ws->tot, s), "depth sort"))) return st;
      order = ws->dv_b;
    }
    // 2. offsets of each primitive's pairs in that order
    if ((st = check_hip(scan_counts(order, counts, ws->n_prims, N, ws->offsets, ws->block_tot, ws->totals + v,
                                    ws->n_eff + v, ws->cap, ws->status + v, s), "count scan")))
      return st;
    // 3. duplicate into (tile, primitive) pairs (with per-tile keys: into the final arrays, which
    //    the key sort then uses as scratch, with the keys in pk_tmp)
    int bits = 1;
    while ((1 << bits) < ntiles) ++bits;
    const int passes = (bits + 7) / 8;
    uint32_t* fk = ws->pair_tiles + (size_t)v * ws->cap;
    uint32_t* fv = ws->pair_prims + (size_t)v * ws->cap;
    if ((st = check_hip(launch_duplicate(ws->scene, ws->views_dev, ws->opts, v, order, ws->offsets, counts,
                                         ws->span_meta + (size_t)v * ws->max_n,
                                         ws->span_rows + (size_t)v * ws->row_cap, tile_keys ? fk : ws->pk_tmp,
                                         tile_keys ? fv : ws->pv_tmp, ws->totals + v, ws->cap, ws->n_prims,
                                         ws->dup_big, ws->dup_count, ws->keygeo + (size_t)v * ws->max_n * KG_N,
                                         tile_keys ? ws->pk_tmp : nullptr, s),
                        "duplicate")))
      return st;
    if (tile_keys) {
      // 3b. stable sort of the pair keys (values: pair ids), then tile and primitive in key order
      uint32_t* kk[5] = {ws->pk_tmp, ws->pk_tmp2, ws->pk_tmp, ws->pk_tmp2, ws->pk_tmp};
      uint32_t* kv[5] = {nullptr, ws->pv_tmp2, ws->pv_tmp, ws->pv_tmp2, ws->pv_tmp};
      if ((st = check_hip(radix_sort(32, ws->n_eff + v, kk, kv, 5, ws->hist, ws->tot, s), "key sort"))) return st;
      if ((st = check_hip(gather_pairs(ws->pv_tmp, fk, fv, ws->n_eff + v, ws->pk_tmp2, ws->pv_tmp2, s), "gather")))
        return st;
    }
    // 4. stable sort of the pairs by tile id -> (tile, key, index) order
    uint32_t* src_k = tile_keys ? ws->pk_tmp2 : ws->pk_tmp;
    uint32_t* src_v = tile_keys ? ws->pv_tmp2 : ws->pv_tmp;
    uint32_t* mid_k = tile_keys ? ws->pk_tmp : ws->pk_tmp2;
    uint32_t* mid_v = tile_keys ? ws->pv_tmp : ws->pv_tmp2;
    // the last pass writes fk/fv; up to 17 key bits (images up to 8192 x 2176) take three passes
    uint32_t* pk[4] = {src_k, passes == 2 ? mid_k : fk, passes == 2 ? fk : mid_k, fk};
    uint32_t* pv[4] = {src_v, passes == 2 ? mid_v : fv, passes == 2 ? fv : mid_v, fv};
    if ((st = check_hip(radix_sort(bits, ws->n_eff + v, pk, pv, 4, ws->hist, ws->tot, s), "tile sort"))) return st;
    // 5. ranges
    uint32_t* rg = ws->ranges + (size_t)v * 2 * ws->max_tiles;
    if ((st = check_hip(tile_ranges(fk, ws->n_eff + v, rg, ntiles, s), "ranges"))) return st;
    // 6. raster launch order: tiles by decreasing list length (stable: equal lengths keep tile order)
    if (ws->opts.launch_order != 0) continue;
    uint32_t* t0 = ws->tk;
    uint32_t* t1 = ws->tk + ws->max_tiles;
    uint32_t* t2 = ws->tk + 2 * (size_t)ws->max_tiles;
    uint32_t* t3 = ws->tk + 3 * (size_t)ws->max_tiles;
    if ((st = check_hip(tile_length_keys(rg, ntiles, t0, t1, s), "tile keys"))) return st;
    if ((st = check_hip(set_u64(ws->n_prims + 1, (uint64_t)ntiles, s), "tile count"))) return st;
    uint32_t* ok_[3] = {t0, t2, t0};
    uint32_t* ov_[3] = {t1, t3, ws->tile_order + (size_t)v * ws->max_tiles};
    if ((st = check_hip(radix_sort(16, ws->n_prims + 1, ok_, ov_, 3, ws->hist, ws->tot, s), "tile order"))) return st;
  }
  ws->have_bins = true;
  return DRK_OK;
}

namespace {

// mode 0 colour, 1 trace (a0 = counts, a1 = indices, a2 = depths), 2 depth (a0) and normal (a2).
drk_status render_views(drk_ws* ws, float* rgb, float* T_final, int mode, int32_t cap, void* a0, int32_t* a1,
                        float* a2, hipStream_t s) {
  size_t off = 0;
  const size_t px_max = (size_t)ws->max_w * ws->max_h;
  for (int v = 0; v < ws->views.nv; ++v) {
    const CamDev& cam = ws->views.cam[v];
    const size_t npx = (size_t)cam.W * cam.H;
    drk_status st = check_hip(
        launch_render_fwd(ws->K, ws->records + (size_t)v * ws->max_n * ws->RF, ws->ranges + (size_t)v * 2 * ws->max_tiles,
                          ws->pair_prims + (size_t)v * ws->cap, &ws->views_dev->cam[v], cam.tiles_x * cam.tiles_y,
                          ws->opts.launch_order == 0 ? ws->tile_order + (size_t)v * ws->max_tiles : nullptr,
                          ws->opts, rgb + 3 * off,
                          T_final ? T_final + off : nullptr, ws->n_emit + v * px_max, ws->consumed + v * px_max,
                          ws->contrib + v * px_max, ws->work_px + 2 * v * px_max, mode,
                          mode == 1 ? (void*)(static_cast<int32_t*>(a0) + off)
                                    : (mode == 2 ? (void*)(static_cast<float*>(a0) + off) : nullptr),
                          mode == 1 ? a1 + off * cap : nullptr,
                          mode == 1 ? a2 + off * cap : (mode == 2 ? a2 + 3 * off : nullptr), cap, s),
        mode == 1 ? "render_trace" : (mode == 2 ? "render_depth_normal" : "render_fwd"));
    if (st) return st;
    off += npx;
  }
  ws->counted = ws->opts.cache_len < kExactOrder && (mode != 0 || ws->opts.counters != 0);
  return DRK_OK;
}

}  // namespace

drk_status drk_render_fwd(drk_ws* ws, float* rgb, float* T_final, void* stream) {
  if (!ws || !rgb) { set_error("null argument"); return DRK_EINVAL; }
  if (!ws->have_bins) { set_error("drk_render_fwd before drk_bin_sort"); return DRK_EINVAL; }
  return render_views(ws, rgb, T_final, 0, 0, nullptr, nullptr, nullptr, reinterpret_cast<hipStream_t>(stream));
}

drk_status drk_render_depth_normal(drk_ws* ws, float* rgb, float* T_final, float* depth, float* normal, void* stream) {
  if (!ws || !rgb || !depth || !normal) { set_error("null argument"); return DRK_EINVAL; }
  if (!ws->have_bins) { set_error("drk_render_depth_normal before drk_bin_sort"); return DRK_EINVAL; }
  if (ws->opts.cache_len >= kExactOrder) { set_error("the exact order renders colour only"); return DRK_EINVAL; }
  return render_views(ws, rgb, T_final, 2, 0, depth, nullptr, normal, reinterpret_cast<hipStream_t>(stream));
}

namespace {

// Checks the shape fields of a raw scene; returns the colour row count, or -1 (error set).
int raw_colour_rows(const drk_scene* raw) {
  if (!raw || raw->n < 0 || raw->K < 3 || raw->K > kMaxK) { set_error("raw scene: n >= 0 and 3 <= K <= %d", kMaxK); return -1; }
  if (raw->color_mode == 0) return 3;
  if (raw->color_mode == 1 && raw->sh_degree >= 0 && raw->sh_degree <= 3) return 3 * (raw->sh_degree + 1) * (raw->sh_degree + 1);
  set_error("raw scene: color_mode 0, or 1 with sh_degree in [0, 3]");
  return -1;
}

bool all_set(const void* const* p, int cnt) {
  for (int i = 0; i < cnt; ++i)
    if (!p[i]) return false;
  return true;
}

}  // namespace

drk_status drk_activate(const drk_scene* raw, const drk_scene_out* out, void* stream) {
  const int ncol = raw_colour_rows(raw);
  if (ncol < 0) return DRK_EINVAL;
  const void* ptrs[16] = {raw->mu, raw->q, raw->scale, raw->theta, raw->eta, raw->tau, raw->opacity, raw->color,
                          out ? out->mu : nullptr, out ? out->q : nullptr, out ? out->scale : nullptr,
                          out ? out->theta : nullptr, out ? out->eta : nullptr, out ? out->tau : nullptr,
                          out ? out->opacity : nullptr, out ? out->color : nullptr};
  if (raw->n > 0 && !all_set(ptrs, 16)) { set_error("null array"); return DRK_EINVAL; }
  return check_hip(launch_activate(*raw, *out, ncol, reinterpret_cast<hipStream_t>(stream)), "activate");
}

drk_status drk_activate_bwd(const drk_scene* raw, const drk_scene_grad* g_act, const drk_scene_out* g_raw,
                            void* stream) {
  const int ncol = raw_colour_rows(raw);
  if (ncol < 0) return DRK_EINVAL;
  if (!g_act || !g_raw) { set_error("null argument"); return DRK_EINVAL; }
  const void* ptrs[24] = {raw->mu, raw->q, raw->scale, raw->theta, raw->eta, raw->tau, raw->opacity, raw->color,
                          g_act->mu, g_act->q, g_act->scale, g_act->theta, g_act->eta, g_act->tau, g_act->opacity,
                          g_act->color, g_raw->mu, g_raw->q, g_raw->scale, g_raw->theta, g_raw->eta, g_raw->tau,
                          g_raw->opacity, g_raw->color};
  if (raw->n > 0 && !all_set(ptrs, 24)) { set_error("null array"); return DRK_EINVAL; }
  return check_hip(launch_activate_bwd(*raw, *g_act, *g_raw, ncol, reinterpret_cast<hipStream_t>(stream)),
                   "activate_bwd");
}

drk_status drk_adam_step(float* param, float* m, float* v, const float* grad, int64_t n, float lr, float beta1,
                         float beta2, float eps, int32_t step, void* stream) {
  if (n < 0 || (n > 0 && (!param || !m || !v || !grad))) { set_error("null array or n < 0"); return DRK_EINVAL; }
  if (step < 1 || !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps > 0.0f)) {
    set_error("adam: step >= 1, betas in [0, 1), eps > 0");
    return DRK_EINVAL;
  }
  return check_hip(launch_adam(param, m, v, grad, n, lr, beta1, beta2, eps, step, reinterpret_cast<hipStream_t>(stream)),
                   "adam");
}

drk_status drk_mesh_to_drk(const float* vertices, int64_t nv, const int32_t* faces, int64_t nf, int32_t m,
                           const float* face_rgb, int32_t K, float tau, float opacity, const drk_scene_out* out,
                           uint32_t* rejected, void* stream) {
  if (!out || (nf > 0 && (!vertices || !faces || !face_rgb || !out->mu || !out->q || !out->scale || !out->theta ||
                          !out->eta || !out->tau || !out->opacity || !out->color))) {
    set_error("null argument");
    return DRK_EINVAL;
  }
  if (nv < 0 || nf < 0 || nv > 0x7FFFFFFF || K < 3 || K > kMaxK || m < 3 || m > K) {
    set_error("mesh sizes out of range (need 3 <= m <= K <= %d, 0 <= nv < 2^31)", kMaxK);
    return DRK_EINVAL;
  }
  if (!(tau > -1.0f && tau < 1.0f) || !(opacity > 0.0f && opacity <= 1.0f)) {
    set_error("tau must be in (-1, 1) and opacity in (0, 1]");
    return DRK_EINVAL;
  }
  return check_hip(launch_mesh_to_drk(vertices, nv, faces, nf, m, face_rgb, K, tau, opacity, *out, rejected,
                                      reinterpret_cast<hipStream_t>(stream)),
                   "mesh_to_drk");
}

drk_status drk_render_trace(drk_ws* ws, float* rgb, float* T_final, int32_t cap, int32_t* trace_n,
                            int32_t* trace_idx, float* trace_z, void* stream) {
  if (!ws || !rgb || !trace_n || !trace_idx || !trace_z) { set_error("null argument"); return DRK_EINVAL; }
  if (!ws->have_bins) { set_error("drk_render_trace before drk_bin_sort"); return DRK_EINVAL; }
  if (ws->opts.cache_len >= kExactOrder) { set_error("the exact order renders colour only"); return DRK_EINVAL; }
  if (cap < 1 || cap > 1024) { set_error("trace cap %d outside [1, 1024]", cap); return DRK_EINVAL; }
  return render_views(ws, rgb, T_final, 1, cap, trace_n, trace_idx, trace_z, reinterpret_cast<hipStream_t>(stream));
}

drk_status drk_trace_metrics(const int32_t* trace_n, const float* trace_z, int64_t npx, int32_t cap, double* out,
                             void* stream) {
  if (!trace_n || !trace_z || !out) { set_error("null argument"); return DRK_EINVAL; }
  if (npx < 0 || cap < 1 || cap > 64) { set_error("npx must be >= 0 and cap in [1, 64]"); return DRK_EINVAL; }
  return check_hip(launch_trace_metrics(trace_n, trace_z, npx, cap, out, reinterpret_cast<hipStream_t>(stream)),
                   "trace metrics");
}

drk_status drk_render_bwd(drk_ws* ws, const drk_scene* scene, const float* rgb, const float* dL_drgb,
                          const drk_scene_grad* grads, void* stream) {
  if (!ws || !scene || !rgb || !dL_drgb || !grads) { set_error("null argument"); return DRK_EINVAL; }
  if (!ws->have_bins) { set_error("drk_render_bwd before drk_bin_sort"); return DRK_EINVAL; }
  if (ws->opts.cache_len >= kExactOrder) { set_error("no backward for the exact order"); return DRK_EINVAL; }
  if (scene->n != ws->scene.n || scene->mu != ws->scene.mu || scene->q != ws->scene.q) {
    set_error("drk_render_bwd: scene differs from the one preprocessed");
    return DRK_EINVAL;
  }
  if (!grads->mu || !grads->q || !grads->scale || !grads->theta || !grads->eta || !grads->tau || !grads->opacity ||
      !grads->color) {
    set_error("gradient array is null");
    return DRK_EINVAL;
  }
  if (!kBackwardEnabled) {
    set_error("drk_render_bwd is switched off: its kernels took an illegal memory access on gfx950 whose "
              "cause is not yet identified");
    return DRK_EDEVICE;
  }
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const int64_t N = ws->scene.n;
  const int GF = grad_fields(ws->K);
  const int64_t stride = ws->max_n;
  drk_status st = check_hip(
      fill_u32(reinterpret_cast<uint32_t*>(ws->grad_rec), 0u, (int64_t)ws->views.nv * GF * stride, s), "clear grads");
  if (st) return st;
  size_t off = 0;
  const size_t px_max = (size_t)ws->max_w * ws->max_h;
  for (int v = 0; v < ws->views.nv; ++v) {
    const CamDev& cam = ws->views.cam[v];
    const size_t npx = (size_t)cam.W * cam.H;
    st = check_hip(launch_render_bwd(ws->K, ws->records + (size_t)v * ws->max_n * ws->RF,
                                     ws->ranges + (size_t)v * 2 * ws->max_tiles, ws->pair_prims + (size_t)v * ws->cap,
                                     &ws->views_dev->cam[v], cam.tiles_x * cam.tiles_y, ws->opts, rgb + 3 * off,
                                     dL_drgb + 3 * off,
                                     ws->grad_rec + (size_t)v * GF * stride, stride, s),
                   "render_bwd");
    if (st) return st;
    off += npx;
  }
  return check_hip(launch_preprocess_bwd(ws->scene, ws->views_dev, ws->opts, ws->tile_counts, ws->grad_rec, ws->max_n,
                                         *grads, s),
                   "preprocess_bwd");
}

drk_status drk_ws_generation(drk_ws* ws, uint64_t* generation) {
  if (!ws || !generation) { set_error("null argument"); return DRK_EINVAL; }
  *generation = ws->generation;
  return DRK_OK;
}

drk_status drk_ws_status(drk_ws* ws, void* stream, int64_t* pairs_needed) {
  if (!ws) { set_error("null workspace"); return DRK_EINVAL; }
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  drk_status st = check_hip(hipStreamSynchronize(s), "stream sync");
  if (st) return st;
  return drk::ws_read_status(ws, pairs_needed);
}

drk_status drk_ws_export(drk_ws* ws, int32_t view, int32_t what, void* dst, int64_t bytes, int64_t* out_count,
                         void* stream) {
  if (!ws || !out_count) { set_error("null argument"); return DRK_EINVAL; }
  if (!ws->have_pre || view < 0 || view >= ws->views.nv) { set_error("view %d not available", view); return DRK_EINVAL; }
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const CamDev& cam = ws->views.cam[view];
  const int64_t N = ws->scene.n;
  const size_t px_max = (size_t)ws->max_w * ws->max_h;
  const void* src = nullptr;
  int64_t count = 0;
  size_t esize = 4;
  if (what >= 5 && what <= 9 && !ws->counted) {
    set_error("per-pixel counters were not written: render with drk_opts.counters = 1");
    return DRK_EINVAL;
  }
  switch (what) {
    case 0: src = ws->depth_keys + (size_t)view * ws->max_n; count = N; break;
    case 1: src = ws->tile_counts + (size_t)view * ws->max_n; count = N; break;
    case 2:
    case 3: {
      if (!ws->have_bins) { set_error("no bins yet"); return DRK_EINVAL; }
      uint64_t ne = 0;
      drk_status st = check_hip(hipStreamSynchronize(s), "sync");
      if (st) return st;
      if ((st = check_hip(hipMemcpy(&ne, ws->n_eff + view, 8, hipMemcpyDeviceToHost), "read n"))) return st;
      count = (int64_t)ne;
      src = (what == 2 ? ws->pair_tiles : ws->pair_prims) + (size_t)view * ws->cap;
      break;
    }
    case 4: src = ws->ranges + (size_t)view * 2 * ws->max_tiles; count = 2LL * cam.tiles_x * cam.tiles_y; break;
    case 5: src = ws->n_emit + view * px_max; count = (int64_t)cam.W * cam.H; break;
    case 6: src = ws->consumed + view * px_max; count = (int64_t)cam.W * cam.H; break;
    case 7: src = ws->contrib + view * px_max; count = (int64_t)cam.W * cam.H; break;
    case 8: src = ws->work_px + 2 * view * px_max; count = (int64_t)cam.W * cam.H; break;
    case 9: src = ws->work_px + 2 * view * px_max + (size_t)cam.W * cam.H; count = (int64_t)cam.W * cam.H; break;
    case 10: {
      if (!ws->have_bins) { set_error("no bins yet"); return DRK_EINVAL; }
      uint64_t ne = 0;
      drk_status st = check_hip(hipStreamSynchronize(s), "sync");
      if (st) return st;
      if ((st = check_hip(hipMemcpy(&ne, ws->n_eff + view, 8, hipMemcpyDeviceToHost), "read n"))) return st;
      *out_count = (int64_t)ne;
      if (!dst) return DRK_OK;
      const int64_t n = std::min<int64_t>((int64_t)ne, bytes / 4);
      return check_hip(launch_pair_keys(ws->views_dev, ws->opts, view, ws->pair_tiles + (size_t)view * ws->cap,
                                        ws->pair_prims + (size_t)view * ws->cap, n,
                                        ws->depth_keys + (size_t)view * ws->max_n,
                                        ws->keygeo + (size_t)view * ws->max_n * KG_N, static_cast<uint32_t*>(dst), s),
                       "pair keys");
    }
    default: set_error("unknown export %d", what); return DRK_EINVAL;
  }
  *out_count = count;
  if (dst && count > 0) {
    const int64_t nbytes = std::min<int64_t>(bytes, count * (int64_t)esize);
    drk_status st = check_hip(hipMemcpyAsync(dst, src, (size_t)nbytes, hipMemcpyDeviceToDevice, s), "export copy");
    if (st) return st;
  }
  return DRK_OK;
}

}  // extern "C"

namespace drk {

// One forward render of one view whose workspace is placed in the caller-given device memory
// [base, base + bytes) with the forward-only layout; the pair capacity is whatever the rest of that
// memory holds.  Enqueued on s, then s is synchronised and the status word read into host stack
// memory, so the call returns the frame's final status.  Allocates nothing.
drk_status render_placed(void* base, size_t bytes, const drk_scene* scene, const drk_camera* cam,
                         const drk_opts* opts, float* rgb, float* T_final, hipStream_t s) {
  if (!scene || !cam || !opts || !rgb) { set_error("null argument"); return DRK_EINVAL; }
  if (scene->n < 0 || scene->K < 3 || scene->K > kMaxK) { set_error("scene: n >= 0 and 3 <= K <= %d", kMaxK); return DRK_EINVAL; }
  drk_ws ws;                       // host bookkeeping on the stack; the device memory is base
  ws.max_n = std::max<int64_t>(scene->n, 1);
  ws.K = scene->K;
  ws.RF = rec_floats(scene->K);
  ws.max_views = 1;
  ws.max_w = cam->width;
  ws.max_h = cam->height;
  if (!valid_ws_args(ws.max_n, ws.K, 1, ws.max_w, ws.max_h, 1)) return DRK_EINVAL;
  ws.max_tiles = ((ws.max_w + kTile - 1) / kTile) * ((ws.max_h + kTile - 1) / kTile);
  ws.row_cap = span_row_capacity(ws.max_n);
  ws.lean = true;
  ws.lean_keys = opts->key_mode != 0;
  ws.cap = 1;
  const size_t fixed = layout(&ws, false, nullptr);
  // six u32 arrays per pair (two ping-pong key/value pairs and the final tile and primitive lists)
  const size_t per_pair = 6 * sizeof(uint32_t), slack = 16 * 256;
  if (fixed + slack + 1024 * per_pair > bytes) {
    set_error("scene of %lld DRKs (K = %d) at %dx%d needs %zu bytes before any tile pair; the fixed device array "
              "holds %zu", (long long)scene->n, scene->K, cam->width, cam->height, fixed, bytes);
    return DRK_ENOMEM;
  }
  int64_t cap = (int64_t)((bytes - fixed - slack) / per_pair);
  cap = std::min<int64_t>(cap, (int64_t)0xFFFFFF00);
  ws.cap = cap;
  while (layout(&ws, false, nullptr) > bytes) ws.cap -= 256;
  layout(&ws, true, static_cast<char*>(base));
  ws.bytes = bytes;
  drk_status st = ws_set_cameras(&ws, cam, 1, s);
  if (st) return st;
  if ((st = ws_preprocess_core(&ws, scene, opts, s))) return st;
  if ((st = drk_bin_sort(&ws, s))) return st;
  if ((st = drk_render_fwd(&ws, rgb, T_final, s))) return st;
  if ((st = check_hip(hipStreamSynchronize(s), "stream sync"))) return st;
  uint32_t status = 0;
  uint64_t total = 0;
  if ((st = check_hip(hipMemcpy(&status, ws.status, sizeof(status), hipMemcpyDeviceToHost), "read status"))) return st;
  if ((st = check_hip(hipMemcpy(&total, ws.totals, sizeof(total), hipMemcpyDeviceToHost), "read pair count"))) return st;
  if (status & ST_INVALID) { set_error("invalid primitive parameters (validate mode)"); return DRK_EINVAL; }
  if (status & ST_OVERFLOW) {
    set_error("the frame needs %llu tile pairs; the fixed device array holds %lld at this scene and image size "
              "(the image is incomplete)", (unsigned long long)total, (long long)ws.cap);
    return DRK_EOVERFLOW;
  }
  return DRK_OK;
}

}  // namespace drk
