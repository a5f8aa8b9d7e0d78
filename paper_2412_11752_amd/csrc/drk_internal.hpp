// Internal definitions shared by the libdrk translation units (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/drk.h"

namespace drk {

constexpr int kTile = 16;            // 16x16 screen tiles (Sec. 4.4 Kernel Culling)
constexpr int kMaxK = 16;            // radial bases per primitive
constexpr int kMaxViews = 8;         // views per launch
constexpr int kMaxTileRows = 136;    // tile rows per view (image height <= 2176)
constexpr int kSpanPools = 64;       // span-row pools per view (one fill counter each)
constexpr int kMaxCache = 8;         // cache slots (Sec. 4.4 Cache Sorting uses 8)
constexpr int32_t kExactOrder = 1 << 30;   // cache_len at or above this: exact per-pixel depth order
constexpr uint32_t kCulledKey = 0xFFFFFFFFu;
constexpr double kGrazing = 1e-6;    // |r_d . n| below this is a grazing ray (no hit)

// ---------------------------------------------------------------------------------------------
// Per (view, primitive) render record, float32, written by the preprocess kernel and read by the
// raster kernels.  The hit of the ray through pixel centre (px, py) is found with a homography
// from pixel offsets to the primitive's tangent plane:
//   dx = px - ax, dy = py - ay,  (U, V, W) = Hm (dx, dy, 1),  u = U/W, v = V/W,
//   view depth of the hit Z = dN / W,  r_d . n = W / |r_d|   (r_d = K^-1 (px, py, 1)).
// Hm = adj[t_u | t_v | mu] (camera frame) * K^-1 * T(ax, ay): the adjugate form of the ray-plane
// intersection of Sec. 3.3, anchored at the quantised projected centre so that FP32 offsets stay
// small where the kernel is evaluated.
enum RecField : int {
  R_H = 0,        // 9 entries, row-major
  R_DN = 9,       // n_c . mu_c
  R_AX = 10, R_AY = 11,       // anchor (pixel coordinates, multiple of 1/256)
  R_OX = 12, R_OY = 13,       // projected centre minus anchor (low-pass centre)
  R_O = 14, R_ETA = 15,
  R_PLO = 16, R_PHI = 17,     // Psi breakpoints (1+tau)/4, (3-tau)/4
  R_PA1 = 18, R_PA2 = 19,     // Psi slopes (1-tau)/(1+tau), (1+tau)/(1-tau)
  R_PB2 = 20, R_PB3 = 21,     // Psi intercepts -tau/(1-tau), 2 tau/(1+tau)
  R_RGB = 22,                 // 3 entries
  R_TAU = 25,
  R_R2CUT = 26,               // u^2 + v^2 beyond which alpha < alpha_min (bound E >= r2 / max_k s_k^2)
  R_LPCUT = 27,               // d^2 |r_d|^2 / W^2 beyond which the low-pass term < alpha_min
  R_BOX = 28,                 // 4 entries: pixel-space box (x0, x1, y0, y1) of the support polygon
  R_ETHR = 32,                // energy beyond which alpha < alpha_min, with margin (c^2 (1 + 1e-3) + 1e-2)
  R_NRM = 33,                 // 3 entries: unit camera-frame plane normal, turned toward the camera
  R_SEC = 36,                 // per-sector arrays follow, each K long (16-byte alignment)
};
// Per-sector arrays (offset R_SEC + field * K + k):
enum SecField : int {
  S_PA = 0,    // pseudo-angle of basis direction k (monotone in theta_k)
  S_C = 1,     // cos theta_k
  S_S = 2,     // sin theta_k
  S_ID = 3,    // 1 / delta_k, delta_k = theta_{k+1} - theta_k (wrapping)
  S_A = 4,     // 1 / (s_k sin delta_k)
  S_B = 5,     // 1 / (s_{k+1} sin delta_k)
  S_IK2 = 6,   // 1 / s_k^2 (1 / s_{k+1}^2 is the next sector's entry)
  S_WLO = 7,   // min(1 / s_k^2, 1 / s_{k+1}^2) (1 - 1e-5): lower bound of the sector's L2 weight
  S_NFIELDS = 8
};
__host__ __device__ constexpr int rec_floats(int K) { return (R_SEC + S_NFIELDS * K + 3) & ~3; }

// ---------------------------------------------------------------------------------------------
struct CamDev {
  int32_t W, H, tiles_x, tiles_y;
  float fx, fy, cx, cy;
  float R[9];
  float t[3];
  float bg[3];
  double campos[3];  // camera centre -R^-1 t (float64; the SH view direction)
};

struct Views {
  CamDev cam[kMaxViews];
  int32_t nv;
};

struct OptsDev {
  float alpha_min, alpha_max, T_min, near_plane, lowpass_sl;
  int32_t cache_len, cull_mode, validate, key_mode, launch_order, counters;
  // polygon kernel choice (results do not depend on it): the small-list length from which the
  // thread-per-primitive walk runs, and the tile rows a primitive may span to join that list
  int32_t small_min, win_admit;
};

// Per (view, primitive) float64 data of the per-tile pre-sort keys (key_mode 1, 2), written by the
// preprocess with the record: the camera-frame plane a . X = dN (a = t_u^c x t_v^c), the centre
// depth, the depth range [zlo, zhi] of the support disc (radius sqrt(2) c max_k s_k; zlo >= near)
// and the pixel box (x0, x1, y0, y1) of the projected support (+-1e30 when cull_mode != 0).
enum KeyGeoField : int { KG_A = 0, KG_DN = 3, KG_ZC = 4, KG_ZLO = 5, KG_ZHI = 6, KG_BOX = 7, KG_N = 12 };

struct SceneDev {
  int64_t n;
  int32_t K, color_mode, sh_degree, ncol;
  const float* mu;
  const float* q;
  const float* scale;
  const float* theta;
  const float* eta;
  const float* tau;
  const float* opacity;
  const float* color;
};

// Structs passed by value as kernel arguments or copied to device memory are laid out alike by
// the host and the device compilations (every translation unit checks these in each pass).
static_assert(sizeof(CamDev) == 120 && offsetof(CamDev, fx) == 16 && offsetof(CamDev, R) == 32 &&
                  offsetof(CamDev, t) == 68 && offsetof(CamDev, bg) == 80 && offsetof(CamDev, campos) == 96,
              "CamDev layout");
static_assert(sizeof(Views) == 968 && offsetof(Views, nv) == 960, "Views layout");
static_assert(sizeof(OptsDev) == 52 && offsetof(OptsDev, cache_len) == 20 && offsetof(OptsDev, counters) == 40 &&
                  offsetof(OptsDev, win_admit) == 48,
              "OptsDev layout");
static_assert(sizeof(SceneDev) == 88 && offsetof(SceneDev, K) == 8 && offsetof(SceneDev, ncol) == 20 &&
                  offsetof(SceneDev, mu) == 24 && offsetof(SceneDev, color) == 80,
              "SceneDev layout");
static_assert(sizeof(drk_scene) == 88 && offsetof(drk_scene, mu) == 24 && offsetof(drk_scene, color) == 80,
              "drk_scene layout");
static_assert(sizeof(drk_scene_grad) == 64 && offsetof(drk_scene_grad, color) == 56, "drk_scene_grad layout");
static_assert(sizeof(drk_scene_out) == 64 && offsetof(drk_scene_out, color) == 56, "drk_scene_out layout");
static_assert(sizeof(drk_camera) == 84 && offsetof(drk_camera, R) == 24 && offsetof(drk_camera, bg) == 72,
              "drk_camera layout");
static_assert(sizeof(drk_opts) == 44 && offsetof(drk_opts, cache_len) == 20 && offsetof(drk_opts, counters) == 40,
              "drk_opts layout");

// Status word bits (device), read back by drk_ws_status.
enum StatusBits : uint32_t { ST_OVERFLOW = 1u, ST_INVALID = 2u };

// Per-primitive gradient of the record quantities (float32, atomically accumulated by the raster
// backward, consumed by the per-primitive backward): layout [field][n].
enum GradField : int {
  G_H = 0,        // 9: dL/dHm
  G_O = 9,        // dL/do (direct)
  G_ETA = 10,
  G_TAU = 11,
  G_RGB = 12,     // 3
  G_OX = 15, G_OY = 16,   // dL/d(low-pass centre offset)
  G_SEC = 17,     // then dL/ds_k [K], dL/dtheta_k [K]
};
__host__ __device__ inline int grad_fields(int K) { return G_SEC + 2 * K; }

}  // namespace drk

// Host-side helpers shared by the host translation units.
namespace drk {
void set_error(const char* fmt, ...);
// Split of drk_preprocess used by the serving loop: the camera is written to device memory by a
// one-thread kernel launched outside any captured graph; the rest reads it from there.
drk_status ws_set_cameras(drk_ws* ws, const drk_camera* cams, int32_t n_views, hipStream_t s);
drk_status ws_preprocess_core(drk_ws* ws, const drk_scene* scene, const drk_opts* opts, hipStream_t s);
drk_status ws_read_status(drk_ws* ws, int64_t* pairs_needed);
float* ws_out_rgb(drk_ws* ws);
// One forward render of one view with its workspace placed in [base, base + bytes) of device memory
// (forward-only layout, pair capacity from what the rest holds); synchronises s and returns the
// frame's final status.  Allocates nothing.
drk_status render_placed(void* base, size_t bytes, const drk_scene* scene, const drk_camera* cam,
                         const drk_opts* opts, float* rgb, float* T_final, hipStream_t s);
size_t ws_bytes(drk_ws* ws);
int64_t ws_capacity(drk_ws* ws);
}
