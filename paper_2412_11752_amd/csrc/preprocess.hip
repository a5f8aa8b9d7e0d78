// Per (view, primitive) preprocessing and tile duplication for the DRK rasterizer.
//
// Float64 geometry (compiled with -ffp-contract=off so every product and sum rounds as written):
// the tile decisions must reproduce a float64 reference exactly.  Outputs are rounded to float32.
//
// Paper passages: rotation / SH colour as in 3D-GS (Sec. 3.1); ray-plane intersection (Sec. 3.3);
// radial basis, L1/L2 blend, sharpening (Sec. 4.1-4.3); calibrated radius and polygon-based tile
// culling on 16x16 tiles (Sec. 4.4, Kernel Culling); centre-depth pre-sort (Sec. 4.4, Cache Sorting).
#include "drk_internal.hpp"

#include <math.h>

#include <algorithm>
#include <type_traits>

namespace drk {

constexpr double kPi = 3.141592653589793;
constexpr double kTwoPi = 2.0 * kPi;
constexpr uint32_t kNoSpans = 0xFFFFFFFFu;
constexpr uint32_t kDupSmall = 32;      // primitives with more tiles are duplicated by a whole workgroup

// ---------------------------------------------------------------------------------------------
// Rotation of a quaternion (w, x, y, z): columns are the tangent axes t_u, t_v and the normal.
__device__ inline void quat_rot(double w, double x, double y, double z, double R[9]) {
  double nrm = sqrt(((w * w + x * x) + y * y) + z * z);
  w = w / nrm; x = x / nrm; y = y / nrm; z = z / nrm;
  R[0] = 1.0 - 2.0 * (y * y + z * z); R[1] = 2.0 * (x * y - w * z); R[2] = 2.0 * (x * z + w * y);
  R[3] = 2.0 * (x * y + w * z); R[4] = 1.0 - 2.0 * (x * x + z * z); R[5] = 2.0 * (y * z - w * x);
  R[6] = 2.0 * (x * z - w * y); R[7] = 2.0 * (y * z + w * x); R[8] = 1.0 - 2.0 * (x * x + y * y);
}

// world -> camera for a point: ((r0 x + r1 y) + r2 z) + t per row
__device__ inline void to_cam(const CamDev& c, const double p[3], double out[3]) {
  for (int i = 0; i < 3; ++i) {
    double a = (double)c.R[3 * i + 0] * p[0];
    a = a + (double)c.R[3 * i + 1] * p[1];
    a = a + (double)c.R[3 * i + 2] * p[2];
    out[i] = a + (double)c.t[i];
  }
}
__device__ inline void rot_cam(const CamDev& c, const double d[3], double out[3]) {
  for (int i = 0; i < 3; ++i) {
    double a = (double)c.R[3 * i + 0] * d[0];
    a = a + (double)c.R[3 * i + 1] * d[1];
    out[i] = a + (double)c.R[3 * i + 2] * d[2];
  }
}

// Inverse of the sharpening remap (Sec. 4.3).
__device__ inline double psi_inv(double y, double tau) {
  if (y < (1.0 - tau) / 4.0) return y * (1.0 + tau) / (1.0 - tau);
  if (y < (3.0 + tau) / 4.0) return (y * (1.0 - tau) + tau) / (1.0 + tau);
  return (y * (1.0 + tau) - 2.0 * tau) / (1.0 - tau);
}

// Real spherical harmonics (orthonormal, degree <= 3), index l*l + l + m.
__device__ inline void real_sh(int deg, double x, double y, double z, double Y[16]) {
  const double c0 = 0.28209479177387814;      // 1 / (2 sqrt(pi))
  const double c1 = 0.4886025119029199;       // sqrt(3 / (4 pi))
  Y[0] = c0;
  if (deg < 1) return;
  Y[1] = c1 * y; Y[2] = c1 * z; Y[3] = c1 * x;
  if (deg < 2) return;
  const double c2a = 1.0925484305920792;      // sqrt(15/pi) / 2
  const double c2b = 0.31539156525252005;     // sqrt(5/pi) / 4
  const double c2c = 0.5462742152960396;      // sqrt(15/pi) / 4
  Y[4] = c2a * x * y; Y[5] = c2a * y * z; Y[6] = c2b * (3.0 * z * z - 1.0);
  Y[7] = c2a * x * z; Y[8] = c2c * (x * x - y * y);
  if (deg < 3) return;
  const double c3a = 0.5900435899266435;      // sqrt(35/(2 pi)) / 4
  const double c3b = 2.890611442640554;       // sqrt(105/pi) / 2
  const double c3c = 0.4570457994644658;      // sqrt(21/(2 pi)) / 4
  const double c3d = 0.3731763325901154;      // sqrt(7/pi) / 4
  const double c3e = 1.445305721320277;       // sqrt(105/pi) / 4
  Y[9] = c3a * y * (3.0 * x * x - y * y);
  Y[10] = c3b * x * y * z;
  Y[11] = c3c * y * (5.0 * z * z - 1.0);
  Y[12] = c3d * (5.0 * z * z * z - 3.0 * z);
  Y[13] = c3c * x * (5.0 * z * z - 1.0);
  Y[14] = c3e * z * (x * x - y * y);
  Y[15] = c3a * x * (x * x - 3.0 * y * y);
}

// ---------------------------------------------------------------------------------------------
// Per-primitive geometry in float64.  GeoBase holds no per-basis arrays (kernels that need the
// bases read them from the scene), so that it lives in registers; Geo adds them for the sequential
// polygon walk of the duplication rebuild.
struct GeoBase {
  double tu[3], tv[3];      // world tangent axes (columns of R(q))
  double mu[3];
  double muc[3];            // camera-frame centre
  double o, tau;
  double c;                 // calibrated radius: {E <= c^2} == {o Psi(g) >= alpha_min}
  double smax;              // max_k s_k
  int K;
};
struct Geo : GeoBase {
  double s[kMaxK], th[kMaxK];
};

// Loads and validates primitive j (the bases streamed from the scene; stored in s_out / th_out when
// given).  Returns false when it can never contribute.
template <typename T>
__device__ inline bool load_geo_core(const SceneDev& sc, int64_t j, const CamDev& cam, const OptsDev& opt, GeoBase& g,
                                     bool* invalid, T* s_out, T* th_out) {
  const int64_t n = sc.n;
  const int K = sc.K;
  g.K = K;
  bool bad = false;
  for (int i = 0; i < 3; ++i) {
    g.mu[i] = (double)sc.mu[i * n + j];
    bad |= !isfinite(g.mu[i]);
  }
  double q[4];
  for (int i = 0; i < 4; ++i) { q[i] = (double)sc.q[i * n + j]; bad |= !isfinite(q[i]); }
  double qq = ((q[0] * q[0] + q[1] * q[1]) + q[2] * q[2]) + q[3] * q[3];
  bad |= !(qq > 0.0);
  double smax = 0.0;
  const double th0 = (double)sc.theta[j];
  double thk = th0;
  for (int k = 0; k < K; ++k) {
    const double sk = (double)sc.scale[k * n + j];
    const double nxt = (k + 1 < K) ? (double)sc.theta[(k + 1) * n + j] : th0 + kTwoPi;
    if (s_out) { s_out[k] = (T)sk; th_out[k] = (T)thk; }
    bad |= !(sk > 0.0) || !isfinite(sk);
    bad |= !(thk >= 0.0) || !(thk < kTwoPi);
    const double gap = nxt - thk;
    bad |= !(gap > 0.0) || !(gap < kPi);
    smax = fmax(smax, sk);
    thk = nxt;
  }
  g.smax = smax;
  g.o = (double)sc.opacity[j];
  g.tau = (double)sc.tau[j];
  double eta = (double)sc.eta[j];
  bad |= !(g.o > 0.0) || !(g.o <= 1.0) || !(g.tau > -1.0) || !(g.tau < 1.0) || !(eta >= 0.0) || !(eta <= 1.0);
  *invalid = bad;
  if (bad) return false;
  double R[9];
  quat_rot(q[0], q[1], q[2], q[3], R);
  g.tu[0] = R[0]; g.tu[1] = R[3]; g.tu[2] = R[6];
  g.tv[0] = R[1]; g.tv[1] = R[4]; g.tv[2] = R[7];
  to_cam(cam, g.mu, g.muc);
  if (!(g.muc[2] > (double)opt.near_plane)) return false;
  if (g.o < (double)opt.alpha_min) return false;
  double gmin = psi_inv((double)opt.alpha_min / g.o, g.tau);
  g.c = sqrt(-2.0 * log(gmin));
  return true;
}

__device__ inline bool load_geo(const SceneDev& sc, int64_t j, const CamDev& cam, const OptsDev& opt, Geo& g,
                                bool* invalid) {
  return load_geo_core(sc, j, cam, opt, g, invalid, g.s, g.th);
}

// ---------------------------------------------------------------------------------------------
// Tile-row spans of the projected support, sequential walk.  Edges of the near-clipped projected
// polygon are streamed in order; each updates the x-extent of the tile rows whose pixel-centre slab
// it crosses.  The row extents live in one of two stores:
//  * RowsAll: every tile row of the view in private memory, indexed relative to the primitive's
//    centre row (wrapping), so that a wave's lanes touch the same slots;
//  * RowsWin: kWinRows rows from `base` on in registers; touching a row outside them sets
//    `overflow` (the caller then takes the primitive to the wave-parallel kernel).
constexpr int kWinRows = 4;

struct RowsAll {
  double lo[kMaxTileRows], hi[kMaxTileRows];
  int base;                         // tile row stored in slot 0
  bool overflow;                    // never set
  __device__ int slot(int r) const {
    const int x = r - base;
    return x < 0 ? x + kMaxTileRows : x;
  }
  __device__ bool holds(int) const { return true; }
  __device__ void clear(int r) { lo[slot(r)] = INFINITY; hi[slot(r)] = -INFINITY; }
  __device__ void fold(int r, double l, double h) {
    const int q = slot(r);
    lo[q] = fmin(lo[q], l);
    hi[q] = fmax(hi[q], h);
  }
  __device__ void get(int r, double& l, double& h) const { l = lo[slot(r)]; h = hi[slot(r)]; }
};

struct RowsWin {
  double lo[kWinRows], hi[kWinRows];
  int base;
  bool overflow;
  __device__ bool holds(int r) const { return r >= base && r < base + kWinRows; }
  __device__ void clear(int r) {
#pragma unroll
    for (int i = 0; i < kWinRows; ++i)
      if (r - base == i) { lo[i] = INFINITY; hi[i] = -INFINITY; }
  }
  __device__ void fold(int r, double l, double h) {
#pragma unroll
    for (int i = 0; i < kWinRows; ++i)
      if (r - base == i) { lo[i] = fmin(lo[i], l); hi[i] = fmax(hi[i], h); }
  }
  __device__ void get(int r, double& l, double& h) const {
    l = INFINITY;
    h = -INFINITY;
#pragma unroll
    for (int i = 0; i < kWinRows; ++i)
      if (r - base == i) { l = lo[i]; h = hi[i]; }
  }
};

template <class Rows>
struct SpansT {
  Rows rows;
  double bx0, bx1, by0, by1;        // box of every projected segment and the low-pass square
  int r0, r1;                       // initialised rows [r0, r1]
  int W, H, tx, ty;
  // near-plane clipping state (Sutherland-Hodgman order); every point in front of the near plane is
  // projected once (its pixel coordinates kept beside it) and reused by both edges it ends
  bool have_prev, prev_in, have_first;
  double prev[3], first[3], prev_xy[2], first_xy[2];
  bool pending_exit, have_first_entry;
  double exit_xy[2], first_entry_xy[2];
};
using Spans = SpansT<RowsAll>;

template <class S>
__device__ inline void spans_init(S& sp, const CamDev& cam) {
  sp.r0 = 1; sp.r1 = 0;
  sp.bx0 = sp.by0 = INFINITY;
  sp.bx1 = sp.by1 = -INFINITY;
  sp.W = cam.W; sp.H = cam.H; sp.tx = cam.tiles_x; sp.ty = cam.tiles_y;
  sp.have_prev = false; sp.have_first = false; sp.pending_exit = false; sp.have_first_entry = false;
  sp.rows.overflow = false;
}

// Row r takes the x-extent [l, h]: the rows [r0, r1] grow to hold it (new rows start empty).
template <class S>
__device__ inline void spans_row(S& sp, int r, double l, double h) {
  if (!sp.rows.holds(r)) { sp.rows.overflow = true; return; }
  if (sp.r0 > sp.r1) {
    sp.r0 = sp.r1 = r;
    sp.rows.clear(r);
  } else {
    while (r < sp.r0) { --sp.r0; sp.rows.clear(sp.r0); }
    while (r > sp.r1) { ++sp.r1; sp.rows.clear(sp.r1); }
  }
  sp.rows.fold(r, l, h);
}

// Screen segment (x0,y0)-(x1,y1) against every tile row slab it may cross.
template <class S>
__device__ inline void spans_segment(S& sp, double x0, double y0, double x1, double y1) {
  double ymin = fmin(y0, y1), ymax = fmax(y0, y1);
  sp.bx0 = fmin(sp.bx0, fmin(x0, x1));
  sp.bx1 = fmax(sp.bx1, fmax(x0, x1));
  sp.by0 = fmin(sp.by0, ymin);
  sp.by1 = fmax(sp.by1, ymax);
  double fa = floor((ymin - 15.5) / 16.0), fb = ceil((ymax - 0.5) / 16.0);
  if (!(fb >= 0.0) || !(fa <= (double)(sp.ty - 1))) return;
  int ra = fa < 0.0 ? 0 : (int)fa;
  int rb = fb > (double)(sp.ty - 1) ? sp.ty - 1 : (int)fb;
  for (int r = ra; r <= rb; ++r) {
    double ya = 16.0 * r + 0.5;
    double yb = fmin(16.0 * r + 15.5, sp.H - 0.5);
    if (ymax < ya || ymin > yb) continue;
    double xa, xb;
    if (y0 == y1) {
      xa = x0; xb = x1;
    } else {
      double ta = (ya - y0) / (y1 - y0);
      double tb = (yb - y0) / (y1 - y0);
      double tlo = fmax(0.0, fmin(ta, tb));
      double thi = fmin(1.0, fmax(ta, tb));
      xa = x0 + tlo * (x1 - x0);
      xb = x0 + thi * (x1 - x0);
    }
    spans_row(sp, r, fmin(xa, xb), fmax(xa, xb));
  }
}

__device__ inline void project(const CamDev& cam, const double p[3], double& x, double& y) {
  x = ((double)cam.fx * p[0]) / p[2] + (double)cam.cx;
  y = ((double)cam.fy * p[1]) / p[2] + (double)cam.cy;
}

// Camera-space polygon vertex stream, clipped to z >= near in Sutherland-Hodgman order.  axy / bxy
// are the pixel coordinates of a / b (used only when the point is in front of the near plane).
template <class S>
__device__ inline void clip_edge(S& sp, const CamDev& cam, double nearp, const double a[3], const double axy[2],
                                 const double b[3], const double bxy[2]) {
  bool ain = a[2] >= nearp, bin = b[2] >= nearp;
  double Ixy[2] = {0.0, 0.0};
  if (ain != bin) {
    double t = (nearp - a[2]) / (b[2] - a[2]);
    double I[3];
    for (int i = 0; i < 3; ++i) I[i] = a[i] + t * (b[i] - a[i]);
    project(cam, I, Ixy[0], Ixy[1]);
  }
  if (ain && bin) {
    spans_segment(sp, axy[0], axy[1], bxy[0], bxy[1]);
  } else if (ain && !bin) {            // exit
    spans_segment(sp, axy[0], axy[1], Ixy[0], Ixy[1]);
    sp.pending_exit = true;
    sp.exit_xy[0] = Ixy[0]; sp.exit_xy[1] = Ixy[1];
  } else if (!ain && bin) {            // entry
    if (sp.pending_exit) {
      spans_segment(sp, sp.exit_xy[0], sp.exit_xy[1], Ixy[0], Ixy[1]);
      sp.pending_exit = false;
    } else if (!sp.have_first_entry) {
      sp.have_first_entry = true;
      sp.first_entry_xy[0] = Ixy[0]; sp.first_entry_xy[1] = Ixy[1];
    }
    spans_segment(sp, Ixy[0], Ixy[1], bxy[0], bxy[1]);
  }
}

template <class S>
__device__ inline void push_vertex(S& sp, const CamDev& cam, double nearp, const double p[3]) {
  double pxy[2] = {0.0, 0.0};
  if (p[2] >= nearp) project(cam, p, pxy[0], pxy[1]);
  if (!sp.have_first) {
    sp.have_first = true;
    for (int i = 0; i < 3; ++i) sp.first[i] = p[i];
    sp.first_xy[0] = pxy[0]; sp.first_xy[1] = pxy[1];
  } else {
    clip_edge(sp, cam, nearp, sp.prev, sp.prev_xy, p, pxy);
  }
  for (int i = 0; i < 3; ++i) sp.prev[i] = p[i];
  sp.prev_xy[0] = pxy[0]; sp.prev_xy[1] = pxy[1];
}

template <class S>
__device__ inline void close_polygon(S& sp, const CamDev& cam, double nearp) {
  if (sp.have_first) clip_edge(sp, cam, nearp, sp.prev, sp.prev_xy, sp.first, sp.first_xy);
  if (sp.pending_exit && sp.have_first_entry)
    spans_segment(sp, sp.exit_xy[0], sp.exit_xy[1], sp.first_entry_xy[0], sp.first_entry_xy[1]);
}

// tangent-plane (x, y) -> camera frame
__device__ inline void lift(const GeoBase& g, const CamDev& cam, double x, double y, double out[3]) {
  double w[3];
  for (int i = 0; i < 3; ++i) w[i] = (g.mu[i] + x * g.tu[i]) + y * g.tv[i];
  to_cam(cam, w, out);
}

// Bases of primitive j as float64: from a loaded Geo, or read from the scene (the same values).
struct GeoBases {
  const Geo& g;
  __device__ double s(int k) const { return g.s[k]; }
  __device__ double th(int k) const { return g.th[k]; }
};
struct SceneBases {
  const SceneDev& sc;
  int64_t j;
  __device__ double s(int k) const { return (double)sc.scale[k * sc.n + j]; }
  __device__ double th(int k) const { return (double)sc.theta[k * sc.n + j]; }
};

// Builds the tile-row spans of primitive g (cull_mode 0: conservative support polygon;
// 1: the paper's endpoint polygon; 2 handled by the caller).  The row store's base is set by the
// caller for RowsWin; RowsAll's is set here.
template <class Rows, class B>
__device__ void build_spans(const GeoBase& g, const B& bs, const CamDev& cam, const OptsDev& opt, SpansT<Rows>& sp) {
  spans_init(sp, cam);
  if constexpr (std::is_same<Rows, RowsAll>::value) {
    const double pyc = fmin(fmax((double)cam.fy * g.muc[1] / g.muc[2] + (double)cam.cy, -1e7), 1e7);
    sp.rows.base = min(max((int)floor(pyc / 16.0), 0), sp.ty - 1);
  }
  const double nearp = (double)opt.near_plane;
  const int K = g.K;
  if (opt.cull_mode == 1) {
    double y = exp(-9.0) / g.o;
    double gm = psi_inv(y < 1.0 ? y : 1.0, g.tau);
    double ml = -log(gm);
    double f = sqrt(ml > 0.0 ? ml : 0.0);
    for (int k = 0; k < K; ++k) {
      double sc = bs.s(k) * f;
      double p[3];
      double sn_, cs_;
      sincos(bs.th(k), &sn_, &cs_);
      lift(g, cam, sc * cs_, sc * sn_, p);
      push_vertex(sp, cam, nearp, p);
    }
  } else {
    // Support polygon.  E is a convex combination of r1^2 and r2^2/sbar^2, so the support reaches at
    // most c * max(chord, sbar) along each direction (chord: distance to the segment e_k e_{k+1},
    // Eq. L1 level set; sbar: Eq. radial).  Both are maximal at the ends of each half sector, where
    // they equal s_k, s_{k+1} or the bisector values below; each half is covered by the quad of its
    // circular sector (half-angle delta/4 < pi/4).
    // cos / sin of theta_k: the previous sector's end angle is this sector's start angle
    double cth, sth;
    sincos(bs.th(0), &sth, &cth);
    for (int k = 0; k < K; ++k) {
      const double thk = bs.th(k);
      const double thn = (k + 1 < K) ? bs.th(k + 1) : bs.th(0) + kTwoPi;
      const double sk = bs.s(k), sn = bs.s((k + 1) % K);
      const double dl = thn - thk;
      const double sbar_mid = 1.0 / sqrt(0.5 * (1.0 / (sk * sk) + 1.0 / (sn * sn)));
      const double chord_mid = 2.0 * cos(0.5 * dl) / (1.0 / sk + 1.0 / sn);
      const double r_mid = fmax(sbar_mid, chord_mid);
      const double rho0 = g.c * fmax(sk, r_mid);
      const double rho1 = g.c * fmax(sn, r_mid);
      const double sec = 1.0 / cos(0.25 * dl);
      const double a1 = thk + 0.5 * dl, m0 = thk + 0.25 * dl, m1 = thk + 0.75 * dl;
      double ca1, sa1;
      sincos(a1, &sa1, &ca1);
      // the six vertices in the tangent plane, then pushed through one call site (one inlined copy
      // of the clip and row walk instead of six keeps the kernel at 3 waves per SIMD)
      double vx[6], vy[6];
      vx[0] = rho0 * cth; vy[0] = rho0 * sth;
      double cm0, sm0, cm1, sm1;
      sincos(m0, &sm0, &cm0);
      sincos(m1, &sm1, &cm1);
      vx[1] = rho0 * sec * cm0; vy[1] = rho0 * sec * sm0;
      vx[2] = rho0 * ca1; vy[2] = rho0 * sa1;
      vx[3] = rho1 * ca1; vy[3] = rho1 * sa1;
      vx[4] = rho1 * sec * cm1; vy[4] = rho1 * sec * sm1;
      sincos(thn, &sth, &cth);
      vx[5] = rho1 * cth; vy[5] = rho1 * sth;
#pragma unroll 1
      for (int q = 0; q < 6; ++q) {
        double p[3];
        lift(g, cam, vx[q], vy[q], p);
        push_vertex(sp, cam, nearp, p);
      }
    }
  }
  close_polygon(sp, cam, nearp);
  // low-pass support: square of half-width s_l sqrt(2 ln(o / alpha_min)) around the projected centre
  if (opt.lowpass_sl > 0.0f) {
    double ratio = g.o / (double)opt.alpha_min;
    double r = (double)opt.lowpass_sl * sqrt(2.0 * log(ratio > 1.0 ? ratio : 1.0));
    double dcx, dcy;
    project(cam, g.muc, dcx, dcy);
    sp.bx0 = fmin(sp.bx0, dcx - r);
    sp.bx1 = fmax(sp.bx1, dcx + r);
    sp.by0 = fmin(sp.by0, dcy - r);
    sp.by1 = fmax(sp.by1, dcy + r);
    for (int row = 0; row < sp.ty; ++row) {
      double ya = 16.0 * row + 0.5;
      double yb = fmin(16.0 * row + 15.5, sp.H - 0.5);
      if (dcy + r >= ya && dcy - r <= yb) spans_row(sp, row, dcx - r, dcx + r);
    }
  }
}

// Tile columns [i0, i1] of row r (false when none).
template <class S>
__device__ inline bool row_tiles(const S& sp, int r, int& i0, int& i1) {
  double l, h;
  sp.rows.get(r, l, h);
  double lo = fmax(l, 0.5);
  double hi = fmin(h, sp.W - 0.5);
  if (lo > hi) return false;
  double a = ceil((lo - 15.5) / 16.0);
  double b = floor((hi - 0.5) / 16.0);
  i0 = a < 0.0 ? 0 : (int)a;
  i1 = b > (double)(sp.tx - 1) ? sp.tx - 1 : (int)b;
  return i0 <= i1;
}

__device__ inline float diamond_angle(float c, float s) {
  // pseudo-angle in [0, 4), strictly increasing with the polar angle of (c, s)
  float r = c / (fabsf(c) + fabsf(s));
  return s >= 0.0f ? 1.0f - r : 3.0f + r;
}

// ---------------------------------------------------------------------------------------------
// Conservative frustum test.  The support polygon lies in the tangent-plane disc of radius
// sqrt(2) c max_k s_k around the centre (its half-sector quads reach rho / cos(h) with
// rho <= c max s_k, h < pi/4); the endpoint polygon of cull mode 1 in that of radius f max_k s_k.  Over that disc a side plane's linear form a . x (pixel x = 0 or W,
// y = 0 or H) ranges over a . mu_c +- R |a - (a . n) n|, n the disc's unit normal; if the whole range
// is on the outer side, no part of the near-clipped polygon can reach a pixel centre (0.5 px inside
// those planes).  The extent carries a margin of 1e-6 |a| (rounding of |a|^2 - (a . n)^2 near zero,
// and of n's length) and R one of 1e-9 relative.  The low-pass square is tested directly.  Culling
// here never removes a tile the polygon would produce.
__device__ inline double disc_extent(double ax, double ay, double az, const double n[3]) {
  const double aa = (ax * ax + ay * ay) + az * az;
  const double an = (ax * n[0] + ay * n[1]) + az * n[2];
  return sqrt(fmax(aa - an * an, 0.0) + 1e-12 * aa);
}

__device__ inline bool outside_view(const GeoBase& g, const CamDev& cam, const OptsDev& opt) {
  // disc radius: sqrt(2) c max_k s_k for the support polygon; for the paper's endpoint polygon
  // (cull mode 1, vertices at s_k f) f max_k s_k
  double rad = 1.4142135623730951 * g.c;
  if (opt.cull_mode == 1) {
    const double y = exp(-9.0) / g.o;
    const double gm = psi_inv(y < 1.0 ? y : 1.0, g.tau);
    const double ml = -log(gm);
    rad = sqrt(ml > 0.0 ? ml : 0.0);
  }
  const double R = rad * g.smax * (1.0 + 1e-9) + 1e-12;
  const double X = g.muc[0], Y = g.muc[1], Z = g.muc[2];
  const double fx = cam.fx, fy = cam.fy, cx = cam.cx, cy = cam.cy, W = cam.W, H = cam.H;
  const double nw[3] = {g.tu[1] * g.tv[2] - g.tu[2] * g.tv[1], g.tu[2] * g.tv[0] - g.tu[0] * g.tv[2],
                        g.tu[0] * g.tv[1] - g.tu[1] * g.tv[0]};
  double n[3];
  rot_cam(cam, nw, n);
  bool out = (fx * X + cx * Z) < -R * disc_extent(fx, 0.0, cx, n) ||
             (fx * X + (cx - W) * Z) > R * disc_extent(fx, 0.0, cx - W, n) ||
             (fy * Y + cy * Z) < -R * disc_extent(0.0, fy, cy, n) ||
             (fy * Y + (cy - H) * Z) > R * disc_extent(0.0, fy, cy - H, n);
  if (out && opt.lowpass_sl > 0.0f) {
    const double ratio = g.o / (double)opt.alpha_min;
    const double r = (double)opt.lowpass_sl * sqrt(2.0 * log(ratio > 1.0 ? ratio : 1.0));
    double dcx, dcy;
    project(cam, g.muc, dcx, dcy);
    const bool sq_out = dcx + r < 0.25 || dcx - r > W - 0.25 || dcy + r < 0.25 || dcy - r > H - 0.25;
    out = sq_out;
  }
  return out;
}

// Per-thread offsets from one atomic per workgroup of NWAVES waves (every thread of the block must
// call it): a wave scan, then the wave totals scanned in LDS by one thread, which also takes the
// block's range from the counter.  One atomic per wave on a single counter serialised a kernel of
// 1M threads.
template <int NWAVES>
__device__ inline uint32_t block_alloc(uint32_t* ctr, uint32_t n) {
  __shared__ uint32_t s_part[NWAVES + 1];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  uint32_t inc = n;
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(inc, o, 64);
    if (lane >= o) inc += y;
  }
  if (lane == 63) s_part[wv] = inc;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t run = 0;
    for (int w = 0; w < NWAVES; ++w) {
      const uint32_t t = s_part[w];
      s_part[w] = run;
      run += t;
    }
    s_part[NWAVES] = run ? atomicAdd(ctr, run) : 0u;
  }
  __syncthreads();
  return s_part[NWAVES] + s_part[wv] + inc - n;
}

// Render record of a visible primitive (layout: RecField / SecField), and its per-tile key data when
// kg is given; the support polygon's box (R_BOX, KG_BOX) is written by the polygon kernel.  The
// bases are read from the scene.
__device__ void write_record(const GeoBase& g, const SceneDev& sc, int64_t j, const CamDev& cam, const OptsDev& opt,
                             float* rec, double* kg) {
  const int64_t n = sc.n;
  const int K = sc.K;
  // homography: adjugate rows of N = [t_u^c | t_v^c | mu_c]
  double tuc[3], tvc[3];
  rot_cam(cam, g.tu, tuc);
  rot_cam(cam, g.tv, tvc);
  const double* m = g.muc;
  double a0[3] = {tvc[1] * m[2] - tvc[2] * m[1], tvc[2] * m[0] - tvc[0] * m[2], tvc[0] * m[1] - tvc[1] * m[0]};
  double a1[3] = {m[1] * tuc[2] - m[2] * tuc[1], m[2] * tuc[0] - m[0] * tuc[2], m[0] * tuc[1] - m[1] * tuc[0]};
  double a2[3] = {tuc[1] * tvc[2] - tuc[2] * tvc[1], tuc[2] * tvc[0] - tuc[0] * tvc[2],
                  tuc[0] * tvc[1] - tuc[1] * tvc[0]};
  double dN = a2[0] * m[0] + a2[1] * m[1] + a2[2] * m[2];
  const double smax = g.smax;
  if (kg) {
    // per-tile key data: the plane, and the depth range of the disc of radius sqrt(2) c max_k s_k
    // around the centre, which holds the support polygon (its half-sector quads reach rho / cos(h)
    // with rho <= c max_k s_k and h < pi/4)
    const double zr = (1.4142135623730951 * (g.c * smax)) * sqrt(tuc[2] * tuc[2] + tvc[2] * tvc[2]);
    for (int i = 0; i < 3; ++i) kg[KG_A + i] = a2[i];
    kg[KG_DN] = dN;
    kg[KG_ZC] = m[2];
    kg[KG_ZLO] = fmax(m[2] - zr, (double)opt.near_plane);
    kg[KG_ZHI] = m[2] + zr;
  }
  double fx = cam.fx, fy = cam.fy, cx = cam.cx, cy = cam.cy;
  double pxc = (fx * m[0]) / m[2] + cx, pyc = (fy * m[1]) / m[2] + cy;
  double axc = fmin(fmax(pxc, -2.0 * cam.W), 3.0 * cam.W);
  double ayc = fmin(fmax(pyc, -2.0 * cam.H), 3.0 * cam.H);
  double ax = rint(axc * 256.0) / 256.0, ay = rint(ayc * 256.0) / 256.0;
  const double* rows[3] = {a0, a1, a2};
  for (int r = 0; r < 3; ++r) {
    const double* a = rows[r];
    rec[R_H + 3 * r + 0] = (float)(a[0] / fx);
    rec[R_H + 3 * r + 1] = (float)(a[1] / fy);
    rec[R_H + 3 * r + 2] = (float)(a[0] * (ax - cx) / fx + a[1] * (ay - cy) / fy + a[2]);
  }
  rec[R_DN] = (float)dN;
  rec[R_AX] = (float)ax;
  rec[R_AY] = (float)ay;
  rec[R_OX] = (float)(pxc - ax);
  rec[R_OY] = (float)(pyc - ay);
  rec[R_O] = (float)g.o;
  rec[R_ETA] = sc.eta[j];
  const double tau = g.tau;
  rec[R_PLO] = (float)((1.0 + tau) / 4.0);
  rec[R_PHI] = (float)((3.0 - tau) / 4.0);
  rec[R_PA1] = (float)((1.0 - tau) / (1.0 + tau));
  rec[R_PA2] = (float)((1.0 + tau) / (1.0 - tau));
  rec[R_PB2] = (float)(-tau / (1.0 - tau));
  rec[R_PB3] = (float)(2.0 * tau / (1.0 + tau));
  rec[R_TAU] = (float)tau;
  // exact early-outs of the raster (with margin): E >= r2 / max_k s_k^2 (both the L1 chord and sbar
  // are bounded by the larger basis length), and the low-pass term needs d^2/den^2 <= 2 s_l^2 ln(o/alpha_min)
  rec[R_R2CUT] = (float)(1.001 * (g.c * smax) * (g.c * smax) + 1e-30);
  const double ratio = g.o / (double)opt.alpha_min;
  const double lpc = opt.lowpass_sl > 0.0f ? 2.0 * (double)opt.lowpass_sl * (double)opt.lowpass_sl *
                                                 log(ratio > 1.0 ? ratio : 1.0)
                                           : 0.0;
  rec[R_LPCUT] = opt.lowpass_sl > 0.0f ? (float)(1.001 * lpc + 1e-6) : -1.0f;
  // alpha = o Psi(exp(-E/2)) is decreasing in E and equals alpha_min at E = c^2; the margin keeps
  // the raster's float32 test conservative against the rounding of exp and Psi
  rec[R_ETHR] = (float)(g.c * g.c * 1.001 + 1e-2);
  {
    // unit normal of the plane, turned toward the camera (n . mu_c < 0), for the normal channel
    const double na = sqrt(a2[0] * a2[0] + a2[1] * a2[1] + a2[2] * a2[2]);
    const double sgn = dN > 0.0 ? -1.0 : 1.0;
    for (int i = 0; i < 3; ++i) rec[R_NRM + i] = (float)(sgn * a2[i] / na);
  }
  if (sc.color_mode == 0) {
    for (int c = 0; c < 3; ++c) rec[R_RGB + c] = sc.color[c * n + j];
  } else {
    double cp[3];
    for (int i = 0; i < 3; ++i)
      cp[i] = cam.campos[i];
    double d[3] = {g.mu[0] - cp[0], g.mu[1] - cp[1], g.mu[2] - cp[2]};
    double dn = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    double Y[16];
    real_sh(sc.sh_degree, d[0] / dn, d[1] / dn, d[2] / dn, Y);
    const int nc = (sc.sh_degree + 1) * (sc.sh_degree + 1);
    for (int c = 0; c < 3; ++c) {
      double acc = 0.0;
      for (int i = 0; i < nc; ++i) acc += Y[i] * (double)sc.color[(3 * i + c) * n + j];
      acc += 0.5;
      rec[R_RGB + c] = (float)(acc > 0.0 ? acc : 0.0);
    }
  }
  for (int k = 0; k < K; ++k) {
    int kn = (k + 1 < K) ? k + 1 : 0;
    double thk = (double)sc.theta[k * n + j];
    double thn = (k + 1 < K) ? (double)sc.theta[(k + 1) * n + j] : (double)sc.theta[j] + kTwoPi;
    double dl = thn - thk;
    double sk = (double)sc.scale[k * n + j], sn = (double)sc.scale[kn * n + j];
    float cf = (float)cos(thk), sf = (float)sin(thk);
    rec[R_SEC + S_PA * K + k] = diamond_angle(cf, sf);
    rec[R_SEC + S_C * K + k] = cf;
    rec[R_SEC + S_S * K + k] = sf;
    rec[R_SEC + S_ID * K + k] = (float)(1.0 / dl);
    double sd = sin(dl);
    rec[R_SEC + S_A * K + k] = (float)(1.0 / (sk * sd));
    rec[R_SEC + S_B * K + k] = (float)(1.0 / (sn * sd));
    rec[R_SEC + S_IK2 * K + k] = (float)(1.0 / (sk * sk));
    rec[R_SEC + S_WLO * K + k] = (float)(fmin(1.0 / (sk * sk), 1.0 / (sn * sn)) * 0.99999);
  }
}

// Pass 1, one thread per (primitive, view): validity, near/opacity/frustum culling and the
// centre-depth key (float32 of ((r20 x + r21 y) + r22 z) + t2, computed in float64).  Primitives
// that may touch the view are appended to the view's work list.  Per-view arrays are
// [view][stride] with stride = the workspace capacity in primitives.
constexpr int kPreBlock = 256;
constexpr int kFixedRows = 8;           // span rows reserved per position of the small work list

// Row buffer of a view (row_cap rows): kFixedRows rows per work-list position, then kSpanPools
// pools filled by atomic counters for primitives with more rows (or for all of them when the buffer
// cannot hold the fixed rows beside pools of at least 64 rows).  Position p of the small list owns
// rows [p kFixedRows, (p + 1) kFixedRows); position p of the big list owns those of position
// stride - 1 - p while that is past the small list's end (the two lists hold at most stride
// primitives unless the small kernel moved some; then the pools).  A primitive whose rows fit
// nowhere gets kNoSpans and is re-derived by the duplication.
struct RowLayout {
  bool fixed;
  int64_t pool_base, pool_rows;
};
__device__ inline RowLayout row_layout(int64_t row_cap, int64_t stride) {
  RowLayout L;
  const int64_t f = (int64_t)kFixedRows * stride;
  L.fixed = row_cap >= f + (int64_t)kSpanPools * 64;
  L.pool_base = L.fixed ? f : 0;
  L.pool_rows = (row_cap - L.pool_base) / kSpanPools;
  return L;
}
constexpr uint32_t kNoItem = 0xFFFFFFFFu;   // a work-list entry taken over by the other list

// Tile rows the support can touch, estimated from the ball of the support disc around the centre:
// for a point (Y + dY, Z + dZ) with dY^2 + dZ^2 <= R^2 and Z - R > 0, |(Y + dY)/(Z + dZ) - Y/Z| <=
// R sqrt(Y^2 + Z^2) / (Z (Z - R)).  True (and the window's first row) when at most opt.win_admit rows
// (kWinRows unless a test asks for more, to make primitives leave their window) are touched and
// no part of the ball is behind the near plane.  The window only chooses the kernel (a primitive
// that touches a row outside it is handed to the wave-parallel one), so float32 is enough here.
__device__ inline bool span_window(const GeoBase& g, const CamDev& cam, const OptsDev& opt, int& base) {
  base = 0;
  if (opt.cull_mode == 2) return true;
  float rad = 1.4142135f * (float)g.c;
  if (opt.cull_mode == 1) {
    const double y = exp(-9.0) / g.o;
    const double gm = psi_inv(y < 1.0 ? y : 1.0, g.tau);
    const float ml = -logf((float)gm);
    rad = sqrtf(ml > 0.0f ? ml : 0.0f);
  }
  const float R = rad * (float)g.smax * 1.001f + 1e-6f;
  const float Y = (float)g.muc[1], Z = (float)g.muc[2];
  if (!(Z - R > opt.near_plane)) return false;
  const float dy = cam.fy * R * sqrtf(Z * Z + Y * Y) / (Z * (Z - R)) * 1.001f;
  const float yc = (cam.fy * Y) / Z + cam.cy;
  float ymin = yc - dy, ymax = yc + dy;
  if (opt.lowpass_sl > 0.0f) {
    const float ratio = (float)g.o / opt.alpha_min;
    const float r = opt.lowpass_sl * sqrtf(2.0f * logf(ratio > 1.0f ? ratio : 1.0f)) * 1.001f;
    ymin = fminf(ymin, yc - r);
    ymax = fmaxf(ymax, yc + r);
  }
  const float last = (float)(cam.tiles_y - 1);
  const float ra = fmaxf(ceilf((ymin - 15.5f) / 16.0f), 0.0f), rb = fminf(floorf((ymax - 0.5f) / 16.0f), last);
  if (!(rb - ra + 1.0f <= (float)opt.win_admit)) return false;
  base = (int)fminf(ra, last);
  return true;
}

__global__ void __launch_bounds__(kPreBlock) k_preprocess(SceneDev sc, const Views* __restrict__ views, OptsDev opt,
                                                    uint32_t* __restrict__ depth_keys,
                                                    uint32_t* __restrict__ tile_counts,
                                                    uint32_t* __restrict__ work_small,
                                                    uint32_t* __restrict__ count_small,
                                                    uint32_t* __restrict__ work_big, uint32_t* __restrict__ count_big,
                                                    uint32_t* __restrict__ status, int64_t stride, int nv) {
  // consecutive workgroups take the same primitives for each view in turn, so that with several
  // views a primitive's parameters are read from memory once and then from the caches
  const int v = (int)(blockIdx.x % (unsigned)nv);
  const int64_t j = (int64_t)(blockIdx.x / (unsigned)nv) * blockDim.x + threadIdx.x;
  const CamDev& cam = views->cam[v];
  bool maybe = false, small = false;
  if (j < sc.n) {
    GeoBase g;
    bool invalid = false;
    const bool alive = load_geo_core<double>(sc, j, cam, opt, g, &invalid, nullptr, nullptr);
    if (invalid && opt.validate) atomicOr(status + v, (uint32_t)ST_INVALID);
    maybe = alive && (opt.cull_mode == 2 || !outside_view(g, cam, opt));
    int base;
    small = maybe && span_window(g, cam, opt, base);
    depth_keys[(int64_t)v * stride + j] = maybe ? __float_as_uint((float)g.muc[2]) : kCulledKey;
    tile_counts[(int64_t)v * stride + j] = 0;
  }
  const uint32_t slot_s = block_alloc<kPreBlock / 64>(count_small + v, small ? 1u : 0u);
  __syncthreads();
  const uint32_t slot_b = block_alloc<kPreBlock / 64>(count_big + v, maybe && !small ? 1u : 0u);
  if (small) work_small[(int64_t)v * stride + slot_s] = (uint32_t)j;
  if (maybe && !small) work_big[(int64_t)v * stride + slot_b] = (uint32_t)j;
}

// Pass 2a, one thread per primitive of the small list: the sequential polygon walk with the rows
// of its window in registers (the same float64 expressions as the wave-parallel kernel, so the
// same spans); a primitive that touches a row outside its window moves to the big list.
__global__ void __launch_bounds__(128) k_polygon_small(SceneDev sc, const Views* __restrict__ views, OptsDev opt,
                                                       float* __restrict__ records, uint32_t* __restrict__ depth_keys,
                                                       uint32_t* __restrict__ tile_counts,
                                                       uint32_t* __restrict__ work_small,
                                                       const uint32_t* __restrict__ count_small,
                                                       uint32_t* __restrict__ work_big, uint32_t* __restrict__ count_big,
                                                       uint2* __restrict__ span_meta, uint32_t* __restrict__ span_rows,
                                                       uint32_t* __restrict__ pool_used, int64_t row_cap,
                                                       int64_t stride, double* __restrict__ keygeo) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int v = blockIdx.y;
  const CamDev& cam = views->cam[v];
  const int K = sc.K;
  const int64_t ns = (int64_t)count_small[v];
  if (ns < (int64_t)opt.small_min) return;   // too few to fill the GPU: the wave kernel takes them
  const bool active = i < ns;
  const int64_t j = active ? (int64_t)work_small[(int64_t)v * stride + i] : 0;
  const int64_t o = (int64_t)v * stride + j;
  bool over = false, ok = false;
  uint32_t count = 0;
  SpansT<RowsWin> sp;
  if (active) {
    GeoBase g;
    bool invalid;
    ok = load_geo_core<double>(sc, j, cam, opt, g, &invalid, nullptr, nullptr);
    if (ok) {
      if (opt.cull_mode == 2) {
        count = (uint32_t)(cam.tiles_x * cam.tiles_y);
      } else {
        int base;
        over = !span_window(g, cam, opt, base);
        if (!over) {
          sp.rows.base = base;
          build_spans(g, SceneBases{sc, j}, cam, opt, sp);
          over = sp.rows.overflow;
        }
        if (!over) {
          for (int r = sp.r0; r <= sp.r1; ++r) {
            int i0, i1;
            if (row_tiles(sp, r, i0, i1)) count += (uint32_t)(i1 - i0 + 1);
          }
        }
      }
    }
  }
  const uint32_t slot_b = block_alloc<2>(count_big + v, over ? 1u : 0u);
  if (!active) return;
  if (over) {
    work_big[(int64_t)v * stride + slot_b] = (uint32_t)j;
    work_small[(int64_t)v * stride + i] = kNoItem;
    return;
  }
  tile_counts[o] = count;
  if (count == 0) {
    depth_keys[o] = kCulledKey;
    return;
  }
  double box[4] = {-1e30, 1e30, -1e30, 1e30};   // only the conservative polygon bounds the support
  if (opt.cull_mode != 2) {
    const uint32_t nrows = (uint32_t)(sp.r1 - sp.r0 + 1);   // at most kWinRows <= kFixedRows
    const RowLayout rl = row_layout(row_cap, stride);
    int64_t at;
    bool fits;
    if (rl.fixed) {
      at = i * kFixedRows;
      fits = true;
    } else {
      const uint32_t pool = (uint32_t)(i % kSpanPools);
      const uint32_t off = atomicAdd(pool_used + (int64_t)v * kSpanPools + pool, nrows);
      at = rl.pool_base + (int64_t)pool * rl.pool_rows + off;
      fits = (int64_t)off + nrows <= rl.pool_rows;
    }
    fits = fits && at + nrows < (int64_t)kNoSpans;
    uint2 meta = make_uint2(kNoSpans, 0u);
    if (fits) {
      uint32_t* out = span_rows + (int64_t)v * row_cap + at;
      for (int r = sp.r0; r <= sp.r1; ++r) {
        int i0, i1;
        out[r - sp.r0] = row_tiles(sp, r, i0, i1) ? ((uint32_t)i0 | ((uint32_t)i1 << 16)) : 0xFFFFFFFFu;
      }
      meta = make_uint2((uint32_t)at, (uint32_t)sp.r0 | (nrows << 16));
    }
    span_meta[o] = meta;
    if (opt.cull_mode == 0) { box[0] = sp.bx0; box[1] = sp.bx1; box[2] = sp.by0; box[3] = sp.by1; }
  }
  float* rec = records + o * rec_floats(K);
  rec[R_BOX + 0] = (float)(box[0] - 0.01);
  rec[R_BOX + 1] = (float)(box[1] + 0.01);
  rec[R_BOX + 2] = (float)(box[2] - 0.01);
  rec[R_BOX + 3] = (float)(box[3] + 0.01);
  if (opt.key_mode != 0) {
    double* kg = keygeo + o * KG_N;
    for (int q = 0; q < 4; ++q) kg[KG_BOX + q] = box[q];
  }
}

// ---------------------------------------------------------------------------------------------
// Pass 2b: the support polygon of each primitive of the big list (supports that may span more than
// kWinRows tile rows or reach the near plane, and those that left the small list), wave-parallel.
// A wave takes a batch of work items, loads their geometry one item per lane, then builds the tile-row spans of one item at
// a time with all its lanes: the lanes take the polygon's vertices, then its edges (each clipped to
// the near plane and cut into tile-row slabs with the float64 expressions of the sequential walk
// above), and the rows' x-extents meet in LDS through exact 64-bit min / max on an order-preserving
// encoding of the doubles.  A minimum or a maximum does not depend on the order of its operands, so
// the spans, tile counts and box equal the sequential walk's bit for bit.  Outputs: the tile count,
// the row spans for the duplication pass (kNoSpans when the item's row pool is full, then the
// duplication re-derives them), and the record's box; the rest of the record is written by k_record.
constexpr int kPolyWaves = 4;           // waves per workgroup
constexpr int kPolyBatch = 8;           // work items per wave batch
constexpr int kMaxPolyV = 6 * kMaxK;    // support polygon vertices (cull mode 0: six per sector)
static_assert(kMaxPolyV <= 128, "edge exit masks cover two 64-edge chunks");

// Order-preserving encoding: unsigned order of the codes is the order of the (non-NaN) doubles.
__device__ inline uint64_t ord_enc(double x) {
  const uint64_t b = (uint64_t)__double_as_longlong(x);
  return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}
__device__ inline double ord_dec(uint64_t e) {
  return __longlong_as_double((long long)((e >> 63) ? (e & 0x7FFFFFFFFFFFFFFFull) : ~e));
}
constexpr uint64_t kEncPosInf = 0xFFF0000000000000ull;   // ord_enc(+inf)
constexpr uint64_t kEncNegInf = 0x000FFFFFFFFFFFFFull;   // ord_enc(-inf)

// Orders this lane's LDS accesses before and after against the other lanes of its wave.
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

struct PolyLds {
  uint64_t lo[kMaxTileRows], hi[kMaxTileRows];       // encoded x-extent of each tile row
  double vx[kMaxPolyV], vy[kMaxPolyV], vz[kMaxPolyV];  // camera-frame vertices
  double px[kMaxPolyV], py[kMaxPolyV];                 // their pixel coordinates (in front of the near plane)
  double ix[kMaxPolyV], iy[kMaxPolyV];                 // pixel coordinates of edge e's near-plane crossing
  GeoBase geo[kPolyBatch];                             // the batch's geometry
  float s[kPolyBatch][kMaxK], th[kPolyBatch][kMaxK];   // and its bases (the scene's float32 values)
  uint32_t item[kPolyBatch];                           // the batch's primitive indices
  double lp[kPolyBatch][3];                            // low-pass square: projected centre, half-width
  double f1[kPolyBatch];                               // cull mode 1: endpoint polygon factor
  uint64_t box[4];                                     // encoded box (x0, -x1, y0, -y1: all minima)
  int rows[2];                                         // touched rows [rows[0], -rows[1]] (minima)
  uint32_t cnt;                                        // tile count
};

// Per-lane part of the spans: box of the lane's segments and the rows they touched.
struct LaneSpans {
  double bx0, bx1, by0, by1;
  int r0, r1;
};

// One screen segment (x0,y0)-(x1,y1) against the tile-row slabs it may cross (the expressions of
// spans_segment; the row extents go to LDS).
__device__ inline void lane_segment(PolyLds& L, LaneSpans& a, int ty, int H, double x0, double y0, double x1,
                                    double y1) {
  const double ymin = fmin(y0, y1), ymax = fmax(y0, y1);
  a.bx0 = fmin(a.bx0, fmin(x0, x1));
  a.bx1 = fmax(a.bx1, fmax(x0, x1));
  a.by0 = fmin(a.by0, ymin);
  a.by1 = fmax(a.by1, ymax);
  const double fa = floor((ymin - 15.5) / 16.0), fb = ceil((ymax - 0.5) / 16.0);
  if (!(fb >= 0.0) || !(fa <= (double)(ty - 1))) return;
  const int ra = fa < 0.0 ? 0 : (int)fa;
  const int rb = fb > (double)(ty - 1) ? ty - 1 : (int)fb;
  for (int r = ra; r <= rb; ++r) {
    const double ya = 16.0 * r + 0.5;
    const double yb = fmin(16.0 * r + 15.5, H - 0.5);
    if (ymax < ya || ymin > yb) continue;
    double xa, xb;
    if (y0 == y1) {
      xa = x0; xb = x1;
    } else {
      const double ta = (ya - y0) / (y1 - y0);
      const double tb = (yb - y0) / (y1 - y0);
      const double tlo = fmax(0.0, fmin(ta, tb));
      const double thi = fmin(1.0, fmax(ta, tb));
      xa = x0 + tlo * (x1 - x0);
      xb = x0 + thi * (x1 - x0);
    }
    a.r0 = min(a.r0, r);
    a.r1 = max(a.r1, r);
    const double xl = fmin(xa, xb), xh = fmax(xa, xb);
    if (xl == xl) atomicMin(&L.lo[r], ord_enc(xl));   // fmin ignores a NaN operand; so does this
    if (xh == xh) atomicMax(&L.hi[r], ord_enc(xh));
  }
}

// Index of the exit edge that precedes edge e around the polygon (exit edges: bits of m0 for edges
// 0-63, of m1 for edges 64-127; at least one is set).
__device__ inline int prev_exit(uint64_t m0, uint64_t m1, int e) {
  if (e >= 64) {
    const int b = e - 64;
    const uint64_t below = b ? (m1 & ((1ull << b) - 1ull)) : 0ull;
    if (below) return 64 + 63 - __clzll((long long)below);
    if (m0) return 63 - __clzll((long long)m0);
    return 64 + 63 - __clzll((long long)m1);
  }
  const uint64_t below = e ? (m0 & ((1ull << e) - 1ull)) : 0ull;
  if (below) return 63 - __clzll((long long)below);
  if (m1) return 64 + 63 - __clzll((long long)m1);
  return 63 - __clzll((long long)m0);
}

__global__ void __launch_bounds__(64 * kPolyWaves) __attribute__((amdgpu_waves_per_eu(3))) k_polygon(SceneDev sc, const Views* __restrict__ views,
                                                            OptsDev opt, float* __restrict__ records,
                                                            uint32_t* __restrict__ depth_keys,
                                                            uint32_t* __restrict__ tile_counts,
                                                            const uint32_t* __restrict__ work_small,
                                                            const uint32_t* __restrict__ count_small,
                                                            const uint32_t* __restrict__ work,
                                                            const uint32_t* __restrict__ work_count,
                                                            uint2* __restrict__ span_meta,
                                                            uint32_t* __restrict__ span_rows,
                                                            uint32_t* __restrict__ pool_used, int64_t row_cap,
                                                            int64_t stride, double* __restrict__ keygeo) {
  __shared__ PolyLds s_lds[kPolyWaves];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  PolyLds& L = s_lds[wv];
  const int v = blockIdx.y;
  const CamDev& cam = views->cam[v];
  // the big list, then the small list too when k_polygon_small left it (fewer than small_min items):
  // the primitives that may span many rows come first, so that they do not finish last
  const int64_t n_small_all = (int64_t)count_small[v];
  const int64_t ns = n_small_all < (int64_t)opt.small_min ? n_small_all : 0;
  const int64_t nbig = (int64_t)work_count[v];
  const int64_t wc = nbig + ns;
  const int64_t n = sc.n;
  const int K = sc.K;
  const int ty = cam.tiles_y, tx = cam.tiles_x, W = cam.W, H = cam.H;
  const double nearp = (double)opt.near_plane;
  const int V = opt.cull_mode == 1 ? K : 6 * K;
  const RowLayout rl = row_layout(row_cap, stride);
  for (int r = lane; r < kMaxTileRows; r += 64) { L.lo[r] = kEncPosInf; L.hi[r] = kEncNegInf; }
  if (lane < 4) L.box[lane] = kEncPosInf;
  if (lane < 2) L.rows[lane] = kMaxTileRows;
  if (lane == 0) L.cnt = 0;
  for (int64_t b = (int64_t)blockIdx.x * kPolyWaves + wv; b * kPolyBatch < wc; b += (int64_t)gridDim.x * kPolyWaves) {
    const int64_t first = b * kPolyBatch;
    const int nb = (int)min((int64_t)kPolyBatch, wc - first);
    wave_sync();   // the previous batch's geometry has been read
    bool mine_ok = false;
    if (lane < nb) {
      const int64_t pos = first + lane;
      const uint32_t mine_j = pos < nbig ? work[(int64_t)v * stride + pos] : work_small[(int64_t)v * stride + (pos - nbig)];
      bool invalid;
      GeoBase mine;
      mine_ok = load_geo_core<float>(sc, mine_j, cam, opt, mine, &invalid, L.s[lane], L.th[lane]);
      L.geo[lane] = mine;
      L.item[lane] = mine_j;
      if (opt.lowpass_sl > 0.0f) {
        const double ratio = mine.o / (double)opt.alpha_min;
        project(cam, mine.muc, L.lp[lane][0], L.lp[lane][1]);
        L.lp[lane][2] = (double)opt.lowpass_sl * sqrt(2.0 * log(ratio > 1.0 ? ratio : 1.0));
      }
      if (opt.cull_mode == 1) {
        const double y = exp(-9.0) / mine.o;
        const double gm = psi_inv(y < 1.0 ? y : 1.0, mine.tau);
        const double ml = -log(gm);
        L.f1[lane] = sqrt(ml > 0.0 ? ml : 0.0);
      }
    }
    const uint64_t ok_mask = __ballot(mine_ok);
    const uint32_t pool = (uint32_t)(b % kSpanPools);
    wave_sync();
    for (int it = 0; it < nb; ++it) {
      if (!((ok_mask >> it) & 1ull)) {
        if (lane == 0) depth_keys[(int64_t)v * stride + L.item[it]] = kCulledKey;
        continue;
      }
      const int64_t j = (int64_t)L.item[it];
      const GeoBase& g = L.geo[it];
      const int64_t o = (int64_t)v * stride + j;
      if (opt.cull_mode == 2) {
        if (lane == 0) {
          tile_counts[o] = (uint32_t)(tx * ty);
          float* rec = records + o * rec_floats(K);
          rec[R_BOX + 0] = (float)(-1e30 - 0.01); rec[R_BOX + 1] = (float)(1e30 + 0.01);
          rec[R_BOX + 2] = (float)(-1e30 - 0.01); rec[R_BOX + 3] = (float)(1e30 + 0.01);
          if (opt.key_mode != 0) {
            double* kg = keygeo + o * KG_N;
            kg[KG_BOX + 0] = -1e30; kg[KG_BOX + 1] = 1e30; kg[KG_BOX + 2] = -1e30; kg[KG_BOX + 3] = 1e30;
          }
        }
        continue;
      }
      wave_sync();   // the previous item's LDS reads are done
      // vertices (lanes over the polygon's vertices), camera frame, and projected when in front
      const double f1 = opt.cull_mode == 1 ? L.f1[it] : 0.0;
      for (int q = lane; q < V; q += 64) {
        double x, y;
        if (opt.cull_mode == 1) {
          const double s1 = (double)L.s[it][q] * f1;
          const double th = (double)L.th[it][q];
          double sn_, cs_;
          sincos(th, &sn_, &cs_);
          x = s1 * cs_;
          y = s1 * sn_;
        } else {
          // half-sector quads of sector k (the sequential walk's expressions)
          const int k = q / 6, m = q - 6 * k;
          const double thk = (double)L.th[it][k];
          const double thn = (k + 1 < K) ? (double)L.th[it][k + 1] : (double)L.th[it][0] + kTwoPi;
          const double sk = (double)L.s[it][k], sn = (double)L.s[it][(k + 1) % K];
          const double dl = thn - thk;
          const double sbar_mid = 1.0 / sqrt(0.5 * (1.0 / (sk * sk) + 1.0 / (sn * sn)));
          const double chord_mid = 2.0 * cos(0.5 * dl) / (1.0 / sk + 1.0 / sn);
          const double r_mid = fmax(sbar_mid, chord_mid);
          double rad = g.c * fmax(m < 3 ? sk : sn, r_mid);
          if (m == 1 || m == 4) rad = rad * (1.0 / cos(0.25 * dl));
          const double ang = m == 0 ? thk : m == 1 ? thk + 0.25 * dl : m == 4 ? thk + 0.75 * dl : m == 5 ? thn
                                                                                                  : thk + 0.5 * dl;
          double sn_, cs_;
          sincos(ang, &sn_, &cs_);
          x = rad * cs_;
          y = rad * sn_;
        }
        double w[3], p[3];
        for (int i = 0; i < 3; ++i) w[i] = (g.mu[i] + x * g.tu[i]) + y * g.tv[i];
        to_cam(cam, w, p);
        L.vx[q] = p[0]; L.vy[q] = p[1]; L.vz[q] = p[2];
        // projected for every lane (no divergent branch); a vertex behind the near plane keeps 0
        double qx, qy;
        project(cam, p, qx, qy);
        const bool front = p[2] >= nearp;
        L.px[q] = front ? qx : 0.0; L.py[q] = front ? qy : 0.0;
      }
      wave_sync();
      // edges: near-plane crossings, and the exit edges as masks
      uint64_t exits[2] = {0ull, 0ull};
      for (int c = 0; c * 64 < V; ++c) {
        const int e = c * 64 + lane;
        bool is_exit = false;
        if (e < V) {
          const int f = e + 1 < V ? e + 1 : 0;
          const double az = L.vz[e], bz = L.vz[f];
          const bool ain = az >= nearp, bin = bz >= nearp;
          if (ain != bin) {
            const double t = (nearp - az) / (bz - az);
            double I[3];
            I[0] = L.vx[e] + t * (L.vx[f] - L.vx[e]);
            I[1] = L.vy[e] + t * (L.vy[f] - L.vy[e]);
            I[2] = az + t * (bz - az);
            double ix, iy;
            project(cam, I, ix, iy);
            L.ix[e] = ix; L.iy[e] = iy;
          }
          is_exit = ain && !bin;
        }
        exits[c] = __ballot(is_exit);
      }
      wave_sync();
      // segments: the kept part of each edge, and from each entry back to the preceding exit
      LaneSpans a;
      a.bx0 = a.by0 = INFINITY;
      a.bx1 = a.by1 = -INFINITY;
      a.r0 = kMaxTileRows; a.r1 = -1;
      for (int e = lane; e < V; e += 64) {
        const int f = e + 1 < V ? e + 1 : 0;
        const bool ain = L.vz[e] >= nearp, bin = L.vz[f] >= nearp;
        // up to two segments per edge, walked through one call site
        const int nseg = ain ? 1 : (bin ? 2 : 0);
        const int x = (!ain && bin) ? prev_exit(exits[0], exits[1], e) : e;
        for (int k = 0; k < nseg; ++k) {
          double x0, y0, x1, y1;
          if (ain) {                      // kept edge, or its part up to the exit
            x0 = L.px[e]; y0 = L.py[e];
            x1 = bin ? L.px[f] : L.ix[e];
            y1 = bin ? L.py[f] : L.iy[e];
          } else if (k == 0) {            // from the preceding exit to this entry
            x0 = L.ix[x]; y0 = L.iy[x]; x1 = L.ix[e]; y1 = L.iy[e];
          } else {                        // from this entry on
            x0 = L.ix[e]; y0 = L.iy[e]; x1 = L.px[f]; y1 = L.py[f];
          }
          lane_segment(L, a, ty, H, x0, y0, x1, y1);
        }
      }
      // low-pass support: square of half-width s_l sqrt(2 ln(o / alpha_min)) around the projected centre
      if (opt.lowpass_sl > 0.0f) {
        const double dcx = L.lp[it][0], dcy = L.lp[it][1], r = L.lp[it][2];
        if (lane == 0) {
          a.bx0 = fmin(a.bx0, dcx - r);
          a.bx1 = fmax(a.bx1, dcx + r);
          a.by0 = fmin(a.by0, dcy - r);
          a.by1 = fmax(a.by1, dcy + r);
        }
        for (int row = lane; row < ty; row += 64) {
          const double ya = 16.0 * row + 0.5;
          const double yb = fmin(16.0 * row + 15.5, H - 0.5);
          if (dcy + r >= ya && dcy - r <= yb) {
            a.r0 = min(a.r0, row);
            a.r1 = max(a.r1, row);
            const double xl = dcx - r, xh = dcx + r;
            if (xl == xl) atomicMin(&L.lo[row], ord_enc(xl));
            if (xh == xh) atomicMax(&L.hi[row], ord_enc(xh));
          }
        }
      }
      // the lanes' boxes and row ranges meet in LDS (a lane with no segment holds the neutral values;
      // its box is never NaN: fmin / fmax above drop NaN operands)
      if (a.r0 <= a.r1) {
        atomicMin(&L.rows[0], a.r0);
        atomicMin(&L.rows[1], -a.r1);
      }
      if (a.bx0 <= a.bx1 || a.by0 <= a.by1) {
        atomicMin(&L.box[0], ord_enc(a.bx0));
        atomicMin(&L.box[1], ord_enc(-a.bx1));
        atomicMin(&L.box[2], ord_enc(a.by0));
        atomicMin(&L.box[3], ord_enc(-a.by1));
      }
      wave_sync();
      const int r0 = L.rows[0], r1 = -L.rows[1];
      // tile columns of each touched row (row_tiles), the count, and the rows reset for the next item
      constexpr int kRowIters = (kMaxTileRows + 63) / 64;
      uint32_t ent[kRowIters];
      uint32_t cnt = 0;
#pragma unroll
      for (int c = 0; c < kRowIters; ++c) {
        const int r = r0 + c * 64 + lane;
        ent[c] = 0xFFFFFFFFu;
        if (r <= r1) {
          const double lo = fmax(ord_dec(L.lo[r]), 0.5);
          const double hi = fmin(ord_dec(L.hi[r]), W - 0.5);
          L.lo[r] = kEncPosInf;
          L.hi[r] = kEncNegInf;
          if (!(lo > hi)) {
            const double ca = ceil((lo - 15.5) / 16.0);
            const double cb = floor((hi - 0.5) / 16.0);
            const int i0 = ca < 0.0 ? 0 : (int)ca;
            const int i1 = cb > (double)(tx - 1) ? tx - 1 : (int)cb;
            if (i0 <= i1) {
              cnt += (uint32_t)(i1 - i0 + 1);
              ent[c] = (uint32_t)i0 | ((uint32_t)i1 << 16);
            }
          }
        }
      }
      if (cnt) atomicAdd(&L.cnt, cnt);
      wave_sync();
      cnt = L.cnt;
      const double bx0 = ord_dec(L.box[0]), bx1 = -ord_dec(L.box[1]);
      const double by0 = ord_dec(L.box[2]), by1 = -ord_dec(L.box[3]);
      wave_sync();
      if (lane < 4) L.box[lane] = kEncPosInf;
      if (lane < 2) L.rows[lane] = kMaxTileRows;
      if (lane == 0) L.cnt = 0;
      if (cnt == 0) {
        if (lane == 0) {
          tile_counts[o] = 0;
          depth_keys[o] = kCulledKey;
        }
        continue;
      }
      const uint32_t nrows = (uint32_t)(r1 - r0 + 1);
      // a fixed slot by list position when it holds the rows, else a pool
      const int64_t pos = first + it;
      const int64_t slot = pos < nbig ? stride - 1 - pos : pos - nbig;   // small-list positions as they are
      int64_t at;
      bool fits;
      if (nrows <= (uint32_t)kFixedRows && rl.fixed && (pos >= nbig || slot >= n_small_all)) {
        at = slot * kFixedRows;
        fits = true;
      } else {
        uint32_t off = 0;
        if (lane == 0) off = atomicAdd(pool_used + (int64_t)v * kSpanPools + pool, nrows);
        off = (uint32_t)__builtin_amdgcn_readlane((int)off, 0);
        at = rl.pool_base + (int64_t)pool * rl.pool_rows + off;
        fits = (int64_t)off + nrows <= rl.pool_rows;
      }
      fits = fits && at + nrows < (int64_t)kNoSpans;   // offsets are stored in 32 bits
      if (fits) {
        uint32_t* out = span_rows + (int64_t)v * row_cap + at;
#pragma unroll
        for (int c = 0; c < kRowIters; ++c) {
          const int r = r0 + c * 64 + lane;
          if (r <= r1) out[r - r0] = ent[c];
        }
      }
      if (lane == 0) {
        tile_counts[o] = cnt;
        uint2 meta;
        meta.x = fits ? (uint32_t)at : kNoSpans;
        meta.y = fits ? ((uint32_t)r0 | (nrows << 16)) : 0u;
        span_meta[o] = meta;
        // only the conservative polygon bounds the support
        const double box[4] = {opt.cull_mode == 0 ? bx0 : -1e30, opt.cull_mode == 0 ? bx1 : 1e30,
                               opt.cull_mode == 0 ? by0 : -1e30, opt.cull_mode == 0 ? by1 : 1e30};
        float* rec = records + o * rec_floats(K);
        rec[R_BOX + 0] = (float)(box[0] - 0.01);
        rec[R_BOX + 1] = (float)(box[1] + 0.01);
        rec[R_BOX + 2] = (float)(box[2] - 0.01);
        rec[R_BOX + 3] = (float)(box[3] + 0.01);
        if (opt.key_mode != 0) {
          double* kg = keygeo + o * KG_N;
          for (int i = 0; i < 4; ++i) kg[KG_BOX + i] = box[i];
        }
      }
    }
  }
}

// Pass 3, one thread per listed primitive with tiles: the rest of its render record.  A thread's
// record fields are written one float at a time, so the wave's records are built in LDS and then
// copied out as float4 rows (each record's 16-byte groups side by side), except the group that
// holds the box (written by k_polygon).
constexpr int kRecWave = 64;
static_assert(R_BOX % 4 == 0, "the box is one float4 group of the record");

__global__ void __launch_bounds__(kRecWave) k_record(SceneDev sc, const Views* __restrict__ views, OptsDev opt,
                                                     float* __restrict__ records,
                                                     const uint32_t* __restrict__ tile_counts,
                                                     const uint32_t* __restrict__ work_small,
                                                     const uint32_t* __restrict__ count_small,
                                                     const uint32_t* __restrict__ work_big,
                                                     const uint32_t* __restrict__ count_big, int64_t stride,
                                                     double* __restrict__ keygeo) {
  extern __shared__ float4 s_rec[];   // kRecWave records of rec_floats(K) floats
  const int lane = threadIdx.x;
  const int v = blockIdx.y;
  const int64_t ns = (int64_t)count_small[v], total = ns + (int64_t)count_big[v];
  const int RF = rec_floats(sc.K), RF4 = RF / 4;
  const CamDev& cam = views->cam[v];
  // positions [0, ns) of the small list, then those of the big list
  const int64_t first = (int64_t)blockIdx.x * kRecWave;
  if (first >= total) return;
  {
    const int64_t i = first + lane;
    int64_t o = -1;
    if (i < total) {
      const uint32_t jj = i < ns ? work_small[(int64_t)v * stride + i] : work_big[(int64_t)v * stride + (i - ns)];
      if (jj != kNoItem && tile_counts[(int64_t)v * stride + jj] != 0) {
        const int64_t j = (int64_t)jj;
        GeoBase g;
        bool invalid;
        if (load_geo_core<double>(sc, j, cam, opt, g, &invalid, nullptr, nullptr)) {
          o = (int64_t)v * stride + j;
          write_record(g, sc, j, cam, opt, reinterpret_cast<float*>(s_rec + lane * RF4),
                       opt.key_mode != 0 ? keygeo + o * KG_N : nullptr);
        }
      }
    }
    const uint64_t has = __ballot(o >= 0);
    __syncthreads();
    for (int q = lane; q < kRecWave * RF4; q += kRecWave) {   // the same trip count in every lane
      const int r = q / RF4, c = q - r * RF4;
      const int64_t orow = __shfl(o, r, 64);
      if (((has >> r) & 1ull) && c != R_BOX / 4) reinterpret_cast<float4*>(records + orow * RF)[c] = s_rec[q];
    }
  }
}

// ---------------------------------------------------------------------------------------------
// Per-tile pre-sort keys (supplement, cache-sorting evaluation), float64 in the order written.
// View depth where the ray through pixel point (x, y) meets the plane; false when it meets it at
// or behind the near plane (or not at all).
__device__ inline bool plane_depth(const double* kg, const CamDev& cam, double nearp, double x, double y, double& z) {
  const double wd = (kg[KG_A] * ((x - (double)cam.cx) / (double)cam.fx) +
                     kg[KG_A + 1] * ((y - (double)cam.cy) / (double)cam.fy)) + kg[KG_A + 2];
  if (wd == 0.0) return false;
  z = kg[KG_DN] / wd;
  return z > nearp && z < INFINITY;
}

// float32 bits of the key of the primitive with key data kg in tile `tile` (key_mode 1: depth on
// the ray through the centre of the tile's pixel-centre rectangle cut to the support box; 2: the
// smallest depth over that rectangle's corner rays), held to [zlo, zhi].
__device__ inline uint32_t tile_key(const double* kg, const CamDev& cam, const OptsDev& opt, uint32_t tile) {
  const int tx = (int)(tile % (uint32_t)cam.tiles_x), ty = (int)(tile / (uint32_t)cam.tiles_x);
  double xa = 16.0 * tx + 0.5, xb = fmin(16.0 * tx + 15.5, cam.W - 0.5);
  double ya = 16.0 * ty + 0.5, yb = fmin(16.0 * ty + 15.5, cam.H - 0.5);
  const double x0 = fmax(xa, kg[KG_BOX + 0]), x1 = fmin(xb, kg[KG_BOX + 1]);
  const double y0 = fmax(ya, kg[KG_BOX + 2]), y1 = fmin(yb, kg[KG_BOX + 3]);
  if (!(x0 > x1) && !(y0 > y1)) { xa = x0; xb = x1; ya = y0; yb = y1; }
  const double nearp = (double)opt.near_plane;
  double z;
  if (opt.key_mode == 1) {
    if (!plane_depth(kg, cam, nearp, 0.5 * (xa + xb), 0.5 * (ya + yb), z)) z = kg[KG_ZC];
  } else {
    z = INFINITY;
    double d;
    if (plane_depth(kg, cam, nearp, xa, ya, d)) z = fmin(z, d);
    if (plane_depth(kg, cam, nearp, xb, ya, d)) z = fmin(z, d);
    if (plane_depth(kg, cam, nearp, xa, yb, d)) z = fmin(z, d);
    if (plane_depth(kg, cam, nearp, xb, yb, d)) z = fmin(z, d);
    if (z == INFINITY) z = kg[KG_ZLO];
  }
  return __float_as_uint((float)fmin(fmax(z, kg[KG_ZLO]), kg[KG_ZHI]));
}

// ---------------------------------------------------------------------------------------------
// Duplication: for the given primitive order (depth-sorted, or index order with per-tile keys),
// write (tile id, primitive) pairs at the scanned offsets, row-major over each primitive's tiles,
// from the stored row spans (recomputed with the same float64 code when they did not fit the row
// buffer), and with key_mode 1 or 2 each pair's key.
__global__ void __launch_bounds__(128) k_duplicate(SceneDev sc, const Views* __restrict__ views, OptsDev opt, int v,
                                                   const uint32_t* __restrict__ sorted_prims,
                                                   const uint32_t* __restrict__ offsets,   // exclusive, per sorted slot
                                                   const uint32_t* __restrict__ tile_counts,
                                                   const uint2* __restrict__ span_meta,
                                                   const uint32_t* __restrict__ span_rows,
                                                   uint32_t* __restrict__ pair_tiles, uint32_t* __restrict__ pair_prims,
                                                   const uint64_t* __restrict__ total_ptr, int64_t capacity,
                                                   const uint64_t* __restrict__ n_sorted,
                                                   uint32_t* __restrict__ big_list, int64_t list_len,
                                                   uint32_t* __restrict__ big_count,
                                                   const double* __restrict__ keygeo, uint32_t* __restrict__ pair_keys) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)*n_sorted) return;
  const uint32_t j = sorted_prims[i];
  const uint32_t cnt = tile_counts[j];
  if (cnt == 0) return;
  if ((int64_t)*total_ptr > capacity) return;   // overflow: the status word already says so
  const uint32_t off = offsets[i];
  const CamDev& cam = views->cam[v];
  const uint2 meta = opt.cull_mode == 2 ? make_uint2(0u, 0u) : span_meta[j];
  if (opt.cull_mode != 2 && meta.x == kNoSpans) {
    // spans not stored (row buffer full): re-derived by k_duplicate_rebuild, listed from the end
    big_list[list_len - 1 - atomicAdd(big_count + 1, 1u)] = (uint32_t)i;
    return;
  }
  if (cnt > kDupSmall) {
    big_list[atomicAdd(big_count, 1u)] = (uint32_t)i;   // written by k_duplicate_big
    return;
  }
  const double* kg = pair_keys ? keygeo + (int64_t)j * KG_N : nullptr;
  if (opt.cull_mode == 2) {
    for (uint32_t t = 0; t < cnt; ++t) {
      pair_tiles[off + t] = t;
      pair_prims[off + t] = j;
      if (kg) pair_keys[off + t] = tile_key(kg, cam, opt, t);
    }
    return;
  }
  uint32_t w = 0;
  const int r0 = (int)(meta.y & 0xFFFFu), nr = (int)(meta.y >> 16);
  const uint32_t* rows = span_rows + meta.x;
  for (int r = 0; r < nr && w < cnt; ++r) {
    const uint32_t e = rows[r];
    if (e == 0xFFFFFFFFu) continue;
    const int i0 = (int)(e & 0xFFFFu), i1 = (int)(e >> 16);
    const uint32_t base = (uint32_t)((r0 + r) * cam.tiles_x);
    for (int c = i0; c <= i1 && w < cnt; ++c, ++w) {
      pair_tiles[off + w] = base + (uint32_t)c;
      pair_prims[off + w] = j;
      if (kg) pair_keys[off + w] = tile_key(kg, cam, opt, base + (uint32_t)c);
    }
  }
}

// Duplication of the primitives whose row spans did not fit the row buffer: rebuilt from the scene
// (the same polygon and spans as k_polygon), one thread per primitive.  Kept apart from
// k_duplicate so that the common path does not carry this code's registers and private arrays.
__global__ void __launch_bounds__(128) k_duplicate_rebuild(SceneDev sc, const Views* __restrict__ views, OptsDev opt,
                                                           int v, const uint32_t* __restrict__ sorted_prims,
                                                           const uint32_t* __restrict__ offsets,
                                                           const uint32_t* __restrict__ tile_counts,
                                                           uint32_t* __restrict__ pair_tiles,
                                                           uint32_t* __restrict__ pair_prims,
                                                           const uint64_t* __restrict__ total_ptr, int64_t capacity,
                                                           const uint32_t* __restrict__ list, int64_t list_len,
                                                           const uint32_t* __restrict__ list_count,
                                                           const double* __restrict__ keygeo,
                                                           uint32_t* __restrict__ pair_keys) {
  if ((int64_t)*total_ptr > capacity) return;
  const uint32_t nreb = list_count[1];
  const CamDev& cam = views->cam[v];
  for (uint32_t item = blockIdx.x * blockDim.x + threadIdx.x; item < nreb; item += gridDim.x * blockDim.x) {
    const uint32_t i = list[list_len - 1 - item];
    const uint32_t j = sorted_prims[i];
    const uint32_t cnt = tile_counts[j];
    const uint32_t off = offsets[i];
    const double* kg = pair_keys ? keygeo + (int64_t)j * KG_N : nullptr;
    Geo g;
    bool invalid;
    if (!load_geo(sc, j, cam, opt, g, &invalid)) continue;
    Spans sp;
    build_spans(g, GeoBases{g}, cam, opt, sp);
    uint32_t w = 0;
    for (int r = sp.r0; r <= sp.r1 && w < cnt; ++r) {
      int i0, i1;
      if (!row_tiles(sp, r, i0, i1)) continue;
      for (int c = i0; c <= i1 && w < cnt; ++c, ++w) {
        pair_tiles[off + w] = (uint32_t)(r * cam.tiles_x + c);
        pair_prims[off + w] = j;
        if (kg) pair_keys[off + w] = tile_key(kg, cam, opt, (uint32_t)(r * cam.tiles_x + c));
      }
    }
  }
}

// Duplication of the primitives with more than kDupSmall tiles: one workgroup per primitive.  The
// lanes load the primitive's stored row entries, an exclusive scan of the rows' tile counts gives
// each row's first output slot, and the lanes then write all the primitive's pairs side by side
// (slot p belongs to the last row whose first slot is <= p), in the same order as a row-by-row walk.
constexpr int kDupBigBlock = 256;
static_assert(kMaxTileRows <= kDupBigBlock, "one lane per stored tile row");

__global__ void __launch_bounds__(kDupBigBlock) k_duplicate_big(const Views* __restrict__ views, OptsDev opt, int v,
                                                       const uint32_t* __restrict__ sorted_prims,
                                                       const uint32_t* __restrict__ offsets,
                                                       const uint32_t* __restrict__ tile_counts,
                                                       const uint2* __restrict__ span_meta,
                                                       const uint32_t* __restrict__ span_rows,
                                                       uint32_t* __restrict__ pair_tiles, uint32_t* __restrict__ pair_prims,
                                                       const uint64_t* __restrict__ total_ptr, int64_t capacity,
                                                       const uint32_t* __restrict__ big_list,
                                                       const uint32_t* __restrict__ big_count,
                                                       const double* __restrict__ keygeo,
                                                       uint32_t* __restrict__ pair_keys) {
  __shared__ uint32_t s_first[kDupBigBlock + 1];   // exclusive scan of the rows' tile counts
  __shared__ uint32_t s_tile0[kDupBigBlock];       // first tile id of each row
  __shared__ uint32_t s_wave[kDupBigBlock / 64];
  if ((int64_t)*total_ptr > capacity) return;
  const uint32_t nbig = *big_count;
  const CamDev& cam = views->cam[v];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  for (uint32_t item = blockIdx.x; item < nbig; item += gridDim.x) {
    const uint32_t i = big_list[item];
    const uint32_t j = sorted_prims[i];
    const uint32_t cnt = tile_counts[j];
    const uint32_t off = offsets[i];
    const double* kg = pair_keys ? keygeo + (int64_t)j * KG_N : nullptr;
    if (opt.cull_mode == 2) {
      for (uint32_t t = tid; t < cnt; t += kDupBigBlock) {
        pair_tiles[off + t] = t;
        pair_prims[off + t] = j;
        if (kg) pair_keys[off + t] = tile_key(kg, cam, opt, t);
      }
      continue;
    }
    const uint2 meta = span_meta[j];
    const int r0 = (int)(meta.y & 0xFFFFu), nr = (int)(meta.y >> 16);
    uint32_t n_row = 0;
    if (tid < nr) {
      const uint32_t e = span_rows[meta.x + tid];
      if (e != 0xFFFFFFFFu) {
        const uint32_t i0 = e & 0xFFFFu, i1 = e >> 16;
        n_row = i1 - i0 + 1u;
        s_tile0[tid] = (uint32_t)((r0 + tid) * cam.tiles_x) + i0;
      }
    }
    // inclusive scan within each wave, then across the four waves
    uint32_t x = n_row;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t y = __shfl_up(x, o, 64);
      if (lane >= o) x += y;
    }
    if (lane == 63) s_wave[wv] = x;
    __syncthreads();
    uint32_t add = 0;
    for (int w = 0; w < wv; ++w) add += s_wave[w];
    s_first[tid + 1] = x + add;
    if (tid == 0) s_first[0] = 0;
    __syncthreads();
    const uint32_t total = min(s_first[nr], cnt);
    for (uint32_t p = tid; p < total; p += kDupBigBlock) {
      int lo = 0, hi = nr - 1;   // last row r with s_first[r] <= p (a non-empty row, as p < s_first[nr])
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (s_first[mid] <= p) lo = mid; else hi = mid - 1;
      }
      const uint32_t tile = s_tile0[lo] + (p - s_first[lo]);
      pair_tiles[off + p] = tile;
      pair_prims[off + p] = j;
      if (kg) pair_keys[off + p] = tile_key(kg, cam, opt, tile);
    }
    __syncthreads();   // the next primitive reuses the shared arrays
  }
}

// Pre-sort key of each sorted pair (inspection): the centre-depth key of its primitive, or the
// per-tile key recomputed from the key data.
__global__ void __launch_bounds__(256) k_pair_keys(const Views* __restrict__ views, OptsDev opt, int v,
                                                   const uint32_t* __restrict__ tiles, const uint32_t* __restrict__ prims,
                                                   int64_t n, const uint32_t* __restrict__ depth_keys,
                                                   const double* __restrict__ keygeo, uint32_t* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t j = prims[i];
  out[i] = opt.key_mode == 0 ? depth_keys[j] : tile_key(keygeo + (int64_t)j * KG_N, views->cam[v], opt, tiles[i]);
}

}  // namespace drk

// Host launchers ------------------------------------------------------------------------------
namespace drk {

__global__ void k_set_views(Views* dst, Views src) { *dst = src; }

hipError_t set_views(Views* d_views, const Views& views, hipStream_t s) {
  hipLaunchKernelGGL(k_set_views, dim3(1), dim3(1), 0, s, d_views, views);
  return hipGetLastError();
}

// work_small / work_big: per view [view][stride] lists; counts: per view; pool_used: kSpanPools
// counters per view.  The counts and pool counters must be zero.
hipError_t launch_preprocess(const SceneDev& sc, const Views* views, int nv, const OptsDev& opt, float* records,
                             uint32_t* depth_keys, uint32_t* tile_counts, uint32_t* work_small, uint32_t* count_small,
                             uint32_t* work_big, uint32_t* count_big, uint2* span_meta, uint32_t* span_rows,
                             uint32_t* pool_used, int64_t row_cap, uint32_t* status, int64_t stride, double* keygeo,
                             hipStream_t s) {
  if (sc.n == 0) return hipSuccess;
  dim3 grid((unsigned)((sc.n + 127) / 128), (unsigned)nv);
  dim3 grid_pre((unsigned)((sc.n + kPreBlock - 1) / kPreBlock * nv));
  hipLaunchKernelGGL(k_preprocess, grid_pre, dim3(kPreBlock), 0, s, sc, views, opt, depth_keys, tile_counts,
                     work_small, count_small, work_big, count_big, status, stride, nv);
  hipLaunchKernelGGL(k_polygon_small, grid, dim3(128), 0, s, sc, views, opt, records, depth_keys, tile_counts,
                     work_small, count_small, work_big, count_big, span_meta, span_rows, pool_used, row_cap, stride,
                     keygeo);
  const int64_t batches = (sc.n + kPolyBatch - 1) / kPolyBatch;
  dim3 grid_poly((unsigned)std::min<int64_t>((batches + kPolyWaves - 1) / kPolyWaves, 2048), (unsigned)nv);
  hipLaunchKernelGGL(k_polygon, grid_poly, dim3(64 * kPolyWaves), 0, s, sc, views, opt, records, depth_keys,
                     tile_counts, work_small, count_small, work_big, count_big, span_meta, span_rows, pool_used,
                     row_cap, stride, keygeo);
  // the two lists hold at most 2 n entries (an entry that moved to the big list stays in the small
  // one as kNoItem)
  dim3 grid_rec((unsigned)((2 * sc.n + kRecWave - 1) / kRecWave), (unsigned)nv);
  const size_t rec_lds = (size_t)kRecWave * rec_floats(sc.K) * sizeof(float);
  hipLaunchKernelGGL(k_record, grid_rec, dim3(kRecWave), rec_lds, s, sc, views, opt, records, tile_counts, work_small,
                     count_small, work_big, count_big, stride, keygeo);
  return hipGetLastError();
}

hipError_t fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t s);

hipError_t launch_duplicate(const SceneDev& sc, const Views* views, const OptsDev& opt, int v,
                            const uint32_t* sorted_prims, const uint32_t* offsets, const uint32_t* tile_counts,
                            const uint2* span_meta, const uint32_t* span_rows, uint32_t* pair_tiles,
                            uint32_t* pair_prims, const uint64_t* total_ptr, int64_t capacity, const uint64_t* n_sorted,
                            uint32_t* big_list, uint32_t* big_count, const double* keygeo, uint32_t* pair_keys,
                            hipStream_t s) {
  if (sc.n == 0) return hipSuccess;
  // big_list holds sc.n entries: big primitives from the front (count big_count[0]) and primitives
  // to rebuild from the back (count big_count[1]); together at most the sorted count <= sc.n
  hipError_t e = fill_u32(big_count, 0u, 2, s);
  if (e != hipSuccess) return e;
  dim3 grid((unsigned)((sc.n + 127) / 128));
  hipLaunchKernelGGL(k_duplicate, grid, dim3(128), 0, s, sc, views, opt, v, sorted_prims, offsets, tile_counts,
                     span_meta, span_rows, pair_tiles, pair_prims, total_ptr, capacity, n_sorted, big_list, sc.n,
                     big_count, keygeo, pair_keys);
  hipLaunchKernelGGL(k_duplicate_big, dim3(4096), dim3(kDupBigBlock), 0, s, views, opt, v, sorted_prims, offsets,
                     tile_counts, span_meta, span_rows, pair_tiles, pair_prims, total_ptr, capacity, big_list, big_count,
                     keygeo, pair_keys);
  hipLaunchKernelGGL(k_duplicate_rebuild, dim3(512), dim3(128), 0, s, sc, views, opt, v, sorted_prims, offsets,
                     tile_counts, pair_tiles, pair_prims, total_ptr, capacity, big_list, sc.n, big_count, keygeo,
                     pair_keys);
  return hipGetLastError();
}

hipError_t launch_pair_keys(const Views* views, const OptsDev& opt, int v, const uint32_t* tiles, const uint32_t* prims,
                            int64_t n, const uint32_t* depth_keys, const double* keygeo, uint32_t* out, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_pair_keys, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, views, opt, v, tiles, prims, n,
                     depth_keys, keygeo, out);
  return hipGetLastError();
}

}  // namespace drk
