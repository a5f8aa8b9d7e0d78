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

namespace drk {

constexpr double kPi = 3.141592653589793;
constexpr double kTwoPi = 2.0 * kPi;

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
// Per-primitive geometry in float64.
struct Geo {
  double tu[3], tv[3];      // world tangent axes (columns of R(q))
  double mu[3];
  double muc[3];            // camera-frame centre
  double o, tau;
  double c;                 // calibrated radius: {E <= c^2} == {o Psi(g) >= alpha_min}
  double s[kMaxK], th[kMaxK];
  int K;
};

// Loads and validates primitive j.  Returns false when it can never contribute.
__device__ inline bool load_geo(const SceneDev& sc, int64_t j, const CamDev& cam, const OptsDev& opt, Geo& g,
                                bool* invalid) {
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
  for (int k = 0; k < K; ++k) {
    g.s[k] = (double)sc.scale[k * n + j];
    g.th[k] = (double)sc.theta[k * n + j];
    bad |= !(g.s[k] > 0.0) || !isfinite(g.s[k]);
    bad |= !(g.th[k] >= 0.0) || !(g.th[k] < kTwoPi);
  }
  for (int k = 0; k < K; ++k) {
    double nxt = (k + 1 < K) ? g.th[k + 1] : g.th[0] + kTwoPi;
    double gap = nxt - g.th[k];
    bad |= !(gap > 0.0) || !(gap < kPi);
  }
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

// Inverse L2 scale 1/sbar along absolute angle a inside the sector [thk, thn] (Sec. 4.1).
__device__ inline double sbar_at(double a, double thk, double thn, double sk, double sn) {
  double dl = (kPi * (a - thk)) / (thn - thk);
  double w = (1.0 + cos(dl)) / ((2.0 * sk) * sk) + (1.0 - cos(dl)) / ((2.0 * sn) * sn);
  return 1.0 / sqrt(w);
}
// Distance from the centre to the segment e_k e_{k+1} along absolute angle a (Sec. 4.2 level set).
__device__ inline double chord_at(double a, double thk, double thn, double sk, double sn) {
  double phi = a - thk;
  double dlt = thn - thk;
  double f = (sin(dlt - phi) / sk + sin(phi) / sn) / sin(dlt);
  return 1.0 / f;
}

// ---------------------------------------------------------------------------------------------
// Tile-row spans of the projected support.  Edges of the near-clipped projected polygon are
// streamed in order; each updates the x-extent of the tile rows whose pixel-centre slab it crosses.
struct Spans {
  double lo[kMaxTileRows], hi[kMaxTileRows];
  int r0, r1;                       // initialised rows [r0, r1]
  int W, H, tx, ty;
  // near-plane clipping state (Sutherland-Hodgman order)
  bool have_prev, prev_in, have_first;
  double prev[3], first[3];
  bool pending_exit, have_first_entry;
  double exit_pt[3], first_entry[3];
};

__device__ inline void spans_init(Spans& sp, const CamDev& cam) {
  sp.r0 = 1; sp.r1 = 0;
  sp.W = cam.W; sp.H = cam.H; sp.tx = cam.tiles_x; sp.ty = cam.tiles_y;
  sp.have_prev = false; sp.have_first = false; sp.pending_exit = false; sp.have_first_entry = false;
}

__device__ inline void spans_touch(Spans& sp, int r) {
  if (sp.r0 > sp.r1) { sp.r0 = sp.r1 = r; sp.lo[r] = INFINITY; sp.hi[r] = -INFINITY; return; }
  while (r < sp.r0) { --sp.r0; sp.lo[sp.r0] = INFINITY; sp.hi[sp.r0] = -INFINITY; }
  while (r > sp.r1) { ++sp.r1; sp.lo[sp.r1] = INFINITY; sp.hi[sp.r1] = -INFINITY; }
}

// Screen segment (x0,y0)-(x1,y1) against every tile row slab it may cross.
__device__ inline void spans_segment(Spans& sp, double x0, double y0, double x1, double y1) {
  double ymin = fmin(y0, y1), ymax = fmax(y0, y1);
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
    spans_touch(sp, r);
    sp.lo[r] = fmin(sp.lo[r], fmin(xa, xb));
    sp.hi[r] = fmax(sp.hi[r], fmax(xa, xb));
  }
}

__device__ inline void project(const CamDev& cam, const double p[3], double& x, double& y) {
  x = ((double)cam.fx * p[0]) / p[2] + (double)cam.cx;
  y = ((double)cam.fy * p[1]) / p[2] + (double)cam.cy;
}

__device__ inline void spans_edge3(Spans& sp, const CamDev& cam, const double a[3], const double b[3]) {
  double x0, y0, x1, y1;
  project(cam, a, x0, y0);
  project(cam, b, x1, y1);
  spans_segment(sp, x0, y0, x1, y1);
}

// Camera-space polygon vertex stream, clipped to z >= near in Sutherland-Hodgman order.
__device__ inline void clip_edge(Spans& sp, const CamDev& cam, double nearp, const double a[3], const double b[3]) {
  bool ain = a[2] >= nearp, bin = b[2] >= nearp;
  double I[3];
  if (ain != bin) {
    double t = (nearp - a[2]) / (b[2] - a[2]);
    for (int i = 0; i < 3; ++i) I[i] = a[i] + t * (b[i] - a[i]);
  }
  if (ain && bin) {
    spans_edge3(sp, cam, a, b);
  } else if (ain && !bin) {            // exit
    spans_edge3(sp, cam, a, I);
    sp.pending_exit = true;
    for (int i = 0; i < 3; ++i) sp.exit_pt[i] = I[i];
  } else if (!ain && bin) {            // entry
    if (sp.pending_exit) {
      spans_edge3(sp, cam, sp.exit_pt, I);
      sp.pending_exit = false;
    } else if (!sp.have_first_entry) {
      sp.have_first_entry = true;
      for (int i = 0; i < 3; ++i) sp.first_entry[i] = I[i];
    }
    spans_edge3(sp, cam, I, b);
  }
}

__device__ inline void push_vertex(Spans& sp, const CamDev& cam, double nearp, const double p[3]) {
  if (!sp.have_first) {
    sp.have_first = true;
    for (int i = 0; i < 3; ++i) sp.first[i] = p[i];
  } else {
    clip_edge(sp, cam, nearp, sp.prev, p);
  }
  for (int i = 0; i < 3; ++i) sp.prev[i] = p[i];
}

__device__ inline void close_polygon(Spans& sp, const CamDev& cam, double nearp) {
  if (sp.have_first) clip_edge(sp, cam, nearp, sp.prev, sp.first);
  if (sp.pending_exit && sp.have_first_entry) spans_edge3(sp, cam, sp.exit_pt, sp.first_entry);
}

// tangent-plane (x, y) -> camera frame
__device__ inline void lift(const Geo& g, const CamDev& cam, double x, double y, double out[3]) {
  double w[3];
  for (int i = 0; i < 3; ++i) w[i] = (g.mu[i] + x * g.tu[i]) + y * g.tv[i];
  to_cam(cam, w, out);
}

// Builds the tile-row spans of primitive g (cull_mode 0: conservative support polygon;
// 1: the paper's endpoint polygon; 2 handled by the caller).
__device__ void build_spans(const Geo& g, const CamDev& cam, const OptsDev& opt, Spans& sp) {
  spans_init(sp, cam);
  const double nearp = (double)opt.near_plane;
  const int K = g.K;
  if (opt.cull_mode == 1) {
    double y = exp(-9.0) / g.o;
    double gm = psi_inv(y < 1.0 ? y : 1.0, g.tau);
    double ml = -log(gm);
    double f = sqrt(ml > 0.0 ? ml : 0.0);
    for (int k = 0; k < K; ++k) {
      double sc = g.s[k] * f;
      double p[3];
      lift(g, cam, sc * cos(g.th[k]), sc * sin(g.th[k]), p);
      push_vertex(sp, cam, nearp, p);
    }
  } else {
    // Support polygon: E is a convex combination of r1^2 and r2^2/sbar^2, so the support lies
    // within radius c * max(sbar, chord) along each direction; both are maximal at sub-arc ends.
    for (int k = 0; k < K; ++k) {
      double thk = g.th[k];
      double thn = (k + 1 < K) ? g.th[k + 1] : g.th[0] + kTwoPi;
      double sk = g.s[k], sn = g.s[(k + 1) % K];
      for (int j = 0; j < kSubArcs; ++j) {
        double a = thk + ((thn - thk) * j) / kSubArcs;
        double b = thk + ((thn - thk) * (j + 1)) / kSubArcs;
        double h = 0.5 * (b - a);
        double mid = a + h;
        double rho = fmax(fmax(sbar_at(a, thk, thn, sk, sn), sbar_at(b, thk, thn, sk, sn)),
                          fmax(chord_at(a, thk, thn, sk, sn), chord_at(b, thk, thn, sk, sn)));
        rho = g.c * rho;
        double rm = rho / cos(h);
        double p[3];
        lift(g, cam, rho * cos(a), rho * sin(a), p);
        push_vertex(sp, cam, nearp, p);
        lift(g, cam, rm * cos(mid), rm * sin(mid), p);
        push_vertex(sp, cam, nearp, p);
        lift(g, cam, rho * cos(b), rho * sin(b), p);
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
    for (int row = 0; row < sp.ty; ++row) {
      double ya = 16.0 * row + 0.5;
      double yb = fmin(16.0 * row + 15.5, sp.H - 0.5);
      if (dcy + r >= ya && dcy - r <= yb) {
        spans_touch(sp, row);
        sp.lo[row] = fmin(sp.lo[row], dcx - r);
        sp.hi[row] = fmax(sp.hi[row], dcx + r);
      }
    }
  }
}

// Tile columns [i0, i1] of row r (false when none).
__device__ inline bool row_tiles(const Spans& sp, int r, int& i0, int& i1) {
  double lo = fmax(sp.lo[r], 0.5);
  double hi = fmin(sp.hi[r], sp.W - 0.5);
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
// Preprocess: one thread per (primitive, view).
__global__ void __launch_bounds__(128) k_preprocess(SceneDev sc, const Views* __restrict__ views, OptsDev opt, float* __restrict__ records,
                                                    uint32_t* __restrict__ depth_keys,
                                                    uint32_t* __restrict__ tile_counts,
                                                    uint32_t* __restrict__ status, int64_t stride) {
  // per-view arrays are [view][stride] (stride = workspace capacity in primitives)
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int v = blockIdx.y;
  if (j >= sc.n) return;
  const CamDev& cam = views->cam[v];
  const int64_t n = sc.n;
  const int K = sc.K;
  const int RF = rec_floats(K);
  Geo g;
  bool invalid = false;
  bool alive = load_geo(sc, j, cam, opt, g, &invalid);
  if (invalid && opt.validate) atomicOr(status + v, (uint32_t)ST_INVALID);
  uint32_t count = 0;
  if (alive) {
    if (opt.cull_mode == 2) {
      count = (uint32_t)(cam.tiles_x * cam.tiles_y);
    } else {
      Spans sp;
      build_spans(g, cam, opt, sp);
      for (int r = sp.r0; r <= sp.r1; ++r) {
        int i0, i1;
        if (row_tiles(sp, r, i0, i1)) count += (uint32_t)(i1 - i0 + 1);
      }
    }
  }
  // centre depth key: float32 of ((r20 x + r21 y) + r22 z) + t2 computed in float64
  depth_keys[(int64_t)v * stride + j] = (alive && count) ? __float_as_uint((float)g.muc[2]) : kCulledKey;
  tile_counts[(int64_t)v * stride + j] = count;
  if (!alive || count == 0) return;

  float* rec = records + ((int64_t)v * stride + j) * RF;
  // homography (see RecField): adjugate rows of N = [t_u^c | t_v^c | mu_c]
  double tuc[3], tvc[3];
  rot_cam(cam, g.tu, tuc);
  rot_cam(cam, g.tv, tvc);
  const double* m = g.muc;
  double a0[3] = {tvc[1] * m[2] - tvc[2] * m[1], tvc[2] * m[0] - tvc[0] * m[2], tvc[0] * m[1] - tvc[1] * m[0]};
  double a1[3] = {m[1] * tuc[2] - m[2] * tuc[1], m[2] * tuc[0] - m[0] * tuc[2], m[0] * tuc[1] - m[1] * tuc[0]};
  double a2[3] = {tuc[1] * tvc[2] - tuc[2] * tvc[1], tuc[2] * tvc[0] - tuc[0] * tvc[2],
                  tuc[0] * tvc[1] - tuc[1] * tvc[0]};
  double dN = a2[0] * m[0] + a2[1] * m[1] + a2[2] * m[2];
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
  // colour
  if (sc.color_mode == 0) {
    for (int c = 0; c < 3; ++c) rec[R_RGB + c] = sc.color[c * n + j];
  } else {
    double cp[3];
    for (int i = 0; i < 3; ++i)
      cp[i] = -(((double)cam.R[i] * (double)cam.t[0] + (double)cam.R[3 + i] * (double)cam.t[1]) +
                (double)cam.R[6 + i] * (double)cam.t[2]);
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
  // per-sector constants
  for (int k = 0; k < K; ++k) {
    int kn = (k + 1 < K) ? k + 1 : 0;
    double thk = g.th[k];
    double thn = (k + 1 < K) ? g.th[k + 1] : g.th[0] + kTwoPi;
    double dl = thn - thk;
    double sk = g.s[k], sn = g.s[kn];
    float cf = (float)cos(thk), sf = (float)sin(thk);
    rec[R_SEC + S_PA * K + k] = diamond_angle(cf, sf);
    rec[R_SEC + S_C * K + k] = cf;
    rec[R_SEC + S_S * K + k] = sf;
    rec[R_SEC + S_ID * K + k] = (float)(1.0 / dl);
    double sd = sin(dl);
    rec[R_SEC + S_A * K + k] = (float)(1.0 / (sk * sd));
    rec[R_SEC + S_B * K + k] = (float)(1.0 / (sn * sd));
    double ik2 = 1.0 / (sk * sk), in2 = 1.0 / (sn * sn);
    rec[R_SEC + S_P * K + k] = (float)(0.5 * (ik2 + in2));
    rec[R_SEC + S_Q * K + k] = (float)(0.5 * (ik2 - in2));
  }
}

// ---------------------------------------------------------------------------------------------
// Duplication: for the depth-sorted primitive order, write (tile id, primitive) pairs at the
// scanned offsets, row-major over each primitive's tiles.  Spans are recomputed with the same
// float64 code as the count, so counts and pairs agree exactly.
__global__ void __launch_bounds__(128) k_duplicate(SceneDev sc, const Views* __restrict__ views, OptsDev opt, int v,
                                                   const uint32_t* __restrict__ sorted_prims,
                                                   const uint32_t* __restrict__ offsets,   // exclusive, per sorted slot
                                                   const uint32_t* __restrict__ tile_counts,
                                                   uint32_t* __restrict__ pair_tiles, uint32_t* __restrict__ pair_prims,
                                                   const uint64_t* __restrict__ total_ptr, int64_t capacity) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= sc.n) return;
  const uint32_t j = sorted_prims[i];
  const uint32_t cnt = tile_counts[j];
  if (cnt == 0) return;
  if ((int64_t)*total_ptr > capacity) return;   // overflow: the status word already says so
  uint32_t off = offsets[i];
  const CamDev& cam = views->cam[v];
  if (opt.cull_mode == 2) {
    for (uint32_t t = 0; t < cnt; ++t) { pair_tiles[off + t] = t; pair_prims[off + t] = j; }
    return;
  }
  Geo g;
  bool invalid;
  if (!load_geo(sc, j, cam, opt, g, &invalid)) return;
  Spans sp;
  build_spans(g, cam, opt, sp);
  uint32_t w = 0;
  for (int r = sp.r0; r <= sp.r1 && w < cnt; ++r) {
    int i0, i1;
    if (!row_tiles(sp, r, i0, i1)) continue;
    for (int c = i0; c <= i1 && w < cnt; ++c, ++w) {
      pair_tiles[off + w] = (uint32_t)(r * cam.tiles_x + c);
      pair_prims[off + w] = j;
    }
  }
}

}  // namespace drk

// Host launchers ------------------------------------------------------------------------------
namespace drk {

__global__ void k_set_views(Views* dst, Views src) { *dst = src; }

hipError_t set_views(Views* d_views, const Views& views, hipStream_t s) {
  hipLaunchKernelGGL(k_set_views, dim3(1), dim3(1), 0, s, d_views, views);
  return hipGetLastError();
}

hipError_t launch_preprocess(const SceneDev& sc, const Views* views, int nv, const OptsDev& opt, float* records,
                             uint32_t* depth_keys, uint32_t* tile_counts, uint32_t* status, int64_t stride,
                             hipStream_t s) {
  if (sc.n == 0) return hipSuccess;
  dim3 grid((unsigned)((sc.n + 127) / 128), (unsigned)nv);
  hipLaunchKernelGGL(k_preprocess, grid, dim3(128), 0, s, sc, views, opt, records, depth_keys, tile_counts, status,
                     stride);
  return hipGetLastError();
}

hipError_t launch_duplicate(const SceneDev& sc, const Views* views, const OptsDev& opt, int v,
                            const uint32_t* sorted_prims, const uint32_t* offsets, const uint32_t* tile_counts,
                            uint32_t* pair_tiles, uint32_t* pair_prims, const uint64_t* total_ptr, int64_t capacity,
                            hipStream_t s) {
  if (sc.n == 0) return hipSuccess;
  dim3 grid((unsigned)((sc.n + 127) / 128));
  hipLaunchKernelGGL(k_duplicate, grid, dim3(128), 0, s, sc, views, opt, v, sorted_prims, offsets, tile_counts,
                     pair_tiles, pair_prims, total_ptr, capacity);
  return hipGetLastError();
}

}  // namespace drk
