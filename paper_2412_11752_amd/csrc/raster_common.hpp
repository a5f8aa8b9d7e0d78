// Per-pixel DRK evaluation shared by the forward and backward raster kernels.
//
// Both kernels call exactly this code (compiled with -ffp-contract=off, explicit fmaf), so the
// backward pass recomputes bit-identical opacities and therefore the identical cache-sorted
// emission sequence of the forward pass.
#pragma once

#include "drk_internal.hpp"

namespace drk {

constexpr int kBatch = 64;          // primitives staged in LDS per round
constexpr int kBlock = kTile * kTile;

struct Pix {
  float px, py;     // pixel centre (x + 0.5, y + 0.5)
  float rd2;        // |r_d|^2 with r_d = ((px - cx)/fx, (py - cy)/fy, 1)
};

struct RasterParams {
  float alpha_min, alpha_max, T_min, near_plane;
  float lp_coef;    // -1 / (2 s_l^2), 0 when the low-pass filter is off
  int32_t lowpass;
  int32_t cache_len;
};

__device__ __forceinline__ float rcpf(float x) { return __builtin_amdgcn_rcpf(x); }

__device__ __forceinline__ float diamond_pa(float u, float v) {
  const float r = u * rcpf(fabsf(u) + fabsf(v));
  return v >= 0.0f ? 1.0f - r : 3.0f + r;
}

// atan2 for the sector angle: atan(a) = a P(a^2) on [0, 1] (odd polynomial fitted by relative-error
// weighted least squares; max relative error 2.2e-7 in float32), then the octant is restored.
__device__ __forceinline__ float atan2_fast(float y, float x) {
  const float ax = fabsf(x), ay = fabsf(y);
  const float mx = fmaxf(ax, ay), mn = fminf(ax, ay);
  const float a = mx > 0.0f ? mn * rcpf(mx) : 0.0f;
  const float s = a * a;
  float p = -0.00469335893820626f;
  p = fmaf(p, s, 0.024252677013602238f);
  p = fmaf(p, s, -0.059486744643040414f);
  p = fmaf(p, s, 0.09914314847813398f);
  p = fmaf(p, s, -0.1401948782422469f);
  p = fmaf(p, s, 0.19969724889612928f);
  p = fmaf(p, s, -0.33331990794665783f);
  p = fmaf(p, s, 0.9999999009920119f);
  float r = a * p;
  r = ay > ax ? 1.5707963267948966f - r : r;
  r = x < 0.0f ? 3.141592653589793f - r : r;
  return copysignf(r, y);
}

// sin(pi x / 2) for x in about [-0.02, 1.02]: odd polynomial (least squares weighted by the relative
// error; max relative error 1.9e-7 in float32).  The L2 weight uses cos^2(pi t/2) = sinhalf(1-t)^2
// and sin^2(pi t/2) = sinhalf(t)^2, both accurate relative to their size.
__device__ __forceinline__ float sinhalf_fast(float x) {
  const float s = x * x;
  float p = 0.00015193128256064164f;
  p = fmaf(p, s, -0.004674595124423347f);
  p = fmaf(p, s, 0.07969015617822843f);
  p = fmaf(p, s, -0.6459637978745842f);
  p = fmaf(p, s, 1.570796320926877f);
  return x * p;
}

__device__ __forceinline__ float exp_fast(float x) { return __builtin_amdgcn_exp2f(x * 1.4426950408889634f); }

// Intermediate values of one (pixel, primitive) evaluation.
struct Eval {
  float dx, dy, U, V, W, iW, u, v;
  float A, B, D, phi, t, ch, sh, ws, r1, r2, E, g, psi, alpha, f;
  int k, piece;
  bool lp_wins;
};

// Evaluates the opacity (after low-pass and clamp) of record r at pixel p.  Returns false when the
// ray misses (grazing, behind the near plane) or when the pixel provably cannot contribute.  Sec. 3.3
// (hit, via the homography), Sec. 4.1-4.3 (kernel), Sec. 4.4 (low-pass).
//
// The L2 weight 1/sbar^2 = (1 + cos pi t)/(2 s_k^2) + (1 - cos pi t)/(2 s_{k+1}^2) (Sec. 4.1) is
// evaluated as cos^2(pi t/2)/s_k^2 + sin^2(pi t/2)/s_{k+1}^2: two positive terms, so that very
// different lengths in one sector do not cancel.
//
// The two early-outs are exact in float32.  cos^2 + sin^2 of the polynomial lies within
// [1 - 1.8e-7, 1 + 4.4e-7], so w_lo = min(1/s_k^2, 1/s_{k+1}^2) (1 - 1e-5) (stored per sector) is below
// the weight after rounding; every other rounding step is monotone, so E >= E_lo = eta r1^2 +
// (1 - eta) r2 w_lo, and E > R_ETHR (c^2 with a margin) gives o Psi(exp(-E/2)) < alpha_min.  Likewise r2 > R_R2CUT bounds E from below by
// r2 / max_k s_k^2.  Either test only rejects when the low-pass term is also below alpha_min.
//
// EARLY_MISS: the grazing, near-plane and radius tests return before the sector search (fewer
// operations where many pixels miss, as with the many small DRKs of a converted mesh); otherwise
// they join the energy cut's branch (one divergent branch less per evaluation).  The results are
// the same either way.
template <int K, bool EARLY_MISS = true>
__device__ __forceinline__ bool drk_eval(const float* __restrict__ r, const Pix& p, const RasterParams& rp, float& at,
                                         float& Z, Eval* ev = nullptr) {
  const float dx = p.px - r[R_AX];
  const float dy = p.py - r[R_AY];
  const float U = fmaf(r[R_H + 0], dx, fmaf(r[R_H + 1], dy, r[R_H + 2]));
  const float V = fmaf(r[R_H + 3], dx, fmaf(r[R_H + 4], dy, r[R_H + 5]));
  const float W = fmaf(r[R_H + 6], dx, fmaf(r[R_H + 7], dy, r[R_H + 8]));
  const float W2 = W * W;
  const float iW = rcpf(W);
  Z = r[R_DN] * iW;
  const float u = U * iW, v = V * iW;
  const float r2 = fmaf(u, u, v * v);
  const float ex = dx - r[R_OX], ey = dy - r[R_OY];
  const float d2 = fmaf(ex, ex, ey * ey);
  // the low-pass term can reach alpha_min (R_LPCUT < 0 when the filter is off)
  const bool lp_in = d2 * p.rd2 <= r[R_LPCUT] * W2;
  // grazing ray (|r_d . n| < 1e-6), hit at or behind the near plane, or beyond the radius cut, in one
  // branch (the values computed for a grazing ray are discarded): divergent branches cost the wave
  // more than the few operations they would skip
  const bool miss = !(W2 >= 1e-12f * p.rd2) | !(Z > rp.near_plane) | ((r2 > r[R_R2CUT]) & !lp_in);
  if (EARLY_MISS && miss) return false;
  float E = 0.0f;
  int k = 0;
  float A = 0.f, B = 0.f, D = 0.f, phi = 0.f, t = 0.f, ch = 1.f, sh = 0.f, ws = 0.f, r1 = 0.f;
  {
    // sector: largest k with pa_k < pa (wrapping to K-1).  No branch on r2 > 0: at the centre
    // (r2 = 0) pa is NaN, the count gives k = K-1, A = B = D = 0 and E = 0
    const float pa = diamond_pa(u, v);
    int cnt = 0;
#pragma unroll
    for (int i = 0; i < K; ++i) cnt += (r[R_SEC + S_PA * K + i] < pa) ? 1 : 0;
    k = (cnt == 0) ? K - 1 : cnt - 1;
    const int kn = (k + 1 == K) ? 0 : k + 1;
    const float* sec = r + R_SEC;
    const float ck = sec[S_C * K + k], sk = sec[S_S * K + k];
    const float cn = sec[S_C * K + kn], sn = sec[S_S * K + kn];
    A = fmaf(ck, v, -(sk * u));          // cross(d_k, p)       = r2 sin(phi)
    B = fmaf(u, sn, -(v * cn));          // cross(p, d_{k+1})   = r2 sin(delta - phi)
    D = fmaf(ck, u, sk * v);             // dot(d_k, p)         = r2 cos(phi)
    r1 = fmaf(sec[S_A * K + k], fabsf(B), sec[S_B * K + k] * fabsf(A));
    const float eta = r[R_ETA];
    const float r1sq = r1 * r1, oeta = 1.0f - eta;
    const float E_lo = fmaf(eta, r1sq, oeta * (r2 * sec[S_WLO * K + k]));
    if ((!EARLY_MISS && miss) | ((E_lo > r[R_ETHR]) & !lp_in)) return false;
    phi = atan2_fast(A, D);
    t = phi * sec[S_ID * K + k];
    sh = sinhalf_fast(t);
    ch = sinhalf_fast(1.0f - t);
    ws = fmaf(ch * ch, sec[S_IK2 * K + k], (sh * sh) * sec[S_IK2 * K + kn]);
    E = fmaf(eta, r1sq, oeta * (r2 * ws));
  }
  const float g = exp_fast(-0.5f * E);
  float psi;
  int piece;
  if (g < r[R_PLO]) { psi = r[R_PA1] * g; piece = 0; }
  else if (g < r[R_PHI]) { psi = fmaf(r[R_PA2], g, r[R_PB2]); piece = 1; }
  else { psi = fmaf(r[R_PA1], g, r[R_PB3]); piece = 2; }
  const float o = r[R_O];
  float alpha = o * psi;
  float f = 0.0f;
  bool lp = false;
  if (rp.lowpass) {
    f = o * exp_fast(rp.lp_coef * ((d2 * p.rd2) * (iW * iW)));
    lp = f > alpha;
    alpha = lp ? f : alpha;
  }
  at = fminf(alpha, rp.alpha_max);
  if (ev) {
    ev->dx = dx; ev->dy = dy; ev->U = U; ev->V = V; ev->W = W; ev->iW = iW; ev->u = u; ev->v = v;
    ev->A = A; ev->B = B; ev->D = D; ev->phi = phi; ev->t = t; ev->ch = ch; ev->sh = sh; ev->ws = ws; ev->r1 = r1;
    ev->r2 = r2;
    ev->E = E; ev->g = g; ev->psi = psi; ev->alpha = alpha; ev->f = f; ev->k = k; ev->piece = piece; ev->lp_wins = lp;
  }
  return true;
}

// Bit i set when staged record i (i < nb) may touch the wave's pixel rectangle.  Lane i tests record
// i; called by every lane of the wave.
template <int RF4>
__device__ __forceinline__ uint64_t batch_box_mask(const float4* lds, int nb, float x0, float x1, float y0, float y1) {
  const int lane = threadIdx.x & 63;
  bool hit = false;
  if (lane < nb) {
    // record i's box (x0, x1, y0, y1) reaches the wave's pixel-centre rectangle; the four tests
    // without short-circuit branches, NaN bounds counting as reaching
    const float4 b = lds[lane * RF4 + R_BOX / 4];
    hit = !(x1 < b.x) & !(x0 > b.y) & !(y1 < b.z) & !(y0 > b.w);
  }
  return __ballot(hit);
}

// Always-full sorted cache of kMaxCache slots (Sec. 4.4 Cache Sorting, Algorithm 1).  Slots hold
// (key, payload...).  Unused capacity holds -inf sentinels (popped first, emit nothing) and, for
// cache_len < kMaxCache, +inf sentinels that never reach the head.  An arriving contributor pops
// the head (the caller reads and emits it first) and is inserted after all entries with key <= its
// key.
template <int NP>
struct Cache {
  float key[kMaxCache];
  float pay[NP][kMaxCache];

  __device__ __forceinline__ void init(int cache_len) {
#pragma unroll
    for (int s = 0; s < kMaxCache; ++s) {
      key[s] = (s < cache_len) ? -INFINITY : INFINITY;
#pragma unroll
      for (int q = 0; q < NP; ++q) pay[q][s] = 0.0f;
    }
  }
  // Drops slot 0 and inserts (z, x).  With b_j = key[j+1] <= z (monotone in j), slot j takes
  // key[j+1] while b_j holds, z at the first j where it fails, and keeps its entry after that.
  __device__ __forceinline__ void pop_insert(float z, const float (&x)[NP]) {
    bool b[kMaxCache - 1];
#pragma unroll
    for (int j = 0; j < kMaxCache - 1; ++j) b[j] = key[j + 1] <= z;
    key[0] = b[0] ? key[1] : z;
#pragma unroll
    for (int q = 0; q < NP; ++q) pay[q][0] = b[0] ? pay[q][1] : x[q];
#pragma unroll
    for (int j = 1; j < kMaxCache - 1; ++j) {
      key[j] = b[j] ? key[j + 1] : (b[j - 1] ? z : key[j]);
#pragma unroll
      for (int q = 0; q < NP; ++q) pay[q][j] = b[j] ? pay[q][j + 1] : (b[j - 1] ? x[q] : pay[q][j]);
    }
    key[kMaxCache - 1] = b[kMaxCache - 2] ? z : key[kMaxCache - 1];
#pragma unroll
    for (int q = 0; q < NP; ++q) pay[q][kMaxCache - 1] = b[kMaxCache - 2] ? x[q] : pay[q][kMaxCache - 1];
  }
};

__device__ inline RasterParams make_params(const OptsDev& o) {
  RasterParams rp;
  rp.alpha_min = o.alpha_min;
  rp.alpha_max = o.alpha_max;
  rp.T_min = o.T_min;
  rp.near_plane = o.near_plane;
  rp.lowpass = o.lowpass_sl > 0.0f;
  rp.lp_coef = rp.lowpass ? -1.0f / (2.0f * o.lowpass_sl * o.lowpass_sl) : 0.0f;
  rp.cache_len = o.cache_len;
  return rp;
}

__device__ inline Pix make_pix(const CamDev& cam, int x, int y) {
  Pix p;
  p.px = (float)x + 0.5f;
  p.py = (float)y + 0.5f;
  const float rx = (p.px - cam.cx) / cam.fx;
  const float ry = (p.py - cam.cy) / cam.fy;
  p.rd2 = fmaf(rx, rx, fmaf(ry, ry, 1.0f));
  return p;
}

}  // namespace drk
