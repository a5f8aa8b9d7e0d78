// Backward DRK raster and per-primitive backward (supplement S4: the backward pass runs front to
// back so that it stays consistent with the cache-sorted forward pass).
//
// k_render_bwd replays each pixel's forward pass exactly: the same staged lists, the same
// drk_eval (bit-identical opacities) and the same cache, so it reproduces the forward emission
// sequence and stopping point.  For every composited contribution i with opacity a_i and colour
// c_i, with G = dL/dC and C the forward colour (background included), A_i the running sum of
// T_j a_j c_j for j <= i:
//   dL/dc_i = T_i a_i G,   dL/da_i = T_i (c_i . G) - ((C - A_i) . G) / (1 - a_i)      (Eq. 1)
// dL/da_i is chained through the clamp, the low-pass max (Sec. 4.4), the sharpening Psi (4.3), the
// L1/L2 energy (4.1, 4.2) and the ray-plane homography (3.3) to record-level quantities of the
// emitted primitive, re-evaluated from its record in global memory, and accumulated with float
// atomics.  k_preprocess_bwd then maps those onto the scene parameters, one thread per primitive.
#include "raster_common.hpp"

#include <math.h>

namespace drk {

__device__ __forceinline__ void gadd(float* p, float v) {
  if (v != 0.0f) unsafeAtomicAdd(p, v);
}

// Gradient terms of one composited (pixel, primitive) pair w.r.t. the record quantities.
struct PairGrad {
  float v[17];       // G_H..G_OY, in GradField order
  float s_k, s_n, th_k, th_n;
  int k, kn;
};

// dL/d(record quantities) of one composited pair with dL/d(alpha~) = gA and colour weight T a.
template <int K>
__device__ void pair_grad(const float* __restrict__ r, const Pix& pix, const RasterParams& rp, float gA, float T_w,
                          float G0, float G1, float G2, PairGrad& out) {
#pragma unroll
  for (int f = 0; f < 17; ++f) out.v[f] = 0.0f;
  out.s_k = out.s_n = out.th_k = out.th_n = 0.0f;
  out.k = 0;
  out.kn = 1 % K;
  out.v[G_RGB + 0] = T_w * G0;   // dL/dc = T a G
  out.v[G_RGB + 1] = T_w * G1;
  out.v[G_RGB + 2] = T_w * G2;
  Eval ev;
  float at, Z;
  // an emitted pair re-evaluates exactly as when it entered the cache; a miss here would mean
  // inconsistent inputs, and contributes nothing rather than reading undefined state
  if (!drk_eval<K>(r, pix, rp, at, Z, &ev)) return;
  if (ev.alpha > rp.alpha_max || gA == 0.0f) return;   // clamped: constant opacity
  const float o = r[R_O];
  float gU = 0.f, gV = 0.f, gW = 0.f;
  if (ev.lp_wins) {
    // f = o exp(arg), arg = lp_coef * d2 * |r_d|^2 / W^2
    out.v[G_O] = gA * (ev.f / o);
    const float garg = gA * ev.f;
    const float ex = ev.dx - r[R_OX], ey = ev.dy - r[R_OY];
    const float iW2 = ev.iW * ev.iW;
    const float gd2 = garg * rp.lp_coef * pix.rd2 * iW2;
    out.v[G_OX] = -2.0f * ex * gd2;
    out.v[G_OY] = -2.0f * ey * gd2;
    const float arg = rp.lp_coef * ((fmaf(ex, ex, ey * ey) * pix.rd2) * iW2);
    gW = garg * (-2.0f * arg * ev.iW);
  } else {
    const float tau = r[R_TAU];
    const float gpsi = gA * o;
    out.v[G_O] = gA * ev.psi;
    float dpsi_dtau, slope;
    if (ev.piece == 0) {
      slope = r[R_PA1];
      dpsi_dtau = -2.0f * ev.g / ((1.0f + tau) * (1.0f + tau));
    } else if (ev.piece == 1) {
      slope = r[R_PA2];
      dpsi_dtau = (2.0f * ev.g - 1.0f) / ((1.0f - tau) * (1.0f - tau));
    } else {
      slope = r[R_PA1];
      dpsi_dtau = 2.0f * (1.0f - ev.g) / ((1.0f + tau) * (1.0f + tau));
    }
    out.v[G_TAU] = gpsi * dpsi_dtau;
    const float gE = -0.5f * ev.g * gpsi * slope;
    const float eta = r[R_ETA];
    out.v[G_ETA] = gE * (ev.r1 * ev.r1 - ev.r2 * ev.ws);
    if (ev.r2 > 0.0f) {
      const int k = ev.k, kn = (k + 1 == K) ? 0 : k + 1;
      const float* sec = r + R_SEC;
      const float ck = sec[S_C * K + k], sk = sec[S_S * K + k];
      const float cn = sec[S_C * K + kn], sn = sec[S_S * K + kn];
      const float id = sec[S_ID * K + k], ak = sec[S_A * K + k], bk = sec[S_B * K + k];
      const float isk2 = sec[S_IK2 * K + k], isn2 = sec[S_IK2 * K + kn];
      const float s_k = 1.0f / sqrtf(isk2), s_n = 1.0f / sqrtf(isn2);
      const float cot = (ck * cn + sk * sn) * (ak * s_k);       // cos(delta) / sin(delta)
      const float g_r1 = gE * 2.0f * eta * ev.r1;
      const float g_ws = gE * (1.0f - eta) * ev.r2;
      const float g_r2 = gE * (1.0f - eta) * ev.ws;
      // ws = ch^2 isk2 + sh^2 isn2 with ch = cos(pi t/2), sh = sin(pi t/2)
      const float g_isk2 = g_ws * (ev.ch * ev.ch);
      const float g_isn2 = g_ws * (ev.sh * ev.sh);
      const float g_t = 3.14159265358979f * (ev.ch * ev.sh) * (isn2 - isk2) * g_ws;
      const float g_phi = g_t * id;
      float g_delta = -g_t * ev.phi * id * id;
      const float sB = ev.B > 0.f ? 1.f : (ev.B < 0.f ? -1.f : 0.f);
      const float sA = ev.A > 0.f ? 1.f : (ev.A < 0.f ? -1.f : 0.f);
      const float gB = g_r1 * ak * sB;
      float gAc = g_r1 * bk * sA;
      const float g_ak = g_r1 * fabsf(ev.B), g_bk = g_r1 * fabsf(ev.A);
      out.s_k = -g_ak * ak / s_k - 2.0f * g_isk2 * isk2 / s_k;
      out.s_n = -g_bk * bk / s_n - 2.0f * g_isn2 * isn2 / s_n;
      g_delta -= (g_ak * ak + g_bk * bk) * cot;
      gAc += g_phi * ev.D / ev.r2;
      const float gD = -g_phi * ev.A / ev.r2;
      const float u = ev.u, v = ev.v;
      const float g_u = -gAc * sk + gB * sn + gD * ck + 2.0f * u * g_r2;
      const float g_v = gAc * ck - gB * cn + gD * sk + 2.0f * v * g_r2;
      out.th_k = -gAc * ev.D + gD * ev.A - g_delta;
      out.th_n = gB * (u * cn + v * sn) + g_delta;
      out.k = k;
      out.kn = kn;
      gU = g_u * ev.iW;
      gV = g_v * ev.iW;
      gW = -(g_u * u + g_v * v) * ev.iW;
    }
  }
  out.v[G_H + 0] = gU * ev.dx;
  out.v[G_H + 1] = gU * ev.dy;
  out.v[G_H + 2] = gU;
  out.v[G_H + 3] = gV * ev.dx;
  out.v[G_H + 4] = gV * ev.dy;
  out.v[G_H + 5] = gV;
  out.v[G_H + 6] = gW * ev.dx;
  out.v[G_H + 7] = gW * ev.dy;
  out.v[G_H + 8] = gW;
}

__device__ __forceinline__ float wave_sum(float x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}

// Accumulates the pair gradients of the lanes with `on` set.  Must be called by every lane of the
// wave.  When all those lanes hold the same primitive the terms are summed across the wave first
// (one atomic per field); otherwise each lane adds its own.
template <int K>
__device__ void accumulate(bool on, uint32_t j, const PairGrad& pg, float* __restrict__ g, int64_t n) {
  const uint64_t m = __ballot(on);
  if (!m) return;
  const int lane = threadIdx.x & 63;
  const int leader = __ffsll((unsigned long long)m) - 1;
  const uint32_t j0 = __shfl(j, leader, 64);
  const bool uniform = __ballot(on && j != j0) == 0;
  if (uniform) {
#pragma unroll
    for (int f = 0; f < 17; ++f) {
      const float t = wave_sum(on ? pg.v[f] : 0.0f);
      if (lane == leader && t != 0.0f) unsafeAtomicAdd(g + (size_t)f * n + j0, t);
    }
    const int k0 = __shfl(pg.k, leader, 64);
    if (__ballot(on && pg.k != k0) == 0) {
      const int kn0 = (k0 + 1 == K) ? 0 : k0 + 1;
      const float a = wave_sum(on ? pg.s_k : 0.0f), b = wave_sum(on ? pg.s_n : 0.0f);
      const float c = wave_sum(on ? pg.th_k : 0.0f), d = wave_sum(on ? pg.th_n : 0.0f);
      if (lane == leader) {
        if (a != 0.0f) unsafeAtomicAdd(g + (size_t)(G_SEC + k0) * n + j0, a);
        if (b != 0.0f) unsafeAtomicAdd(g + (size_t)(G_SEC + kn0) * n + j0, b);
        if (c != 0.0f) unsafeAtomicAdd(g + (size_t)(G_SEC + K + k0) * n + j0, c);
        if (d != 0.0f) unsafeAtomicAdd(g + (size_t)(G_SEC + K + kn0) * n + j0, d);
      }
      return;
    }
  } else if (on) {
#pragma unroll
    for (int f = 0; f < 17; ++f)
      if (pg.v[f] != 0.0f) unsafeAtomicAdd(g + (size_t)f * n + j, pg.v[f]);
  }
  if (on) {
    if (pg.s_k != 0.0f) unsafeAtomicAdd(g + (size_t)(G_SEC + pg.k) * n + j, pg.s_k);
    if (pg.s_n != 0.0f) unsafeAtomicAdd(g + (size_t)(G_SEC + pg.kn) * n + j, pg.s_n);
    if (pg.th_k != 0.0f) unsafeAtomicAdd(g + (size_t)(G_SEC + K + pg.k) * n + j, pg.th_k);
    if (pg.th_n != 0.0f) unsafeAtomicAdd(g + (size_t)(G_SEC + K + pg.kn) * n + j, pg.th_n);
  }
}

template <int K>
__global__ void __launch_bounds__(kBlock) k_render_bwd(const float* __restrict__ records, const uint32_t* __restrict__ ranges,
                                                       const uint32_t* __restrict__ prims, const CamDev* __restrict__ camp,
                                                       OptsDev opt, const float* __restrict__ rgb,
                                                       const float* __restrict__ dL, float* __restrict__ grad,
                                                       int64_t n) {
  constexpr int RF = (R_SEC + S_NFIELDS * K + 3) & ~3;
  constexpr int RF4 = RF / 4;
  __shared__ float4 lds[kBatch * RF4];
  __shared__ uint32_t lidx[kBatch];
  const CamDev& cam = *camp;
  const int tile = blockIdx.x;
  const int tx = tile % cam.tiles_x, ty = tile / cam.tiles_x;
  const int tid = threadIdx.x;
  const int x = tx * kTile + (tid & (kTile - 1));
  const int y = ty * kTile + (tid >> 4);
  const bool inside = x < cam.W && y < cam.H;
  const RasterParams rp = make_params(opt);
  const Pix pix = make_pix(cam, x, y);
  // pixel-centre rectangle of this wave (16 x 4 pixels)
  const float wx0 = (float)(tx * kTile) + 0.5f, wx1 = wx0 + (float)(kTile - 1);
  const float wy0 = (float)(ty * kTile + (tid >> 6) * 4) + 0.5f, wy1 = wy0 + 3.0f;
  const uint32_t start = ranges[2 * tile], end = ranges[2 * tile + 1];
  const size_t plane = (size_t)cam.W * cam.H;
  const size_t pidx = inside ? (size_t)y * cam.W + x : 0;
  float Cf0 = 0.f, Cf1 = 0.f, Cf2 = 0.f, G0 = 0.f, G1 = 0.f, G2 = 0.f;
  if (inside) {
    Cf0 = rgb[pidx]; Cf1 = rgb[plane + pidx]; Cf2 = rgb[2 * plane + pidx];
    G0 = dL[pidx]; G1 = dL[plane + pidx]; G2 = dL[2 * plane + pidx];
  }
  float T = 1.0f, A0 = 0.f, A1 = 0.f, A2 = 0.f;
  bool done = !inside || (G0 == 0.f && G1 == 0.f && G2 == 0.f);
  Cache<2> cache;
  cache.init(rp.cache_len);

  // Composites the popped entries (alpha a, primitive j) of the lanes with `have` set, exactly as the
  // forward pass does, and accumulates their gradients.  Called by every lane of the wave.
  auto emit = [&](bool have, float a, uint32_t j) {
    PairGrad pg;
    bool on = false;
    if (have) {
      const float test = T * (1.0f - a);
      if (test < rp.T_min) {
        done = true;
      } else {
        const float* rg = records + (size_t)j * RF;
        const float c0 = rg[R_RGB + 0], c1 = rg[R_RGB + 1], c2 = rg[R_RGB + 2];
        const float w = a * T;
        A0 = fmaf(w, c0, A0);
        A1 = fmaf(w, c1, A1);
        A2 = fmaf(w, c2, A2);
        const float rest = (Cf0 - A0) * G0 + (Cf1 - A1) * G1 + (Cf2 - A2) * G2;
        const float gA = T * (c0 * G0 + c1 * G1 + c2 * G2) - rest / (1.0f - a);
        pair_grad<K>(rg, pix, rp, gA, w, G0, G1, G2, pg);
        T = test;
        on = true;
      }
    }
    accumulate<K>(on, j, pg, grad, n);
  };

  for (uint32_t b0 = start; b0 < end; b0 += kBatch) {
    if (__syncthreads_count(!done) == 0) break;
    const int nb = (int)min((uint32_t)kBatch, end - b0);
    for (int q = tid; q < nb * RF4; q += kBlock) {
      const int ri = q / RF4, c = q - ri * RF4;
      const uint32_t j = prims[b0 + ri];
      lds[q] = reinterpret_cast<const float4*>(records + (size_t)j * RF)[c];
    }
    if (tid < nb) lidx[tid] = prims[b0 + tid];
    __syncthreads();
    const uint64_t mask = batch_box_mask<RF4>(lds, nb, wx0, wx1, wy0, wy1);
    for (uint64_t m = mask; m; m &= m - 1) {
      if (__ballot(!done) == 0) break;
      const int i = __builtin_ctzll(m);
      const float* r = reinterpret_cast<const float*>(lds + i * RF4);
      bool contrib = false;
      float at = 0.0f, Z = 0.0f;
      if (!done) contrib = drk_eval<K>(r, pix, rp, at, Z) && at >= rp.alpha_min;
      // a contributor pops the head (emitted when real), then is inserted
      const bool have = contrib && cache.pay[0][0] > 0.0f;
      if (__ballot(have)) emit(have, cache.pay[0][0], __float_as_uint(cache.pay[1][0]));
      if (contrib) {
        const float x2[2] = {at, __uint_as_float(lidx[i])};
        cache.pop_insert(Z, x2);
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int s = 0; s < kMaxCache; ++s) {
    const bool have = !done && cache.pay[0][s] > 0.0f;
    if (__ballot(have)) emit(have, cache.pay[0][s], __float_as_uint(cache.pay[1][s]));
  }
}

template <int K>
static hipError_t launch_bwd_k(const float* records, const uint32_t* ranges, const uint32_t* prims, const CamDev* cam,
                               int ntiles, const OptsDev& opt, const float* rgb, const float* dL, float* grad, int64_t n,
                               hipStream_t s) {
  hipLaunchKernelGGL(k_render_bwd<K>, dim3(ntiles), dim3(kBlock), 0, s, records, ranges, prims, cam, opt, rgb, dL, grad, n);
  return hipGetLastError();
}

hipError_t launch_render_bwd(int K, const float* records, const uint32_t* ranges, const uint32_t* prims,
                             const CamDev* cam, int ntiles, const OptsDev& opt, const float* rgb, const float* dL, float* grad,
                             int64_t n, hipStream_t s) {
  switch (K) {
#define DRK_CASE(k) \
  case k: return launch_bwd_k<k>(records, ranges, prims, cam, ntiles, opt, rgb, dL, grad, n, s);
    DRK_CASE(3) DRK_CASE(4) DRK_CASE(5) DRK_CASE(6) DRK_CASE(7) DRK_CASE(8) DRK_CASE(9) DRK_CASE(10)
    DRK_CASE(11) DRK_CASE(12) DRK_CASE(13) DRK_CASE(14) DRK_CASE(15) DRK_CASE(16)
#undef DRK_CASE
    default: return hipErrorInvalidValue;
  }
}

// ---------------------------------------------------------------------------------------------
// Per-primitive backward (float64): record gradients of every view -> scene parameter gradients.

__device__ inline void cross3(const double a[3], const double b[3], double o[3]) {
  o[0] = a[1] * b[2] - a[2] * b[1];
  o[1] = a[2] * b[0] - a[0] * b[2];
  o[2] = a[0] * b[1] - a[1] * b[0];
}

// gradient of the real SH basis (degree <= 3) w.r.t. the direction components (polynomial form)
__device__ inline void real_sh_grad(int deg, double x, double y, double z, double Y[16], double dY[16][3]) {
  const double c0 = 0.28209479177387814, c1 = 0.4886025119029199;
  for (int i = 0; i < 16; ++i) { Y[i] = 0.0; dY[i][0] = dY[i][1] = dY[i][2] = 0.0; }
  Y[0] = c0;
  if (deg >= 1) {
    Y[1] = c1 * y; dY[1][1] = c1;
    Y[2] = c1 * z; dY[2][2] = c1;
    Y[3] = c1 * x; dY[3][0] = c1;
  }
  if (deg >= 2) {
    const double a = 1.0925484305920792, b = 0.31539156525252005, c = 0.5462742152960396;
    Y[4] = a * x * y; dY[4][0] = a * y; dY[4][1] = a * x;
    Y[5] = a * y * z; dY[5][1] = a * z; dY[5][2] = a * y;
    Y[6] = b * (3.0 * z * z - 1.0); dY[6][2] = 6.0 * b * z;
    Y[7] = a * x * z; dY[7][0] = a * z; dY[7][2] = a * x;
    Y[8] = c * (x * x - y * y); dY[8][0] = 2.0 * c * x; dY[8][1] = -2.0 * c * y;
  }
  if (deg >= 3) {
    const double a = 0.5900435899266435, b = 2.890611442640554, c = 0.4570457994644658;
    const double d = 0.3731763325901154, e = 1.445305721320277;
    Y[9] = a * y * (3.0 * x * x - y * y);
    dY[9][0] = 6.0 * a * x * y; dY[9][1] = a * (3.0 * x * x - 3.0 * y * y);
    Y[10] = b * x * y * z;
    dY[10][0] = b * y * z; dY[10][1] = b * x * z; dY[10][2] = b * x * y;
    Y[11] = c * y * (5.0 * z * z - 1.0);
    dY[11][1] = c * (5.0 * z * z - 1.0); dY[11][2] = 10.0 * c * y * z;
    Y[12] = d * (5.0 * z * z * z - 3.0 * z);
    dY[12][2] = d * (15.0 * z * z - 3.0);
    Y[13] = c * x * (5.0 * z * z - 1.0);
    dY[13][0] = c * (5.0 * z * z - 1.0); dY[13][2] = 10.0 * c * x * z;
    Y[14] = e * z * (x * x - y * y);
    dY[14][0] = 2.0 * e * x * z; dY[14][1] = -2.0 * e * y * z; dY[14][2] = e * (x * x - y * y);
    Y[15] = a * x * (x * x - 3.0 * y * y);
    dY[15][0] = a * (3.0 * x * x - 3.0 * y * y); dY[15][1] = -6.0 * a * x * y;
  }
}

__global__ void __launch_bounds__(128) __attribute__((amdgpu_waves_per_eu(4))) k_preprocess_bwd(SceneDev sc, const Views* __restrict__ views, OptsDev opt,
                                                        const uint32_t* __restrict__ tile_counts,
                                                        const float* __restrict__ grec, int64_t stride,
                                                        drk_scene_grad out) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= sc.n) return;
  const int64_t n = sc.n;
  const int K = sc.K;
  const int GF = grad_fields(K);
  double gmu[3] = {0, 0, 0}, gq[4] = {0, 0, 0, 0};
  double go = 0, geta = 0, gtau = 0;
  double gs[kMaxK], gth[kMaxK];
  for (int k = 0; k < K; ++k) gs[k] = gth[k] = 0.0;
  const int nc = sc.color_mode == 1 ? (sc.sh_degree + 1) * (sc.sh_degree + 1) : 1;
  double gcol[48];
  for (int i = 0; i < 3 * nc; ++i) gcol[i] = 0.0;
  double mu[3], q[4];
  for (int i = 0; i < 3; ++i) mu[i] = (double)sc.mu[i * n + j];
  for (int i = 0; i < 4; ++i) q[i] = (double)sc.q[i * n + j];
  const double qn = sqrt(((q[0] * q[0] + q[1] * q[1]) + q[2] * q[2]) + q[3] * q[3]);
  const double w = q[0] / qn, x = q[1] / qn, y = q[2] / qn, z = q[3] / qn;
  const double tu[3] = {1.0 - 2.0 * (y * y + z * z), 2.0 * (x * y + w * z), 2.0 * (x * z - w * y)};
  const double tv[3] = {2.0 * (x * y - w * z), 1.0 - 2.0 * (x * x + z * z), 2.0 * (y * z + w * x)};
  double gtu[3] = {0, 0, 0}, gtv[3] = {0, 0, 0};

  for (int v = 0; v < views->nv; ++v) {
    if (tile_counts[(int64_t)v * stride + j] == 0) continue;
    const float* gr = grec + (size_t)v * GF * stride;
    auto G = [&](int f) { return (double)gr[(size_t)f * stride + j]; };
    const CamDev& cam = views->cam[v];
    double R[9];
    for (int i = 0; i < 9; ++i) R[i] = cam.R[i];
    double muc[3], tuc[3], tvc[3];
    for (int i = 0; i < 3; ++i) {
      muc[i] = R[3 * i] * mu[0] + R[3 * i + 1] * mu[1] + R[3 * i + 2] * mu[2] + (double)cam.t[i];
      tuc[i] = R[3 * i] * tu[0] + R[3 * i + 1] * tu[1] + R[3 * i + 2] * tu[2];
      tvc[i] = R[3 * i] * tv[0] + R[3 * i + 1] * tv[1] + R[3 * i + 2] * tv[2];
    }
    const double fx = cam.fx, fy = cam.fy, cx = cam.cx, cy = cam.cy;
    // anchor exactly as the forward record (piecewise constant: no gradient)
    const double pxc = (fx * muc[0]) / muc[2] + cx, pyc = (fy * muc[1]) / muc[2] + cy;
    const double axc = fmin(fmax(pxc, -2.0 * cam.W), 3.0 * cam.W), ayc = fmin(fmax(pyc, -2.0 * cam.H), 3.0 * cam.H);
    const double ax = rint(axc * 256.0) / 256.0, ay = rint(ayc * 256.0) / 256.0;
    // dL/dHm -> dL/d(adjugate rows)
    double ga[3][3];
    for (int r = 0; r < 3; ++r) {
      const double h0 = G(G_H + 3 * r), h1 = G(G_H + 3 * r + 1), h2 = G(G_H + 3 * r + 2);
      ga[r][0] = h0 / fx + h2 * (ax - cx) / fx;
      ga[r][1] = h1 / fy + h2 * (ay - cy) / fy;
      ga[r][2] = h2;
    }
    // a0 = tvc x muc, a1 = muc x tuc, a2 = tuc x tvc ; for a = b x c: gb = c x ga, gc = ga x b
    double t1[3], gmuc[3] = {0, 0, 0}, gtuc[3] = {0, 0, 0}, gtvc[3] = {0, 0, 0};
    cross3(muc, ga[0], t1); for (int i = 0; i < 3; ++i) gtvc[i] += t1[i];
    cross3(ga[0], tvc, t1); for (int i = 0; i < 3; ++i) gmuc[i] += t1[i];
    cross3(tuc, ga[1], t1); for (int i = 0; i < 3; ++i) gmuc[i] += t1[i];
    cross3(ga[1], muc, t1); for (int i = 0; i < 3; ++i) gtuc[i] += t1[i];
    cross3(tvc, ga[2], t1); for (int i = 0; i < 3; ++i) gtuc[i] += t1[i];
    cross3(ga[2], tuc, t1); for (int i = 0; i < 3; ++i) gtvc[i] += t1[i];
    // low-pass centre: (ox, oy) = projection of mu_c - anchor
    const double gox = G(G_OX), goy = G(G_OY);
    gmuc[0] += gox * fx / muc[2];
    gmuc[1] += goy * fy / muc[2];
    gmuc[2] += -(gox * fx * muc[0] + goy * fy * muc[1]) / (muc[2] * muc[2]);
    // camera -> world
    for (int i = 0; i < 3; ++i) {
      gmu[i] += R[i] * gmuc[0] + R[3 + i] * gmuc[1] + R[6 + i] * gmuc[2];
      gtu[i] += R[i] * gtuc[0] + R[3 + i] * gtuc[1] + R[6 + i] * gtuc[2];
      gtv[i] += R[i] * gtvc[0] + R[3 + i] * gtvc[1] + R[6 + i] * gtvc[2];
    }
    go += G(G_O);
    geta += G(G_ETA);
    gtau += G(G_TAU);
    for (int k = 0; k < K; ++k) {
      gs[k] += G(G_SEC + k);
      gth[k] += G(G_SEC + K + k);
    }
    // colour
    const double grgb[3] = {G(G_RGB), G(G_RGB + 1), G(G_RGB + 2)};
    if (sc.color_mode == 0) {
      for (int c = 0; c < 3; ++c) gcol[c] += grgb[c];
    } else {
      double cp[3];
      for (int i = 0; i < 3; ++i)
        cp[i] = cam.campos[i];
      double d[3] = {mu[0] - cp[0], mu[1] - cp[1], mu[2] - cp[2]};
      const double dn = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
      const double dh[3] = {d[0] / dn, d[1] / dn, d[2] / dn};
      double Y[16], dY[16][3];
      real_sh_grad(sc.sh_degree, dh[0], dh[1], dh[2], Y, dY);
      double gdh[3] = {0, 0, 0};
      for (int c = 0; c < 3; ++c) {
        double val = 0.5;
        for (int i = 0; i < nc; ++i) val += Y[i] * (double)sc.color[(3 * i + c) * n + j];
        if (val < 0.0) continue;                     // clamped at 0: no gradient
        for (int i = 0; i < nc; ++i) {
          gcol[3 * i + c] += grgb[c] * Y[i];
          const double co = (double)sc.color[(3 * i + c) * n + j];
          for (int a = 0; a < 3; ++a) gdh[a] += grgb[c] * co * dY[i][a];
        }
      }
      const double dd = gdh[0] * dh[0] + gdh[1] * dh[1] + gdh[2] * dh[2];
      for (int a = 0; a < 3; ++a) gmu[a] += (gdh[a] - dh[a] * dd) / dn;
    }
  }
  // tangent axes -> unit quaternion -> raw quaternion
  double gw = 2.0 * z * gtu[1] - 2.0 * y * gtu[2] - 2.0 * z * gtv[0] + 2.0 * x * gtv[2];
  double gx = 2.0 * y * gtu[1] + 2.0 * z * gtu[2] + 2.0 * y * gtv[0] - 4.0 * x * gtv[1] + 2.0 * w * gtv[2];
  double gy = -4.0 * y * gtu[0] + 2.0 * x * gtu[1] - 2.0 * w * gtu[2] + 2.0 * x * gtv[0] + 2.0 * z * gtv[2];
  double gz = -4.0 * z * gtu[0] + 2.0 * w * gtu[1] + 2.0 * x * gtu[2] - 2.0 * w * gtv[0] - 4.0 * z * gtv[1] +
              2.0 * y * gtv[2];
  const double dot = gw * w + gx * x + gy * y + gz * z;
  gq[0] = (gw - w * dot) / qn;
  gq[1] = (gx - x * dot) / qn;
  gq[2] = (gy - y * dot) / qn;
  gq[3] = (gz - z * dot) / qn;
  for (int i = 0; i < 3; ++i) out.mu[i * n + j] = (float)gmu[i];
  for (int i = 0; i < 4; ++i) out.q[i * n + j] = (float)gq[i];
  for (int k = 0; k < K; ++k) {
    out.scale[k * n + j] = (float)gs[k];
    out.theta[k * n + j] = (float)gth[k];
  }
  out.eta[j] = (float)geta;
  out.tau[j] = (float)gtau;
  out.opacity[j] = (float)go;
  const int ncol = sc.color_mode == 1 ? 3 * nc : 3;
  for (int i = 0; i < ncol; ++i) out.color[(int64_t)i * n + j] = (float)gcol[i];
}

hipError_t launch_preprocess_bwd(const SceneDev& sc, const Views* views, const OptsDev& opt, const uint32_t* tile_counts,
                                 const float* grec, int64_t stride, const drk_scene_grad& out, hipStream_t s) {
  if (sc.n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_preprocess_bwd, dim3((unsigned)((sc.n + 127) / 128)), dim3(128), 0, s, sc, views, opt,
                     tile_counts, grec, stride, out);
  return hipGetLastError();
}

}  // namespace drk
