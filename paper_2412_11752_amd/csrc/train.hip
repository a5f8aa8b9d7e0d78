// Parametrization and optimizer step (supplement S4, Parametrization and Model Training).
//
// Raw, unconstrained parameters map to the renderer's: o = sigmoid, s_k = exp, q normalised,
// tau = -0.1 + 1.09 sigmoid, eta = sigmoid, centre and colour unchanged.  Angles: the K sector gaps
// are proportional to a_k = sigmoid(raw_k) + 1/(K - 2) and sum to 2 pi, theta_k being their sum
// before k (theta_0 = 0); a_k in (1/(K-2), 1 + 1/(K-2)) keeps every gap below pi.
// One thread per primitive: every row of the SoA arrays is read and written coalesced.
#include "drk_internal.hpp"

#include <math.h>

namespace drk {

constexpr float kTwoPiF = 6.28318530717958647692f;
constexpr float kTauLo = -0.1f, kTauSpan = 1.09f;

__device__ inline float sigmoidf(float x) { return 1.0f / (1.0f + expf(-x)); }

__global__ void __launch_bounds__(256) k_activate(drk_scene raw, drk_scene_out out, int ncol) {
  const int64_t n = raw.n, j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const int K = raw.K;
  for (int c = 0; c < 3; ++c) out.mu[c * n + j] = raw.mu[c * n + j];
  float q[4], qq = 0.0f;
  for (int c = 0; c < 4; ++c) { q[c] = raw.q[c * n + j]; qq = fmaf(q[c], q[c], qq); }
  const float iq = 1.0f / sqrtf(qq);
  for (int c = 0; c < 4; ++c) out.q[c * n + j] = q[c] * iq;
  for (int k = 0; k < K; ++k) out.scale[k * n + j] = expf(raw.scale[k * n + j]);
  const float r = 1.0f / (float)(K - 2);
  float a[kMaxK], S = 0.0f;
  for (int k = 0; k < K; ++k) { a[k] = sigmoidf(raw.theta[k * n + j]) + r; S += a[k]; }
  const float f = kTwoPiF / S;
  float C = 0.0f;
  for (int k = 0; k < K; ++k) { out.theta[k * n + j] = f * C; C += a[k]; }
  out.eta[j] = sigmoidf(raw.eta[j]);
  out.tau[j] = fmaf(kTauSpan, sigmoidf(raw.tau[j]), kTauLo);
  out.opacity[j] = sigmoidf(raw.opacity[j]);
  for (int c = 0; c < ncol; ++c) out.color[c * n + j] = raw.color[c * n + j];
}

// dL/d(raw) from dL/d(activated) (same shapes), recomputing the activation's intermediates.
__global__ void __launch_bounds__(256) k_activate_bwd(drk_scene raw, drk_scene_grad g, drk_scene_out out, int ncol) {
  const int64_t n = raw.n, j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const int K = raw.K;
  for (int c = 0; c < 3; ++c) out.mu[c * n + j] = g.mu[c * n + j];
  // q = p / |p|: dp = (dq - q (q . dq)) / |p|
  float p[4], pp = 0.0f, dq[4];
  for (int c = 0; c < 4; ++c) { p[c] = raw.q[c * n + j]; pp = fmaf(p[c], p[c], pp); dq[c] = g.q[c * n + j]; }
  const float ip = 1.0f / sqrtf(pp);
  float qd = 0.0f;
  for (int c = 0; c < 4; ++c) qd = fmaf(p[c] * ip, dq[c], qd);
  for (int c = 0; c < 4; ++c) out.q[c * n + j] = (dq[c] - p[c] * ip * qd) * ip;
  for (int k = 0; k < K; ++k) out.scale[k * n + j] = g.scale[k * n + j] * expf(raw.scale[k * n + j]);
  // theta_k = 2 pi C_k / S: d a_j = (2 pi / S) (sum_{k > j} dtheta_k - sum_k dtheta_k C_k / S)
  const float r = 1.0f / (float)(K - 2);
  float sg[kMaxK], S = 0.0f;
  for (int k = 0; k < K; ++k) { sg[k] = sigmoidf(raw.theta[k * n + j]); S += sg[k] + r; }
  float dot = 0.0f, C = 0.0f;
  for (int k = 0; k < K; ++k) { dot = fmaf(g.theta[k * n + j], C, dot); C += sg[k] + r; }
  const float f = kTwoPiF / S, mean = dot / S;
  float tail = 0.0f;
  for (int k = K - 1; k >= 0; --k) {
    out.theta[k * n + j] = f * (tail - mean) * sg[k] * (1.0f - sg[k]);
    tail += g.theta[k * n + j];
  }
  const float se = sigmoidf(raw.eta[j]), st = sigmoidf(raw.tau[j]), so = sigmoidf(raw.opacity[j]);
  out.eta[j] = g.eta[j] * se * (1.0f - se);
  out.tau[j] = g.tau[j] * kTauSpan * st * (1.0f - st);
  out.opacity[j] = g.opacity[j] * so * (1.0f - so);
  for (int c = 0; c < ncol; ++c) out.color[c * n + j] = g.color[c * n + j];
}

// Adam (bias-corrected), one element per lane, grid-stride.
__global__ void __launch_bounds__(256) k_adam(float* __restrict__ p, float* __restrict__ m, float* __restrict__ v,
                                              const float* __restrict__ g, int64_t n, float lr, float b1, float b2,
                                              float eps, float c1, float c2) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const float gi = g[i];
    const float mi = fmaf(b1, m[i], (1.0f - b1) * gi);
    const float vi = fmaf(b2, v[i], (1.0f - b2) * gi * gi);
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
  }
}

hipError_t launch_activate(const drk_scene& raw, const drk_scene_out& out, int ncol, hipStream_t s) {
  if (raw.n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_activate, dim3((unsigned)((raw.n + 255) / 256)), dim3(256), 0, s, raw, out, ncol);
  return hipGetLastError();
}

hipError_t launch_activate_bwd(const drk_scene& raw, const drk_scene_grad& g, const drk_scene_out& out, int ncol,
                               hipStream_t s) {
  if (raw.n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_activate_bwd, dim3((unsigned)((raw.n + 255) / 256)), dim3(256), 0, s, raw, g, out, ncol);
  return hipGetLastError();
}

hipError_t launch_adam(float* p, float* m, float* v, const float* g, int64_t n, float lr, float b1, float b2, float eps,
                       int step, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const float c1 = (float)(1.0 / (1.0 - pow((double)b1, (double)step)));
  const float c2 = (float)(1.0 / (1.0 - pow((double)b2, (double)step)));
  int64_t blocks = (n + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(k_adam, dim3((unsigned)blocks), dim3(256), 0, s, p, m, v, g, n, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}

}  // namespace drk
