// Mesh to DRK (the section "Converting Mesh to DRK" and its supplement): one DRK per planar convex
// face, basis endpoints at the vertices, no optimisation.  One thread per face, float64.
//
// The level: with eta = 1 the energy is r1^2 (Eq. L1), whose level sets are the polygons through
// s_k e_k scaled by r1; placing the vertices at r1 = sqrt(2 ln 2) gives g = exp(-E/2) = 1/2 there,
// and Psi(1/2) = 1/2 for every tau (Sec. 4.3), so the face outline is the alpha = o/2 contour and
// tau sets how sharply alpha falls across it.
#include "drk_internal.hpp"

#include <math.h>

namespace drk {

constexpr double kTwoPiM = 6.283185307179586;
constexpr double kPiM = 3.141592653589793;
constexpr double kMeshLevel = 1.1774100225154747;   // sqrt(2 ln 2)

__device__ inline void cross3d(const double a[3], const double b[3], double o[3]) {
  o[0] = a[1] * b[2] - a[2] * b[1];
  o[1] = a[2] * b[0] - a[0] * b[2];
  o[2] = a[0] * b[1] - a[1] * b[0];
}

// (w, x, y, z) of the rotation with columns t_u, t_v, n (Shepperd's method: the largest of
// 1 + trace and 1 + 2 R_ii - trace under the square root).
__device__ inline void quat_from_frame(const double tu[3], const double tv[3], const double n[3], double q[4]) {
  const double R[3][3] = {{tu[0], tv[0], n[0]}, {tu[1], tv[1], n[1]}, {tu[2], tv[2], n[2]}};
  const double t = R[0][0] + R[1][1] + R[2][2];
  if (t > 0.0) {
    const double r = sqrt(1.0 + t);
    q[0] = 0.5 * r;
    q[1] = (R[2][1] - R[1][2]) / (2.0 * r);
    q[2] = (R[0][2] - R[2][0]) / (2.0 * r);
    q[3] = (R[1][0] - R[0][1]) / (2.0 * r);
    return;
  }
  int i = 0;
  if (R[1][1] > R[i][i]) i = 1;
  if (R[2][2] > R[i][i]) i = 2;
  const int j = (i + 1) % 3, k = (i + 2) % 3;
  const double r = sqrt(1.0 + R[i][i] - R[j][j] - R[k][k]);
  q[0] = (R[k][j] - R[j][k]) / (2.0 * r);
  q[1 + i] = 0.5 * r;
  q[1 + j] = (R[j][i] + R[i][j]) / (2.0 * r);
  q[1 + k] = (R[k][i] + R[i][k]) / (2.0 * r);
}

__global__ void __launch_bounds__(128) k_mesh_to_drk(const float* __restrict__ V, int64_t nv, const int32_t* __restrict__ F,
                                                     int64_t nf, int m, const float* __restrict__ rgb, int K, float tau,
                                                     float opacity, drk_scene_out out, uint32_t* __restrict__ rejected) {
  const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= nf) return;
  double P[kMaxK][3];
  int mv = 0;
  bool ok = true;
  for (int i = 0; i < m; ++i) {
    const int32_t id = F[f * m + i];
    if (id < 0) break;
    if ((int64_t)id >= nv) { ok = false; break; }
    for (int c = 0; c < 3; ++c) P[mv][c] = (double)V[(int64_t)c * nv + id];
    ++mv;
  }
  ok = ok && mv >= 3;
  double mu[3] = {0.0, 0.0, 0.0}, q[4] = {1.0, 0.0, 0.0, 0.0};
  double th[kMaxK], s[kMaxK];
  if (ok) {
    for (int i = 0; i < mv; ++i)
      for (int c = 0; c < 3; ++c) mu[c] += P[i][c];
    for (int c = 0; c < 3; ++c) mu[c] /= (double)mv;
    for (int i = 0; i < mv; ++i)
      for (int c = 0; c < 3; ++c) P[i][c] -= mu[c];
    // normal of the winding: sum of the cross products of consecutive centred vertices
    double a[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < mv; ++i) {
      double cr[3];
      cross3d(P[i], P[(i + 1) % mv], cr);
      for (int c = 0; c < 3; ++c) a[c] += cr[c];
    }
    const double na = sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
    const double d0 = sqrt(P[0][0] * P[0][0] + P[0][1] * P[0][1] + P[0][2] * P[0][2]);
    ok = na > 0.0 && d0 > 0.0;
    if (ok) {
      double n[3], tu[3], tv[3];
      for (int c = 0; c < 3; ++c) { n[c] = a[c] / na; tu[c] = P[0][c] / d0; }
      cross3d(n, tu, tv);
      double x[kMaxK], y[kMaxK], ang[kMaxK];
      for (int i = 0; i < mv; ++i) {
        x[i] = P[i][0] * tu[0] + P[i][1] * tu[1] + P[i][2] * tu[2];
        y[i] = P[i][0] * tv[0] + P[i][1] * tv[1] + P[i][2] * tv[2];
        double t = atan2(y[i], x[i]);
        ang[i] = i == 0 ? 0.0 : (t < 0.0 ? t + kTwoPiM : t);
      }
      // endpoints of the DRK: the vertices, with the extra endpoints on the edges in between
      const int extra_all = K - mv, base = extra_all / mv, more = extra_all % mv;
      int k = 0;
      double px[kMaxK], py[kMaxK];
      for (int i = 0; i < mv; ++i) {
        const int i1 = (i + 1 == mv) ? 0 : i + 1;
        px[k] = x[i]; py[k] = y[i]; th[k] = ang[i]; ++k;
        const int e = base + (i < more ? 1 : 0);
        for (int c = 1; c <= e; ++c) {
          const double fr = (double)c / (double)(e + 1);
          px[k] = x[i] + fr * (x[i1] - x[i]);
          py[k] = y[i] + fr * (y[i1] - y[i]);
          const double t = atan2(py[k], px[k]);
          th[k] = t < 0.0 ? t + kTwoPiM : t;
          ++k;
        }
      }
      for (int i = 1; i < K; ++i) {
        const double gap = th[i] - th[i - 1];
        ok = ok && gap > 0.0 && gap < kPiM;
      }
      const double wrap = th[0] + kTwoPiM - th[K - 1];
      ok = ok && wrap > 0.0 && wrap < kPiM;
      for (int i = 0; i < K; ++i) s[i] = sqrt(px[i] * px[i] + py[i] * py[i]) / kMeshLevel;
      if (ok) quat_from_frame(tu, tv, n, q);
    }
  }
  if (!ok) {
    mu[0] = mu[1] = mu[2] = 0.0;
    q[0] = 1.0; q[1] = q[2] = q[3] = 0.0;
    for (int i = 0; i < K; ++i) { s[i] = 1.0; th[i] = i * (kTwoPiM / K); }
    if (rejected) atomicAdd(rejected, 1u);
  }
  const float below_two_pi = 6.2831850f;   // largest float32 below 2 pi
  for (int c = 0; c < 3; ++c) out.mu[c * nf + f] = (float)mu[c];
  for (int c = 0; c < 4; ++c) out.q[c * nf + f] = (float)q[c];
  for (int i = 0; i < K; ++i) {
    out.scale[i * nf + f] = (float)s[i];
    out.theta[i * nf + f] = fminf((float)th[i], below_two_pi);
  }
  out.eta[f] = 1.0f;
  out.tau[f] = tau;
  out.opacity[f] = ok ? opacity : 0.0f;
  for (int c = 0; c < 3; ++c) out.color[c * nf + f] = rgb[c * nf + f];
}

__global__ void k_zero_u32(uint32_t* p) { *p = 0u; }

hipError_t launch_mesh_to_drk(const float* V, int64_t nv, const int32_t* F, int64_t nf, int m, const float* rgb, int K,
                              float tau, float opacity, const drk_scene_out& out, uint32_t* rejected, hipStream_t s) {
  if (rejected) hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(1), 0, s, rejected);
  if (nf > 0)
    hipLaunchKernelGGL(k_mesh_to_drk, dim3((unsigned)((nf + 127) / 128)), dim3(128), 0, s, V, nv, F, nf, m, rgb, K, tau,
                       opacity, out, rejected);
  return hipGetLastError();
}

}  // namespace drk
