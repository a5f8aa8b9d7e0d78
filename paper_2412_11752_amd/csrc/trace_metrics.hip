// Sorting-accuracy measures of recorded front-to-back traces (supplement, cache-sorting
// evaluation: accuracy, Kendall's tau and MAE of the composited depths against their sorted order).
//
// One wave64 per pixel, lane i holding the i-th recorded depth (at most 64).  The stable rank of
// each depth places it in the sorted sequence (through LDS); a position is correct when it holds
// the depth the sorted sequence holds there; Kendall's tau counts concordant minus discordant
// pairs (ties count as neither) over m (m - 1) / 2.  Per-block sums go to the six outputs with
// float64 atomics.
#include "drk_internal.hpp"

namespace drk {

constexpr int kMetricWaves = 4;

__global__ void __launch_bounds__(64 * kMetricWaves) k_trace_metrics(const int32_t* __restrict__ trace_n,
                                                                  const float* __restrict__ trace_z, int64_t npx,
                                                                  int cap, double* __restrict__ out) {
  __shared__ float sorted[kMetricWaves][64];
  __shared__ double part[kMetricWaves][6];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t p = (int64_t)blockIdx.x * kMetricWaves + w;
  const int n = p < npx ? trace_n[p] : 0;
  const int m = n < cap ? n : cap;
  const bool on = lane < m;
  const float z = on ? trace_z[p * cap + lane] : 0.0f;
  int rank = 0, cd = 0;
  for (int k = 0; k < m; ++k) {
    const float zk = __shfl(z, k, 64);
    rank += (zk < z || (zk == z && k < lane)) ? 1 : 0;
    if (k > lane) cd += (zk > z) ? 1 : ((zk < z) ? -1 : 0);
  }
  if (on) sorted[w][rank] = z;
  __syncthreads();
  const float zs = on ? sorted[w][lane] : 0.0f;
  double v_ok = (on && zs == z) ? 1.0 : 0.0;
  double v_err = on ? (double)fabsf(z - zs) : 0.0;
  double v_cd = (double)cd;
  for (int o = 32; o > 0; o >>= 1) {
    v_ok += __shfl_xor(v_ok, o, 64);
    v_err += __shfl_xor(v_err, o, 64);
    v_cd += __shfl_xor(v_cd, o, 64);
  }
  if (lane == 0) {
    part[w][0] = (double)m;
    part[w][1] = v_ok;
    part[w][2] = m >= 2 ? v_cd / (0.5 * (double)m * (double)(m - 1)) : 0.0;
    part[w][3] = m >= 2 ? 1.0 : 0.0;
    part[w][4] = v_err;
    part[w][5] = n > cap ? 1.0 : 0.0;
  }
  __syncthreads();
  if (threadIdx.x < 6) {
    double acc = 0.0;
    for (int i = 0; i < kMetricWaves; ++i) acc += part[i][threadIdx.x];
    if (acc != 0.0) atomicAdd(out + threadIdx.x, acc);
  }
}

__global__ void k_zero6(double* out) {
  if (threadIdx.x < 6) out[threadIdx.x] = 0.0;
}

hipError_t launch_trace_metrics(const int32_t* trace_n, const float* trace_z, int64_t npx, int cap, double* out,
                                hipStream_t s) {
  hipLaunchKernelGGL(k_zero6, dim3(1), dim3(64), 0, s, out);
  if (npx > 0)
    hipLaunchKernelGGL(k_trace_metrics, dim3((unsigned)((npx + kMetricWaves - 1) / kMetricWaves)), dim3(64 * kMetricWaves),
                       0, s, trace_n, trace_z, npx, cap, out);
  return hipGetLastError();
}

}  // namespace drk
