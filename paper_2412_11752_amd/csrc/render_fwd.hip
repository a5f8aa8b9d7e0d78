// Forward DRK raster (Eq. 1; Sec. 3.3; Sec. 4.1-4.4; Algorithm 1 of the supplement).
//
// One 256-lane workgroup (four wave64s) per 16x16 tile; lane = pixel.  The tile's primitive list
// (ordered by centre depth) is streamed through LDS in rounds of fwd_round(K) records loaded with
// coalesced float4 reads.  Every lane evaluates every staged primitive at its pixel whose box
// reaches its wave's pixels; contributors enter the per-pixel sorted cache (keys in VGPRs,
// payloads in LDS slots), the popped head is composited front to back, and a pixel stops when its
// transmittance would drop below T_min.  The workgroup leaves the list as soon as all 256 pixels
// are done.  The exact-order kernel below keeps rounds of kBatch records.
#include "raster_common.hpp"

#include <type_traits>

namespace drk {

// Output variants: MODE 0 colour only; MODE 1 (trace) also records, per pixel, the primitive index
// and hit depth of its first trace_cap composited contributions (and their count), for the
// sorting-accuracy measures; MODE 2 also blends the hit depth and the plane normal with the
// colour's weights into the depth and normal channels (aux0 = trace_n or depth, aux1 = trace_idx,
// aux2 = trace_z or normal).
constexpr int kFwdPlain = 0, kFwdTrace = 1, kFwdDepthNormal = 2;


// Cache of the forward raster (Sec. 4.4 Cache Sorting, Algorithm 1) with its payloads in LDS.
// Registers hold the kMaxCache keys in order and one word of 4-bit slot ids: nibble j names the LDS
// slot that holds the (alpha, primitive index) of the entry at order position j.  An insertion
// moves keys and one id word instead of keys and two payload arrays, and writes the newcomer's
// payload into the slot of the popped head.  The head's payload is also kept in registers, so an
// emission reads no LDS.  Same entries, same order and same ties as Cache<2>.
struct CacheSlots {
  float key[kMaxCache];
  uint32_t ids;
  float head_a;
  uint32_t head_i;
  uint2* slots;       // this lane's slots, kBlock apart

  __device__ __forceinline__ void init(int cache_len, uint2* lds_slots, int tid) {
#pragma unroll
    for (int s = 0; s < kMaxCache; ++s) key[s] = (s < cache_len) ? -INFINITY : INFINITY;
    ids = 0x76543210u;
    head_a = 0.0f;
    head_i = 0u;
    slots = lds_slots + tid;
#pragma unroll
    for (int s = 0; s < kMaxCache; ++s) slots[s * kBlock] = make_uint2(0u, 0u);
  }
  __device__ __forceinline__ uint2 at_position(int j) const {
    return slots[((ids >> (4 * j)) & 0xFu) * kBlock];
  }
  __device__ __forceinline__ float key_at(int j) const { return key[j]; }
  // Drops position 0 and inserts (z; a, idx) after every key <= z (the caller has read the head).
  __device__ __forceinline__ void pop_insert(float z, float a, uint32_t idx) {
    static_assert(kMaxCache == 8, "eight 4-bit slot ids in one word");
    bool b[kMaxCache - 1];
    uint32_t p = 0;
#pragma unroll
    for (int j = 0; j < kMaxCache - 1; ++j) {
      b[j] = key[j + 1] <= z;
      p += b[j] ? 1u : 0u;
    }
    key[0] = b[0] ? key[1] : z;
#pragma unroll
    for (int j = 1; j < kMaxCache - 1; ++j) key[j] = b[j] ? key[j + 1] : (b[j - 1] ? z : key[j]);
    key[kMaxCache - 1] = b[kMaxCache - 2] ? z : key[kMaxCache - 1];
    // positions < p take the ids of positions 1..p, position p the freed slot, the rest stay
    const uint32_t freed = ids & 0xFu;
    slots[freed * kBlock] = make_uint2(__float_as_uint(a), idx);
    const uint32_t sh = 4u * p;
    const uint32_t low = (1u << sh) - 1u;
    const uint32_t t = (ids & ~(0xFu << sh)) | (freed << sh);
    ids = (t & ~low) | ((ids >> 4) & low);
    if (p == 0) {
      head_a = a;
      head_i = idx;
    } else {
      const uint2 h = slots[(ids & 0xFu) * kBlock];
      head_a = __uint_as_float(h.x);
      head_i = h.y;
    }
  }
};

// The register cache (Cache<2>: keys, alphas and indices in VGPRs) behind the same interface, for
// the depth / normal variant: it carries more per-pixel state, so its occupancy is bound by VGPRs
// rather than LDS, and it keeps rounds of kBatch records.
struct CacheRegs {
  Cache<2> c;
  float head_a;
  uint32_t head_i;
  __device__ __forceinline__ void init(int cache_len, uint2*, int) {
    c.init(cache_len);
    head_a = 0.0f;
    head_i = 0u;
  }
  __device__ __forceinline__ uint2 at_position(int j) const {
    return make_uint2(__float_as_uint(c.pay[0][j]), __float_as_uint(c.pay[1][j]));
  }
  __device__ __forceinline__ float key_at(int j) const { return c.key[j]; }
  __device__ __forceinline__ void pop_insert(float z, float a, uint32_t idx) {
    const float x2[2] = {a, __uint_as_float(idx)};
    c.pop_insert(z, x2);
    head_a = c.pay[0][0];
    head_i = __float_as_uint(c.pay[1][0]);
  }
};

// Records staged per round by the colour and trace rasters: as many as keep a workgroup's LDS
// (records and their indices, the cache slots above, the exit flags) within 20 KB, so that 8
// workgroups of 256 lanes (8 waves per SIMD) fit on a CU: 10 records of K = 8, 6 of K = 16, at
// most 16.
constexpr int fwd_round(int K) {
  constexpr int kFree = 20480 - kMaxCache * kBlock * (int)sizeof(uint2) - 2 * (int)sizeof(uint32_t);
  return kFree / (rec_floats(K) * 4 + 4) > 16 ? 16 : kFree / (rec_floats(K) * 4 + 4);
}

template <int MODE, int K>
struct FwdCfg {
  static constexpr bool kSlots = MODE != 2;
  static constexpr int kRound = kSlots ? fwd_round(K) : kBatch;
  using CacheT = typename std::conditional<kSlots, CacheSlots, CacheRegs>::type;
};

// COUNT: also write the per-pixel work counters (instrumentation; the production launch of MODE 0
// leaves them out).
template <int K, int MODE, bool COUNT>
__global__ void __launch_bounds__(kBlock) k_render_fwd(const float* __restrict__ records, const uint32_t* __restrict__ ranges,
                                                       const uint32_t* __restrict__ prims, const CamDev* __restrict__ camp,
                                                       const uint32_t* __restrict__ tile_order, OptsDev opt,
                                                       float* __restrict__ rgb, float* __restrict__ T_out,
                                                       int32_t* __restrict__ n_emit_out,
                                                       int32_t* __restrict__ consumed_out,
                                                       int32_t* __restrict__ contrib_out,
                                                       int32_t* __restrict__ work_out,
                                                       void* __restrict__ aux0, int32_t* __restrict__ aux1,
                                                       float* __restrict__ aux2, int trace_cap) {
  constexpr bool TRACE = MODE == kFwdTrace;
  constexpr bool GEOM = MODE == kFwdDepthNormal;
  int32_t* trace_n = TRACE ? static_cast<int32_t*>(aux0) : nullptr;
  int32_t* trace_idx = aux1;
  float* trace_z = aux2;
  constexpr int RF = (R_SEC + S_NFIELDS * K + 3) & ~3;
  constexpr int RF4 = RF / 4;
  constexpr int kRound = FwdCfg<MODE, K>::kRound;
  __shared__ float4 lds[kRound * RF4];
  __shared__ uint32_t lidx[kRound];
  __shared__ uint2 s_slots[FwdCfg<MODE, K>::kSlots ? kMaxCache * kBlock : 1];
  __shared__ uint32_t s_live[2];   // round r sets s_live[r & 1] when a pixel is still compositing
  const CamDev& cam = *camp;
  const int tile = tile_order ? (int)tile_order[blockIdx.x] : (int)blockIdx.x;   // launch order
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
  const size_t trace_base = TRACE && inside ? ((size_t)y * cam.W + x) * (size_t)trace_cap : 0;

  float T = 1.0f, C0 = 0.0f, C1 = 0.0f, C2 = 0.0f;
  float Dz = 0.0f, N0 = 0.0f, N1 = 0.0f, N2 = 0.0f;   // depth / normal channels (MODE 2)
  int n_emit = 0, n_contrib = 0, n_hit = 0, n_full = 0;
  int consumed = (int)(end - start);
  bool done = !inside;
  // cache payload: (alpha, primitive index); the colour is gathered from the record at emission
  typename FwdCfg<MODE, K>::CacheT cache;
  cache.init(rp.cache_len, s_slots, tid);
  if (tid < 2) s_live[tid] = 0u;

  // The workgroup leaves the list once no pixel is compositing.  The waves of round r set
  // s_live[r & 1] after their evaluations; round r + 1 reads it after the end-of-round barrier, and
  // thread 0 clears it again after round r + 1's staging barrier (it is next set in round r + 2).
  uint32_t round = 0;
  for (uint32_t b0 = start; b0 < end; b0 += kRound, ++round) {
    if (round > 0 && s_live[(round - 1) & 1u] == 0u) break;
    const int nb = (int)min((uint32_t)kRound, end - b0);
    for (int q = tid; q < nb * RF4; q += kBlock) {
      const int ri = q / RF4, c = q - ri * RF4;
      const uint32_t j = prims[b0 + ri];
      lds[q] = reinterpret_cast<const float4*>(records + (size_t)j * RF)[c];
    }
    if (tid < nb) lidx[tid] = prims[b0 + tid];
    __syncthreads();
    if (tid == 0 && round > 0) s_live[(round - 1) & 1u] = 0u;
    const uint64_t mask = batch_box_mask<RF4>(lds, nb, wx0, wx1, wy0, wy1);
    // one exit for the loop (the mask); a pixel that stops only leaves the rest of the round's steps
    for (uint64_t m = mask; m; m &= m - 1) {
      if (done) continue;
      const int i = __builtin_ctzll(m);
      const float* r = reinterpret_cast<const float*>(lds + i * RF4);
      if constexpr (COUNT) ++n_hit;
      float at, Z;
      if (!drk_eval<K, MODE == kFwdDepthNormal>(r, pix, rp, at, Z)) continue;
      if constexpr (COUNT) ++n_full;
      if (at >= rp.alpha_min) {
        if constexpr (COUNT) ++n_contrib;
        // pop the head (emit it), then insert the newcomer
        const float a = cache.head_a;
        if (a > 0.0f) {
          const float test = T * (1.0f - a);
          if (test < rp.T_min) {
            done = true;
            if constexpr (COUNT) consumed = (int)(b0 - start) + i + 1;
            continue;
          }
          const float* c = records + (size_t)cache.head_i * RF + R_RGB;
          const float w = a * T;
          C0 = fmaf(w, c[0], C0);
          C1 = fmaf(w, c[1], C1);
          C2 = fmaf(w, c[2], C2);
          T = test;
          if constexpr (TRACE) {
            if (n_emit < trace_cap) {
              trace_idx[trace_base + n_emit] = (int32_t)cache.head_i;
              trace_z[trace_base + n_emit] = cache.key_at(0);
            }
          }
          if constexpr (GEOM) {
            const float* nr = c - R_RGB + R_NRM;
            Dz = fmaf(w, cache.key_at(0), Dz);
            N0 = fmaf(w, nr[0], N0);
            N1 = fmaf(w, nr[1], N1);
            N2 = fmaf(w, nr[2], N2);
          }
          ++n_emit;
        }
        cache.pop_insert(Z, at, lidx[i]);
      }
    }
    const bool live = __ballot(!done) != 0ull;
    if ((tid & 63) == 0 && live) s_live[round & 1u] = 1u;
    __syncthreads();
  }
  if (!done) {
#pragma unroll
    for (int s = 0; s < kMaxCache; ++s) {
      const uint2 e = cache.at_position(s);
      const float a = __uint_as_float(e.x);
      if (!done && a > 0.0f) {
        const float test = T * (1.0f - a);
        if (test < rp.T_min) {
          done = true;
        } else {
          const float* c = records + (size_t)e.y * RF + R_RGB;
          const float w = a * T;
          C0 = fmaf(w, c[0], C0);
          C1 = fmaf(w, c[1], C1);
          C2 = fmaf(w, c[2], C2);
          T = test;
          if constexpr (TRACE) {
            if (n_emit < trace_cap) {
              trace_idx[trace_base + n_emit] = (int32_t)e.y;
              trace_z[trace_base + n_emit] = cache.key_at(s);
            }
          }
          if constexpr (GEOM) {
            const float* nr = c - R_RGB + R_NRM;
            Dz = fmaf(w, cache.key_at(s), Dz);
            N0 = fmaf(w, nr[0], N0);
            N1 = fmaf(w, nr[1], N1);
            N2 = fmaf(w, nr[2], N2);
          }
          ++n_emit;
        }
      }
    }
  }
  if (inside) {
    const size_t plane = (size_t)cam.W * cam.H;
    const size_t pidx = (size_t)y * cam.W + x;
    rgb[pidx] = fmaf(T, cam.bg[0], C0);
    rgb[plane + pidx] = fmaf(T, cam.bg[1], C1);
    rgb[2 * plane + pidx] = fmaf(T, cam.bg[2], C2);
    if (T_out) T_out[pidx] = T;
    if constexpr (COUNT) {
      n_emit_out[pidx] = n_emit;
      consumed_out[pidx] = consumed;
      contrib_out[pidx] = n_contrib;
      work_out[pidx] = n_hit;               // entries whose hit was evaluated (wave box passed)
      work_out[plane + pidx] = n_full;      // entries that went through the full kernel
    }
    if constexpr (TRACE) trace_n[pidx] = n_emit;
    if constexpr (GEOM) {
      static_cast<float*>(aux0)[pidx] = Dz;
      aux2[pidx] = N0;
      aux2[plane + pidx] = N1;
      aux2[2 * plane + pidx] = N2;
    }
  }
}

// Exact per-pixel order (cache_len >= 2^30): every contribution of the tile's list composited in
// the order of its hit depth Z (ties by primitive index), with the same stop rule, i.e. the ideal
// order the cache of Algorithm 1 approximates.  Each pass over the list gathers, per pixel, the
// kExactChunk contributions nearest behind the last one composited, in a sorted register buffer of
// (Z, index, alpha) that keeps the smallest, and composites them; passes repeat until every pixel of
// the tile has stopped or has no contribution left.  A pass cannot end early, so the cost is about
// one full list scan per kExactChunk composited contributions.
constexpr int kExactChunk = 8;

template <int K>
__global__ void __launch_bounds__(kBlock) k_render_exact(const float* __restrict__ records,
                                                         const uint32_t* __restrict__ ranges,
                                                         const uint32_t* __restrict__ prims,
                                                         const CamDev* __restrict__ camp,
                                                         const uint32_t* __restrict__ tile_order, OptsDev opt,
                                                         float* __restrict__ rgb, float* __restrict__ T_out) {
  constexpr int RF = (R_SEC + S_NFIELDS * K + 3) & ~3;
  constexpr int RF4 = RF / 4;
  __shared__ float4 lds[kBatch * RF4];
  __shared__ uint32_t lidx[kBatch];
  const CamDev& cam = *camp;
  const int tile = tile_order ? (int)tile_order[blockIdx.x] : (int)blockIdx.x;
  const int tx = tile % cam.tiles_x, ty = tile / cam.tiles_x;
  const int tid = threadIdx.x;
  const int x = tx * kTile + (tid & (kTile - 1));
  const int y = ty * kTile + (tid >> 4);
  const bool inside = x < cam.W && y < cam.H;
  const RasterParams rp = make_params(opt);
  const Pix pix = make_pix(cam, x, y);
  const float wx0 = (float)(tx * kTile) + 0.5f, wx1 = wx0 + (float)(kTile - 1);
  const float wy0 = (float)(ty * kTile + (tid >> 6) * 4) + 0.5f, wy1 = wy0 + 3.0f;
  const uint32_t start = ranges[2 * tile], end = ranges[2 * tile + 1];
  float T = 1.0f, C0 = 0.0f, C1 = 0.0f, C2 = 0.0f;
  bool done = !inside;
  float last_z = -INFINITY;         // (Z, index) of the last composited contribution
  uint32_t last_j = 0;
  bool have_last = false;
  while (__syncthreads_count(!done) != 0) {
    float bz[kExactChunk], ba[kExactChunk];
    uint32_t bj[kExactChunk];
#pragma unroll
    for (int s = 0; s < kExactChunk; ++s) { bz[s] = INFINITY; bj[s] = 0xFFFFFFFFu; ba[s] = 0.0f; }
    for (uint32_t b0 = start; b0 < end; b0 += kBatch) {
      const int nb = (int)min((uint32_t)kBatch, end - b0);
      for (int q = tid; q < nb * RF4; q += kBlock) {
        const int ri = q / RF4, c = q - ri * RF4;
        lds[q] = reinterpret_cast<const float4*>(records + (size_t)prims[b0 + ri] * RF)[c];
      }
      if (tid < nb) lidx[tid] = prims[b0 + tid];
      __syncthreads();
      const uint64_t mask = batch_box_mask<RF4>(lds, nb, wx0, wx1, wy0, wy1);
      if (!done) {
        for (uint64_t m = mask; m; m &= m - 1) {
          const int i = __builtin_ctzll(m);
          float at, Z;
          if (!drk_eval<K>(reinterpret_cast<const float*>(lds + i * RF4), pix, rp, at, Z)) continue;
          if (!(at >= rp.alpha_min)) continue;
          const uint32_t j = lidx[i];
          if (have_last && !(Z > last_z || (Z == last_z && j > last_j))) continue;   // already composited
          // lt[s]: the newcomer goes before slot s (monotone in s, the buffer being sorted)
          bool lt[kExactChunk];
#pragma unroll
          for (int s = 0; s < kExactChunk; ++s) lt[s] = Z < bz[s] || (Z == bz[s] && j < bj[s]);
          if (!lt[kExactChunk - 1]) continue;
#pragma unroll
          for (int s = kExactChunk - 1; s > 0; --s) {
            bz[s] = lt[s - 1] ? bz[s - 1] : (lt[s] ? Z : bz[s]);
            bj[s] = lt[s - 1] ? bj[s - 1] : (lt[s] ? j : bj[s]);
            ba[s] = lt[s - 1] ? ba[s - 1] : (lt[s] ? at : ba[s]);
          }
          bz[0] = lt[0] ? Z : bz[0];
          bj[0] = lt[0] ? j : bj[0];
          ba[0] = lt[0] ? at : ba[0];
        }
      }
      __syncthreads();
    }
    int got = 0;
#pragma unroll
    for (int s = 0; s < kExactChunk; ++s) {
      if (!done && bj[s] != 0xFFFFFFFFu) {
        ++got;
        const float a = ba[s];
        const float test = T * (1.0f - a);
        if (test < rp.T_min) {
          done = true;
        } else {
          const float* c = records + (size_t)bj[s] * RF + R_RGB;
          const float w = a * T;
          C0 = fmaf(w, c[0], C0);
          C1 = fmaf(w, c[1], C1);
          C2 = fmaf(w, c[2], C2);
          T = test;
          last_z = bz[s];
          last_j = bj[s];
          have_last = true;
        }
      }
    }
    if (got < kExactChunk) done = true;   // nothing behind: the list is exhausted for this pixel
  }
  if (inside) {
    const size_t plane = (size_t)cam.W * cam.H;
    const size_t pidx = (size_t)y * cam.W + x;
    rgb[pidx] = fmaf(T, cam.bg[0], C0);
    rgb[plane + pidx] = fmaf(T, cam.bg[1], C1);
    rgb[2 * plane + pidx] = fmaf(T, cam.bg[2], C2);
    if (T_out) T_out[pidx] = T;
  }
}

template <int K>
static hipError_t launch_fwd_k(const float* records, const uint32_t* ranges, const uint32_t* prims, const CamDev* cam,
                               int ntiles, const uint32_t* order, const OptsDev& opt, float* rgb, float* T, int32_t* ne, int32_t* cons, int32_t* nc,
                               int32_t* wk, int mode, void* a0, int32_t* a1, float* a2, int cap, hipStream_t s) {
  if (opt.cache_len >= kExactOrder) {
    if (mode != kFwdPlain) return hipErrorInvalidValue;   // exact order: colour and transmittance only
    hipLaunchKernelGGL((k_render_exact<K>), dim3(ntiles), dim3(kBlock), 0, s, records, ranges, prims, cam, order, opt,
                       rgb, T);
  } else if (mode == kFwdTrace)
    hipLaunchKernelGGL((k_render_fwd<K, kFwdTrace, true>), dim3(ntiles), dim3(kBlock), 0, s, records, ranges, prims, cam, order,
                       opt, rgb, T, ne, cons, nc, wk, a0, a1, a2, cap);
  else if (mode == kFwdDepthNormal)
    hipLaunchKernelGGL((k_render_fwd<K, kFwdDepthNormal, true>), dim3(ntiles), dim3(kBlock), 0, s, records, ranges, prims,
                       cam, order, opt, rgb, T, ne, cons, nc, wk, a0, nullptr, a2, 0);
  else if (opt.counters)
    hipLaunchKernelGGL((k_render_fwd<K, kFwdPlain, true>), dim3(ntiles), dim3(kBlock), 0, s, records, ranges, prims, cam,
                       order, opt, rgb, T, ne, cons, nc, wk, nullptr, nullptr, nullptr, 0);
  else
    hipLaunchKernelGGL((k_render_fwd<K, kFwdPlain, false>), dim3(ntiles), dim3(kBlock), 0, s, records, ranges, prims, cam,
                       order, opt, rgb, T, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, 0);
  return hipGetLastError();
}

// mode 0: colour only (per-pixel counters when opt.counters); 1: trace (a0 = counts, a1 = indices,
// a2 = depths, cap entries per pixel); 2: depth (a0) and normal (a2) channels.  Modes 1 and 2 always
// write the counters.  Pointers are those of this view.
hipError_t launch_render_fwd(int K, const float* records, const uint32_t* ranges, const uint32_t* prims,
                             const CamDev* cam, int ntiles, const uint32_t* order, const OptsDev& opt, float* rgb, float* T, int32_t* ne, int32_t* cons,
                             int32_t* nc, int32_t* wk, int mode, void* a0, int32_t* a1, float* a2, int cap, hipStream_t s) {
  switch (K) {
#define DRK_CASE(k) \
  case k: return launch_fwd_k<k>(records, ranges, prims, cam, ntiles, order, opt, rgb, T, ne, cons, nc, wk, mode, a0, a1, a2, cap, s);
    DRK_CASE(3) DRK_CASE(4) DRK_CASE(5) DRK_CASE(6) DRK_CASE(7) DRK_CASE(8) DRK_CASE(9) DRK_CASE(10)
    DRK_CASE(11) DRK_CASE(12) DRK_CASE(13) DRK_CASE(14) DRK_CASE(15) DRK_CASE(16)
#undef DRK_CASE
    default: return hipErrorInvalidValue;
  }
}

}  // namespace drk
