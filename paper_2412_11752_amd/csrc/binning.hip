// Binning for the DRK rasterizer: stable LSD radix sort (u32 keys, u32 values), exclusive scan of
// per-primitive tile counts, and per-tile ranges.
//
// The sort runs on a fixed grid whose element count is read from device memory, so the host never
// waits for the pair count (the sequence can be captured in a HIP graph).  Block b owns a
// contiguous chunk; each pass is upsweep (per-block digit histogram) -> per-digit scan over blocks
// -> stable scatter.  Within a block the scatter ranks 256 keys per round with wave64 ballots
// (lanes holding the same digit) and a cross-wave prefix in LDS, so equal keys keep input order.
#include "drk_internal.hpp"

namespace drk {

constexpr int kRsThreads = 256;
constexpr int kRsBlocks = 1024;
constexpr int kRsWaves = kRsThreads / 64;

__device__ inline uint64_t chunk_begin(uint64_t n, int b) {
  uint64_t chunk = (n + kRsBlocks - 1) / kRsBlocks;
  uint64_t s = chunk * (uint64_t)b;
  return s < n ? s : n;
}

__global__ void __launch_bounds__(kRsThreads) k_rs_upsweep(const uint32_t* __restrict__ keys, const uint64_t* __restrict__ d_n,
                                                           int shift, uint32_t mask, uint32_t* __restrict__ hist) {
  __shared__ uint32_t h[256];
  const int tid = threadIdx.x, b = blockIdx.x;
  h[tid] = 0;
  __syncthreads();
  const uint64_t n = *d_n;
  const uint64_t s = chunk_begin(n, b), e = chunk_begin(n, b + 1);
  for (uint64_t i = s + tid; i < e; i += kRsThreads) atomicAdd(&h[(keys[i] >> shift) & mask], 1u);
  __syncthreads();
  hist[(size_t)tid * kRsBlocks + b] = h[tid];
}

// One block per digit: exclusive scan of hist[d][0..kRsBlocks) in place, digit total to tot[d].
__global__ void __launch_bounds__(1024) k_rs_scan_rows(uint32_t* __restrict__ hist, uint32_t* __restrict__ tot) {
  __shared__ uint32_t wsum[16];
  const int tid = threadIdx.x, d = blockIdx.x;
  const int lane = tid & 63, w = tid >> 6;
  uint32_t x = hist[(size_t)d * kRsBlocks + tid];
  // inclusive wave scan
  uint32_t inc = x;
  for (int o = 1; o < 64; o <<= 1) {
    uint32_t y = __shfl_up(inc, o, 64);
    if (lane >= o) inc += y;
  }
  if (lane == 63) wsum[w] = inc;
  __syncthreads();
  if (tid < 16) {
    uint32_t v = wsum[tid];
    uint32_t acc = v;
    for (int o = 1; o < 16; o <<= 1) {
      uint32_t y = __shfl_up(acc, o, 16);
      if (tid >= o) acc += y;
    }
    wsum[tid] = acc - v;   // exclusive
    if (tid == 15) tot[d] = acc;
  }
  __syncthreads();
  hist[(size_t)d * kRsBlocks + tid] = inc - x + wsum[w];
}

// Stable scatter of one pass.  A block walks its chunk in tiles of kRsTile keys.  Wave w of a tile
// takes its kRsItems * 64 consecutive keys in rounds of 64 and ranks each key among the equal digits
// of its wave (ballots over the digit bits, a running per-digit count in LDS that the wave alone
// updates), so a key's rank follows input order: wave, then round, then lane.  The tile's digit
// counts are then scanned, the keys are placed in LDS in digit order, and written out from there:
// consecutive threads write consecutive slots of a digit's run, instead of one scattered word each.
constexpr int kRsItems = 8;
constexpr int kRsTile = kRsThreads * kRsItems;

__device__ inline void rs_wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__global__ void __launch_bounds__(kRsThreads) k_rs_scatter(const uint32_t* __restrict__ kin, const uint32_t* __restrict__ vin,
                                                           uint32_t* __restrict__ kout, uint32_t* __restrict__ vout,
                                                           const uint64_t* __restrict__ d_n, int shift, int bits,
                                                           const uint32_t* __restrict__ hist,
                                                           const uint32_t* __restrict__ tot) {
  __shared__ uint32_t base[256];              // global slot of each digit's next key from this block
  __shared__ uint32_t wrun[kRsWaves][256];    // per wave: keys of each digit ranked so far in the tile
  __shared__ uint32_t tstart[256];            // start of each digit's run in the tile
  __shared__ uint32_t part[kRsWaves];
  __shared__ uint32_t sk[kRsTile], sv[kRsTile];
  const int tid = threadIdx.x, b = blockIdx.x;
  const int lane = tid & 63, w = tid >> 6;
  const uint32_t mask = (bits >= 32) ? 0xFFFFFFFFu : ((1u << bits) - 1u);
  // digit bases: exclusive scan of the digit totals + this block's offset inside each digit
  {
    uint32_t x = tot[tid];
    uint32_t inc = x;
    for (int o = 1; o < 64; o <<= 1) {
      uint32_t y = __shfl_up(inc, o, 64);
      if (lane >= o) inc += y;
    }
    if (lane == 63) part[w] = inc;
    __syncthreads();
    uint32_t pre = 0;
    for (int i = 0; i < w; ++i) pre += part[i];
    base[tid] = pre + inc - x + hist[(size_t)tid * kRsBlocks + b];
    for (int i = 0; i < kRsWaves; ++i) wrun[i][tid] = 0;
  }
  __syncthreads();
  const uint64_t n = *d_n;
  const uint64_t s = chunk_begin(n, b), e = chunk_begin(n, b + 1);
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  for (uint64_t t0 = s; t0 < e; t0 += kRsTile) {
    const uint32_t tn = (uint32_t)((e - t0) < (uint64_t)kRsTile ? (e - t0) : (uint64_t)kRsTile);
    uint32_t key[kRsItems], val[kRsItems], pos[kRsItems];
#pragma unroll
    for (int k = 0; k < kRsItems; ++k) {
      const uint32_t li = (uint32_t)(w * kRsItems + k) * 64u + (uint32_t)lane;   // slot in the tile
      const bool valid = li < tn;
      key[k] = 0;
      val[k] = 0;
      pos[k] = 0;
      if ((uint32_t)(w * kRsItems + k) * 64u >= tn) continue;   // the wave's round is past the tile's end
      if (valid) {
        key[k] = kin[t0 + li];
        val[k] = vin ? vin[t0 + li] : (uint32_t)(t0 + li);
      }
      const uint32_t d = (key[k] >> shift) & mask;
      uint64_t peers = __ballot(valid);
      for (int bb = 0; bb < bits; ++bb) {
        const bool set = (d >> bb) & 1u;
        const uint64_t m = __ballot(set);
        peers &= set ? m : ~m;
      }
      const uint32_t rank = (uint32_t)__popcll(peers & lt);
      if (valid) pos[k] = wrun[w][d] + rank;
      rs_wave_sync();
      if (valid && rank == 0) wrun[w][d] += (uint32_t)__popcll(peers);
      rs_wave_sync();
    }
    __syncthreads();
    // per digit (thread tid = digit): the waves' offsets and the tile's run starts
    {
      uint32_t c = 0;
      for (int i = 0; i < kRsWaves; ++i) {
        const uint32_t x = wrun[i][tid];
        wrun[i][tid] = c;        // now the exclusive prefix over the waves
        c += x;
      }
      uint32_t inc = c;
      for (int o = 1; o < 64; o <<= 1) {
        uint32_t y = __shfl_up(inc, o, 64);
        if (lane >= o) inc += y;
      }
      if (lane == 63) part[w] = inc;
      __syncthreads();
      uint32_t pre = 0;
      for (int i = 0; i < w; ++i) pre += part[i];
      tstart[tid] = pre + inc - c;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kRsItems; ++k) {
      const uint32_t li = (uint32_t)(w * kRsItems + k) * 64u + (uint32_t)lane;
      if (li < tn) {
        const uint32_t d = (key[k] >> shift) & mask;
        const uint32_t at = tstart[d] + wrun[w][d] + pos[k];
        sk[at] = key[k];
        sv[at] = val[k];
      }
    }
    __syncthreads();
    for (uint32_t i = (uint32_t)tid; i < tn; i += kRsThreads) {
      const uint32_t k = sk[i];
      const uint32_t d = (k >> shift) & mask;
      const uint32_t at = base[d] + (i - tstart[d]);
      kout[at] = k;
      vout[at] = sv[i];
    }
    __syncthreads();
    {
      // advance the digit bases by the tile's counts (next run start minus this one)
      const uint32_t next = (tid + 1 < 256) ? tstart[tid + 1] : tn;
      base[tid] += next - tstart[tid];
      for (int i = 0; i < kRsWaves; ++i) wrun[i][tid] = 0;
    }
    __syncthreads();
  }
}

// Stable sort of n (device) pairs by key bits [0, key_bits).  Pass p reads bufs[p] and writes
// bufs[p + 1]; bufs must hold passes + 1 entries.  vin of the first pass may be null (value = index).
hipError_t radix_sort(int key_bits, const uint64_t* d_n, uint32_t* const* kbufs, uint32_t* const* vbufs, int nbufs,
                      uint32_t* hist, uint32_t* tot, hipStream_t s) {
  const int passes = (key_bits + 7) / 8;
  // pass p reads buffer p and writes buffer p + 1
  if (key_bits < 1 || key_bits > 32 || passes + 1 > nbufs) return hipErrorInvalidValue;
  for (int p = 0; p < passes; ++p) {
    const int shift = 8 * p;
    const int bits = (key_bits - shift) < 8 ? (key_bits - shift) : 8;
    const uint32_t mask = (1u << bits) - 1u;
    hipLaunchKernelGGL(k_rs_upsweep, dim3(kRsBlocks), dim3(kRsThreads), 0, s, kbufs[p], d_n, shift, mask, hist);
    hipLaunchKernelGGL(k_rs_scan_rows, dim3(256), dim3(1024), 0, s, hist, tot);
    hipLaunchKernelGGL(k_rs_scatter, dim3(kRsBlocks), dim3(kRsThreads), 0, s, kbufs[p], vbufs[p], kbufs[p + 1],
                       vbufs[p + 1], d_n, shift, bits, hist, tot);
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------------
// Exclusive scan of tile counts gathered in depth order: offsets[i] = sum_{i' < i} counts[prim[i']].
constexpr int kScanItems = 4;
constexpr int kScanBlock = 256 * kScanItems;

__global__ void __launch_bounds__(256) k_scan_local(const uint32_t* __restrict__ prims, const uint32_t* __restrict__ counts,
                                                    const uint64_t* __restrict__ d_n, uint32_t* __restrict__ offsets,
                                                    uint64_t* __restrict__ block_tot) {
  __shared__ uint64_t part[4];
  const int64_t n = (int64_t)*d_n;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int64_t base = (int64_t)blockIdx.x * kScanBlock + (int64_t)tid * kScanItems;
  uint32_t c[kScanItems];
  uint64_t sum = 0;
  for (int i = 0; i < kScanItems; ++i) {
    c[i] = (base + i < n) ? counts[prims[base + i]] : 0u;
    sum += c[i];
  }
  uint64_t inc = sum;
  for (int o = 1; o < 64; o <<= 1) {
    uint64_t y = __shfl_up(inc, o, 64);
    if (lane >= o) inc += y;
  }
  if (lane == 63) part[w] = inc;
  __syncthreads();
  uint64_t pre = 0;
  for (int i = 0; i < w; ++i) pre += part[i];
  uint64_t run = pre + inc - sum;
  for (int i = 0; i < kScanItems; ++i) {
    if (base + i < n) offsets[base + i] = (uint32_t)run;
    run += c[i];
  }
  if (tid == 255) block_tot[blockIdx.x] = pre + inc;
}

// Single block: exclusive scan of the block totals; grand total (pairs needed) to *total.
__global__ void __launch_bounds__(1024) k_scan_blocks(uint64_t* __restrict__ block_tot, int nb,
                                                      uint64_t* __restrict__ total, uint64_t* __restrict__ n_eff,
                                                      int64_t capacity, uint32_t* __restrict__ status) {
  __shared__ uint64_t part[16];
  __shared__ uint64_t carry;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  if (tid == 0) carry = 0;
  __syncthreads();
  for (int b0 = 0; b0 < nb; b0 += 1024) {
    const int i = b0 + tid;
    uint64_t x = (i < nb) ? block_tot[i] : 0;
    uint64_t inc = x;
    for (int o = 1; o < 64; o <<= 1) {
      uint64_t y = __shfl_up(inc, o, 64);
      if (lane >= o) inc += y;
    }
    if (lane == 63) part[w] = inc;
    __syncthreads();
    uint64_t pre = carry;
    for (int k = 0; k < w; ++k) pre += part[k];
    if (i < nb) block_tot[i] = pre + inc - x;
    __syncthreads();
    if (tid == 1023) carry = pre + inc;
    __syncthreads();
  }
  if (tid == 0) {
    *total = carry;
    const bool over = (int64_t)carry > capacity;
    *n_eff = over ? 0 : carry;
    if (over) atomicOr(status, (uint32_t)ST_OVERFLOW);
  }
}

__global__ void __launch_bounds__(256) k_scan_add(uint32_t* __restrict__ offsets, const uint64_t* __restrict__ d_n,
                                                  const uint64_t* __restrict__ block_off) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t n = (int64_t)*d_n;
  if (i < n) offsets[i] += (uint32_t)block_off[i / kScanBlock];
}

// n: device count (at most n_max) of depth-sorted primitives.
hipError_t scan_counts(const uint32_t* prims, const uint32_t* counts, const uint64_t* d_n, int64_t n_max,
                       uint32_t* offsets, uint64_t* block_tot, uint64_t* total, uint64_t* n_eff, int64_t capacity,
                       uint32_t* status, hipStream_t s) {
  const int nb = (int)((n_max + kScanBlock - 1) / kScanBlock);
  if (nb > 0) hipLaunchKernelGGL(k_scan_local, dim3(nb), dim3(256), 0, s, prims, counts, d_n, offsets, block_tot);
  hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(1024), 0, s, block_tot, nb, total, n_eff, capacity, status);
  if (n_max > 0)
    hipLaunchKernelGGL(k_scan_add, dim3((unsigned)((n_max + 255) / 256)), dim3(256), 0, s, offsets, d_n, block_tot);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------------
// Stable compaction of the primitives that touch at least one tile (index order kept), with their
// depth keys: the depth sort then only sees visible primitives, and equal keys stay in index order.
__global__ void __launch_bounds__(256) k_flag_scan(const uint32_t* __restrict__ counts, int64_t n,
                                                   uint32_t* __restrict__ pos, uint64_t* __restrict__ block_tot) {
  __shared__ uint32_t part[4];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int64_t base = (int64_t)blockIdx.x * kScanBlock + (int64_t)tid * kScanItems;
  uint32_t f[kScanItems], sum = 0;
  for (int i = 0; i < kScanItems; ++i) {
    f[i] = (base + i < n && counts[base + i] > 0) ? 1u : 0u;
    sum += f[i];
  }
  uint32_t inc = sum;
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(inc, o, 64);
    if (lane >= o) inc += y;
  }
  if (lane == 63) part[w] = inc;
  __syncthreads();
  uint32_t pre = 0;
  for (int i = 0; i < w; ++i) pre += part[i];
  uint32_t run = pre + inc - sum;
  for (int i = 0; i < kScanItems; ++i) {
    if (base + i < n) pos[base + i] = f[i] ? run : 0xFFFFFFFFu;
    run += f[i];
  }
  if (tid == 255) block_tot[blockIdx.x] = pre + inc;
}

__global__ void __launch_bounds__(256) k_compact(const uint32_t* __restrict__ pos, const uint64_t* __restrict__ block_off,
                                                 const uint32_t* __restrict__ keys, int64_t n,
                                                 uint32_t* __restrict__ out_k, uint32_t* __restrict__ out_v) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const uint32_t p = pos[i];
  if (p == 0xFFFFFFFFu) return;
  const uint64_t q = p + block_off[i / kScanBlock];
  out_k[q] = keys[i];
  out_v[q] = (uint32_t)i;
}

hipError_t compact_visible(const uint32_t* counts, const uint32_t* keys, int64_t n, uint32_t* pos,
                           uint64_t* block_tot, uint64_t* n_vis, uint64_t* scratch_u64, uint32_t* out_k,
                           uint32_t* out_v, uint32_t* dummy_status, hipStream_t s) {
  const int nb = (int)((n + kScanBlock - 1) / kScanBlock);
  if (nb > 0) hipLaunchKernelGGL(k_flag_scan, dim3(nb), dim3(256), 0, s, counts, n, pos, block_tot);
  hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(1024), 0, s, block_tot, nb, n_vis, scratch_u64,
                     (int64_t)0x7FFFFFFFFFFFFFFF, dummy_status);
  if (n > 0)
    hipLaunchKernelGGL(k_compact, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, pos, block_tot, keys, n, out_k,
                       out_v);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------------
// Per-tile [start, end) of the tile-sorted pair list.
__global__ void __launch_bounds__(256) k_ranges_clear(uint32_t* __restrict__ ranges, int ntiles) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < 2 * ntiles) ranges[i] = 0;
}

__global__ void __launch_bounds__(256) k_ranges(const uint32_t* __restrict__ tiles, const uint64_t* __restrict__ d_n,
                                                uint32_t* __restrict__ ranges) {
  const uint64_t n = *d_n;
  for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (uint64_t)gridDim.x * 256) {
    const uint32_t t = tiles[i];
    if (i == 0 || tiles[i - 1] != t) ranges[2 * t] = (uint32_t)i;
    if (i + 1 == n || tiles[i + 1] != t) ranges[2 * t + 1] = (uint32_t)(i + 1);
  }
}

// Sort keys of the tiles by decreasing list length (lengths above 65535 tie), values = tile ids.
__global__ void __launch_bounds__(256) k_tile_keys(const uint32_t* __restrict__ ranges, int ntiles,
                                                   uint32_t* __restrict__ keys, uint32_t* __restrict__ vals) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t >= ntiles) return;
  const uint32_t len = ranges[2 * t + 1] - ranges[2 * t];
  keys[t] = 0xFFFFu - (len < 0xFFFFu ? len : 0xFFFFu);
  vals[t] = (uint32_t)t;
}

hipError_t tile_length_keys(const uint32_t* ranges, int ntiles, uint32_t* keys, uint32_t* vals, hipStream_t s) {
  hipLaunchKernelGGL(k_tile_keys, dim3((ntiles + 255) / 256), dim3(256), 0, s, ranges, ntiles, keys, vals);
  return hipGetLastError();
}

hipError_t tile_ranges(const uint32_t* tiles, const uint64_t* d_n, uint32_t* ranges, int ntiles, hipStream_t s) {
  hipLaunchKernelGGL(k_ranges_clear, dim3((2 * ntiles + 255) / 256), dim3(256), 0, s, ranges, ntiles);
  hipLaunchKernelGGL(k_ranges, dim3(2048), dim3(256), 0, s, tiles, d_n, ranges);
  return hipGetLastError();
}

// After the stable sort of pair keys (values = pair ids): tile and primitive of each pair in key
// order, ready for the stable sort by tile.
__global__ void __launch_bounds__(256) k_gather_pairs(const uint32_t* __restrict__ ids, const uint32_t* __restrict__ tiles,
                                                      const uint32_t* __restrict__ prims, const uint64_t* __restrict__ d_n,
                                                      uint32_t* __restrict__ tiles_out, uint32_t* __restrict__ prims_out) {
  const uint64_t n = *d_n;
  for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (uint64_t)gridDim.x * 256) {
    const uint32_t id = ids[i];
    tiles_out[i] = tiles[id];
    prims_out[i] = prims[id];
  }
}

hipError_t gather_pairs(const uint32_t* ids, const uint32_t* tiles, const uint32_t* prims, const uint64_t* d_n,
                        uint32_t* tiles_out, uint32_t* prims_out, hipStream_t s) {
  hipLaunchKernelGGL(k_gather_pairs, dim3(2048), dim3(256), 0, s, ids, tiles, prims, d_n, tiles_out, prims_out);
  return hipGetLastError();
}

__global__ void k_set_u64(uint64_t* p, uint64_t v) { *p = v; }

__global__ void __launch_bounds__(256) k_fill_u32(uint32_t* __restrict__ p, uint32_t v, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) p[i] = v;
}

hipError_t fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}

hipError_t set_u64(uint64_t* p, uint64_t v, hipStream_t s) {
  hipLaunchKernelGGL(k_set_u64, dim3(1), dim3(1), 0, s, p, v);
  return hipGetLastError();
}

}  // namespace drk
