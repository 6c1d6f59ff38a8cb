// Tile binning (Sec. III-A depth order, Sec. III-D.2 footprint tiles):
//   exclusive scan of per-(view, Gaussian) tile counts -> instance offsets,
//   duplicate each Gaussian once per tile its footprint reaches with the key
//   (global tile << 32 | float bits of depth),
//   stable LSD radix sort of (key, Gaussian) pairs on the significant key bits,
//   [start, end) of every tile in the sorted list.
// Kernels that depend on the instance count read it from device memory, so the whole
// sequence has host-known launch shapes (graph-capturable); instances beyond the buffer
// capacity are dropped and an overflow flag is raised.
#include "gs_common.h"
#include "kernels.h"

namespace gs {

constexpr int kScanBlock = 256;
constexpr int kScanItems = 8;   // 2048 elements per block
constexpr int kScanTile = kScanBlock * kScanItems;

// Block-wide exclusive scan of one value per thread; returns the block total.
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t x, uint32_t* s_warp, uint32_t& total) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  uint32_t incl = x;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(incl, o, 64);
    if (lane >= o) incl += y;
  }
  if (lane == 63) s_warp[wid] = incl;
  __syncthreads();
  uint32_t wbase = 0;
  total = 0;
  for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
    const uint32_t t = s_warp[w];
    if (w < wid) wbase += t;
    total += t;
  }
  __syncthreads();
  return wbase + incl - x;
}

// Pass 1: per-block local exclusive scan and block sums.
__global__ void __launch_bounds__(kScanBlock)
k_scan_local(const uint32_t* __restrict__ in, uint32_t* __restrict__ out, uint32_t* __restrict__ sums, int64_t n) {
  __shared__ uint32_t s_warp[kScanBlock / 64];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  uint32_t v[kScanItems];
  uint32_t tsum = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    v[k] = (base + k < n) ? in[base + k] : 0u;
    tsum += v[k];
  }
  uint32_t total;
  uint32_t run = block_exclusive_scan(tsum, s_warp, total);
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    if (base + k < n) out[base + k] = run;
    run += v[k];
  }
  if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

// Pass 3: add the scanned block sums.
__global__ void __launch_bounds__(kScanBlock)
k_scan_add(uint32_t* __restrict__ out, const uint32_t* __restrict__ sums, int64_t n) {
  const uint32_t add = sums[blockIdx.x];
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  for (int k = threadIdx.x; k < kScanTile; k += kScanBlock)
    if (base + k < n) out[base + k] += add;
}

// total = last offset + last count
__global__ void k_scan_total(const uint32_t* __restrict__ in, const uint32_t* __restrict__ out, int64_t n,
                             uint32_t* __restrict__ total) {
  total[0] = n > 0 ? out[n - 1] + in[n - 1] : 0u;
}

int64_t scan_temp_elems(int64_t n) {
  int64_t t = 0;
  while (n > 1) {
    n = (n + kScanTile - 1) / kScanTile;
    t += n;
  }
  return t + 1;
}

// Exclusive scan of n u32 values (in may equal out); temp holds scan_temp_elems(n).
hipError_t exclusive_scan(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* temp, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t nb = (n + kScanTile - 1) / kScanTile;
  uint32_t* sums = temp;
  hipLaunchKernelGGL(k_scan_local, dim3((unsigned)nb), dim3(kScanBlock), 0, s, in, out, sums, n);
  if (nb > 1) {
    hipError_t e = exclusive_scan(sums, sums, nb, temp + nb, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_scan_add, dim3((unsigned)nb), dim3(kScanBlock), 0, s, out, sums, n);
  }
  return hipGetLastError();
}

hipError_t scan_counts(const uint32_t* counts, uint32_t* offsets, int64_t n, uint32_t* temp,
                       uint32_t* total, hipStream_t s) {
  hipError_t e = exclusive_scan(counts, offsets, n, temp, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_scan_total, dim3(1), dim3(1), 0, s, counts, offsets, n, total);
  return hipGetLastError();
}

// ------------------------------------------------------------------- duplicate
__global__ void __launch_bounds__(256)
k_duplicate(const float4* __restrict__ rec, const uint32_t* __restrict__ counts,
            const uint32_t* __restrict__ offsets, int32_t N, ViewsArg va, uint64_t* __restrict__ keys,
            uint32_t* __restrict__ vals, int64_t capacity, uint32_t* __restrict__ overflow) {
  const int64_t vi = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (vi >= (int64_t)va.n * N) return;
  const uint32_t cnt = counts[vi];
  if (cnt == 0) return;
  const int v = (int)(vi / N);
  const uint32_t g = (uint32_t)(vi - (int64_t)v * N);
  const ViewDev& V = va.v[v];
  const float4 r0 = rec[vi * 4], r1 = rec[vi * 4 + 1], r2 = rec[vi * 4 + 2], r3 = rec[vi * 4 + 3];
  const uint32_t a = __float_as_uint(r3.x), b = __float_as_uint(r3.y);
  const int x0 = a & 0xffff, y0 = a >> 16, x1 = b & 0xffff, y1 = b >> 16;
  const uint64_t dbits = __float_as_uint(r2.y);
  int64_t o = offsets[vi];
  if (o + cnt > capacity) {
    atomicOr(overflow, 1u);
    return;
  }
  // Same predicate as the count pass; writes never leave this Gaussian's [o, o + cnt).
  const int64_t end = o + cnt;
  for (int ty = y0; ty <= y1 && o < end; ++ty)
    for (int tx = x0; tx <= x1 && o < end; ++tx)
      if (key_tile_hit(r0.x, r0.y, r0.z, r0.w, r1.x, r2.w, tx, ty)) {
        const uint64_t tile = (uint64_t)(V.tile_base + ty * V.tiles_x + tx);
        keys[o] = (tile << 32) | dbits;
        vals[o] = g;
        ++o;
      }
  // unreachable when both passes agree; a sentinel tile sorts last and is never ranged
  for (; o < end; ++o) {
    keys[o] = ~0ull;
    vals[o] = 0u;
  }
}

hipError_t duplicate_keys(const float4* rec, const uint32_t* counts, const uint32_t* offsets, int32_t N,
                          const ViewsArg& va, uint64_t* keys, uint32_t* vals, int64_t capacity,
                          uint32_t* overflow, hipStream_t s) {
  const int64_t n = (int64_t)va.n * N;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_duplicate, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, rec, counts, offsets,
                     N, va, keys, vals, capacity, overflow);
  return hipGetLastError();
}

// ------------------------------------------------------------------ radix sort
// Stable LSD sort with 8-bit digits. Each pass: per-block digit histograms
// (digit-major), an exclusive scan of the histograms, then a stable scatter in which
// every wave ranks its keys in order with ballot-based peer masks.
constexpr int kSortBlock = 256;
constexpr int kSortItems = 8;                       // keys per thread
constexpr int kSortTile = kSortBlock * kSortItems;  // 2048 keys per block
constexpr int kWaves = kSortBlock / 64;

// Instances to process: all of them when they fit, none after an overflow (the render
// is then empty and the overflow flag tells the host to re-plan).
__device__ __forceinline__ uint32_t sort_count(const uint32_t* n_dev, int64_t cap) {
  const uint32_t n = n_dev[0];
  return (int64_t)n <= cap ? n : 0u;
}

__global__ void __launch_bounds__(kSortBlock)
k_radix_hist(const uint64_t* __restrict__ keys, const uint32_t* __restrict__ n_dev, int64_t cap, int shift,
             uint32_t* __restrict__ hist, int nblocks) {
  __shared__ uint32_t s_h[256];
  s_h[threadIdx.x] = 0;
  __syncthreads();
  const uint32_t n = sort_count(n_dev, cap);
  const int64_t base = (int64_t)blockIdx.x * kSortTile;
  for (int k = threadIdx.x; k < kSortTile; k += kSortBlock) {
    const int64_t idx = base + k;
    if (idx < n) atomicAdd(&s_h[(uint32_t)(keys[idx] >> shift) & 255u], 1u);
  }
  __syncthreads();
  hist[(int64_t)threadIdx.x * nblocks + blockIdx.x] = s_h[threadIdx.x];
}

__global__ void __launch_bounds__(kSortBlock)
k_radix_scatter(const uint64_t* __restrict__ kin, const uint32_t* __restrict__ vin, uint64_t* __restrict__ kout,
                uint32_t* __restrict__ vout, const uint32_t* __restrict__ n_dev, int64_t cap, int shift,
                const uint32_t* __restrict__ hist_scan, int nblocks) {
  __shared__ uint32_t s_cnt[kWaves][256];
  __shared__ uint32_t s_base[kWaves][256];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int d = lane; d < 256; d += 64) s_cnt[wid][d] = 0;
  __syncthreads();
  const uint32_t n = sort_count(n_dev, cap);
  const int64_t base = (int64_t)blockIdx.x * kSortTile + (int64_t)wid * (64 * kSortItems);
  uint64_t key[kSortItems];
  uint32_t val[kSortItems], rank[kSortItems], dig[kSortItems];
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
#pragma unroll
  for (int r = 0; r < kSortItems; ++r) {
    const int64_t idx = base + r * 64 + lane;
    const bool ok = idx < n;
    key[r] = ok ? kin[idx] : 0ull;
    val[r] = ok ? vin[idx] : 0u;
    const uint32_t d = (uint32_t)(key[r] >> shift) & 255u;
    dig[r] = d;
    uint64_t peers = __ballot(ok);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const uint64_t m = __ballot((d >> b) & 1u);
      peers &= ((d >> b) & 1u) ? m : ~m;
    }
    uint32_t prev = 0;
    const int leader = peers ? (__ffsll((long long)peers) - 1) : 0;
    if (ok && lane == leader) {
      prev = s_cnt[wid][d];
      s_cnt[wid][d] = prev + (uint32_t)__popcll(peers);
    }
    prev = __shfl(prev, leader, 64);
    rank[r] = prev + (uint32_t)__popcll(peers & lt);
  }
  __syncthreads();
  // per-digit offsets of each wave inside the block, plus the block's global offset
  {
    const int d = threadIdx.x;
    uint32_t run = hist_scan[(int64_t)d * nblocks + blockIdx.x];
#pragma unroll
    for (int w = 0; w < kWaves; ++w) {
      s_base[w][d] = run;
      run += s_cnt[w][d];
    }
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kSortItems; ++r) {
    const int64_t idx = base + r * 64 + lane;
    if (idx < n) {
      const uint32_t pos = s_base[wid][dig[r]] + rank[r];
      kout[pos] = key[r];
      vout[pos] = val[r];
    }
  }
}

int64_t sort_temp_elems(int64_t cap) {
  const int64_t nb = (cap + kSortTile - 1) / kSortTile;
  return 256 * nb + scan_temp_elems(256 * nb);
}

// Sorts (keys[0], vals[0]) on bits [0, nbits) using (keys[1], vals[1]) as the double buffer;
// returns in *which the index of the buffer that holds the result.
hipError_t radix_sort(uint64_t* keys[2], uint32_t* vals[2], const uint32_t* n_dev, int64_t cap, int nbits,
                      uint32_t* temp, int* which, hipStream_t s) {
  *which = 0;
  if (cap <= 0) return hipSuccess;
  const int nb = (int)((cap + kSortTile - 1) / kSortTile);
  uint32_t* hist = temp;
  uint32_t* stemp = temp + (int64_t)256 * nb;
  int cur = 0;
  for (int shift = 0; shift < nbits; shift += 8) {
    hipLaunchKernelGGL(k_radix_hist, dim3(nb), dim3(kSortBlock), 0, s, keys[cur], n_dev, cap, shift, hist, nb);
    hipError_t e = exclusive_scan(hist, hist, (int64_t)256 * nb, stemp, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_radix_scatter, dim3(nb), dim3(kSortBlock), 0, s, keys[cur], vals[cur], keys[cur ^ 1],
                       vals[cur ^ 1], n_dev, cap, shift, hist, nb);
    cur ^= 1;
  }
  *which = cur;
  return hipGetLastError();
}

// ---------------------------------------------------------------------- ranges
__global__ void __launch_bounds__(256)
k_ranges(const uint64_t* __restrict__ keys, const uint32_t* __restrict__ n_dev, int64_t cap,
         uint2* __restrict__ ranges, uint32_t n_tiles) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t n = sort_count(n_dev, cap);
  if (i >= n) return;
  const uint32_t t = (uint32_t)(keys[i] >> 32);
  if (i == 0) {
    if (t < n_tiles) ranges[t].x = 0;
  } else {
    const uint32_t tp = (uint32_t)(keys[i - 1] >> 32);
    if (tp != t) {
      if (tp < n_tiles) ranges[tp].y = (uint32_t)i;
      if (t < n_tiles) ranges[t].x = (uint32_t)i;
    }
  }
  if (i == (int64_t)n - 1 && t < n_tiles) ranges[t].y = n;
}

hipError_t tile_ranges(const uint64_t* keys, const uint32_t* n_dev, int64_t cap, uint2* ranges, int64_t n_tiles,
                       hipStream_t s) {
  if (cap <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_ranges, dim3((unsigned)((cap + 255) / 256)), dim3(256), 0, s, keys, n_dev, cap, ranges,
                     (uint32_t)n_tiles);
  return hipGetLastError();
}

}  // namespace gs
