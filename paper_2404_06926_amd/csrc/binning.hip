// Tile binning (Sec. III-A depth order, Sec. III-D.2 footprint tiles).
//
// The order the blend needs is (global tile, depth, Gaussian index). It is reached in two
// small sorts instead of one wide one:
//   1. a stable LSD radix sort of the (view, Gaussian) pairs by the float bits of their
//      depth (4 passes over V*N 32-bit keys; pairs that reach no tile get the largest key);
//   2. an exclusive scan of the tile counts in that order, then every pair emits its tile
//      ids at its offset, so the instance list comes out in (depth, view-major index)
//      order;
//   3. a stable LSD radix sort of the instances by global tile id only
//      (ceil(log2(tiles + 1)) bits, 2 passes up to 65535 tiles);
//   4. [start, end) of every tile in the sorted list.
// Stability makes the result identical to sorting the 64-bit keys tile << 32 | depth bits
// with ties in emission order, at about a fifth of the bytes.
// Kernels that depend on the instance count read it from device memory, so the sequence
// has host-known launch shapes (graph-capturable). Instances beyond the buffer capacity
// are dropped and flagged; the render is then empty.
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

// Pass 1: per-block local exclusive scan and block sums; element k is in[idx[k]] when idx
// is given (a gather in another order), else in[k].
__global__ void __launch_bounds__(kScanBlock)
k_scan_local(const uint32_t* __restrict__ in, const uint32_t* __restrict__ idx, uint32_t* __restrict__ out,
             uint32_t* __restrict__ sums, int64_t n) {
  __shared__ uint32_t s_warp[kScanBlock / 64];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  uint32_t v[kScanItems];
  uint32_t tsum = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    v[k] = 0u;
    if (base + k < n) v[k] = idx ? in[idx[base + k]] : in[base + k];
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
__global__ void k_scan_total(const uint32_t* __restrict__ in, const uint32_t* __restrict__ idx,
                             const uint32_t* __restrict__ out, int64_t n, uint32_t* __restrict__ total) {
  total[0] = n > 0 ? out[n - 1] + (idx ? in[idx[n - 1]] : in[n - 1]) : 0u;
}

int64_t scan_temp_elems(int64_t n) {
  int64_t t = 0;
  while (n > 1) {
    n = (n + kScanTile - 1) / kScanTile;
    t += n;
  }
  return t + 1;
}

static hipError_t scan_impl(const uint32_t* in, const uint32_t* idx, uint32_t* out, int64_t n, uint32_t* temp,
                            hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t nb = (n + kScanTile - 1) / kScanTile;
  uint32_t* sums = temp;
  hipLaunchKernelGGL(k_scan_local, dim3((unsigned)nb), dim3(kScanBlock), 0, s, in, idx, out, sums, n);
  if (nb > 1) {
    hipError_t e = scan_impl(sums, nullptr, sums, nb, temp + nb, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_scan_add, dim3((unsigned)nb), dim3(kScanBlock), 0, s, out, sums, n);
  }
  return hipGetLastError();
}

// Exclusive scan of n u32 values (in may equal out); temp holds scan_temp_elems(n).
hipError_t exclusive_scan(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* temp, hipStream_t s) {
  return scan_impl(in, nullptr, out, n, temp, s);
}

// offsets[k] = sum of counts[order[j]] for j < k; total = sum of all.
hipError_t scan_counts(const uint32_t* counts, const uint32_t* order, uint32_t* offsets, int64_t n,
                       uint32_t* temp, uint32_t* total, hipStream_t s) {
  hipError_t e = scan_impl(counts, order, offsets, n, temp, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_scan_total, dim3(1), dim3(1), 0, s, counts, order, offsets, n, total);
  return hipGetLastError();
}

// ------------------------------------------------------------------ radix sort
// Stable LSD sort with 8-bit digits. Each pass: per-block digit histograms
// (digit-major), an exclusive scan of the histograms, then a stable scatter in which
// every wave ranks its keys in order with ballot-based peer masks.
constexpr int kSortBlock = 256;
constexpr int kSortItems = 8;                       // keys per thread (16 measured slower: too few
constexpr int kSortTile = kSortBlock * kSortItems;  // blocks for the 1M-key depth sort); 2048 per block
constexpr int kWaves = kSortBlock / 64;

// Elements to process: all of them when they fit, none after an overflow (the render is
// then empty and the overflow flag tells the host to re-plan).
__device__ __forceinline__ uint32_t sort_count(const uint32_t* n_dev, int64_t cap) {
  const uint32_t n = n_dev[0];
  return (int64_t)n <= cap ? n : 0u;
}

// Lanes of the wave whose digit equals this lane's (8 ballots), restricted to `ok` lanes.
__device__ __forceinline__ uint64_t digit_peers(uint32_t d, bool ok) {
  uint64_t peers = __ballot(ok);
#pragma unroll
  for (int b = 0; b < 8; ++b) {
    const uint64_t m = __ballot((d >> b) & 1u);
    peers &= ((d >> b) & 1u) ? m : ~m;
  }
  return peers;
}

template <typename K>
__global__ void __launch_bounds__(kSortBlock)
k_radix_hist(const K* __restrict__ keys, const uint32_t* __restrict__ n_dev, int64_t cap, int shift,
             uint32_t* __restrict__ hist, int nblocks) {
  __shared__ uint32_t s_h[kWaves][256];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int d = lane; d < 256; d += 64) s_h[wid][d] = 0;
  __syncthreads();
  const uint32_t n = sort_count(n_dev, cap);
  const int64_t base = (int64_t)blockIdx.x * kSortTile + (int64_t)wid * (64 * kSortItems);
#pragma unroll
  for (int r = 0; r < kSortItems; ++r) {
    const int64_t idx = base + r * 64 + lane;
    const bool ok = idx < n;
    const uint32_t d = ok ? (uint32_t)(keys[idx] >> shift) & 255u : 0u;
    // one LDS add per distinct digit of the wave
    const uint64_t peers = digit_peers(d, ok);
    if (ok && lane == __ffsll((long long)peers) - 1) s_h[wid][d] += (uint32_t)__popcll(peers);
  }
  __syncthreads();
  const int d = threadIdx.x;
  hist[(int64_t)d * nblocks + blockIdx.x] = s_h[0][d] + s_h[1][d] + s_h[2][d] + s_h[3][d];
}

// The block's keys are first placed in LDS in (digit, original order) order, then written
// out by consecutive lanes, so each digit's run goes to consecutive global addresses.
template <typename K>
__global__ void __launch_bounds__(kSortBlock)
k_radix_scatter(const K* __restrict__ kin, const uint32_t* __restrict__ vin, K* __restrict__ kout,
                uint32_t* __restrict__ vout, const uint32_t* __restrict__ n_dev, int64_t cap, int shift,
                const uint32_t* __restrict__ hist_scan, int nblocks) {
  __shared__ uint32_t s_cnt[kWaves][256];   // keys per (wave, digit), then the wave's offset
  __shared__ uint32_t s_start[256];         // first LDS slot of each digit
  __shared__ uint32_t s_gbase[256];         // global position of the block's first key of each digit
  __shared__ uint32_t s_warp[kWaves];
  __shared__ K s_key[kSortTile];
  __shared__ uint32_t s_val[kSortTile];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int d = lane; d < 256; d += 64) s_cnt[wid][d] = 0;
  __syncthreads();
  const uint32_t n = sort_count(n_dev, cap);
  const int64_t blk0 = (int64_t)blockIdx.x * kSortTile;
  const int64_t base = blk0 + (int64_t)wid * (64 * kSortItems);
  K key[kSortItems];
  uint32_t val[kSortItems], rank[kSortItems], dig[kSortItems];
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
#pragma unroll
  for (int r = 0; r < kSortItems; ++r) {
    const int64_t idx = base + r * 64 + lane;
    const bool ok = idx < n;
    key[r] = ok ? kin[idx] : (K)0;
    val[r] = ok ? vin[idx] : 0u;
    const uint32_t d = (uint32_t)(key[r] >> shift) & 255u;
    dig[r] = d;
    const uint64_t peers = digit_peers(d, ok);
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
  // digit totals of the block, their exclusive scan (LDS start of each digit) and each
  // wave's offset inside its digit run
  {
    const int d = threadIdx.x;
    uint32_t tot = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) {
      const uint32_t c = s_cnt[w][d];
      s_cnt[w][d] = tot;
      tot += c;
    }
    uint32_t all;
    const uint32_t start = block_exclusive_scan(tot, s_warp, all);
    s_start[d] = start;
    s_gbase[d] = hist_scan[(int64_t)d * nblocks + blockIdx.x];
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kSortItems; ++r) {
    const int64_t idx = base + r * 64 + lane;
    if (idx < n) {
      const uint32_t slot = s_start[dig[r]] + s_cnt[wid][dig[r]] + rank[r];
      s_key[slot] = key[r];
      s_val[slot] = val[r];
    }
  }
  __syncthreads();
  const int64_t nblk = min((int64_t)kSortTile, (int64_t)n - blk0);
  for (int t = threadIdx.x; t < nblk; t += kSortBlock) {
    const K k = s_key[t];
    const uint32_t d = (uint32_t)(k >> shift) & 255u;
    const uint32_t pos = s_gbase[d] + ((uint32_t)t - s_start[d]);
    kout[pos] = k;
    vout[pos] = s_val[t];
  }
}

int64_t sort_temp_elems(int64_t cap) {
  const int64_t nb = (cap + kSortTile - 1) / kSortTile;
  return 256 * nb + scan_temp_elems(256 * nb);
}

// Sorts (keys[0], vals[0]) on bits [0, nbits) using (keys[1], vals[1]) as the double buffer;
// *which receives the index of the buffer that holds the result.
hipError_t radix_sort_u32(uint32_t* keys[2], uint32_t* vals[2], const uint32_t* n_dev, int64_t cap, int nbits,
                          uint32_t* temp, int* which, hipStream_t s) {
  *which = 0;
  if (cap <= 0) return hipSuccess;
  const int nb = (int)((cap + kSortTile - 1) / kSortTile);
  uint32_t* hist = temp;
  uint32_t* stemp = temp + (int64_t)256 * nb;
  int cur = 0;
  for (int shift = 0; shift < nbits; shift += 8) {
    hipLaunchKernelGGL(k_radix_hist<uint32_t>, dim3(nb), dim3(kSortBlock), 0, s, keys[cur], n_dev, cap, shift,
                       hist, nb);
    hipError_t e = exclusive_scan(hist, hist, (int64_t)256 * nb, stemp, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_radix_scatter<uint32_t>, dim3(nb), dim3(kSortBlock), 0, s, keys[cur], vals[cur],
                       keys[cur ^ 1], vals[cur ^ 1], n_dev, cap, shift, hist, nb);
    cur ^= 1;
  }
  *which = cur;
  return hipGetLastError();
}

// Instances are emitted in depth order: pair k of the depth order ((view, Gaussian) id
// order[k]) owns the instance range [offsets[k], offsets[k] + count). One lane per
// instance, so the work does not depend on how unevenly the counts fall: block b covers
// instances [256 b, 256 b + 256); it stages the offsets and ids of the (at most 256) pairs
// from block_start[b] in LDS, finds its instance's pair by binary search and takes the
// tile from the pair's 64-bit hit mask (its r-th set bit, row-major in the pair's tile
// rectangle). Pairs whose rectangle has more than 64 tiles were listed by the projection;
// one wave each evaluates the tile predicate over the rectangle and places the hits with
// a ballot prefix sum. Instances past the capacity are not written; the overflow flag is
// raised and the render is emptied downstream.
constexpr int kLb = 256;

// block_start[b] = the pair that owns instance 256 b.
__global__ void __launch_bounds__(256)
k_block_starts(const uint32_t* __restrict__ offsets, const uint32_t* __restrict__ n_dev, int64_t n_pairs,
               int64_t capacity, uint32_t* __restrict__ block_start) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n_pairs) return;
  const int64_t total = n_dev[0];
  const int64_t o = offsets[k];
  const int64_t e = min(k + 1 < n_pairs ? (int64_t)offsets[k + 1] : total, min(total, capacity));
  for (int64_t b = (o + kLb - 1) / kLb; b * kLb < e; ++b) block_start[b] = (uint32_t)k;
}

// position of the r-th set bit (r counted from 0) of a 32-bit word that has more than r
__device__ __forceinline__ int nth_set_bit32(uint32_t w, uint32_t r) {
  int pos = 0;
#pragma unroll
  for (int sh = 16; sh >= 1; sh >>= 1) {
    const uint32_t c = (uint32_t)__popc(w & ((1u << sh) - 1u));
    if (r >= c) {
      r -= c;
      w >>= sh;
      pos += sh;
    }
  }
  return pos;
}

__global__ void __launch_bounds__(kLb)
k_dup_lb(const float4* __restrict__ rec, const uint32_t* __restrict__ order, const uint32_t* __restrict__ offsets,
         const uint32_t* __restrict__ block_start, const uint32_t* __restrict__ n_dev, int64_t n_pairs, int32_t N,
         ViewsArg va, int64_t capacity, uint32_t* __restrict__ tiles_out, uint32_t* __restrict__ vals_out,
         uint32_t* __restrict__ emit_g, uint32_t* __restrict__ inst_off, uint32_t* __restrict__ overflow) {
  __shared__ uint32_t s_off[kLb + 1];
  __shared__ uint32_t s_vi[kLb];
  const int64_t total = n_dev[0];
  if (blockIdx.x == 0 && threadIdx.x == 0 && total > capacity) atomicOr(overflow, 1u);
  const int64_t lim = min(total, capacity);
  const int64_t slot0 = (int64_t)blockIdx.x * kLb;
  if (slot0 >= lim) return;
  const int64_t k0 = block_start[blockIdx.x];
  {
    const int64_t k = k0 + threadIdx.x;
    s_off[threadIdx.x] = k < n_pairs ? offsets[k] : (uint32_t)total;
    s_vi[threadIdx.x] = k < n_pairs ? order[k] : 0u;
    if (threadIdx.x == 0) s_off[kLb] = k0 + kLb < n_pairs ? offsets[k0 + kLb] : (uint32_t)total;
  }
  __syncthreads();
  const int64_t slot = slot0 + threadIdx.x;
  if (slot >= lim) return;
  // the pairs k0 .. k0 + 255 cover this block (every pair before the unused ones has a
  // tile): the last staged offset <= slot is the owner
  int lo = 0, hi = kLb - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if ((int64_t)s_off[mid] <= slot) lo = mid;
    else hi = mid - 1;
  }
  const uint32_t vi = s_vi[lo];
  const uint32_t r = (uint32_t)(slot - (int64_t)s_off[lo]);
  if (r == 0) inst_off[vi] = (uint32_t)slot;
  const float4 r3 = rec[(size_t)vi * 4 + 3];
  const uint32_t a = __float_as_uint(r3.x), b = __float_as_uint(r3.y);
  const int x0 = a & 0xffff, y0 = a >> 16, x1 = b & 0xffff, y1 = b >> 16;
  const int rw = x1 - x0 + 1;
  if (rw * (y1 - y0 + 1) > 64) return;  // a listed pair: k_dup_big writes it
  const uint32_t mlo = __float_as_uint(r3.z), mhi = __float_as_uint(r3.w);
  const uint32_t clo = (uint32_t)__popc(mlo);
  const int pos = r < clo ? nth_set_bit32(mlo, r) : 32 + nth_set_bit32(mhi, r - clo);
  const int v = (int)(vi / (uint32_t)N);
  const uint32_t g = vi - (uint32_t)v * (uint32_t)N;
  const ViewDev& V = va.v[v];
  tiles_out[slot] = (uint32_t)(V.tile_base + (y0 + pos / rw) * V.tiles_x + (x0 + pos % rw));
  vals_out[slot] = (uint32_t)slot;
  emit_g[slot] = g;
}

// One wave per listed pair (tile rectangle of more than 64 tiles).
__global__ void __launch_bounds__(256)
k_dup_big(const float4* __restrict__ rec, const uint32_t* __restrict__ big_list, const uint32_t* __restrict__ big_n,
          const uint32_t* __restrict__ counts, const uint32_t* __restrict__ inst_off,
          const uint32_t* __restrict__ n_dev, int32_t N, ViewsArg va, int64_t capacity,
          uint32_t* __restrict__ tiles_out, uint32_t* __restrict__ vals_out, uint32_t* __restrict__ emit_g) {
  const int lane = threadIdx.x & 63;
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  if ((int64_t)n_dev[0] > capacity) return;
  const int64_t nb = big_n[0];
  const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;  // lanes under this one
  for (int64_t w = wave; w < nb; w += nwaves) {
    const uint32_t vi = big_list[w];
    const int v = (int)(vi / (uint32_t)N);
    const uint32_t g = vi - (uint32_t)v * (uint32_t)N;
    const ViewDev& V = va.v[v];
    const float4* rp = rec + (size_t)vi * 4;
    const float4 r0 = rp[0], r1 = rp[1], r2 = rp[2], r3 = rp[3];
    const uint32_t a = __float_as_uint(r3.x), b = __float_as_uint(r3.y);
    const int x0 = a & 0xffff, y0 = a >> 16, x1 = b & 0xffff, y1 = b >> 16;
    const int rw = x1 - x0 + 1, area = rw * (y1 - y0 + 1);
    const int64_t o = inst_off[vi];
    const uint32_t cnt = counts[vi];
    uint32_t base = 0;
    for (int t0 = 0; t0 < area; t0 += 64) {
      const int t = t0 + lane;
      int tx = 0, ty = 0;
      bool hit = false;
      if (t < area) {
        tx = x0 + t % rw;
        ty = y0 + t / rw;
        hit = key_tile_hit(r0.x, r0.y, r0.z, r0.w, r1.x, r2.w, tx, ty);
      }
      const uint64_t m = __ballot(hit);
      const uint32_t p = base + (uint32_t)__popcll(m & below);
      if (hit && p < cnt) {
        const int64_t slot = o + p;
        tiles_out[slot] = (uint32_t)(V.tile_base + ty * V.tiles_x + tx);
        vals_out[slot] = (uint32_t)slot;
        emit_g[slot] = g;
      }
      base += (uint32_t)__popcll(m);
    }
    // unreachable when both passes agree; the sentinel tile sorts after every real tile
    for (uint32_t p = base + lane; p < cnt; p += 64) {
      tiles_out[o + p] = 0xffffffffu;
      vals_out[o + p] = (uint32_t)(o + p);
      emit_g[o + p] = 0u;
    }
  }
}

int64_t block_start_elems(int64_t capacity) { return capacity / kLb + 2; }

hipError_t duplicate_keys(const float4* rec, const uint32_t* counts, const uint32_t* order, const uint32_t* offsets,
                          const uint32_t* n_dev, const uint32_t* big_list, const uint32_t* big_n, int32_t N,
                          const ViewsArg& va, uint32_t* tiles, uint32_t* vals, uint32_t* emit_g, uint32_t* inst_off,
                          uint32_t* block_start, int64_t capacity, uint32_t* overflow, hipStream_t s) {
  const int64_t n = (int64_t)va.n * N;
  if (n <= 0 || capacity <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_block_starts, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, offsets, n_dev, n, capacity,
                     block_start);
  hipLaunchKernelGGL(k_dup_lb, dim3((unsigned)((capacity + kLb - 1) / kLb)), dim3(kLb), 0, s, rec, order, offsets,
                     block_start, n_dev, n, N, va, capacity, tiles, vals, emit_g, inst_off, overflow);
  hipLaunchKernelGGL(k_dup_big, dim3(512), dim3(256), 0, s, rec, big_list, big_n, counts, inst_off, n_dev, N, va,
                     capacity, tiles, vals, emit_g);
  return hipGetLastError();
}

// Gaussian index of every instance in blend order (for inspection).
__global__ void __launch_bounds__(256)
k_gather_g(const uint32_t* __restrict__ vals, const uint32_t* __restrict__ emit_g, const uint32_t* __restrict__ n_dev,
           int64_t cap, uint32_t* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < sort_count(n_dev, cap)) out[i] = emit_g[vals[i]];
}

hipError_t gather_gaussians(const uint32_t* vals, const uint32_t* emit_g, const uint32_t* n_dev, int64_t cap,
                            uint32_t* out, hipStream_t s) {
  if (cap <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_g, dim3((unsigned)((cap + 255) / 256)), dim3(256), 0, s, vals, emit_g, n_dev, cap, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------- ranges
__global__ void __launch_bounds__(256)
k_ranges(const uint32_t* __restrict__ tiles, const uint32_t* __restrict__ n_dev, int64_t cap,
         uint2* __restrict__ ranges, uint32_t n_tiles) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t n = sort_count(n_dev, cap);
  if (i >= n) return;
  const uint32_t t = tiles[i];
  if (i == 0) {
    if (t < n_tiles) ranges[t].x = 0;
  } else {
    const uint32_t tp = tiles[i - 1];
    if (tp != t) {
      if (tp < n_tiles) ranges[tp].y = (uint32_t)i;
      if (t < n_tiles) ranges[t].x = (uint32_t)i;
    }
  }
  if (i == (int64_t)n - 1 && t < n_tiles) ranges[t].y = n;
}

hipError_t tile_ranges(const uint32_t* tiles, const uint32_t* n_dev, int64_t cap, uint2* ranges, int64_t n_tiles,
                       hipStream_t s) {
  if (cap <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_ranges, dim3((unsigned)((cap + 255) / 256)), dim3(256), 0, s, tiles, n_dev, cap, ranges,
                     (uint32_t)n_tiles);
  return hipGetLastError();
}

}  // namespace gs
