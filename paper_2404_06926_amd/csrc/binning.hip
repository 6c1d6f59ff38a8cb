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

// Exclusive scan over a fixed grid of at most kScanGrid blocks, each owning a contiguous
// run of 2048-element tiles (every block at least one): the up pass sums each block's run,
// the down pass takes the sum of the earlier blocks' runs as its start and scans its tiles
// in order. Element k is in[idx[k]] when idx is given (a gather in another order; the up
// pass stores the gathered values in order so that the down pass reads them contiguously),
// else in[k]; in may equal out.
constexpr int kScanGrid = 4096;

static int scan_grid(int64_t n) {
  return (int)std::min<int64_t>(kScanGrid, std::max<int64_t>(1, (n + kScanTile - 1) / kScanTile));
}

__device__ __forceinline__ void scan_share(int64_t n, int G, int64_t& t0, int64_t& t1) {
  const int64_t nt = (n + kScanTile - 1) / kScanTile;
  t0 = (int64_t)blockIdx.x * nt / G;
  t1 = (int64_t)(blockIdx.x + 1) * nt / G;
}

__global__ void __launch_bounds__(kScanBlock)
k_scan_up(const uint32_t* __restrict__ in, const uint32_t* __restrict__ idx, int64_t n, uint32_t* __restrict__ sums,
          int G, uint32_t* __restrict__ gathered) {
  __shared__ uint32_t s_warp[kScanBlock / 64];
  int64_t t0, t1;
  scan_share(n, G, t0, t1);
  uint32_t tsum = 0;
  for (int64_t t = t0; t < t1; ++t) {
    const int64_t base = t * kScanTile + (int64_t)threadIdx.x;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
      const int64_t e = base + (int64_t)k * kScanBlock;  // coalesced over the lanes
      if (e < n) {
        const uint32_t v = idx ? in[idx[e]] : in[e];
        if (idx) gathered[e] = v;
        tsum += v;
      }
    }
  }
  uint32_t total;
  block_exclusive_scan(tsum, s_warp, total);
  if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

// total (optional): the sum of all elements, written by the last block.
__global__ void __launch_bounds__(kScanBlock)
k_scan_down(const uint32_t* __restrict__ in, const uint32_t* __restrict__ idx, uint32_t* __restrict__ out, int64_t n,
            const uint32_t* __restrict__ sums, int G, uint32_t* __restrict__ total_out) {
  __shared__ uint32_t s_warp[kScanBlock / 64];
  // start of this block's run: the sums of the blocks before it (G <= 4096: 16 per thread)
  uint32_t before = 0;
#pragma unroll
  for (int k = 0; k < kScanGrid / kScanBlock; ++k) {
    const int b = (int)threadIdx.x + k * kScanBlock;
    if (b < (int)blockIdx.x) before += sums[b];
  }
  uint32_t carry;
  block_exclusive_scan(before, s_warp, carry);
  int64_t t0, t1;
  scan_share(n, G, t0, t1);
  for (int64_t t = t0; t < t1; ++t) {
    const int64_t base = t * kScanTile + (int64_t)threadIdx.x * kScanItems;
    const bool full = base + kScanItems <= n;  // the lane's 8 elements as two 16-B accesses
    uint32_t v[kScanItems];
    uint32_t tsum = 0;
    if (full && !idx) {
      const uint4 a = *(const uint4*)(in + base), b = *(const uint4*)(in + base + 4);
      v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w; v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
    } else {
#pragma unroll
      for (int k = 0; k < kScanItems; ++k) {
        v[k] = 0u;
        if (base + k < n) v[k] = idx ? in[idx[base + k]] : in[base + k];
      }
    }
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) tsum += v[k];
    uint32_t tile_total;
    uint32_t run = carry + block_exclusive_scan(tsum, s_warp, tile_total);
    uint32_t o[kScanItems];
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
      o[k] = run;
      run += v[k];
    }
    if (full) {
      *(uint4*)(out + base) = make_uint4(o[0], o[1], o[2], o[3]);
      *(uint4*)(out + base + 4) = make_uint4(o[4], o[5], o[6], o[7]);
    } else {
#pragma unroll
      for (int k = 0; k < kScanItems; ++k)
        if (base + k < n) out[base + k] = o[k];
    }
    carry += tile_total;
  }
  if (total_out && blockIdx.x == (unsigned)(G - 1) && threadIdx.x == 0) total_out[0] = carry;
}

// block sums, then room for n gathered values
int64_t scan_temp_elems(int64_t n) { return kScanGrid + n + 1; }

static hipError_t scan_impl(const uint32_t* in, const uint32_t* idx, uint32_t* out, int64_t n, uint32_t* temp,
                            uint32_t* total, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int G = scan_grid(n);
  uint32_t* gathered = temp + kScanGrid;
  hipLaunchKernelGGL(k_scan_up, dim3(G), dim3(kScanBlock), 0, s, in, idx, n, temp, G, gathered);
  if (idx)
    hipLaunchKernelGGL(k_scan_down, dim3(G), dim3(kScanBlock), 0, s, gathered, nullptr, out, n, temp, G, total);
  else
    hipLaunchKernelGGL(k_scan_down, dim3(G), dim3(kScanBlock), 0, s, in, nullptr, out, n, temp, G, total);
  return hipGetLastError();
}

// Exclusive scan of n u32 values (in may equal out); temp holds scan_temp_elems(n).
hipError_t exclusive_scan(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* temp, hipStream_t s) {
  return scan_impl(in, nullptr, out, n, temp, nullptr, s);
}

// offsets[k] = sum of counts[order[j]] for j < k; total = sum of all.
hipError_t scan_counts(const uint32_t* counts, const uint32_t* order, uint32_t* offsets, int64_t n,
                       uint32_t* temp, uint32_t* total, hipStream_t s) {
  return scan_impl(counts, order, offsets, n, temp, total, s);
}

// ------------------------------------------------------------------ radix sort
// Stable LSD sort with 8-bit digits over a fixed grid of G blocks (even share: block g
// owns a contiguous run of 2048-key tiles, whatever the key count). Each pass:
//   up:      per-block digit counts (digit-major, counts[d * G + g]);
//   rowscan: one block per digit scans its row over the G blocks and writes the digit
//            total;
//   down:    each block takes the exclusive scan of the 256 digit totals plus its row
//            prefix as the global start of each digit, then walks its tiles in order:
//            every wave ranks its keys with ballot-based peer masks, the tile is placed
//            in LDS in (digit, original order) order and written out by consecutive lanes
//            (each digit's run goes to consecutive addresses), and the digit starts
//            advance by the tile's counts.
// Three launches per pass and a count matrix of 256 x G entries, independent of n.
constexpr int kSortBlock = 256;
constexpr int kSortItems = 8;
constexpr int kSortTile = kSortBlock * kSortItems;  // 2048 keys per tile
constexpr int kWaves = kSortBlock / 64;
constexpr int kSortGrid = 1024;                     // blocks of the up and down sweeps

// Elements to process: all of them when they fit, none after an overflow (the render is
// then empty and the overflow flag tells the host to re-plan).
__device__ __forceinline__ uint32_t sort_count(const uint32_t* n_dev, int64_t cap) {
  const uint32_t n = n_dev[0];
  return (int64_t)n <= cap ? n : 0u;
}

// Tiles [t0, t1) of block g among G for n keys.
__device__ __forceinline__ void sort_share(uint32_t n, int G, int64_t& t0, int64_t& t1) {
  const int64_t nt = ((int64_t)n + kSortTile - 1) / kSortTile;
  t0 = (int64_t)blockIdx.x * nt / G;
  t1 = (int64_t)(blockIdx.x + 1) * nt / G;
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
k_radix_up(const K* __restrict__ keys, const uint32_t* __restrict__ n_dev, int64_t cap, int shift,
           uint32_t mask, uint32_t* __restrict__ counts, int G) {
  __shared__ uint32_t s_h[kWaves][256];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int d = lane; d < 256; d += 64) s_h[wid][d] = 0;
  __syncthreads();
  const uint32_t n = sort_count(n_dev, cap);
  int64_t t0, t1;
  sort_share(n, G, t0, t1);
  for (int64_t t = t0; t < t1; ++t) {
    const int64_t base = t * kSortTile + (int64_t)wid * (64 * kSortItems);
#pragma unroll
    for (int r = 0; r < kSortItems; ++r) {
      const int64_t idx = base + r * 64 + lane;
      const bool ok = idx < n;
      const uint32_t d = ok ? (uint32_t)(keys[idx] >> shift) & mask : 0u;
      // one LDS add per distinct digit of the wave
      const uint64_t peers = digit_peers(d, ok);
      if (ok && lane == __ffsll((long long)peers) - 1) s_h[wid][d] += (uint32_t)__popcll(peers);
    }
  }
  __syncthreads();
  const int d = threadIdx.x;
  counts[(int64_t)d * G + blockIdx.x] = s_h[0][d] + s_h[1][d] + s_h[2][d] + s_h[3][d];
}

// Block d: exclusive scan of row d (G <= kSortGrid entries) in place, its total to totals[d].
__global__ void __launch_bounds__(256)
k_radix_rowscan(uint32_t* __restrict__ counts, int G, uint32_t* __restrict__ totals) {
  constexpr int kPer = kSortGrid / 256;
  __shared__ uint32_t s_warp[4];
  uint32_t* row = counts + (int64_t)blockIdx.x * G;
  uint32_t v[kPer], sum = 0;
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    const int i = (int)threadIdx.x * kPer + k;
    v[k] = i < G ? row[i] : 0u;
    sum += v[k];
  }
  uint32_t total;
  uint32_t run = block_exclusive_scan(sum, s_warp, total);
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    const int i = (int)threadIdx.x * kPer + k;
    if (i < G) row[i] = run;
    run += v[k];
  }
  if (threadIdx.x == 0) totals[blockIdx.x] = total;
}

template <typename K>
__global__ void __launch_bounds__(kSortBlock)
k_radix_down(const K* __restrict__ kin, const uint32_t* __restrict__ vin, K* __restrict__ kout,
             uint32_t* __restrict__ vout, const uint32_t* __restrict__ n_dev, int64_t cap, int shift, uint32_t mask,
             const uint32_t* __restrict__ counts, const uint32_t* __restrict__ totals, int G) {
  __shared__ uint32_t s_cnt[kWaves][256];   // keys per (wave, digit), then the wave's offset
  __shared__ uint32_t s_start[256];         // first LDS slot of each digit in the tile
  __shared__ uint32_t s_tot[256];           // keys of each digit in the tile
  __shared__ uint32_t s_base[256];          // global position of the block's next key of each digit
  __shared__ uint32_t s_warp[kWaves];
  __shared__ K s_key[kSortTile];
  __shared__ uint32_t s_val[kSortTile];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const uint32_t n = sort_count(n_dev, cap);
  int64_t t0, t1;
  sort_share(n, G, t0, t1);
  if (t0 >= t1) return;
  {
    const int d = threadIdx.x;
    uint32_t all;
    const uint32_t start = block_exclusive_scan(totals[d], s_warp, all);
    s_base[d] = start + counts[(int64_t)d * G + blockIdx.x];
  }
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  for (int64_t t = t0; t < t1; ++t) {
    for (int d = lane; d < 256; d += 64) s_cnt[wid][d] = 0;
    __syncthreads();
    const int64_t blk0 = t * kSortTile;
    const int64_t base = blk0 + (int64_t)wid * (64 * kSortItems);
    K key[kSortItems];
    uint32_t val[kSortItems], rank[kSortItems], dig[kSortItems];
#pragma unroll
    for (int r = 0; r < kSortItems; ++r) {
      const int64_t idx = base + r * 64 + lane;
      const bool ok = idx < n;
      key[r] = ok ? kin[idx] : (K)0;
      val[r] = ok ? vin[idx] : 0u;
      const uint32_t d = (uint32_t)(key[r] >> shift) & mask;
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
    // digit totals of the tile, their exclusive scan (LDS start of each digit) and each
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
      s_start[d] = block_exclusive_scan(tot, s_warp, all);
      s_tot[d] = tot;
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
    for (int i = threadIdx.x; i < nblk; i += kSortBlock) {
      const K k = s_key[i];
      const uint32_t d = (uint32_t)(k >> shift) & mask;
      const uint32_t pos = s_base[d] + ((uint32_t)i - s_start[d]);
      kout[pos] = k;
      vout[pos] = s_val[i];
    }
    __syncthreads();
    s_base[threadIdx.x] += s_tot[threadIdx.x];
  }
}

static int sort_grid(int64_t cap) {
  return (int)std::min<int64_t>(kSortGrid, std::max<int64_t>(1, (cap + kSortTile - 1) / kSortTile));
}

int64_t sort_temp_elems(int64_t cap) { return 256 * (int64_t)sort_grid(cap) + 256; }

// Sorts (keys[0], vals[0]) on bits [0, nbits) using (keys[1], vals[1]) as the double buffer;
// *which receives the index of the buffer that holds the result.
hipError_t radix_sort_u32(uint32_t* keys[2], uint32_t* vals[2], const uint32_t* n_dev, int64_t cap, int nbits,
                          uint32_t* temp, int* which, hipStream_t s) {
  *which = 0;
  if (cap <= 0) return hipSuccess;
  const int G = sort_grid(cap);
  uint32_t* counts = temp;
  uint32_t* totals = temp + (int64_t)256 * G;
  // as many passes as 8-bit digits need, the bits spread evenly over them: fewer digit
  // values per pass give longer runs of equal digits in each tile, so the scatter writes
  // longer contiguous pieces (12-bit tile ids: two 6-bit passes rather than 8 + 4)
  const int passes = (nbits + 7) / 8;
  const int width = passes ? (nbits + passes - 1) / passes : 8;
  int cur = 0;
  for (int shift = 0; shift < nbits; shift += width) {
    const int w = std::min(width, nbits - shift);
    const uint32_t mask = (w >= 32) ? 0xFFFFFFFFu : ((1u << w) - 1u);
    hipLaunchKernelGGL(k_radix_up<uint32_t>, dim3(G), dim3(kSortBlock), 0, s, keys[cur], n_dev, cap, shift, mask,
                       counts, G);
    hipLaunchKernelGGL(k_radix_rowscan, dim3(256), dim3(256), 0, s, counts, G, totals);
    hipLaunchKernelGGL(k_radix_down<uint32_t>, dim3(G), dim3(kSortBlock), 0, s, keys[cur], vals[cur], keys[cur ^ 1],
                       vals[cur ^ 1], n_dev, cap, shift, mask, counts, totals, G);
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
