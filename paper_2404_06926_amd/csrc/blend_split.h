// Long-list split of the blend (see blend.hip): the per-chunk state a split forward
// leaves, the chunk length and ranges, and the work item of each workgroup of a blend
// launch. Shared by the pixel-order and the per-Gaussian blend kernels (internal).
#pragma once

#include "gs_common.h"
#include "kernels.h"

namespace gs {

// ---- split lists -------------------------------------------------------------------
// State of one chunk of a split tile, per pixel of the tile (field-major, 256 floats):
//   0    the chunk's own transmittance factor (product of its entries' 1 - alpha)
//   1-3  colour the chunk adds (sum of c a T, T the transmittance in front of the entry)
//   4    depth the chunk adds
//   5    transmittance after the chunk (where the pixel stopped, if it stopped in it)
//   6    bits: list position after the chunk's last contributor | kStopped | kDead
constexpr uint32_t kStopped = 1u << 31;   // the pixel's transmittance fell below kTMin here
constexpr uint32_t kDead = 1u << 30;      // ... before the chunk: the chunk adds nothing
constexpr uint32_t kPosMask = kDead - 1u;

__device__ __forceinline__ float* split_field(const SplitArg& sp, uint32_t slot, int f) {
  return sp.state + ((size_t)slot * kSplitFields + f) * (kTile * kTile);
}

// What the chunks c0, c0 + 1, ... of a split tile add at pixel q onto `acc`, in chunk order,
// up to the chunk the pixel stopped in and before a chunk it was dead for: the colour and
// depth sums, the transmittance after the last chunk taken and the largest
// last-contributor position.
// The state is read four chunks at a time, all loads issued before the first is used
// (a chunk-by-chunk walk waits one memory round trip per chunk); the sums still add chunk
// by chunk, so the result is the walk's.
struct ChunkSums {
  float c0, c1, c2, d, T;
  uint32_t last;
};
__device__ inline ChunkSums sum_chunks(const SplitArg& sp, uint32_t slot0, int c0, int nch, int q, ChunkSums acc) {
  ChunkSums r = acc;
  bool go = true;
  for (int cb = c0; cb < nch && go; cb += 4) {
    uint32_t bits[4];
    float f[4][5];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      bits[u] = kDead;
      if (cb + u < nch) {
        const uint32_t s = slot0 + (uint32_t)(cb + u);
        bits[u] = __float_as_uint(split_field(sp, s, 6)[q]);
#pragma unroll
        for (int k = 0; k < 5; ++k) f[u][k] = split_field(sp, s, 1 + k)[q];
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (go && (bits[u] & kDead)) go = false;
      if (go) {
        r.c0 += f[u][0];
        r.c1 += f[u][1];
        r.c2 += f[u][2];
        r.d += f[u][3];
        r.T = f[u][4];
        r.last = max(r.last, bits[u] & kPosMask);
        if (bits[u] & kStopped) go = false;
      }
    }
  }
  return r;
}

// Chunk length for a render with n_inst instances (par > 0).
__device__ __forceinline__ uint32_t chunk_len(uint32_t n_inst, int32_t par, int32_t min_len) {
  const uint32_t L = max((n_inst + (uint32_t)par - 1u) / (uint32_t)par, (uint32_t)min_len);
  return (L + 63u) & ~63u;
}

// Chunk c of a list of n entries cut into nch near-equal chunks: [begin, end).
__device__ __forceinline__ void chunk_range(int n, int nch, int c, int& begin, int& end) {
  begin = (int)((int64_t)c * n / nch);
  end = (int)((int64_t)(c + 1) * n / nch);
}

struct BlendItem {
  int tile, c, nch, begin, end;  // chunk c of nch covers list positions [begin, end)
  uint32_t slot0;                // first state slot of the tile, kNoSlot if not split
};

// Work of block b: blocks [0, par) take the chunks >= 1 of split tiles (the long lists
// start first), blocks [par, par + tiles) take tile b - par, whole or its chunk 0.
// Returns false (uniformly over the block) for a block without work.
__device__ __forceinline__ bool blend_item(const SplitArg& sp, const uint2* __restrict__ ranges, BlendItem& it) {
  const int b = (int)blockIdx.x;
  int tile = b - sp.par, c = 0;
  if (b < sp.par) {
    if ((uint32_t)b >= min(sp.counts[0], (uint32_t)sp.par)) return false;
    const uint2 e = sp.extra[b];
    if (e.x == kNoSlot) return false;
    tile = (int)e.x;
    c = (int)e.y;
  }
  const uint2 rg = ranges[tile];
  const int n = (int)(rg.y - rg.x);
  it.tile = tile;
  it.c = c;
  it.slot0 = sp.par > 0 ? sp.tile_slot[tile] : kNoSlot;
  if (it.slot0 == kNoSlot) {
    it.nch = 1;
    it.begin = 0;
    it.end = n;
  } else {
    const int L = (int)chunk_len(*sp.n_inst, sp.par, sp.min_len);
    it.nch = (n + L - 1) / L;
    chunk_range(n, it.nch, c, it.begin, it.end);
  }
  return true;
}


// blocks [0, par) for the chunks >= 1 of split tiles, then one per tile
inline dim3 item_grid(const ViewsArg& va, const SplitArg& sp) {
  return dim3((unsigned)(va.total_tiles + (sp.par > 0 ? sp.par : 0)));
}

}  // namespace gs
