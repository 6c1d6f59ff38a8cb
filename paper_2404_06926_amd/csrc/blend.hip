// Front-to-back blending (Sec. III-A Eq. 4-5, 7) with the per-keyframe exposure affine
// (Sec. III-C.3), and its reverse-order adjoint.
//
// One workgroup of 256 lanes (4 waves) per 16x16 tile; each wave owns one 8x8 quadrant,
// one pixel per lane. The tile's depth-sorted list is staged through LDS in batches of
// 256 entries (one gather of 36 B per lane from the 64-B projection record). While
// staging, each lane also tests its entry's footprint against the four quadrants; a wave
// skips entries whose footprint misses its quadrant. The test uses the footprint
// threshold widened by 1e-4 (relative and absolute), so a skipped entry would have been
// skipped by the per-pixel alpha cut-off as well and the outputs are unchanged.
//
// Launch shapes: PX pixels per lane (1, 2 or 4), 256 / PX lanes per tile, so the per-entry
// LDS reads and the per-Gaussian wave reductions of the backward are shared by PX pixels.
//
// The forward also writes, for views that ask, the depth map (Eq. 6) and the opacity map
// (Eq. 7, as 1 - T_final).
//
// The forward saves per pixel the final transmittance and the list position after the
// last contributor; the backward starts from them (no forward replay), walks the list
// from that position down to 0, recovers T_i = T_{i+1} / (1 - alpha_i), keeps the colour
// seen behind the current Gaussian, and reduces each Gaussian's nine gradient terms over
// the 64 lanes of a wave with DPP row operations before one atomic add per wave and field.
//
// Long lists. A workgroup walks its tile's list serially per pixel, so a tile whose list
// is much longer than the others (the horizon of a street scene gathers thousands of
// pixel-sized Gaussians) sets the duration of the whole launch. Such lists are cut into
// chunks (SplitArg, kernels.h) that separate workgroups blend:
//   1. k_blend_trans: for every chunk but the last, each pixel's product of (1 - alpha)
//      over the chunk's entries.
//   2. k_blend_fwd: each chunk starts from the product of the earlier chunks' factors and
//      blends its entries with the cut-offs of the serial walk (a pixel whose
//      transmittance in front of the chunk is already below the stop threshold takes
//      nothing from it), leaving its partial colour, depth, transmittance and last
//      contributor per pixel.
//   3. k_split_merge: adds the chunks up in depth order and writes the pixel outputs.
//   4. k_blend_bwd: each chunk starts its reverse walk from its own transmittance and the
//      colour, depth and opacity seen behind it (the later chunks and the background)
//      instead of from the final transmittance and the background.
// The passes are separate launches: the kernel boundary is what makes one workgroup's
// writes visible to another, with no cache write-back per workgroup.
// Front-to-back compositing is associative (C = C_front + T_front C_back, T = T_front
// T_back), so the split changes results only by FP32 rounding order; a stop decision
// within rounding of the threshold may fall one entry differently, as between any two
// orders of evaluation.
#include "blend_split.h"
#include "gs_common.h"
#include "kernels.h"

namespace gs {

constexpr int kBlendBlock = 256;
#define NW_OF(PX) (kBlendBlock / (PX) / 64)

// 4-bit mask of the tile's 8x8 quadrants (bit q: x half q & 1, y half q >> 1) that the
// footprint {q <= thr (1 + 1e-4) + 1e-4} reaches at some pixel centre, with
// q = A dx^2 + 2B dx dy + C dy^2 (offsets from the mean). A quadrant is reached when it
// holds the mean, else when the smaller of the 1-D minima of q, clamped to the quadrant, on
// its edges nearest the mean passes (the segment from any point of the quadrant to the mean,
// along which the convex q falls, crosses one of them inside the quadrant). The two x
// halves share their nearest x edge and its unclamped minimiser, the two y halves likewise,
// so each quadrant adds only its clamps and two quadratics. iA = 1/A, iC = 1/C: the
// hardware reciprocal, whose rounding moves a clamped minimum's position by an ulp and so q
// only at second order, well inside the margin. A projected conic is positive definite
// (A, C > 0), so the minimisers are finite and each clamp is one median of three.
__device__ __forceinline__ uint32_t quadrant_mask(float4 r0, float4 r1, float thr, int tx, int ty) {
  const float t = thr * 1.0001f + 1e-4f;
  const float A = r0.z, B = r0.w, C = r1.x;
  const float iA = __builtin_amdgcn_rcpf(A), iC = __builtin_amdgcn_rcpf(C);
  float xl[2], xh[2], ex[2], dyu[2], ax[2], bx[2], yl[2], yh[2], ey[2], dxu[2], cy[2], by[2];
  bool inx[2], iny[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    xl[h] = (float)(tx * kTile + 8 * h) + 0.5f - r0.x;  // pixel-centre offsets of the half
    xh[h] = xl[h] + 7.f;
    inx[h] = xl[h] <= 0.f && xh[h] >= 0.f;
    ex[h] = xl[h] > 0.f ? xl[h] : xh[h];
    dyu[h] = -(B * ex[h]) * iC;  // minimiser of q along the edge x = ex
    ax[h] = A * ex[h] * ex[h];   // q(ex, dy) = ax + bx dy + C dy^2
    bx[h] = 2.f * B * ex[h];
    yl[h] = (float)(ty * kTile + 8 * h) + 0.5f - r0.y;
    yh[h] = yl[h] + 7.f;
    iny[h] = yl[h] <= 0.f && yh[h] >= 0.f;
    ey[h] = yl[h] > 0.f ? yl[h] : yh[h];
    dxu[h] = -(B * ey[h]) * iA;  // minimiser of q along the edge y = ey
    cy[h] = C * ey[h] * ey[h];   // q(dx, ey) = cy + by dx + A dx^2
    by[h] = 2.f * B * ey[h];
  }
  uint32_t m = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int h = q & 1, v = q >> 1;
    const float dy = __builtin_amdgcn_fmed3f(dyu[h], yl[v], yh[v]);
    const float dx = __builtin_amdgcn_fmed3f(dxu[v], xl[h], xh[h]);
    const float qx = fmaf(C * dy, dy, fmaf(bx[h], dy, ax[h]));
    const float qy = fmaf(A * dx, dx, fmaf(by[v], dx, cy[v]));
    if ((inx[h] && iny[v]) || (!inx[h] && qx <= t) || (!iny[v] && qy <= t)) m |= 1u << q;
  }
  return m;
}

template <int CTRL, int ROWS>
__device__ __forceinline__ float dpp_f(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROWS, 0xf, false));
}

// Sum over each row of 16 lanes with DPP row operations, valid in every lane of the row.
__device__ __forceinline__ float row_sum16(float x) {
  x += dpp_f<0xB1, 0xf>(x);   // quad_perm [1,0,3,2]
  x += dpp_f<0x4E, 0xf>(x);   // quad_perm [2,3,0,1]
  x += dpp_f<0x141, 0xf>(x);  // row_half_mirror: 8-lane sums
  x += dpp_f<0x140, 0xf>(x);  // row_mirror: 16-lane sums
  return x;
}

// Sum over the 64 lanes with DPP row operations; the total is valid in lane 63.
__device__ __forceinline__ float wave_sum_to_63(float x) {
  x = row_sum16(x);
  x += dpp_f<0x142, 0xa>(x);  // row_bcast:15 into rows 1 and 3
  x += dpp_f<0x143, 0xc>(x);  // row_bcast:31 into rows 2 and 3
  return x;
}

// dst = src(lane - n) + src on the lanes of banks 1 and 3 (lane bit 2 set; n = 4) or of
// banks 2 and 3 (lane bit 3 set; n = 8) of every row of 16; the other lanes keep dst. DPP's
// bank mask has no intrinsic form that keeps dst, hence the instruction is written out; the
// two wait states a DPP read of a freshly written register needs come first.
__device__ __forceinline__ void add_from_below4(float& dst, float src) {
  asm("s_nop 1\n\tv_add_f32_dpp %0, %1, %1 row_shr:4 row_mask:0xf bank_mask:0xa" : "+v"(dst) : "v"(src));
}
__device__ __forceinline__ void add_from_below8(float& dst, float src) {
  asm("s_nop 1\n\tv_add_f32_dpp %0, %1, %1 row_shr:8 row_mask:0xf bank_mask:0xc" : "+v"(dst) : "v"(src));
}

// Sums over each row of 16 lanes of eight values at once, transposing while reducing:
// each exchange step halves the values a lane carries (the lane keeps one half, its partner
// the other), so 8 values cost 4 + 2 + 1 exchanges instead of 8 per step. The steps over
// lane bits 2 and 3 (partners in the same row) need no selects: one DPP add from the lane
// above writes every lane, a bank-masked DPP add from the lane below then overwrites the
// lanes that keep the other half. Then lane bit 0 (a select pair and a quad_perm add) and
// lane bit 1 (quad_perm). On return lane L holds its row's total of v[term_of_lane(L)]
// (lanes with bit 1 set repeat their partner's).
__device__ __forceinline__ float row_sum8_transposed(const float (&v)[8], int lane) {
#pragma clang fp contract(off)  // each first add must stay a DPP add, not fuse with a product
  float w[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {  // lane bit 2: keep v[k] (bit clear) or v[k + 4]
    w[k] = v[k] + dpp_f<0x104, 0xf>(v[k]);  // row_shl:4, from lane + 4
    add_from_below4(w[k], v[k + 4]);
  }
  float x[2];
#pragma unroll
  for (int k = 0; k < 2; ++k) {  // lane bit 3: keep w[k] or w[k + 2]
    x[k] = w[k] + dpp_f<0x108, 0xf>(w[k]);  // row_shl:8, from lane + 8
    add_from_below8(x[k], w[k + 2]);
  }
  const bool b0 = lane & 1;  // lane bit 0: keep x[0] or x[1]
  const float send = b0 ? x[0] : x[1];
  const float keep = b0 ? x[1] : x[0];
  float y = keep + dpp_f<0xB1, 0xf>(send);  // quad_perm [1,0,3,2]: from lane ^ 1
  y += dpp_f<0x4E, 0xf>(y);                 // quad_perm [2,3,0,1]: lane bit 1
  return y;
}

// Adds the four rows of 16 lanes: on return every lane holds the sum of its value over the
// lanes L, L ^ 16, L ^ 32 and L ^ 48 (two lane swaps and two adds, no LDS round trip).
__device__ __forceinline__ float add_rows(float y) {
  const auto h = __builtin_amdgcn_permlane32_swap(__float_as_uint(y), __float_as_uint(y), false, false);
  y = __uint_as_float(h[0]) + __uint_as_float(h[1]);
  const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(y), __float_as_uint(y), false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

// index of the value whose total lane L holds after row_sum8_transposed: lane bits 2, 3, 0
// give bits 2, 1, 0 of the index (lanes 0, 1, 4, 5, 8, 9, 12, 13 of a row hold the eight
// totals)
__device__ __forceinline__ int term_of_lane(int lane) {
  return (((lane >> 2) & 1) << 2) | (((lane >> 3) & 1) << 1) | (lane & 1);
}

__device__ __forceinline__ uint32_t wave_max_u32(uint32_t x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x = max(x, (uint32_t)__shfl_xor((int)x, o, 64));
  return x;
}

// Pixels of a lane. PX pixels per lane, 256 / PX lanes (4 / PX waves) per tile:
//   PX = 1: wave w owns quadrant w, one pixel per lane;
//   PX = 2: wave w owns the 8-wide column half w, pixels (x, y) and (x, y + 8);
//   PX = 4: one wave owns the tile, pixel k of a lane lies in quadrant k.
// Quadrant q covers x half q & 1 and y half q >> 1 of the tile.
template <int PX>
__device__ __forceinline__ void lane_pixel(int wid, int lane, int k, int& lx, int& ly) {
  if (PX == 1) {
    lx = 8 * (wid & 1) + (lane & 7);
    ly = 8 * (wid >> 1) + (lane >> 3);
  } else if (PX == 2) {
    lx = 8 * wid + (lane & 7);
    ly = 8 * k + (lane >> 3);
  } else {
    lx = 8 * (k & 1) + (lane & 7);
    ly = 8 * (k >> 1) + (lane >> 3);
  }
}

template <int PX>
__device__ __forceinline__ int pixel_quadrant(int wid, int k) {
  return PX == 1 ? wid : (PX == 2 ? wid + 2 * k : k);
}

// quadrants covered by wave w
template <int PX>
__device__ __forceinline__ uint32_t wave_quadrants(int w) {
  return PX == 1 ? (1u << w) : (PX == 2 ? ((1u << w) | (1u << (w + 2))) : 0xFu);
}

// Per-wave lists of the staged batch: the entries t < cnt whose quadrant mask meets wave
// w's quadrants, in batch (depth) order, in s_list[w][0 .. s_len[w]). A wave then walks
// only the entries that can reach its pixels: with pixel-sized footprints (long lists of
// small Gaussians) most entries meet one quadrant. Called by every thread of the block.
template <int PX, int NW, int NT>
__device__ __forceinline__ void build_wave_lists(uint32_t m_own, int cnt, uint8_t (*s_list)[NT], int* s_len,
                                                 uint32_t (*s_wc)[NW]) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int t = threadIdx.x;
  const uint32_t m = t < cnt ? m_own : 0u;
  const uint64_t lt = lane ? (~0ull >> (64 - lane)) : 0ull;
  bool hit[NW];
  uint32_t rank[NW];
#pragma unroll
  for (int w2 = 0; w2 < NW; ++w2) {
    hit[w2] = (m & wave_quadrants<PX>(w2)) != 0u;
    const uint64_t b = __ballot(hit[w2]);
    rank[w2] = (uint32_t)__popcll(b & lt);
    if (lane == 0) s_wc[w2][wid] = (uint32_t)__popcll(b);
  }
  __syncthreads();
#pragma unroll
  for (int w2 = 0; w2 < NW; ++w2) {
    uint32_t off = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
      const uint32_t c = s_wc[w2][w];
      if (w < wid) off += c;
      tot += c;
    }
    if (hit[w2]) s_list[w2][off + rank[w2]] = (uint8_t)t;
    if (t == 0) s_len[w2] = (int)tot;
  }
  __syncthreads();
}

// One pixel's outputs from its pre-exposure colour (blended colour without background),
// final transmittance, list position after the last contributor and depth.
template <bool DEPTH>
__device__ __forceinline__ void write_pixel(const ViewDev& V, int64_t p, float c0, float c1, float c2, float T,
                                            uint32_t last, float D) {
  const int64_t P = (int64_t)V.W * V.H;
  const float pre0 = c0 + T * V.bg[0], pre1 = c1 + T * V.bg[1], pre2 = c2 + T * V.bg[2];
  float o0 = pre0, o1 = pre1, o2 = pre2;
  if (V.exposure) {
    const float* E = V.exposure;
    o0 = E[0] * pre0 + E[1] * pre1 + E[2] * pre2 + E[3];
    o1 = E[4] * pre0 + E[5] * pre1 + E[6] * pre2 + E[7];
    o2 = E[8] * pre0 + E[9] * pre1 + E[10] * pre2 + E[11];
  }
  V.out_rgb[p] = o0;
  V.out_rgb[P + p] = o1;
  V.out_rgb[2 * P + p] = o2;
  V.out_T[p] = T;
  V.out_nc[p] = last;
  if (DEPTH && V.out_depth) V.out_depth[p] = D;
  if (V.out_opac) V.out_opac[p] = 1.0f - T;  // Eq. 7 telescoped: sum a_i T_i = 1 - T_final
}

// Pass 3 of a split tile: block b merges the tile of extra item b when that item is the
// tile's chunk 1 (one block per split tile); one pixel per lane. Per pixel the chunks are
// taken in depth order up to the one the pixel stopped in.
template <bool DEPTH>
__global__ void __launch_bounds__(kTile * kTile)
k_split_merge(ViewsArg va, const uint2* __restrict__ ranges, SplitArg sp) {
  if (blockIdx.x >= min(sp.counts[0], (uint32_t)sp.par)) return;
  const uint2 e = sp.extra[blockIdx.x];
  if (e.x == kNoSlot || e.y != 1u) return;
  const int tile = (int)e.x;
  const uint32_t slot0 = sp.tile_slot[tile];
  const uint2 rg = ranges[tile];
  const int n = (int)(rg.y - rg.x);
  const int L = (int)chunk_len(*sp.n_inst, sp.par, sp.min_len);
  const int nch = (n + L - 1) / L;
  const ViewDev& V = va.v[view_of_tile(va, tile)];
  const int lt = tile - V.tile_base;
  const int tx = lt % V.tiles_x, ty = lt / V.tiles_x;
  const int q = (int)threadIdx.x;
  const int px = tx * kTile + (q & 15), py = ty * kTile + (q >> 4);
  if (px >= V.W || py >= V.H) return;
  const ChunkSums r = sum_chunks(sp, slot0, 0, nch, q, ChunkSums{0.f, 0.f, 0.f, 0.f, 1.0f, 0u});
  write_pixel<DEPTH>(V, (int64_t)py * V.W + px, r.c0, r.c1, r.c2, r.T, r.last, r.d);
}

// Pass 1 of a split tile: block b takes chunk extra[b].y - 1 of tile extra[b].x (every
// chunk but the last), one pixel per lane as k_blend_fwd with PX = 1.
__global__ void __launch_bounds__(kBlendBlock)
k_blend_trans(ViewsArg va, const float4* __restrict__ rec, int32_t N, const uint32_t* __restrict__ vals,
              const uint32_t* __restrict__ emit_g, const uint2* __restrict__ ranges, SplitArg sp) {
  constexpr int NT = kBlendBlock, NW = NT / 64;
  __shared__ float4 s_a[NT];  // mx, my, A, B
  __shared__ float2 s_b[NT];  // C, o
  __shared__ uint8_t s_list[NW][NT];
  __shared__ int s_len[NW];
  __shared__ uint32_t s_wc[NW][NW];
  if (blockIdx.x >= min(sp.counts[0], (uint32_t)sp.par)) return;
  const uint2 e = sp.extra[blockIdx.x];
  if (e.x == kNoSlot) return;
  const int tile = (int)e.x, c = (int)e.y - 1;
  const uint32_t slot0 = sp.tile_slot[tile];
  const uint2 rg = ranges[tile];
  const int n = (int)(rg.y - rg.x);
  const int L = (int)chunk_len(*sp.n_inst, sp.par, sp.min_len);
  int begin, end;
  chunk_range(n, (n + L - 1) / L, c, begin, end);
  const int v = view_of_tile(va, tile);
  const ViewDev& V = va.v[v];
  const int lt = tile - V.tile_base;
  const int tx = lt % V.tiles_x, ty = lt / V.tiles_x;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const float4* vrec = rec + (size_t)v * N * 4;
  int lx, ly;
  lane_pixel<1>(wid, lane, 0, lx, ly);
  const float pxc = (float)(tx * kTile + lx) + 0.5f, pyc = (float)(ty * kTile + ly) + 0.5f;
  // T carries the pixel's state in its sign, as in the forward: a pixel outside the image or
  // whose product fell below the stop threshold keeps -T
  float T = (tx * kTile + lx < V.W && ty * kTile + ly < V.H) ? 1.0f : -1.0f;
  for (int base = begin; base < end; base += NT) {
    if (__syncthreads_count(T < 0.0f) == NT) break;
    const int kk = base + (int)threadIdx.x;
    uint32_t qm = 0;
    if (kk < end) {
      const uint32_t g = emit_g[vals[rg.x + kk]];
      const float4* r = vrec + (size_t)g * 4;
      const float4 r0 = r[0], r1 = r[1], r2 = r[2];
      s_a[threadIdx.x] = blend_stage_a(r0);
      s_b[threadIdx.x] = make_float2(blend_stage_c(r1.x), r1.y);
      qm = quadrant_mask(r0, r1, r2.w, tx, ty);
    }
    build_wave_lists<1, NW, NT>(qm, min(NT, end - base), s_list, s_len, s_wc);
    // wave-uniform and branch-free, as the forward's loop: a pixel that does not take an
    // entry keeps its T by selection
    const int len = __builtin_amdgcn_readfirstlane(s_len[wid]);
    for (int jj = 0; jj < len; ++jj) {
      const bool live = !(T < 0.0f);
      if (!__any(live)) break;
      const int j = __builtin_amdgcn_readfirstlane((int)s_list[wid][jj]);
      const float4 a = s_a[j];
      const float2 b = s_b[j];
      float dx, dy;
      const float power = blend_power2(a.x, a.y, a.z, a.w, b.x, pxc, pyc, dx, dy);
      const float alpha = fminf(kAlphaMax, b.y * blend_exp2(power));
      const bool ok = live && !(power > 0.0f) && alpha >= kAlphaMin;
      const float Tn = T * (1.0f - alpha);
      // below the threshold every later chunk is dead for this pixel whatever lies in
      // front: the product so far is kept, marked done
      T = ok ? (Tn < kTMin ? -Tn : Tn) : T;
    }
  }
  split_field(sp, slot0 + c, 0)[ly * kTile + lx] = fabsf(T);
}

// Items of a render: every tile longer than the chunk length and than `balance` times the
// mean list takes ceil(n / L) state slots and lists its chunks >= 1 as extra items. counts[0..1]
// are zero on entry.
__global__ void k_split_items(const uint2* __restrict__ ranges, int32_t n_tiles, SplitArg sp) {
  const int t = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (t >= n_tiles) return;
  const uint2 r = ranges[t];
  const uint32_t n = r.y > r.x ? r.y - r.x : 0u;
  const uint32_t n_inst = *sp.n_inst;
  const uint32_t L = chunk_len(n_inst, sp.par, sp.min_len);
  // lists within `balance` times the mean keep the launch balanced without a split
  const float keep = sp.balance * (float)n_inst / (float)n_tiles;
  uint32_t slot = kNoSlot;
  if (n > L && (float)n > keep) {
    const uint32_t nch = (n + L - 1u) / L;
    const uint32_t s0 = atomicAdd(&sp.counts[1], nch);
    const uint32_t e0 = atomicAdd(&sp.counts[0], nch - 1u);
    const uint32_t par = (uint32_t)sp.par;
    if (s0 + nch <= 2u * par && e0 + nch - 1u <= par) {
      slot = s0;
      for (uint32_t c = 1; c < nch; ++c) sp.extra[e0 + c - 1u] = make_uint2((uint32_t)t, c);
    } else {
      // cannot happen with L >= instances / par; kept consistent anyway: the tile is
      // blended whole and its reserved items are marked empty
      for (uint32_t c = 1; c < nch && e0 + c - 1u < par; ++c) sp.extra[e0 + c - 1u] = make_uint2(kNoSlot, 0u);
    }
  }
  sp.tile_slot[t] = slot;
}

hipError_t split_items(const uint2* ranges, int32_t n_tiles, const SplitArg& sp, hipStream_t s) {
  if (n_tiles <= 0 || sp.par <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_split_items, dim3((n_tiles + 255) / 256), dim3(256), 0, s, ranges, n_tiles, sp);
  return hipGetLastError();
}

// DEPTH: also accumulate the depth map D = sum d_i a_i T_i (Eq. 6) for views that ask.
template <int PX, bool DEPTH>
__global__ void __launch_bounds__(kBlendBlock / PX)
k_blend_fwd(ViewsArg va, const float4* __restrict__ rec, int32_t N, const uint32_t* __restrict__ vals,
            const uint32_t* __restrict__ emit_g, const uint2* __restrict__ ranges, SplitArg sp) {
  constexpr int NT = kBlendBlock / PX;
  // per entry: (mx, my, A, B), (C, o, r, g), (b, camera-frame depth, quadrant mask bits, -):
  // one 48-B record, so a wave-uniform entry index addresses all of it from one register
  __shared__ float4 s_r[NT][3];
  __shared__ uint8_t s_list[NW_OF(PX)][NT];   // per-wave entry lists of the batch
  __shared__ int s_len[NW_OF(PX)];
  __shared__ uint32_t s_wc[NW_OF(PX)][NW_OF(PX)];
  BlendItem it;
  if (!blend_item(sp, ranges, it)) return;
  const int tile = it.tile;
  const bool split = it.slot0 != kNoSlot;
  const uint32_t slot = it.slot0 + (uint32_t)it.c;
  // the depth sum is always accumulated (one FMA): a split tile carries it in its chunk
  // state whether or not this render outputs the map, since a backward through the depth
  // map needs the depth seen behind each chunk
  const int v = view_of_tile(va, tile);
  const ViewDev& V = va.v[v];
  const int lt = tile - V.tile_base;
  const int tx = lt % V.tiles_x, ty = lt / V.tiles_x;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const uint2 rg = ranges[tile];
  const float4* vrec = rec + (size_t)v * N * 4;

  // T carries the pixel's state in its sign: a pixel that is done (outside the image,
  // stopped in an earlier chunk or at an entry of this one) keeps -T, so one comparison
  // gives both its transmittance and whether it still blends
  float pxc[PX], pyc[PX], T[PX], C0[PX], C1[PX], C2[PX], Dm[PX];
  uint32_t last[PX];
  bool inside[PX], dead[PX];
#pragma unroll
  for (int k = 0; k < PX; ++k) {
    int lx, ly;
    lane_pixel<PX>(wid, lane, k, lx, ly);
    const int px = tx * kTile + lx, py = ty * kTile + ly;
    pxc[k] = (float)px + 0.5f;
    pyc[k] = (float)py + 0.5f;
    inside[k] = px < V.W && py < V.H;
    dead[k] = false;
    T[k] = 1.0f;
    if (split && it.c > 0 && inside[k]) {
      // transmittance in front of the chunk: the earlier chunks' factors
      const int q = ly * kTile + lx;
      for (int c = 0; c < it.c; ++c) T[k] *= split_field(sp, it.slot0 + c, 0)[q];
      dead[k] = T[k] < kTMin;  // stopped in an earlier chunk
    }
    if (!inside[k] || dead[k]) T[k] = -T[k];
    C0[k] = C1[k] = C2[k] = Dm[k] = 0.0f;
    last[k] = 0;
  }
  auto all_done = [&]() {
    bool d = true;
#pragma unroll
    for (int k = 0; k < PX; ++k) d = d && T[k] < 0.0f;
    return d;
  };
  for (int base = it.begin; base < it.end; base += NT) {
    if (__syncthreads_count(all_done()) == NT) break;
    const int kk = base + (int)threadIdx.x;
    uint32_t qm = 0;
    if (kk < it.end) {
      const uint32_t g = emit_g[vals[rg.x + kk]];
      const float4* r = vrec + (size_t)g * 4;
      const float4 r0 = r[0], r1 = r[1], r2 = r[2];
      qm = quadrant_mask(r0, r1, r2.w, tx, ty);
      s_r[threadIdx.x][0] = blend_stage_a(r0);
      s_r[threadIdx.x][1] = make_float4(blend_stage_c(r1.x), r1.y, r1.z, r1.w);
      s_r[threadIdx.x][2] = make_float4(r2.x, r2.y, __uint_as_float(qm), 0.f);
    }
    const int cnt = min(NT, it.end - base);
    build_wave_lists<PX, NW_OF(PX), NT>(qm, cnt, s_list, s_len, s_wc);
    // wave-uniform loop (list length and entry index scalar); a pixel that does not take an
    // entry (done, outside the entry's quadrants, power > 0, alpha below the cut-off, or
    // stopping at it) runs the same arithmetic with weight 0, which adds exact zeros, and
    // keeps its T and last contributor by selection: no per-pixel branches
    const int len = __builtin_amdgcn_readfirstlane(s_len[wid]);
    for (int jj = 0; jj < len; ++jj) {
      // one comparison per pixel gives both the wave's exit test and the pixel's own
      bool live[PX], any_live = false;
#pragma unroll
      for (int k = 0; k < PX; ++k) {
        live[k] = !(T[k] < 0.0f);
        any_live = any_live || live[k];
      }
      if (!__any(any_live)) break;
      const int j = __builtin_amdgcn_readfirstlane((int)s_list[wid][jj]);
      const float4 a = s_r[j][0];
      const float4 b = s_r[j][1];
      const float4 cr = s_r[j][2];
      // with one pixel per lane a wave's list holds only entries that meet its quadrant
      const uint32_t m = PX == 1 ? 1u : __float_as_uint(cr.z);
      const uint32_t pos1 = (uint32_t)(base + j + 1);
#pragma unroll
      for (int k = 0; k < PX; ++k) {
        float dx, dy;
        const float power = blend_power2(a.x, a.y, a.z, a.w, b.x, pxc[k], pyc[k], dx, dy);
        const float alpha = fminf(kAlphaMax, b.y * blend_exp2(power));
        const bool ok = (PX == 1 || ((m >> pixel_quadrant<PX>(wid, k)) & 1u)) && live[k] &&
                        !(power > 0.0f) && alpha >= kAlphaMin;
        const float Tn = T[k] * (1.0f - alpha);
        const bool below = Tn < kTMin;
        const bool take = ok && !below;
        const float w = take ? alpha * T[k] : 0.0f;
        C0[k] += b.z * w;
        C1[k] += b.w * w;
        C2[k] += cr.x * w;
        Dm[k] += cr.y * w;  // (kept only where the depth is wanted: one FMA, no select)
        // taken: T after the entry; stopping here: done, T kept (as -T)
        const float Tnext = below ? -T[k] : Tn;
        T[k] = ok ? Tnext : T[k];
        last[k] = take ? pos1 : last[k];
      }
    }
  }
  if (!split) {
#pragma unroll
    for (int k = 0; k < PX; ++k) {
      if (!inside[k]) continue;
      const int64_t p = (int64_t)(int)pyc[k] * V.W + (int)pxc[k];
      write_pixel<DEPTH>(V, p, C0[k], C1[k], C2[k], fabsf(T[k]), last[k], Dm[k]);
    }
    return;
  }
#pragma unroll
  for (int k = 0; k < PX; ++k) {
    int lx, ly;
    lane_pixel<PX>(wid, lane, k, lx, ly);
    const int q = ly * kTile + lx;
    const bool done = T[k] < 0.0f;
    T[k] = fabsf(T[k]);
    const uint32_t bits = last[k] | (dead[k] ? kDead : (inside[k] && done ? kStopped : 0u));
    split_field(sp, slot, 1)[q] = C0[k];
    split_field(sp, slot, 2)[q] = C1[k];
    split_field(sp, slot, 3)[q] = C2[k];
    split_field(sp, slot, 4)[q] = Dm[k];
    split_field(sp, slot, 5)[q] = T[k];
    split_field(sp, slot, 6)[q] = __uint_as_float(bits);
  }
}

// DET = false: the waves' per-Gaussian sums of a batch meet in LDS (LDS float atomics), and
// after the batch one float atomic per entry and term goes to g2d, with the terms of an
// entry on neighbouring lanes (one 48-B record per entry): a Gaussian that reaches several
// quadrants of the tile costs one set of global atomics, not one per wave.
// DET = true: the waves' sums are added in wave order in LDS and every instance's
// gradient is written to inst_grad[emission index]; the exposure gradient of each tile is
// written to exp_part[tile] for a fixed-order reduction. No atomics, so the result does not
// depend on scheduling.
// MAPS: views may carry dL/dD and dL/dO (Eq. 6-7); they add to dL/dalpha through the same
// behind-the-Gaussian recursion with d_i and 1 in place of the colour (no background), and
// give a tenth gradient, dL/d(camera-frame depth) = sum_px a_i T_i dL/dD.
template <int PX, bool DET, bool MAPS>
__global__ void __launch_bounds__(kBlendBlock / PX)
k_blend_bwd(ViewsArg va, const float4* __restrict__ rec, int32_t N, const uint32_t* __restrict__ vals,
            const uint32_t* __restrict__ emit_g, const uint2* __restrict__ ranges, float* __restrict__ g2d,
            float* __restrict__ inst_grad, float* __restrict__ exp_part, SplitArg sp) {
  constexpr int NT = kBlendBlock / PX;
  constexpr int NW = NT / 64;
  constexpr int NG = MAPS ? 10 : 9;  // gradient terms per Gaussian
  // per entry: (mx, my, A, B), (C, o, r, g), (b, depth, -, -): one 48-B record, so a
  // wave-uniform entry index addresses all of it from one register
  __shared__ float4 s_r[NT][3];
  __shared__ uint32_t s_g[NT];
  __shared__ uint32_t s_e[DET ? NT : 1];
  __shared__ float s_part[DET ? NW : 1][DET ? NT : 1][NG];
  __shared__ float s_acc[DET ? 1 : NT][NG];  // batch sums (DET = false), zero between batches
  __shared__ uint8_t s_m[NT];
  __shared__ uint8_t s_list[NW][NT];   // per-wave entry lists of the batch
  __shared__ int s_len[NW];
  __shared__ uint32_t s_wc[NW][NW];
  __shared__ float s_red[NW][12];
  __shared__ uint32_t s_wmax[NW];
  BlendItem it;
  if (render_dropped(va) || !blend_item(sp, ranges, it)) return;
  if (!DET)
    for (int k = (int)threadIdx.x; k < NT * NG; k += NT) (&s_acc[0][0])[k] = 0.0f;
  const int tile = it.tile;
  const bool split = it.slot0 != kNoSlot;
  const uint32_t slot = it.slot0 + (uint32_t)it.c;
  const int v = view_of_tile(va, tile);
  const ViewDev& V = va.v[v];
  const int lt = tile - V.tile_base;
  const int tx = lt % V.tiles_x, ty = lt / V.tiles_x;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const uint2 rg = ranges[tile];
  const float4* vrec = rec + (size_t)v * N * 4;
  float* vg = g2d + (size_t)v * N * kGradFloats;
  const int64_t P = (int64_t)V.W * V.H;

  // per pixel: transmittance (recovered backwards), last contributor, dL/d(out), dL/d(pre)
  float pxc[PX], pyc[PX], T[PX], g0[PX], g1[PX], g2[PX], G0[PX], G1[PX], G2[PX];
  float B0[PX], B1[PX], B2[PX];  // colour seen behind the current Gaussian, normalised
  float gD[PX], gO[PX], BD[PX], BO[PX];  // map gradients and the maps seen behind (MAPS)
  uint32_t nc[PX];
  bool inside[PX];
  uint32_t ncmax = 0;
#pragma unroll
  for (int k = 0; k < PX; ++k) {
    int lx, ly;
    lane_pixel<PX>(wid, lane, k, lx, ly);
    const int px = tx * kTile + lx, py = ty * kTile + ly;
    pxc[k] = (float)px + 0.5f;
    pyc[k] = (float)py + 0.5f;
    inside[k] = px < V.W && py < V.H;
    T[k] = 1.0f;
    g0[k] = g1[k] = g2[k] = 0.0f;
    gD[k] = gO[k] = BD[k] = BO[k] = 0.0f;
    nc[k] = 0;
    if (inside[k]) {
      const int64_t p = (int64_t)py * V.W + px;
      T[k] = V.out_T[p];
      nc[k] = V.out_nc[p];
      g0[k] = V.dl_drgb[p];
      g1[k] = V.dl_drgb[P + p];
      g2[k] = V.dl_drgb[2 * P + p];
      if (MAPS) {
        if (V.dl_ddepth) gD[k] = V.dl_ddepth[p];
        if (V.dl_dopac) gO[k] = V.dl_dopac[p];
      }
    }
    // dL/d(pre-exposure colour) = A^T g
    G0[k] = g0[k];
    G1[k] = g1[k];
    G2[k] = g2[k];
    if (V.exposure) {
      const float* E = V.exposure;
      G0[k] = E[0] * g0[k] + E[4] * g1[k] + E[8] * g2[k];
      G1[k] = E[1] * g0[k] + E[5] * g1[k] + E[9] * g2[k];
      G2[k] = E[2] * g0[k] + E[6] * g1[k] + E[10] * g2[k];
    }
    B0[k] = V.bg[0];
    B1[k] = V.bg[1];
    B2[k] = V.bg[2];
    if (split && inside[k]) {
      // start after this chunk: its own transmittance, and what the later chunks up to the
      // one the pixel stopped in, then the background, add behind it (normalised)
      const int q = ly * kTile + lx;
      const float Tf = T[k];
      const ChunkSums cs = sum_chunks(sp, it.slot0, it.c + 1, it.nch, q,
                                      ChunkSums{Tf * B0[k], Tf * B1[k], Tf * B2[k], 0.f, 0.f, 0u});
      const float r0 = cs.c0, r1 = cs.c1, r2 = cs.c2, rd = cs.d;
      T[k] = split_field(sp, slot, 5)[q];
      // a chunk past the pixel's stop has no contributor there; keep its state finite
      const float inv = T[k] > 0.0f ? 1.0f / T[k] : 0.0f;
      B0[k] = r0 * inv;
      B1[k] = r1 * inv;
      B2[k] = r2 * inv;
      BD[k] = rd * inv;
      BO[k] = 1.0f - Tf * inv;
    }
    ncmax = max(ncmax, nc[k]);
  }
  // the gradient term whose wave total lane L < 16 holds after the entry loop's reduction
  const int term = lane == 2 ? 8 : ((MAPS && lane == 3) ? NG - 1 : term_of_lane(lane));
  const bool takes = lane < 16 && (!(lane & 2) || lane == 2 || (MAPS && lane == 3));
  float* const acc_lane = &s_acc[0][0] + term;
  const uint32_t wmax = wave_max_u32(ncmax);
  if (lane == 0) s_wmax[wid] = wmax;
  __syncthreads();
  int nmax = 0;
#pragma unroll
  for (int w = 0; w < NW; ++w) nmax = max(nmax, (int)s_wmax[w]);

  for (int end = min(nmax, it.end); end > it.begin; end -= NT) {
    const int base = __builtin_amdgcn_readfirstlane(max(it.begin, end - NT));
    const int cnt = end - base;
    __syncthreads();
    uint32_t qm = 0;
    if ((int)threadIdx.x < cnt) {
      const uint32_t e = vals[rg.x + base + threadIdx.x];
      const uint32_t g = emit_g[e];
      const float4* r = vrec + (size_t)g * 4;
      const float4 r0 = r[0], r1 = r[1], r2 = r[2];
      s_r[threadIdx.x][0] = blend_stage_a(r0);
      s_r[threadIdx.x][1] = make_float4(blend_stage_c(r1.x), r1.y, r1.z, r1.w);
      s_r[threadIdx.x][2] = make_float4(r2.x, r2.y, 0.f, 0.f);
      s_g[threadIdx.x] = g;
      qm = quadrant_mask(r0, r1, r2.w, tx, ty);
      s_m[threadIdx.x] = (uint8_t)qm;
      if (DET) {
        s_e[threadIdx.x] = e;
#pragma unroll
        for (int w = 0; w < NW; ++w)
#pragma unroll
          for (int f = 0; f < NG; ++f) s_part[w][threadIdx.x][f] = 0.f;
      }
    }
    build_wave_lists<PX, NW, NT>(qm, cnt, s_list, s_len, s_wc);
    // entries at or past the wave's max are idle (wave-uniform bounds and entry index: a
    // scalar loop)
    const int jtop = __builtin_amdgcn_readfirstlane(min(cnt, (int)wmax - base) - 1);
    for (int jj = __builtin_amdgcn_readfirstlane(s_len[wid]) - 1; jj >= 0; --jj) {
      const int j = __builtin_amdgcn_readfirstlane((int)s_list[wid][jj]);
      if (j > jtop) continue;
      const uint32_t m = PX == 1 ? 1u : s_m[j];  // (a wave's list meets its quadrant)
      const int pos = base + j;
      const float4 a = s_r[j][0];
      const float4 b = s_r[j][1];
      const float4 cr = s_r[j][2];
      const float c2 = cr.x;
      const float dep = MAPS ? cr.y : 0.0f;
      // per-lane sums of the gradient terms over the lane's pixels (the first pixel sets
      // them: adding to 0 would cost an operation, as 0 + x differs from x for x = -0)
      float gv[NG];
      auto add = [&](int k, int f, float x) { gv[f] = k == 0 ? x : gv[f] + x; };
      bool any = false;
      // Branch-free: a pixel that does not take this entry (outside the Gaussian's quadrant
      // mask, past its last contributor, power > 0 or alpha below the cut-off) runs the same
      // arithmetic with alpha = 0, which leaves its T and colour behind unchanged exactly
      // (T is selected, B + 0 (c - B) = B) and adds exact zeros to the sums.
#pragma unroll
      for (int k = 0; k < PX; ++k) {
        float dx, dy;
        const float power = blend_power2(a.x, a.y, a.z, a.w, b.x, pxc[k], pyc[k], dx, dy);
        const float ex = blend_exp2(power);
        const float araw = b.y * ex;
        const float alpha = fminf(kAlphaMax, araw);
        const bool on = (PX == 1 || ((m >> pixel_quadrant<PX>(wid, k)) & 1u)) && pos < (int)nc[k] &&
                        power <= 0.0f && alpha >= kAlphaMin;
        any = any || on;
        const float al = on ? alpha : 0.0f;
        // transmittance in front of this Gaussian (al = 0 leaves it as it is: the
        // reciprocal of 1 is exactly 1)
        T[k] = T[k] * __builtin_amdgcn_rcpf(1.0f - al);
        const float w = al * T[k];
        add(k, 6, w * G0[k]);
        add(k, 7, w * G1[k]);
        add(k, 8, w * G2[k]);
        // colour in front minus colour behind, per channel: dL/dalpha's factors, and the
        // step of the colour behind to the one in front of this Gaussian,
        // B <- alpha c + (1 - alpha) B = B + alpha (c - B)
        const float d0 = b.z - B0[k], d1 = b.w - B1[k], d2 = c2 - B2[k];
        // dL/dalpha = T (c - B) . G (+ the maps' terms)
        float dot = d0 * G0[k] + d1 * G1[k] + d2 * G2[k];
        B0[k] = fmaf(al, d0, B0[k]);
        B1[k] = fmaf(al, d1, B1[k]);
        B2[k] = fmaf(al, d2, B2[k]);
        if (MAPS) {
          const float dd = dep - BD[k], dO = 1.0f - BO[k];
          dot += dd * gD[k] + dO * gO[k];
          BD[k] = fmaf(al, dd, BD[k]);
          BO[k] = fmaf(al, dO, BO[k]);
          add(k, 9, w * gD[k]);
        }
        // dL/dpower = dL/dalpha * alpha = (alpha T) dot (no gradient through the clamp at
        // kAlphaMax; selected to zero where the pixel does not take the entry, whose colour
        // behind may not be finite there); its moments over the pixels, which the projection
        // backward turns into the 2D mean, conic and opacity gradients
        const float dpow = (on && araw <= kAlphaMax) ? w * dot : 0.0f;
        const float px_ = dpow * dx, py_ = dpow * dy;
        add(k, 0, px_);
        add(k, 1, py_);
        add(k, 2, px_ * dx);
        add(k, 3, px_ * dy);
        add(k, 4, py_ * dy);
        add(k, 5, dpow);
      }
      if (!__any(any)) continue;
      // wave totals: terms 0..7 transposed within each row of 16 lanes, which leaves lanes
      // 2 and 3 of a row as repeats; they take the row sums of terms 8 (and 9), then the
      // rows are added. Lane L < 16 ends with the total of term `term` (see above), and the
      // lanes that take one write or add it, one LDS instruction per entry.
      float g8[8];
#pragma unroll
      for (int f = 0; f < 8; ++f) g8[f] = gv[f];
      float val = row_sum8_transposed(g8, lane);   // (the cross-lane sums run on every lane)
      const float t8 = row_sum16(gv[8]);
      const float t9 = MAPS ? row_sum16(gv[NG - 1]) : 0.0f;
      val = (lane & 15) == 2 ? t8 : val;
      if (MAPS) val = (lane & 15) == 3 ? t9 : val;
      val = add_rows(val);
      if (DET) {
        if (takes) s_part[wid][j][term] = val;
      } else if (takes && val != 0.0f) {
        __hip_atomic_fetch_add(acc_lane + j * NG, val, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      }
    }
    if (!DET) {
      // the batch's sums to g2d; each read slot is cleared for the next batch
      __syncthreads();
      for (int idx = (int)threadIdx.x; idx < cnt * NG; idx += NT) {
        const int e = idx / NG, f = idx - e * NG;
        const float val = s_acc[e][f];
        if (val != 0.0f) {
          unsafeAtomicAdd(vg + (size_t)s_g[e] * kGradFloats + f, val);
          s_acc[e][f] = 0.0f;
        }
      }
    }
    if (DET) {
      __syncthreads();
      if ((int)threadIdx.x < cnt) {
        float sum[NG];
#pragma unroll
        for (int f = 0; f < NG; ++f) {
          sum[f] = s_part[0][threadIdx.x][f];
#pragma unroll
          for (int w = 1; w < NW; ++w) sum[f] += s_part[w][threadIdx.x][f];
        }
        float4* dst = (float4*)(inst_grad + (size_t)s_e[threadIdx.x] * 12);
        dst[0] = make_float4(sum[0], sum[1], sum[2], sum[3]);
        dst[1] = make_float4(sum[4], sum[5], sum[6], sum[7]);
        dst[2] = make_float4(sum[8], MAPS ? sum[NG - 1] : 0.f, 0.f, 0.f);
      }
    }
  }
  if (DET) {
    // entries past every pixel's last contributor carry no gradient
    for (int k = max(nmax, it.begin) + (int)threadIdx.x; k < it.end; k += NT) {
      float4* dst = (float4*)(inst_grad + (size_t)vals[rg.x + k] * 12);
      const float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
      dst[0] = z;
      dst[1] = z;
      dst[2] = z;
    }
  }
  // exposure gradient: dL/dA = sum g pre^T, dL/db = sum g (pre = B after the walk down to
  // list position 0, so only the tile's first chunk has it)
  if (V.dl_dexp && it.c == 0) {
    float e[12] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int k = 0; k < PX; ++k) {
      if (!inside[k]) continue;
      e[0] += g0[k] * B0[k]; e[1] += g0[k] * B1[k]; e[2] += g0[k] * B2[k]; e[3] += g0[k];
      e[4] += g1[k] * B0[k]; e[5] += g1[k] * B1[k]; e[6] += g1[k] * B2[k]; e[7] += g1[k];
      e[8] += g2[k] * B0[k]; e[9] += g2[k] * B1[k]; e[10] += g2[k] * B2[k]; e[11] += g2[k];
    }
#pragma unroll
    for (int f = 0; f < 12; ++f) e[f] = wave_sum_to_63(e[f]);
    __syncthreads();
    if (lane == 63)
#pragma unroll
      for (int f = 0; f < 12; ++f) s_red[wid][f] = e[f];
    __syncthreads();
    if (threadIdx.x < 12) {
      float s = 0.f;
      for (int w = 0; w < NW; ++w) s += s_red[w][threadIdx.x];
      if (DET)
        exp_part[(size_t)tile * 12 + threadIdx.x] = s;
      else
        unsafeAtomicAdd(V.dl_dexp + threadIdx.x, s);
    }
  }
}

// Deterministic exposure gradient: per view and entry, the tiles' partial sums in tile order.
__global__ void k_exposure_reduce(ViewsArg va, const float* __restrict__ exp_part) {
  const int v = blockIdx.x, f = threadIdx.x;
  if (v >= va.n || f >= 12 || render_dropped(va)) return;
  const ViewDev& V = va.v[v];
  if (!V.dl_dexp) return;
  const int T = V.tiles_x * V.tiles_y;
  float s = 0.f;
  for (int t = 0; t < T; ++t) s += exp_part[(size_t)(V.tile_base + t) * 12 + f];
  V.dl_dexp[f] += s;
}


template <int PX>
static void launch_fwd(const ViewsArg& va, const float4* rec, int32_t N, const uint32_t* vals,
                       const uint32_t* emit_g, const uint2* ranges, const SplitArg& sp, hipStream_t s) {
  bool depth = false;
  for (int v = 0; v < va.n; ++v) depth = depth || va.v[v].out_depth != nullptr;
  if (depth)
    hipLaunchKernelGGL((k_blend_fwd<PX, true>), item_grid(va, sp), dim3(kBlendBlock / PX), 0, s, va, rec, N, vals,
                       emit_g, ranges, sp);
  else
    hipLaunchKernelGGL((k_blend_fwd<PX, false>), item_grid(va, sp), dim3(kBlendBlock / PX), 0, s, va, rec, N, vals,
                       emit_g, ranges, sp);
}

template <int PX, bool MAPS>
static void launch_bwd_maps(const ViewsArg& va, const float4* rec, int32_t N, const uint32_t* vals,
                            const uint32_t* emit_g, const uint2* ranges, float* g2d, float* inst_grad,
                            float* exp_part, const SplitArg& sp, hipStream_t s) {
  if (inst_grad) {
    hipLaunchKernelGGL((k_blend_bwd<PX, true, MAPS>), item_grid(va, sp), dim3(kBlendBlock / PX), 0, s, va, rec, N,
                       vals, emit_g, ranges, g2d, inst_grad, exp_part, sp);
    hipLaunchKernelGGL(k_exposure_reduce, dim3(va.n), dim3(64), 0, s, va, exp_part);
  } else {
    hipLaunchKernelGGL((k_blend_bwd<PX, false, MAPS>), item_grid(va, sp), dim3(kBlendBlock / PX), 0, s, va, rec, N,
                       vals, emit_g, ranges, g2d, inst_grad, exp_part, sp);
  }
}

template <int PX>
static void launch_bwd(const ViewsArg& va, const float4* rec, int32_t N, const uint32_t* vals,
                       const uint32_t* emit_g, const uint2* ranges, float* g2d, float* inst_grad, float* exp_part,
                       const SplitArg& sp, hipStream_t s) {
  bool maps = false;
  for (int v = 0; v < va.n; ++v) maps = maps || va.v[v].dl_ddepth != nullptr || va.v[v].dl_dopac != nullptr;
  if (maps)
    launch_bwd_maps<PX, true>(va, rec, N, vals, emit_g, ranges, g2d, inst_grad, exp_part, sp, s);
  else
    launch_bwd_maps<PX, false>(va, rec, N, vals, emit_g, ranges, g2d, inst_grad, exp_part, sp, s);
}

hipError_t exposure_reduce(const ViewsArg& va, const float* exp_part, hipStream_t s) {
  hipLaunchKernelGGL(k_exposure_reduce, dim3(va.n), dim3(64), 0, s, va, exp_part);
  return hipGetLastError();
}

hipError_t blend_forward(const ViewsArg& va, const float4* rec, int32_t N, const uint32_t* vals,
                         const uint32_t* emit_g, const uint2* ranges, const SplitArg& sp, int px,
                         hipStream_t s) {
  if (va.total_tiles <= 0) return hipSuccess;
  if (px != 1 && px != 2 && px != 4) return hipErrorInvalidValue;
  if (sp.par > 0)
    hipLaunchKernelGGL(k_blend_trans, dim3((unsigned)sp.par), dim3(kBlendBlock), 0, s, va, rec, N, vals, emit_g,
                       ranges, sp);
  switch (px) {
    case 1: launch_fwd<1>(va, rec, N, vals, emit_g, ranges, sp, s); break;
    case 2: launch_fwd<2>(va, rec, N, vals, emit_g, ranges, sp, s); break;
    default: launch_fwd<4>(va, rec, N, vals, emit_g, ranges, sp, s); break;
  }
  if (sp.par > 0) {
    bool depth = false;
    for (int v = 0; v < va.n; ++v) depth = depth || va.v[v].out_depth != nullptr;
    if (depth)
      hipLaunchKernelGGL(k_split_merge<true>, dim3((unsigned)sp.par), dim3(kTile * kTile), 0, s, va, ranges, sp);
    else
      hipLaunchKernelGGL(k_split_merge<false>, dim3((unsigned)sp.par), dim3(kTile * kTile), 0, s, va, ranges, sp);
  }
  return hipGetLastError();
}

hipError_t blend_backward(const ViewsArg& va, const float4* rec, int32_t N, const uint32_t* vals,
                          const uint32_t* emit_g, const uint2* ranges, float* g2d, float* inst_grad,
                          float* exp_part, const SplitArg& sp, int px, hipStream_t s) {
  if (va.total_tiles <= 0) return hipSuccess;
  switch (px) {
    case 1: launch_bwd<1>(va, rec, N, vals, emit_g, ranges, g2d, inst_grad, exp_part, sp, s); break;
    case 2: launch_bwd<2>(va, rec, N, vals, emit_g, ranges, g2d, inst_grad, exp_part, sp, s); break;
    case 4: launch_bwd<4>(va, rec, N, vals, emit_g, ranges, g2d, inst_grad, exp_part, sp, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace gs
