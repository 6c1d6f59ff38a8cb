// Per-Gaussian backward of the blend (the parallelisation Sec. III-D.1 adopts for the
// backward pass: lanes own Gaussians, not pixels).
//
// One workgroup of four waves per 16x16 tile, wave w owning the pixels of the tile's 8x8
// quadrant w. The tile's depth-sorted list is taken in chunks of 64 entries, from the chunk
// holding the last contributor back to the first, one entry per lane with the chunk's
// deepest entry in lane 0 (every wave holds the same chunk). For every pixel of its
// quadrant still open at the chunk (its last contributor lies at or past the chunk start)
// a wave evaluates the 64 entries at that pixel and forms, across lanes (inclusive or
// exclusive scans from the back of the chunk):
//   Q_i    = prod_{k >= i} (1 - a_k)                    (suffix product, DPP scan)
//   T_i    = T_after / Q_i                              (transmittance in front of i)
//   S_i    = S_after + sum_{k > i} c_k a_k T_k          (colour behind i, incl. background)
//   dL/da_i = sum_ch G_ch (T_i c_i,ch - S_i,ch / (1 - a_i))
// with G = A^T dL/dout, and (T_after, S_after) the transmittance after the chunk and the
// colour behind it, which start at (T_final, T_final bg) and move to the previous chunk
// through LDS. Every sum adds positive terms from the back, so the colour behind a deep
// entry keeps its relative precision however small the transmittance has become. Each
// lane adds its Gaussian's nine gradient terms over its wave's pixels in registers; the
// four waves' sums meet in LDS and are added in wave order, then written once per
// instance: one atomic add per term, or, deterministic, the instance's record. A pixel that
// no entry of the chunk reaches skips the scans (its state passes the chunk unchanged). After the first chunk S_after is the pixel's pre-exposure colour,
// which gives the exposure gradient. Contribution decisions follow the forward: entry i
// contributes at pixel p iff i is before the pixel's saved list position and its alpha
// passes the cut-off.
#include "blend_split.h"
#include "gs_common.h"
#include "kernels.h"

namespace gs {

template <int CTRL, int ROWS>
__device__ __forceinline__ float dpp_or(float v, float identity) {
  return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(identity), __float_as_int(v), CTRL, ROWS, 0xf,
                                                    false));
}

// inclusive scans over the 64 lanes (lanes with no source take the identity)
__device__ __forceinline__ float wave_scan_add(float x) {
  x += dpp_or<0x111, 0xf>(x, 0.f);  // row_shr:1
  x += dpp_or<0x112, 0xf>(x, 0.f);  // row_shr:2
  x += dpp_or<0x114, 0xf>(x, 0.f);  // row_shr:4
  x += dpp_or<0x118, 0xf>(x, 0.f);  // row_shr:8
  x += dpp_or<0x142, 0xa>(x, 0.f);  // row_bcast:15 into rows 1 and 3
  x += dpp_or<0x143, 0xc>(x, 0.f);  // row_bcast:31 into rows 2 and 3
  return x;
}

__device__ __forceinline__ float wave_scan_mul(float x) {
  x *= dpp_or<0x111, 0xf>(x, 1.f);
  x *= dpp_or<0x112, 0xf>(x, 1.f);
  x *= dpp_or<0x114, 0xf>(x, 1.f);
  x *= dpp_or<0x118, 0xf>(x, 1.f);
  x *= dpp_or<0x142, 0xa>(x, 1.f);
  x *= dpp_or<0x143, 0xc>(x, 1.f);
  return x;
}

// the value of the lane below (lane 0: 0), by the DPP whole-wave shift, not an LDS permute
__device__ __forceinline__ float wave_shr1(float x) { return dpp_or<0x138, 0xf>(x, 0.f); }

__device__ __forceinline__ float wave_sum_all(float x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}

template <bool DET>
__global__ void __launch_bounds__(256)
k_blend_bwd_pg(ViewsArg va, const float4* __restrict__ rec, int32_t N, const uint32_t* __restrict__ vals,
               const uint32_t* __restrict__ emit_g, const uint2* __restrict__ ranges, float* __restrict__ g2d,
               float* __restrict__ inst_grad, float* __restrict__ exp_part, SplitArg sp) {
  // pixel slot ps = 64 w + lane: wave w owns the tile's 8x8 quadrant w
  __shared__ float s_T[256];          // transmittance after the current chunk
  __shared__ float s_S[3][256];       // colour behind the current chunk (incl. background)
  __shared__ float s_G[3][256];       // dL/d(pre-exposure colour)
  __shared__ uint32_t s_nc[256];      // list position after the pixel's last contributor
  __shared__ float s_acc[4][9][64];   // each wave's sums of an entry's nine terms over its pixels
  __shared__ float s_e[4][12];        // each wave's exposure-gradient sums
  __shared__ uint32_t s_wmax[4];
  BlendItem it;
  if (render_dropped(va) || !blend_item(sp, ranges, it)) return;
  const int tile = it.tile;
  const bool split = it.slot0 != kNoSlot;
  const int v = view_of_tile(va, tile);
  const ViewDev& V = va.v[v];
  const int lt = tile - V.tile_base;
  const int tx = lt % V.tiles_x, ty = lt / V.tiles_x;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const uint2 rg = ranges[tile];
  const float4* vrec = rec + (size_t)v * N * 4;
  float* vg = g2d + (size_t)v * N * kGradFloats;
  const int64_t P = (int64_t)V.W * V.H;
  // the lane's pixel of the wave's quadrant
  const int qx = tx * kTile + 8 * (wid & 1), qy = ty * kTile + 8 * (wid >> 1);
  auto pixel_of = [&](int l, int& px, int& py) {
    px = qx + (l & 7);
    py = qy + (l >> 3);
  };

  float gl[3];  // dL/dout of the lane's pixel (exposure gradient)
  {
    int px, py;
    pixel_of(lane, px, py);
    float g0 = 0.f, g1 = 0.f, g2 = 0.f, T = 1.0f;
    uint32_t nc = 0;
    if (px < V.W && py < V.H) {
      const int64_t o = (int64_t)py * V.W + px;
      nc = V.out_nc[o];
      T = V.out_T[o];
      g0 = V.dl_drgb[o];
      g1 = V.dl_drgb[P + o];
      g2 = V.dl_drgb[2 * P + o];
    }
    gl[0] = g0;
    gl[1] = g1;
    gl[2] = g2;
    float G0 = g0, G1 = g1, G2 = g2;
    if (V.exposure) {
      const float* E = V.exposure;
      G0 = E[0] * g0 + E[4] * g1 + E[8] * g2;
      G1 = E[1] * g0 + E[5] * g1 + E[9] * g2;
      G2 = E[2] * g0 + E[6] * g1 + E[10] * g2;
    }
    const int ps = 64 * wid + lane;
    // state after this work item's entries: the final transmittance and the background,
    // or, for a chunk of a split tile, the transmittance after the chunk and the colour the
    // later chunks add up to the one the pixel stopped in, then the background
    float S0 = T * V.bg[0], S1 = T * V.bg[1], S2 = T * V.bg[2];
    if (split && px < V.W && py < V.H) {
      const int q = (py - ty * kTile) * kTile + (px - tx * kTile);
      const ChunkSums cs = sum_chunks(sp, it.slot0, it.c + 1, it.nch, q, ChunkSums{S0, S1, S2, 0.f, 0.f, 0u});
      S0 = cs.c0;
      S1 = cs.c1;
      S2 = cs.c2;
      T = split_field(sp, it.slot0 + it.c, 5)[q];
    }
    s_T[ps] = T;
    s_S[0][ps] = S0;
    s_S[1][ps] = S1;
    s_S[2][ps] = S2;
    s_G[0][ps] = G0;
    s_G[1][ps] = G1;
    s_G[2][ps] = G2;
    s_nc[ps] = nc;
    uint32_t m = nc;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m = max(m, (uint32_t)__shfl_xor((int)m, o, 64));
    if (lane == 0) s_wmax[wid] = m;
  }
  __syncthreads();
  const uint32_t nmax = max(max(s_wmax[0], s_wmax[1]), max(s_wmax[2], s_wmax[3]));
  const int nlist = min((int)nmax, it.end);  // entries of the item before every last contributor

  // sub-chunks of 64 entries aligned at the item's start, from the back
  for (int c0 = it.begin + ((nlist - it.begin - 1) / 64) * 64; nlist > it.begin && c0 >= it.begin; c0 -= 64) {
    const int j = c0 + 63 - lane;  // lane 0 holds the deepest entry of the chunk
    const bool live = j < nlist;
    uint32_t e_idx = 0, g = 0;
    float4 a = make_float4(0.f, 0.f, 0.f, 0.f), b = make_float4(0.f, 0.f, 0.f, 0.f);
    float c2 = 0.f;
    if (live) {
      e_idx = vals[rg.x + j];
      g = emit_g[e_idx];
      const float4* r = vrec + (size_t)g * 4;
      a = blend_stage_a(r[0]);
      b = r[1];
      b.x = blend_stage_c(b.x);
      c2 = r[2].x;
    }
    float acc[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    for (int l = 0; l < 64; ++l) {  // the wave's pixels, one after another
      const int ps = 64 * wid + l;
      const uint32_t ncp = s_nc[ps];
      if ((int)ncp <= c0) continue;  // every contributor of this pixel lies before the chunk
      int pxi, pyi;
      pixel_of(l, pxi, pyi);
      const float pxc = (float)pxi + 0.5f, pyc = (float)pyi + 0.5f;
      float dx = 0.f, dy = 0.f, ex = 0.f, araw = 0.f, alpha = 0.f;
      if (live && j < (int)ncp) {
        const float power = blend_power2(a.x, a.y, a.z, a.w, b.x, pxc, pyc, dx, dy);
        if (power <= 0.0f) {
          ex = blend_exp2(power);
          araw = b.y * ex;
          alpha = fminf(kAlphaMax, araw);
          if (alpha < kAlphaMin) alpha = 0.0f;
        }
      }
      // no entry of the chunk reaches the pixel: its transmittance and colour behind pass
      // the chunk unchanged and it adds no gradient (exactly what the scans would give)
      if (!__any(alpha > 0.0f)) continue;
      const float oma = 1.0f - alpha;
      const float Q = wave_scan_mul(oma);   // prod over this entry and the deeper ones
      const float Ta = s_T[ps];
      const float T = Ta * __builtin_amdgcn_rcpf(Q);  // in front of this entry
      const float w = alpha * T;
      // colour the deeper entries of the chunk add (exclusive scan: the lane below's sum)
      const float k0 = wave_scan_add(wave_shr1(b.z * w)), k1 = wave_scan_add(wave_shr1(b.w * w));
      const float k2 = wave_scan_add(wave_shr1(c2 * w));
      const float S0 = s_S[0][ps] + k0, S1 = s_S[1][ps] + k1, S2 = s_S[2][ps] + k2;
      if (alpha > 0.0f) {
        const float G0 = s_G[0][ps], G1 = s_G[1][ps], G2 = s_G[2][ps];
        const float iom = __builtin_amdgcn_rcpf(oma);
        const float dalpha = G0 * (T * b.z - S0 * iom) + G1 * (T * b.w - S1 * iom) + G2 * (T * c2 - S2 * iom);
        acc[6] += w * G0;
        acc[7] += w * G1;
        acc[8] += w * G2;
        if (araw <= kAlphaMax) {
          // moments of dL/dpower = dL/dalpha * alpha (the 2D-gradient record's form)
          const float dpow = dalpha * alpha;
          const float px_ = dpow * dx, py_ = dpow * dy;
          acc[0] += px_;
          acc[1] += py_;
          acc[2] += px_ * dx;
          acc[3] += px_ * dy;
          acc[4] += py_ * dy;
          acc[5] += dpow;
        }
      }
      // carry the pixel state to the previous chunk (lane 63 holds the front entry)
      if (lane == 63) {
        s_T[ps] = T;
        s_S[0][ps] = S0 + b.z * w;
        s_S[1][ps] = S1 + b.w * w;
        s_S[2][ps] = S2 + c2 * w;
      }
    }
    // the four waves' sums of each entry, added in wave order by the first wave
#pragma unroll
    for (int f = 0; f < 9; ++f) s_acc[wid][f][lane] = acc[f];
    __syncthreads();
    if (wid == 0 && live) {
      float t[9];
#pragma unroll
      for (int f = 0; f < 9; ++f) t[f] = ((s_acc[0][f][lane] + s_acc[1][f][lane]) + s_acc[2][f][lane]) + s_acc[3][f][lane];
      if (DET) {
        float4* dst = (float4*)(inst_grad + (size_t)e_idx * 12);
        dst[0] = make_float4(t[0], t[1], t[2], t[3]);
        dst[1] = make_float4(t[4], t[5], t[6], t[7]);
        dst[2] = make_float4(t[8], 0.f, 0.f, 0.f);
      } else {
        float* dst = vg + (size_t)g * kGradFloats;
#pragma unroll
        for (int f = 0; f < 9; ++f)
          if (t[f] != 0.0f) unsafeAtomicAdd(dst + f, t[f]);
      }
    }
    __syncthreads();  // s_acc is written again by the next chunk
  }
  if (DET) {
    // entries past every pixel's last contributor carry no gradient
    for (int k = max(nlist, it.begin) + (int)threadIdx.x; k < it.end; k += 256) {
      float4* dst = (float4*)(inst_grad + (size_t)vals[rg.x + k] * 12);
      const float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
      dst[0] = z;
      dst[1] = z;
      dst[2] = z;
    }
  }
  if (V.dl_dexp && it.c == 0) {
    // dL/dA = sum g pre^T, dL/db = sum g, with pre the colour behind list position 0 (so
    // only a tile's first chunk has it; each wave's pixel state is its own: no barrier
    // needed before reading it)
    const int ps = 64 * wid + lane;
    const float p0 = s_S[0][ps], p1 = s_S[1][ps], p2 = s_S[2][ps];
    float e[12];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      e[4 * r + 0] = gl[r] * p0;
      e[4 * r + 1] = gl[r] * p1;
      e[4 * r + 2] = gl[r] * p2;
      e[4 * r + 3] = gl[r];
    }
#pragma unroll
    for (int f = 0; f < 12; ++f) e[f] = wave_sum_all(e[f]);
    if (lane < 12) {
      float sv = 0.f;
#pragma unroll
      for (int f = 0; f < 12; ++f) sv = lane == f ? e[f] : sv;
      s_e[wid][lane] = sv;
    }
    __syncthreads();
    if (threadIdx.x < 12) {
      const float sv = ((s_e[0][threadIdx.x] + s_e[1][threadIdx.x]) + s_e[2][threadIdx.x]) + s_e[3][threadIdx.x];
      if (DET)
        exp_part[(size_t)tile * 12 + threadIdx.x] = sv;
      else
        unsafeAtomicAdd(V.dl_dexp + threadIdx.x, sv);
    }
  }
}

hipError_t blend_backward_per_gaussian(const ViewsArg& va, const float4* rec, int32_t N, const uint32_t* vals,
                                       const uint32_t* emit_g, const uint2* ranges, float* g2d, float* inst_grad,
                                       float* exp_part, const SplitArg& sp, hipStream_t s) {
  if (va.total_tiles <= 0) return hipSuccess;
  if (inst_grad) {
    hipLaunchKernelGGL(k_blend_bwd_pg<true>, item_grid(va, sp), dim3(256), 0, s, va, rec, N, vals, emit_g, ranges,
                       g2d, inst_grad, exp_part, sp);
    return exposure_reduce(va, exp_part, s);
  } else
    hipLaunchKernelGGL(k_blend_bwd_pg<false>, item_grid(va, sp), dim3(256), 0, s, va, rec, N, vals, emit_g, ranges,
                       g2d, inst_grad, exp_part, sp);
  return hipGetLastError();
}

}  // namespace gs
