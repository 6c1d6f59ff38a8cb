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
#include "gs_common.h"
#include "kernels.h"

namespace gs {

constexpr int kBlendBlock = 256;

// Minimum of q = A dx^2 + 2B dx dy + C dy^2 over [x0, x1] x [y0, y1] (offsets from the
// mean) compared with thr: 0 inside; else the clamped 1-D minimum on the separating edges.
__device__ __forceinline__ bool footprint_hits_rect(float A, float B, float C, float thr, float x0, float x1,
                                                    float y0, float y1) {
  if (x0 <= 0.f && x1 >= 0.f && y0 <= 0.f && y1 >= 0.f) return true;
  float qmin = __builtin_huge_valf();
  if (x0 > 0.f || x1 < 0.f) {
    const float dx = (x0 > 0.f) ? x0 : x1;
    const float dy = fminf(fmaxf(-(B * dx) / C, y0), y1);
    qmin = fminf(qmin, A * dx * dx + 2.f * B * dx * dy + C * dy * dy);
  }
  if (y0 > 0.f || y1 < 0.f) {
    const float dy = (y0 > 0.f) ? y0 : y1;
    const float dx = fminf(fmaxf(-(B * dy) / A, x0), x1);
    qmin = fminf(qmin, A * dx * dx + 2.f * B * dx * dy + C * dy * dy);
  }
  return qmin <= thr;
}

// 4-bit mask of the tile's 8x8 quadrants (bit q: x half q & 1, y half q >> 1) that the
// footprint {q <= thr (1 + 1e-4) + 1e-4} reaches at some pixel centre.
__device__ __forceinline__ uint32_t quadrant_mask(float4 r0, float4 r1, float thr, int tx, int ty) {
  const float t = thr * 1.0001f + 1e-4f;
  uint32_t m = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const float x0 = (float)(tx * kTile + 8 * (q & 1)) + 0.5f - r0.x;
    const float y0 = (float)(ty * kTile + 8 * (q >> 1)) + 0.5f - r0.y;
    if (footprint_hits_rect(r0.z, r0.w, r1.x, t, x0, x0 + 7.f, y0, y0 + 7.f)) m |= 1u << q;
  }
  return m;
}

template <int CTRL, int ROWS>
__device__ __forceinline__ float dpp_f(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROWS, 0xf, false));
}

// Sum over the 64 lanes with DPP row operations; the total is valid in lane 63.
__device__ __forceinline__ float wave_sum_to_63(float x) {
  x += dpp_f<0xB1, 0xf>(x);   // quad_perm [1,0,3,2]
  x += dpp_f<0x4E, 0xf>(x);   // quad_perm [2,3,0,1]
  x += dpp_f<0x141, 0xf>(x);  // row_half_mirror: 8-lane sums
  x += dpp_f<0x140, 0xf>(x);  // row_mirror: 16-lane sums
  x += dpp_f<0x142, 0xa>(x);  // row_bcast:15 into rows 1 and 3
  x += dpp_f<0x143, 0xc>(x);  // row_bcast:31 into rows 2 and 3
  return x;
}

// Sums over the wave of eight values at once, transposing while reducing: each exchange
// step halves the values a lane carries (the lane keeps one half, its partner the other),
// so 8 values cost 4 + 2 + 1 exchanges instead of 8 per step. Steps: lane ^ 1 and lane ^ 2
// (DPP quad_perm), lane ^ 4 (ds_swizzle), then the single value over lane bit 3 (DPP
// row_shr:8, valid in lanes 8..15 of each row of 16) and lane bits 4, 5 (shuffles). On
// return lane 8 + j of each row holds the wave total of v[rev3(j)], rev3 reversing the
// three bits of j; other lanes hold partial sums.
__device__ __forceinline__ float wave_sum8_transposed(const float (&v)[8], int lane) {
  const bool b0 = lane & 1, b1 = lane & 2, b2 = lane & 4;
  float w[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const float send = b0 ? v[k] : v[k + 4];
    const float keep = b0 ? v[k + 4] : v[k];
    w[k] = keep + dpp_f<0xB1, 0xf>(send);  // from lane ^ 1
  }
  float x[2];
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const float send = b1 ? w[k] : w[k + 2];
    const float keep = b1 ? w[k + 2] : w[k];
    x[k] = keep + dpp_f<0x4E, 0xf>(send);  // from lane ^ 2
  }
  const float send = b2 ? x[0] : x[1];
  const float keep = b2 ? x[1] : x[0];
  // ds_swizzle bit-mask mode: and 0x1f, or 0, xor 4 (from lane ^ 4 within 32 lanes)
  float y = keep + __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(send), 0x101F));
  y += dpp_f<0x118, 0xf>(y);  // row_shr:8: lanes 8..15 of a row add lanes 0..7
  y += __shfl_xor(y, 16, 64);
  y += __shfl_xor(y, 32, 64);
  return y;
}

// index of the value whose total lane 8 + j (j = lane & 7) holds after wave_sum8_transposed
__device__ __forceinline__ int rev3(int j) { return ((j & 1) << 2) | (j & 2) | ((j >> 2) & 1); }

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

// DEPTH: also accumulate the depth map D = sum d_i a_i T_i (Eq. 6) for views that ask.
template <int PX, bool DEPTH>
__global__ void __launch_bounds__(kBlendBlock / PX)
k_blend_fwd(ViewsArg va, const float4* __restrict__ rec, int32_t N, const uint32_t* __restrict__ vals,
            const uint32_t* __restrict__ emit_g, const uint2* __restrict__ ranges) {
  constexpr int NT = kBlendBlock / PX;
  __shared__ float4 s_a[NT];   // mx, my, A, B
  __shared__ float4 s_b[NT];   // C, o, r, g
  __shared__ float s_c[NT];    // b
  __shared__ float s_d[DEPTH ? NT : 1];  // camera-frame depth
  __shared__ uint8_t s_m[NT];  // quadrant mask
  const int tile = blockIdx.x;
  const int v = view_of_tile(va, tile);
  const ViewDev& V = va.v[v];
  const int lt = tile - V.tile_base;
  const int tx = lt % V.tiles_x, ty = lt / V.tiles_x;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const uint2 rg = ranges[tile];
  const int n = (int)(rg.y - rg.x);
  const float4* vrec = rec + (size_t)v * N * 4;

  float pxc[PX], pyc[PX], T[PX], C0[PX], C1[PX], C2[PX], Dm[PX];
  uint32_t last[PX];
  bool done[PX];
#pragma unroll
  for (int k = 0; k < PX; ++k) {
    int lx, ly;
    lane_pixel<PX>(wid, lane, k, lx, ly);
    const int px = tx * kTile + lx, py = ty * kTile + ly;
    pxc[k] = (float)px + 0.5f;
    pyc[k] = (float)py + 0.5f;
    done[k] = !(px < V.W && py < V.H);
    T[k] = 1.0f;
    C0[k] = C1[k] = C2[k] = Dm[k] = 0.0f;
    last[k] = 0;
  }
  auto all_done = [&]() {
    bool d = true;
#pragma unroll
    for (int k = 0; k < PX; ++k) d = d && done[k];
    return d;
  };
  bool lane_done = all_done();
  for (int base = 0; base < n; base += NT) {
    if (__syncthreads_count(lane_done) == NT) break;
    const int kk = base + (int)threadIdx.x;
    if (kk < n) {
      const uint32_t g = emit_g[vals[rg.x + kk]];
      const float4* r = vrec + (size_t)g * 4;
      const float4 r0 = r[0], r1 = r[1], r2 = r[2];
      s_a[threadIdx.x] = r0;
      s_b[threadIdx.x] = r1;
      s_c[threadIdx.x] = r2.x;
      if (DEPTH) s_d[threadIdx.x] = r2.y;
      s_m[threadIdx.x] = (uint8_t)quadrant_mask(r0, r1, r2.w, tx, ty);
    }
    __syncthreads();
    const int cnt = min(NT, n - base);
    if (!lane_done) {
      for (int j = 0; j < cnt; ++j) {
        const uint32_t m = s_m[j];
        const float4 a = s_a[j];
        const float4 b = s_b[j];
#pragma unroll
        for (int k = 0; k < PX; ++k) {
          if (!((m >> pixel_quadrant<PX>(wid, k)) & 1u) || done[k]) continue;
          float dx, dy;
          const float power = blend_power(a.x, a.y, a.z, a.w, b.x, pxc[k], pyc[k], dx, dy);
          if (power > 0.0f) continue;
          const float alpha = fminf(kAlphaMax, b.y * __expf(power));
          if (alpha < kAlphaMin) continue;
          const float Tn = T[k] * (1.0f - alpha);
          if (Tn < kTMin) {
            done[k] = true;
            continue;
          }
          const float w = alpha * T[k];
          C0[k] += b.z * w;
          C1[k] += b.w * w;
          C2[k] += s_c[j] * w;
          if (DEPTH) Dm[k] += s_d[j] * w;
          T[k] = Tn;
          last[k] = (uint32_t)(base + j + 1);
        }
        lane_done = all_done();
        if (lane_done) break;
      }
    }
  }
  const int64_t P = (int64_t)V.W * V.H;
#pragma unroll
  for (int k = 0; k < PX; ++k) {
    const int px = (int)pxc[k], py = (int)pyc[k];
    if (px >= V.W || py >= V.H) continue;
    const int64_t p = (int64_t)py * V.W + px;
    const float pre0 = C0[k] + T[k] * V.bg[0], pre1 = C1[k] + T[k] * V.bg[1], pre2 = C2[k] + T[k] * V.bg[2];
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
    V.out_T[p] = T[k];
    V.out_nc[p] = last[k];
    if (V.out_pre) {
      V.out_pre[p] = pre0;
      V.out_pre[P + p] = pre1;
      V.out_pre[2 * P + p] = pre2;
    }
    if (DEPTH && V.out_depth) V.out_depth[p] = Dm[k];
    if (V.out_opac) V.out_opac[p] = 1.0f - T[k];  // Eq. 7 telescoped: sum a_i T_i = 1 - T_final
  }
}

// DET = false: each wave's per-Gaussian sums go to g2d with float atomics.
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
            float* __restrict__ inst_grad, float* __restrict__ exp_part) {
  constexpr int NT = kBlendBlock / PX;
  constexpr int NW = NT / 64;
  constexpr int NG = MAPS ? 10 : 9;  // gradient terms per Gaussian
  __shared__ float4 s_a[NT];
  __shared__ float4 s_b[NT];
  __shared__ float s_c[NT];
  __shared__ float s_d[MAPS ? NT : 1];
  __shared__ uint32_t s_g[NT];
  __shared__ uint32_t s_e[DET ? NT : 1];
  __shared__ float s_part[DET ? NW : 1][DET ? NT : 1][NG];
  __shared__ uint8_t s_m[NT];
  __shared__ float s_red[NW][12];
  __shared__ uint32_t s_wmax[NW];
  const int tile = blockIdx.x;
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
    ncmax = max(ncmax, nc[k]);
  }
  const uint32_t wmax = wave_max_u32(ncmax);
  if (lane == 0) s_wmax[wid] = wmax;
  __syncthreads();
  int nmax = 0;
#pragma unroll
  for (int w = 0; w < NW; ++w) nmax = max(nmax, (int)s_wmax[w]);

  for (int end = nmax; end > 0; end -= NT) {
    const int base = max(0, end - NT);
    const int cnt = end - base;
    __syncthreads();
    if ((int)threadIdx.x < cnt) {
      const uint32_t e = vals[rg.x + base + threadIdx.x];
      const uint32_t g = emit_g[e];
      const float4* r = vrec + (size_t)g * 4;
      const float4 r0 = r[0], r1 = r[1], r2 = r[2];
      s_a[threadIdx.x] = r0;
      s_b[threadIdx.x] = r1;
      s_c[threadIdx.x] = r2.x;
      if (MAPS) s_d[threadIdx.x] = r2.y;
      s_g[threadIdx.x] = g;
      s_m[threadIdx.x] = (uint8_t)quadrant_mask(r0, r1, r2.w, tx, ty);
      if (DET) {
        s_e[threadIdx.x] = e;
#pragma unroll
        for (int w = 0; w < NW; ++w)
#pragma unroll
          for (int f = 0; f < NG; ++f) s_part[w][threadIdx.x][f] = 0.f;
      }
    }
    __syncthreads();
    const int jtop = min(cnt, (int)wmax - base) - 1;  // entries at or past the wave's max are idle
    for (int j = jtop; j >= 0; --j) {
      const uint32_t m = s_m[j];
      const int pos = base + j;
      const float4 a = s_a[j];
      const float4 b = s_b[j];
      const float c2 = s_c[j];
      const float dep = MAPS ? s_d[j] : 0.0f;
      float gv[NG];
#pragma unroll
      for (int f = 0; f < NG; ++f) gv[f] = 0.f;
      bool any = false;
#pragma unroll
      for (int k = 0; k < PX; ++k) {
        if (!((m >> pixel_quadrant<PX>(wid, k)) & 1u)) continue;
        if (pos >= (int)nc[k]) continue;
        float dx, dy;
        const float power = blend_power(a.x, a.y, a.z, a.w, b.x, pxc[k], pyc[k], dx, dy);
        if (power > 0.0f) continue;
        const float ex = __expf(power);
        const float araw = b.y * ex;
        const float alpha = fminf(kAlphaMax, araw);
        if (alpha < kAlphaMin) continue;
        any = true;
        const float oma = 1.0f - alpha;
        T[k] = T[k] * __builtin_amdgcn_rcpf(oma);  // transmittance in front of this Gaussian
        const float w = alpha * T[k];
        gv[6] += w * G0[k];
        gv[7] += w * G1[k];
        gv[8] += w * G2[k];
        float dalpha = T[k] * ((b.z - B0[k]) * G0[k] + (b.w - B1[k]) * G1[k] + (c2 - B2[k]) * G2[k]);
        B0[k] = alpha * b.z + oma * B0[k];
        B1[k] = alpha * b.w + oma * B1[k];
        B2[k] = alpha * c2 + oma * B2[k];
        if (MAPS) {
          dalpha += T[k] * ((dep - BD[k]) * gD[k] + (1.0f - BO[k]) * gO[k]);
          BD[k] = alpha * dep + oma * BD[k];
          BO[k] = alpha + oma * BO[k];
          gv[9] += w * gD[k];
        }
        if (araw <= kAlphaMax) {
          const float dpow = dalpha * alpha;
          gv[0] += dpow * (a.z * dx + a.w * dy);
          gv[1] += dpow * (a.w * dx + b.x * dy);
          gv[2] += -0.5f * dpow * dx * dx;
          gv[3] += -dpow * dx * dy;
          gv[4] += -0.5f * dpow * dy * dy;
          gv[5] += dalpha * ex;
        }
      }
      if (!__any(any)) continue;
      // terms 0..7 transposed (lanes 8..15 end with the totals), the rest by DPP rows
      float g8[8];
#pragma unroll
      for (int f = 0; f < 8; ++f) g8[f] = gv[f];
      const float tot = wave_sum8_transposed(g8, lane);
#pragma unroll
      for (int f = 8; f < NG; ++f) gv[f] = wave_sum_to_63(gv[f]);
      if (lane >= 8 && lane < 16) {
        const int f = rev3(lane & 7);
        if (DET)
          s_part[wid][j][f] = tot;
        else if (tot != 0.0f)
          unsafeAtomicAdd(vg + (size_t)s_g[j] * kGradFloats + f, tot);
      }
      if (lane == 63) {
#pragma unroll
        for (int f = 8; f < NG; ++f) {
          if (DET)
            s_part[wid][j][f] = gv[f];
          else if (gv[f] != 0.0f)
            unsafeAtomicAdd(vg + (size_t)s_g[j] * kGradFloats + f, gv[f]);
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
    const int n = (int)(rg.y - rg.x);
    for (int k = nmax + (int)threadIdx.x; k < n; k += NT) {
      float4* dst = (float4*)(inst_grad + (size_t)vals[rg.x + k] * 12);
      const float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
      dst[0] = z;
      dst[1] = z;
      dst[2] = z;
    }
  }
  // exposure gradient: dL/dA = sum g pre^T, dL/db = sum g (pre = B after the walk)
  if (V.dl_dexp) {
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
  if (v >= va.n || f >= 12) return;
  const ViewDev& V = va.v[v];
  if (!V.dl_dexp) return;
  const int T = V.tiles_x * V.tiles_y;
  float s = 0.f;
  for (int t = 0; t < T; ++t) s += exp_part[(size_t)(V.tile_base + t) * 12 + f];
  V.dl_dexp[f] += s;
}

template <int PX>
static void launch_fwd(const ViewsArg& va, const float4* rec, int32_t N, const uint32_t* vals,
                       const uint32_t* emit_g, const uint2* ranges, hipStream_t s) {
  bool depth = false;
  for (int v = 0; v < va.n; ++v) depth = depth || va.v[v].out_depth != nullptr;
  if (depth)
    hipLaunchKernelGGL((k_blend_fwd<PX, true>), dim3(va.total_tiles), dim3(kBlendBlock / PX), 0, s, va, rec, N,
                       vals, emit_g, ranges);
  else
    hipLaunchKernelGGL((k_blend_fwd<PX, false>), dim3(va.total_tiles), dim3(kBlendBlock / PX), 0, s, va, rec, N,
                       vals, emit_g, ranges);
}

template <int PX, bool MAPS>
static void launch_bwd_maps(const ViewsArg& va, const float4* rec, int32_t N, const uint32_t* vals,
                            const uint32_t* emit_g, const uint2* ranges, float* g2d, float* inst_grad,
                            float* exp_part, hipStream_t s) {
  if (inst_grad) {
    hipLaunchKernelGGL((k_blend_bwd<PX, true, MAPS>), dim3(va.total_tiles), dim3(kBlendBlock / PX), 0, s, va, rec,
                       N, vals, emit_g, ranges, g2d, inst_grad, exp_part);
    hipLaunchKernelGGL(k_exposure_reduce, dim3(va.n), dim3(64), 0, s, va, exp_part);
  } else {
    hipLaunchKernelGGL((k_blend_bwd<PX, false, MAPS>), dim3(va.total_tiles), dim3(kBlendBlock / PX), 0, s, va, rec,
                       N, vals, emit_g, ranges, g2d, inst_grad, exp_part);
  }
}

template <int PX>
static void launch_bwd(const ViewsArg& va, const float4* rec, int32_t N, const uint32_t* vals,
                       const uint32_t* emit_g, const uint2* ranges, float* g2d, float* inst_grad, float* exp_part,
                       hipStream_t s) {
  bool maps = false;
  for (int v = 0; v < va.n; ++v) maps = maps || va.v[v].dl_ddepth != nullptr || va.v[v].dl_dopac != nullptr;
  if (maps)
    launch_bwd_maps<PX, true>(va, rec, N, vals, emit_g, ranges, g2d, inst_grad, exp_part, s);
  else
    launch_bwd_maps<PX, false>(va, rec, N, vals, emit_g, ranges, g2d, inst_grad, exp_part, s);
}

hipError_t exposure_reduce(const ViewsArg& va, const float* exp_part, hipStream_t s) {
  hipLaunchKernelGGL(k_exposure_reduce, dim3(va.n), dim3(64), 0, s, va, exp_part);
  return hipGetLastError();
}

hipError_t blend_forward(const ViewsArg& va, const float4* rec, int32_t N, const uint32_t* vals,
                         const uint32_t* emit_g, const uint2* ranges, int px, hipStream_t s) {
  if (va.total_tiles <= 0) return hipSuccess;
  switch (px) {
    case 1: launch_fwd<1>(va, rec, N, vals, emit_g, ranges, s); break;
    case 2: launch_fwd<2>(va, rec, N, vals, emit_g, ranges, s); break;
    case 4: launch_fwd<4>(va, rec, N, vals, emit_g, ranges, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t blend_backward(const ViewsArg& va, const float4* rec, int32_t N, const uint32_t* vals,
                          const uint32_t* emit_g, const uint2* ranges, float* g2d, float* inst_grad,
                          float* exp_part, int px, hipStream_t s) {
  if (va.total_tiles <= 0) return hipSuccess;
  switch (px) {
    case 1: launch_bwd<1>(va, rec, N, vals, emit_g, ranges, g2d, inst_grad, exp_part, s); break;
    case 2: launch_bwd<2>(va, rec, N, vals, emit_g, ranges, g2d, inst_grad, exp_part, s); break;
    case 4: launch_bwd<4>(va, rec, N, vals, emit_g, ranges, g2d, inst_grad, exp_part, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace gs
