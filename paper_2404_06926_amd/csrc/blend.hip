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

__device__ __forceinline__ uint32_t wave_max_u32(uint32_t x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x = max(x, (uint32_t)__shfl_xor((int)x, o, 64));
  return x;
}

__global__ void __launch_bounds__(kBlendBlock)
k_blend_fwd(ViewsArg va, const float4* __restrict__ rec, int32_t N, const uint32_t* __restrict__ vals,
            const uint32_t* __restrict__ emit_g, const uint2* __restrict__ ranges) {
  __shared__ float4 s_a[kBlendBlock];   // mx, my, A, B
  __shared__ float4 s_b[kBlendBlock];   // C, o, r, g
  __shared__ float s_c[kBlendBlock];    // b
  __shared__ uint8_t s_m[kBlendBlock];  // quadrant mask
  const int tile = blockIdx.x;
  const int v = view_of_tile(va, tile);
  const ViewDev& V = va.v[v];
  const int lt = tile - V.tile_base;
  const int tx = lt % V.tiles_x, ty = lt / V.tiles_x;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int px = tx * kTile + 8 * (wid & 1) + (lane & 7);
  const int py = ty * kTile + 8 * (wid >> 1) + (lane >> 3);
  const bool inside = px < V.W && py < V.H;
  const float pxc = (float)px + 0.5f, pyc = (float)py + 0.5f;
  const uint2 rg = ranges[tile];
  const int n = (int)(rg.y - rg.x);
  const float4* vrec = rec + (size_t)v * N * 4;

  float T = 1.0f, C0 = 0.0f, C1 = 0.0f, C2 = 0.0f;
  uint32_t last = 0;
  bool done = !inside;
  for (int base = 0; base < n; base += kBlendBlock) {
    if (__syncthreads_count(done) == kBlendBlock) break;
    const int k = base + (int)threadIdx.x;
    if (k < n) {
      const uint32_t g = emit_g[vals[rg.x + k]];
      const float4* r = vrec + (size_t)g * 4;
      const float4 r0 = r[0], r1 = r[1], r2 = r[2];
      s_a[threadIdx.x] = r0;
      s_b[threadIdx.x] = r1;
      s_c[threadIdx.x] = r2.x;
      s_m[threadIdx.x] = (uint8_t)quadrant_mask(r0, r1, r2.w, tx, ty);
    }
    __syncthreads();
    const int cnt = min(kBlendBlock, n - base);
    if (!done) {
      for (int j = 0; j < cnt; ++j) {
        if (!((s_m[j] >> wid) & 1u)) continue;
        const float4 a = s_a[j];
        const float4 b = s_b[j];
        float dx, dy;
        const float power = blend_power(a.x, a.y, a.z, a.w, b.x, pxc, pyc, dx, dy);
        if (power > 0.0f) continue;
        const float alpha = fminf(kAlphaMax, b.y * __expf(power));
        if (alpha < kAlphaMin) continue;
        const float Tn = T * (1.0f - alpha);
        if (Tn < kTMin) {
          done = true;
          break;
        }
        const float w = alpha * T;
        C0 += b.z * w;
        C1 += b.w * w;
        C2 += s_c[j] * w;
        T = Tn;
        last = (uint32_t)(base + j + 1);
      }
    }
  }
  if (!inside) return;
  const int64_t p = (int64_t)py * V.W + px;
  const int64_t P = (int64_t)V.W * V.H;
  const float pre0 = C0 + T * V.bg[0], pre1 = C1 + T * V.bg[1], pre2 = C2 + T * V.bg[2];
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
}

// DET = false: each wave's per-Gaussian sums go to g2d with float atomics.
// DET = true: the four waves' sums are added in wave order in LDS and every instance's
// gradient is written to inst_grad[emission index]; the exposure gradient of each tile is
// written to exp_part[tile] for a fixed-order reduction. No atomics, so the result does not
// depend on scheduling.
template <bool DET>
__global__ void __launch_bounds__(kBlendBlock)
k_blend_bwd(ViewsArg va, const float4* __restrict__ rec, int32_t N, const uint32_t* __restrict__ vals,
            const uint32_t* __restrict__ emit_g, const uint2* __restrict__ ranges, float* __restrict__ g2d,
            float* __restrict__ inst_grad, float* __restrict__ exp_part) {
  __shared__ float4 s_a[kBlendBlock];
  __shared__ float4 s_b[kBlendBlock];
  __shared__ float s_c[kBlendBlock];
  __shared__ uint32_t s_g[kBlendBlock];
  __shared__ uint32_t s_e[DET ? kBlendBlock : 1];
  __shared__ float s_part[DET ? kBlendBlock / 64 : 1][DET ? kBlendBlock : 1][9];
  __shared__ uint8_t s_m[kBlendBlock];
  __shared__ float s_red[kBlendBlock / 64][12];
  __shared__ uint32_t s_wmax[kBlendBlock / 64];
  const int tile = blockIdx.x;
  const int v = view_of_tile(va, tile);
  const ViewDev& V = va.v[v];
  const int lt = tile - V.tile_base;
  const int tx = lt % V.tiles_x, ty = lt / V.tiles_x;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int px = tx * kTile + 8 * (wid & 1) + (lane & 7);
  const int py = ty * kTile + 8 * (wid >> 1) + (lane >> 3);
  const bool inside = px < V.W && py < V.H;
  const float pxc = (float)px + 0.5f, pyc = (float)py + 0.5f;
  const uint2 rg = ranges[tile];
  const float4* vrec = rec + (size_t)v * N * 4;
  float* vg = g2d + (size_t)v * N * kGradFloats;

  const int64_t p = (int64_t)py * V.W + px;
  const int64_t P = (int64_t)V.W * V.H;
  float T = 1.0f, g0 = 0.f, g1 = 0.f, g2 = 0.f;
  uint32_t nc = 0;
  if (inside) {
    T = V.out_T[p];
    nc = V.out_nc[p];
    g0 = V.dl_drgb[p];
    g1 = V.dl_drgb[P + p];
    g2 = V.dl_drgb[2 * P + p];
  }
  // dL/d(pre-exposure colour) = A^T g
  float G0 = g0, G1 = g1, G2 = g2;
  if (V.exposure) {
    const float* E = V.exposure;
    G0 = E[0] * g0 + E[4] * g1 + E[8] * g2;
    G1 = E[1] * g0 + E[5] * g1 + E[9] * g2;
    G2 = E[2] * g0 + E[6] * g1 + E[10] * g2;
  }
  const uint32_t wmax = wave_max_u32(nc);
  if (lane == 0) s_wmax[wid] = wmax;
  __syncthreads();
  const int nmax = (int)max(max(s_wmax[0], s_wmax[1]), max(s_wmax[2], s_wmax[3]));
  // colour seen behind the current Gaussian, normalised by the transmittance in front of it
  float B0 = V.bg[0], B1 = V.bg[1], B2 = V.bg[2];

  for (int end = nmax; end > 0; end -= kBlendBlock) {
    const int base = max(0, end - kBlendBlock);
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
      s_g[threadIdx.x] = g;
      s_m[threadIdx.x] = (uint8_t)quadrant_mask(r0, r1, r2.w, tx, ty);
      if (DET) {
        s_e[threadIdx.x] = e;
#pragma unroll
        for (int w = 0; w < kBlendBlock / 64; ++w)
#pragma unroll
          for (int f = 0; f < 9; ++f) s_part[w][threadIdx.x][f] = 0.f;
      }
    }
    __syncthreads();
    const int jtop = min(cnt, (int)wmax - base) - 1;  // entries at or past the wave's max are idle
    for (int j = jtop; j >= 0; --j) {
      if (!((s_m[j] >> wid) & 1u)) continue;
      const int pos = base + j;
      const float4 a = s_a[j];
      const float4 b = s_b[j];
      bool contrib = pos < (int)nc;
      float dx = 0.f, dy = 0.f, ex = 0.f, araw = 0.f, alpha = 0.f;
      if (contrib) {
        const float power = blend_power(a.x, a.y, a.z, a.w, b.x, pxc, pyc, dx, dy);
        if (power > 0.0f) {
          contrib = false;
        } else {
          ex = __expf(power);
          araw = b.y * ex;
          alpha = fminf(kAlphaMax, araw);
          if (alpha < kAlphaMin) contrib = false;
        }
      }
      if (!__any(contrib)) continue;
      float gv[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
      if (contrib) {
        const float c0 = b.z, c1 = b.w, c2 = s_c[j];
        const float oma = 1.0f - alpha;
        T = T * __builtin_amdgcn_rcpf(oma);  // transmittance in front of this Gaussian
        const float w = alpha * T;
        gv[6] = w * G0;
        gv[7] = w * G1;
        gv[8] = w * G2;
        const float dalpha = T * ((c0 - B0) * G0 + (c1 - B1) * G1 + (c2 - B2) * G2);
        B0 = alpha * c0 + oma * B0;
        B1 = alpha * c1 + oma * B1;
        B2 = alpha * c2 + oma * B2;
        if (araw <= kAlphaMax) {
          const float dpow = dalpha * alpha;
          gv[0] = dpow * (a.z * dx + a.w * dy);
          gv[1] = dpow * (a.w * dx + b.x * dy);
          gv[2] = -0.5f * dpow * dx * dx;
          gv[3] = -dpow * dx * dy;
          gv[4] = -0.5f * dpow * dy * dy;
          gv[5] = dalpha * ex;
        }
      }
#pragma unroll
      for (int f = 0; f < 9; ++f) gv[f] = wave_sum_to_63(gv[f]);
      if (lane == 63) {
        if (DET) {
#pragma unroll
          for (int f = 0; f < 9; ++f) s_part[wid][j][f] = gv[f];
        } else {
          float* dst = vg + (size_t)s_g[j] * kGradFloats;
#pragma unroll
          for (int f = 0; f < 9; ++f)
            if (gv[f] != 0.0f) unsafeAtomicAdd(dst + f, gv[f]);
        }
      }
    }
    if (DET) {
      __syncthreads();
      if ((int)threadIdx.x < cnt) {
        float sum[9];
#pragma unroll
        for (int f = 0; f < 9; ++f)
          sum[f] = ((s_part[0][threadIdx.x][f] + s_part[1][threadIdx.x][f]) + s_part[2][threadIdx.x][f]) +
                   s_part[3][threadIdx.x][f];
        float4* dst = (float4*)(inst_grad + (size_t)s_e[threadIdx.x] * 12);
        dst[0] = make_float4(sum[0], sum[1], sum[2], sum[3]);
        dst[1] = make_float4(sum[4], sum[5], sum[6], sum[7]);
        dst[2] = make_float4(sum[8], 0.f, 0.f, 0.f);
      }
    }
  }
  if (DET) {
    // entries past every pixel's last contributor carry no gradient
    const int n = (int)(rg.y - rg.x);
    for (int k = nmax + (int)threadIdx.x; k < n; k += kBlendBlock) {
      float4* dst = (float4*)(inst_grad + (size_t)vals[rg.x + k] * 12);
      const float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
      dst[0] = z;
      dst[1] = z;
      dst[2] = z;
    }
  }
  // exposure gradient: dL/dA = sum g pre^T, dL/db = sum g (pre = B after the walk)
  if (V.dl_dexp) {
    float e[12];
    e[0] = g0 * B0; e[1] = g0 * B1; e[2] = g0 * B2; e[3] = g0;
    e[4] = g1 * B0; e[5] = g1 * B1; e[6] = g1 * B2; e[7] = g1;
    e[8] = g2 * B0; e[9] = g2 * B1; e[10] = g2 * B2; e[11] = g2;
#pragma unroll
    for (int f = 0; f < 12; ++f) e[f] = wave_sum_to_63(inside ? e[f] : 0.0f);
    __syncthreads();
    if (lane == 63)
#pragma unroll
      for (int f = 0; f < 12; ++f) s_red[wid][f] = e[f];
    __syncthreads();
    if (threadIdx.x < 12) {
      float s = 0.f;
      for (int w = 0; w < kBlendBlock / 64; ++w) s += s_red[w][threadIdx.x];
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

hipError_t blend_forward(const ViewsArg& va, const float4* rec, int32_t N, const uint32_t* vals,
                         const uint32_t* emit_g, const uint2* ranges, hipStream_t s) {
  if (va.total_tiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_blend_fwd, dim3(va.total_tiles), dim3(kBlendBlock), 0, s, va, rec, N, vals, emit_g, ranges);
  return hipGetLastError();
}

hipError_t blend_backward(const ViewsArg& va, const float4* rec, int32_t N, const uint32_t* vals,
                          const uint32_t* emit_g, const uint2* ranges, float* g2d, float* inst_grad,
                          float* exp_part, hipStream_t s) {
  if (va.total_tiles <= 0) return hipSuccess;
  if (inst_grad) {
    hipLaunchKernelGGL(k_blend_bwd<true>, dim3(va.total_tiles), dim3(kBlendBlock), 0, s, va, rec, N, vals, emit_g,
                       ranges, g2d, inst_grad, exp_part);
    hipLaunchKernelGGL(k_exposure_reduce, dim3(va.n), dim3(64), 0, s, va, exp_part);
  } else {
    hipLaunchKernelGGL(k_blend_bwd<false>, dim3(va.total_tiles), dim3(kBlendBlock), 0, s, va, rec, N, vals, emit_g,
                       ranges, g2d, inst_grad, exp_part);
  }
  return hipGetLastError();
}

}  // namespace gs
