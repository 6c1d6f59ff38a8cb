// Front-to-back blending (Sec. III-A Eq. 4-5, 7) with the per-keyframe exposure affine
// (Sec. III-C.3), and its reverse-order adjoint.
//
// One workgroup of 256 lanes (4 waves) per 16x16 tile, one pixel per lane. The tile's
// depth-sorted list is staged through LDS in batches of 256 records (one gather of 36 B
// per lane from the 64-B projection record), then every lane walks the batch.
// The forward saves per pixel the final transmittance and the list position after the
// last contributor; the backward starts from them (no forward replay), walks the list
// from that position down to 0, recovers T_i = T_{i+1} / (1 - alpha_i), keeps the colour
// seen behind the current Gaussian, and reduces each Gaussian's gradient over the 64
// lanes of a wave before one atomic add per wave and field.
#include "gs_common.h"
#include "kernels.h"

namespace gs {

constexpr int kBlendBlock = 256;

__global__ void __launch_bounds__(kBlendBlock)
k_blend_fwd(ViewsArg va, const float4* __restrict__ rec, int32_t N, const uint32_t* __restrict__ vals,
            const uint2* __restrict__ ranges) {
  __shared__ float4 s_a[kBlendBlock];   // mx, my, A, B
  __shared__ float4 s_b[kBlendBlock];   // C, o, r, g
  __shared__ float s_c[kBlendBlock];    // b
  const int tile = blockIdx.x;
  const int v = view_of_tile(va, tile);
  const ViewDev& V = va.v[v];
  const int lt = tile - V.tile_base;
  const int tx = lt % V.tiles_x, ty = lt / V.tiles_x;
  const int px = tx * kTile + (threadIdx.x & 15), py = ty * kTile + (threadIdx.x >> 4);
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
      const uint32_t g = vals[rg.x + k];
      const float4* r = vrec + (size_t)g * 4;
      s_a[threadIdx.x] = r[0];
      s_b[threadIdx.x] = r[1];
      s_c[threadIdx.x] = r[2].x;
    }
    __syncthreads();
    const int cnt = min(kBlendBlock, n - base);
    if (!done) {
      for (int j = 0; j < cnt; ++j) {
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

__global__ void __launch_bounds__(kBlendBlock)
k_blend_bwd(ViewsArg va, const float4* __restrict__ rec, int32_t N, const uint32_t* __restrict__ vals,
            const uint2* __restrict__ ranges, float* __restrict__ g2d) {
  __shared__ float4 s_a[kBlendBlock];
  __shared__ float4 s_b[kBlendBlock];
  __shared__ float s_c[kBlendBlock];
  __shared__ uint32_t s_g[kBlendBlock];
  __shared__ float s_red[kBlendBlock / 64][12];
  __shared__ uint32_t s_max;
  const int tile = blockIdx.x;
  const int v = view_of_tile(va, tile);
  const ViewDev& V = va.v[v];
  const int lt = tile - V.tile_base;
  const int tx = lt % V.tiles_x, ty = lt / V.tiles_x;
  const int px = tx * kTile + (threadIdx.x & 15), py = ty * kTile + (threadIdx.x >> 4);
  const bool inside = px < V.W && py < V.H;
  const float pxc = (float)px + 0.5f, pyc = (float)py + 0.5f;
  const uint2 rg = ranges[tile];
  const float4* vrec = rec + (size_t)v * N * 4;
  float* vg = g2d + (size_t)v * N * kGradFloats;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;

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
  if (threadIdx.x == 0) s_max = 0;
  __syncthreads();
  if (nc) atomicMax(&s_max, nc);
  __syncthreads();
  const int nmax = (int)s_max;
  // colour seen behind the current Gaussian, normalised by the transmittance in front of it
  float B0 = V.bg[0], B1 = V.bg[1], B2 = V.bg[2];

  for (int end = nmax; end > 0; end -= kBlendBlock) {
    const int base = max(0, end - kBlendBlock);
    const int cnt = end - base;
    __syncthreads();
    if ((int)threadIdx.x < cnt) {
      const uint32_t g = vals[rg.x + base + threadIdx.x];
      const float4* r = vrec + (size_t)g * 4;
      s_a[threadIdx.x] = r[0];
      s_b[threadIdx.x] = r[1];
      s_c[threadIdx.x] = r[2].x;
      s_g[threadIdx.x] = g;
    }
    __syncthreads();
    for (int j = cnt - 1; j >= 0; --j) {
      const int pos = base + j;
      const float4 a = s_a[j];
      const float4 b = s_b[j];
      bool contrib = inside && pos < (int)nc;
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
        T = T / oma;  // transmittance in front of this Gaussian
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
      for (int f = 0; f < 9; ++f) gv[f] = wave_sum(gv[f]);
      if (lane == 0) {
        float* dst = vg + (size_t)s_g[j] * kGradFloats;
#pragma unroll
        for (int f = 0; f < 9; ++f)
          if (gv[f] != 0.0f) unsafeAtomicAdd(dst + f, gv[f]);
      }
    }
  }
  // exposure gradient: dL/dA = sum g pre^T, dL/db = sum g (pre = B after the walk)
  if (V.dl_dexp) {
    float e[12];
    e[0] = g0 * B0; e[1] = g0 * B1; e[2] = g0 * B2; e[3] = g0;
    e[4] = g1 * B0; e[5] = g1 * B1; e[6] = g1 * B2; e[7] = g1;
    e[8] = g2 * B0; e[9] = g2 * B1; e[10] = g2 * B2; e[11] = g2;
#pragma unroll
    for (int f = 0; f < 12; ++f) e[f] = wave_sum(inside ? e[f] : 0.0f);
    __syncthreads();
    if (lane == 0)
#pragma unroll
      for (int f = 0; f < 12; ++f) s_red[wid][f] = e[f];
    __syncthreads();
    if (threadIdx.x < 12) {
      float s = 0.f;
      for (int w = 0; w < kBlendBlock / 64; ++w) s += s_red[w][threadIdx.x];
      unsafeAtomicAdd(V.dl_dexp + threadIdx.x, s);
    }
  }
}

hipError_t blend_forward(const ViewsArg& va, const float4* rec, int32_t N, const uint32_t* vals,
                         const uint2* ranges, hipStream_t s) {
  if (va.total_tiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_blend_fwd, dim3(va.total_tiles), dim3(kBlendBlock), 0, s, va, rec, N, vals, ranges);
  return hipGetLastError();
}

hipError_t blend_backward(const ViewsArg& va, const float4* rec, int32_t N, const uint32_t* vals,
                          const uint2* ranges, float* g2d, hipStream_t s) {
  if (va.total_tiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_blend_bwd, dim3(va.total_tiles), dim3(kBlendBlock), 0, s, va, rec, N, vals, ranges, g2d);
  return hipGetLastError();
}

}  // namespace gs
