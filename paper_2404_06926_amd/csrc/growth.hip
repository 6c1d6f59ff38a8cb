// Map growth: expansion by the opacity mask (Sec. III-C.2, Eq. 8) and sky Gaussians
// initialised from nearest-neighbour distances (Sec. III-C.1).
//
// Expansion: one lane per candidate point projects it into the keyframe view, finds the
// pixel it falls on and keeps it when the pixel's opacity O = 1 - T_final is below tau.
// The kept points are compacted in input order (exclusive scan of the flags) and become
// Gaussians by the point initialisation rule. The pixel is an integer decision taken in
// FP32 with a fixed operation order and no contraction:
//   x_c = ((R00 x + R01 y) + R02 z) + t0 (same for y_c, z_c), u = f_x (x_c / z_c) + c_x,
//   inside = z_c > near and 0 <= u < W and 0 <= v < H, pixel = (floor u, floor v).
#include "gs_common.h"
#include "kernels.h"

namespace gs {

__global__ void __launch_bounds__(256)
k_expand_flags(const float* __restrict__ xyz, int64_t n, ViewDev V, const float* __restrict__ T, float tau,
               float near_z, uint32_t* __restrict__ flags) {
#pragma clang fp contract(off)
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const float x = xyz[3 * j], y = xyz[3 * j + 1], z = xyz[3 * j + 2];
  const float xc = ((V.R[0] * x + V.R[1] * y) + V.R[2] * z) + V.t[0];
  const float yc = ((V.R[3] * x + V.R[4] * y) + V.R[5] * z) + V.t[1];
  const float zc = ((V.R[6] * x + V.R[7] * y) + V.R[8] * z) + V.t[2];
  uint32_t keep = 0;
  if (zc > near_z) {
    const float u = V.fx * __fdiv_rn(xc, zc) + V.cx;
    const float v = V.fy * __fdiv_rn(yc, zc) + V.cy;
    if (u >= 0.0f && u < (float)V.W && v >= 0.0f && v < (float)V.H) {
      const int px = min((int)floorf(u), V.W - 1), py = min((int)floorf(v), V.H - 1);
      const float O = 1.0f - T[(int64_t)py * V.W + px];
      keep = O < tau ? 1u : 0u;
    }
  }
  flags[j] = keep;
}

// Sec. III-C.1 row initialisation shared by every point source: mean, isotropic
// log-scale, identity rotation, opacity logit, SH DC from a colour (colour = Y00 dc + 0.5),
// higher SH zero; gradients and Adam moments zero; not visible.
__device__ __forceinline__ void init_row(float* __restrict__ buf, int64_t cap, int32_t F, int32_t K, int64_t i,
                                         float x, float y, float z, float ls, float logit0, float r, float g,
                                         float b, uint8_t* __restrict__ vis) {
  float* P = buf;
  P[i] = x;
  P[cap + i] = y;
  P[2 * cap + i] = z;
  P[3 * cap + i] = ls;
  P[4 * cap + i] = ls;
  P[5 * cap + i] = ls;
  P[6 * cap + i] = 1.0f;
  P[7 * cap + i] = 0.0f;
  P[8 * cap + i] = 0.0f;
  P[9 * cap + i] = 0.0f;
  P[10 * cap + i] = logit0;
  P[11 * cap + i] = (r - 0.5f) / kSH0;
  P[12 * cap + i] = (g - 0.5f) / kSH0;
  P[13 * cap + i] = (b - 0.5f) / kSH0;
  for (int f = 14; f < 11 + 3 * K; ++f) P[f * cap + i] = 0.0f;
  for (int f = 0; f < F; ++f) {
    buf[(int64_t)(F + f) * cap + i] = 0.0f;
    buf[(int64_t)(2 * F + f) * cap + i] = 0.0f;
    buf[(int64_t)(3 * F + f) * cap + i] = 0.0f;
  }
  vis[i] = 0;
}

// Kept points (flags[j] = 1) go to row n0 + offsets[j]; scale d / f_x with d the point's
// camera-frame depth clamped below at near.
__global__ void __launch_bounds__(256)
k_init_selected(float* __restrict__ buf, int64_t cap, int32_t F, int32_t K, int64_t n0, int64_t n,
                const float* __restrict__ xyz, const float* __restrict__ rgb, const uint32_t* __restrict__ flags,
                const uint32_t* __restrict__ offsets, ViewDev V, float near_z, float logit0,
                uint8_t* __restrict__ vis) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n || !flags[j]) return;
  const float x = xyz[3 * j], y = xyz[3 * j + 1], z = xyz[3 * j + 2];
  const float d = V.R[6] * x + V.R[7] * y + V.R[8] * z + V.t[2];
  init_row(buf, cap, F, K, n0 + offsets[j], x, y, z, logf(fmaxf(d, near_z) / V.fx), logit0, rgb[3 * j],
           rgb[3 * j + 1], rgb[3 * j + 2], vis);
}

// Squared distance from each point to its closest other point: every lane owns one point
// and sweeps all points through LDS in tiles of 256.
__global__ void __launch_bounds__(256) k_nn_dist2(const float* __restrict__ xyz, int64_t n, float* __restrict__ d2) {
  __shared__ float s_p[3][256];
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  float x = 0.f, y = 0.f, z = 0.f;
  if (j < n) {
    x = xyz[3 * j];
    y = xyz[3 * j + 1];
    z = xyz[3 * j + 2];
  }
  float best = __builtin_huge_valf();
  for (int64_t base = 0; base < n; base += 256) {
    __syncthreads();
    const int64_t k = base + threadIdx.x;
    if (k < n) {
      s_p[0][threadIdx.x] = xyz[3 * k];
      s_p[1][threadIdx.x] = xyz[3 * k + 1];
      s_p[2][threadIdx.x] = xyz[3 * k + 2];
    }
    __syncthreads();
    const int cnt = (int)min((int64_t)256, n - base);
    for (int t = 0; t < cnt; ++t) {
      const float dx = s_p[0][t] - x, dy = s_p[1][t] - y, dz = s_p[2][t] - z;
      const float e = dx * dx + dy * dy + dz * dz;
      if (base + t != j) best = fminf(best, e);
    }
  }
  if (j < n) d2[j] = best;
}

// Sky rows: white DC, opacity logit0, isotropic scale = nearest-neighbour distance.
__global__ void __launch_bounds__(256)
k_init_sky(float* __restrict__ buf, int64_t cap, int32_t F, int32_t K, int64_t n0, int64_t n,
           const float* __restrict__ xyz, const float* __restrict__ d2, float logit0, uint8_t* __restrict__ vis) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  init_row(buf, cap, F, K, n0 + j, xyz[3 * j], xyz[3 * j + 1], xyz[3 * j + 2], 0.5f * logf(d2[j]), logit0, 1.0f,
           1.0f, 1.0f, vis);
}

static unsigned blocks(int64_t n) { return (unsigned)((n + 255) / 256); }

hipError_t expand_flags(const float* xyz, int64_t n, const ViewDev& V, const float* T, float tau, float near_z,
                        uint32_t* flags, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_expand_flags, dim3(blocks(n)), dim3(256), 0, s, xyz, n, V, T, tau, near_z, flags);
  return hipGetLastError();
}

hipError_t init_selected(float* buf, int64_t cap, int32_t F, int32_t K, int64_t n0, int64_t n, const float* xyz,
                         const float* rgb, const uint32_t* flags, const uint32_t* offsets, const ViewDev& V,
                         float near_z, float logit0, uint8_t* vis, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_init_selected, dim3(blocks(n)), dim3(256), 0, s, buf, cap, F, K, n0, n, xyz, rgb, flags,
                     offsets, V, near_z, logit0, vis);
  return hipGetLastError();
}

hipError_t init_sky(float* buf, int64_t cap, int32_t F, int32_t K, int64_t n0, int64_t n, const float* xyz,
                    float* d2, float logit0, uint8_t* vis, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_nn_dist2, dim3(blocks(n)), dim3(256), 0, s, xyz, n, d2);
  hipLaunchKernelGGL(k_init_sky, dim3(blocks(n)), dim3(256), 0, s, buf, cap, F, K, n0, n, xyz, d2, logit0, vis);
  return hipGetLastError();
}

}  // namespace gs
