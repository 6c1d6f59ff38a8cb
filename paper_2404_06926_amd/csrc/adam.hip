// Sparse Adam (Sec. III-D.2; Adam with the vanilla-3DGS learning rates, Sec. IV-A.1),
// Gaussian initialisation from points (Sec. III-C.1), appends, fills and plane copies.
#include "gs_common.h"
#include "kernels.h"

namespace gs {

// Device step counter and bias corrections: t += 1; bc1 = 1 - b1^t; bc2 = 1 - b2^t.
// Kept on the device so that a replayed graph advances t.
__global__ void k_adam_prepare(int64_t* step, float* bc, float beta1, float beta2) {
  const int64_t t = step[0] + 1;
  step[0] = t;
  bc[0] = (float)(1.0 - pow((double)beta1, (double)t));
  bc[1] = (float)(1.0 - pow((double)beta2, (double)t));
}

// One lane per (row, plane); rows with vis = 0 are left untouched.
__global__ void __launch_bounds__(256)
k_adam(float* __restrict__ p, float* __restrict__ g, float* __restrict__ m, float* __restrict__ v,
       const uint8_t* __restrict__ vis, int64_t cap, int32_t N, LrArg lr, const float* __restrict__ bc,
       float beta1, float beta2, float eps) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int f = blockIdx.y;
  if (i >= N || !vis[i]) return;
  const int64_t k = (int64_t)f * cap + i;
  float pp = p[k], mm = m[k], vv = v[k];
  adam_update(pp, mm, vv, g[k], lr.lr[f], beta1, beta2, eps, bc[0], bc[1]);
  p[k] = pp;
  m[k] = mm;
  v[k] = vv;
  g[k] = 0.0f;
}

// Exposure states: [E(12) | grad(12) | m(12) | v(12)] each.
__global__ void k_adam_exposure(ExpArg ea, const float* __restrict__ bc, float lr, float beta1, float beta2,
                                float eps) {
  const int e = blockIdx.x, k = threadIdx.x;
  if (e >= ea.n || k >= 12) return;
  float* s = ea.p[e];
  float pp = s[k], mm = s[24 + k], vv = s[36 + k];
  adam_update(pp, mm, vv, s[12 + k], lr, beta1, beta2, eps, bc[0], bc[1]);
  s[k] = pp;
  s[24 + k] = mm;
  s[36 + k] = vv;
  s[12 + k] = 0.0f;
}

__global__ void __launch_bounds__(256) k_fill_u32(uint32_t* __restrict__ d, uint32_t val, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) d[i] = val;
}

// rows [n0, n0 + n) of every plane: params from AoS inputs, grads/m/v = 0, vis = 0
__global__ void __launch_bounds__(256)
k_append(float* __restrict__ buf, int64_t cap, int32_t F, int32_t K, int64_t n0, int64_t n,
         const float* __restrict__ means, const float* __restrict__ ls, const float* __restrict__ quats,
         const float* __restrict__ logits, const float* __restrict__ sh, uint8_t* __restrict__ vis) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const int64_t i = n0 + j;
  float* P = buf;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    P[c * cap + i] = means[3 * j + c];
    P[(3 + c) * cap + i] = ls[3 * j + c];
  }
#pragma unroll
  for (int c = 0; c < 4; ++c) P[(6 + c) * cap + i] = quats[4 * j + c];
  P[10 * cap + i] = logits[j];
  for (int f = 0; f < 3 * K; ++f) P[(11 + f) * cap + i] = sh[3 * K * j + f];
  for (int f = 0; f < F; ++f) {
    buf[(int64_t)(F + f) * cap + i] = 0.0f;
    buf[(int64_t)(2 * F + f) * cap + i] = 0.0f;
    buf[(int64_t)(3 * F + f) * cap + i] = 0.0f;
  }
  vis[i] = 0;
}

// Sec. III-C.1: a point becomes a Gaussian centred on it, with SH DC chosen so that it
// renders as the point's colour (colour = Y00 dc + 0.5), other SH 0, opacity o_init,
// identity rotation and isotropic scale d / f, d = depth of the point in the view.
__global__ void __launch_bounds__(256)
k_init_points(float* __restrict__ buf, int64_t cap, int32_t F, int32_t K, int64_t n0, int64_t n,
              const float* __restrict__ xyz, const float* __restrict__ rgb, ViewDev V, float near_z,
              float logit0, uint8_t* __restrict__ vis) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const int64_t i = n0 + j;
  const float x = xyz[3 * j], y = xyz[3 * j + 1], z = xyz[3 * j + 2];
  const float d = V.R[6] * x + V.R[7] * y + V.R[8] * z + V.t[2];
  const float ls = logf(fmaxf(d, near_z) / V.fx);
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
#pragma unroll
  for (int c = 0; c < 3; ++c) P[(11 + c) * cap + i] = (rgb[3 * j + c] - 0.5f) / kSH0;
  for (int f = 14; f < 11 + 3 * K; ++f) P[f * cap + i] = 0.0f;
  for (int f = 0; f < F; ++f) {
    buf[(int64_t)(F + f) * cap + i] = 0.0f;
    buf[(int64_t)(2 * F + f) * cap + i] = 0.0f;
    buf[(int64_t)(3 * F + f) * cap + i] = 0.0f;
  }
  vis[i] = 0;
}

// copy rows [0, n) of nplanes planes from stride cap0 to stride cap1
__global__ void __launch_bounds__(256)
k_copy_planes(const float* __restrict__ src, int64_t cap0, float* __restrict__ dst, int64_t cap1, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int f = blockIdx.y;
  if (i < n) dst[(int64_t)f * cap1 + i] = src[(int64_t)f * cap0 + i];
}

hipError_t adam_prepare(int64_t* step, float* bc, float beta1, float beta2, hipStream_t s) {
  hipLaunchKernelGGL(k_adam_prepare, dim3(1), dim3(1), 0, s, step, bc, beta1, beta2);
  return hipGetLastError();
}

hipError_t adam_exposures(const ExpArg& ea, const float* bc, float lr, float beta1, float beta2, float eps,
                          hipStream_t s) {
  if (ea.n > 0) hipLaunchKernelGGL(k_adam_exposure, dim3(ea.n), dim3(64), 0, s, ea, bc, lr, beta1, beta2, eps);
  return hipGetLastError();
}

hipError_t adam_step(float* buf, int64_t cap, int32_t F, int32_t N, const uint8_t* vis, const LrArg& lr,
                     int64_t* step, float* bc, float beta1, float beta2, float eps, const ExpArg& ea,
                     float lr_exposure, hipStream_t s) {
  hipLaunchKernelGGL(k_adam_prepare, dim3(1), dim3(1), 0, s, step, bc, beta1, beta2);
  if (N > 0) {
    hipLaunchKernelGGL(k_adam, dim3((unsigned)((N + 255) / 256), (unsigned)F), dim3(256), 0, s, buf, buf + F * cap,
                       buf + 2 * F * cap, buf + 3 * F * cap, vis, cap, N, lr, bc, beta1, beta2, eps);
  }
  if (ea.n > 0)
    hipLaunchKernelGGL(k_adam_exposure, dim3(ea.n), dim3(64), 0, s, ea, bc, lr_exposure, beta1, beta2, eps);
  return hipGetLastError();
}

hipError_t fill_u32(uint32_t* d, uint32_t val, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, d, val, n);
  return hipGetLastError();
}

hipError_t append_rows(float* buf, int64_t cap, int32_t F, int32_t K, int64_t n0, int64_t n, const float* means,
                       const float* ls, const float* quats, const float* logits, const float* sh, uint8_t* vis,
                       hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_append, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, buf, cap, F, K, n0, n, means,
                     ls, quats, logits, sh, vis);
  return hipGetLastError();
}

hipError_t init_points(float* buf, int64_t cap, int32_t F, int32_t K, int64_t n0, int64_t n, const float* xyz,
                       const float* rgb, const ViewDev& V, float near_z, float logit0, uint8_t* vis,
                       hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_init_points, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, buf, cap, F, K, n0, n,
                     xyz, rgb, V, near_z, logit0, vis);
  return hipGetLastError();
}

hipError_t copy_planes(const float* src, int64_t cap0, float* dst, int64_t cap1, int64_t n, int nplanes,
                       hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy_planes, dim3((unsigned)((n + 255) / 256), (unsigned)nplanes), dim3(256), 0, s, src,
                     cap0, dst, cap1, n);
  return hipGetLastError();
}

}  // namespace gs
