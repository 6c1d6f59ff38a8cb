// Eq. 9 loss: L = (1 - lambda) mean|out - gt| + lambda (1 - mean SSIM(out, gt)) and its
// gradient. SSIM per channel with an 11x11 Gaussian window (sigma 1.5, separable),
// C1 = 0.01^2, C2 = 0.03^2, zero padding outside the image.
//
// Pass 1 (per 16x16 pixel block, per channel): out and gt with a 5-pixel halo go to LDS,
// a horizontal then a vertical window pass forms the five local moments, and the pass
// writes the partial derivatives of SSIM with respect to mu_x, E[x^2] and E[xy] (already
// scaled by dL/dSSIM) plus per-block sums of SSIM and |out - gt|.
// Pass 2: the same separable window applied to those partial maps (the window is
// symmetric, so the adjoint of the zero-padded correlation is the same correlation)
// gives dL/dout = blur(d_mu) + 2 x blur(d_xx) + y blur(d_xy) + L1 term.
// Pass 3: one block adds the per-block sums in a fixed order.
#include <cmath>

#include "gs_common.h"
#include "kernels.h"

namespace gs {

constexpr int kLB = 16;          // output block edge
constexpr int kHalo = 5;
constexpr int kLE = kLB + 2 * kHalo;  // 26

// Normalised 1-D Gaussian window (sigma 1.5), passed by value to the kernels.
struct Win {
  float w[11];
};

static Win make_window() {
  Win W;
  double g[11], s = 0.0;
  for (int i = 0; i < 11; ++i) {
    g[i] = std::exp(-((i - 5) * (i - 5)) / (2.0 * 1.5 * 1.5));
    s += g[i];
  }
  for (int i = 0; i < 11; ++i) W.w[i] = (float)(g[i] / s);
  return W;
}

template <int NQ>
__device__ __forceinline__ void sep_blur(const Win& c_win, float (*src)[kLE][kLE], float (*hbuf)[kLE][kLB],
                                         float* outv) {
  // horizontal: rows 0..25, output columns 0..15
  for (int t = threadIdx.x; t < kLE * kLB; t += 256) {
    const int r = t / kLB, c = t % kLB;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      float acc = 0.f;
#pragma unroll
      for (int j = 0; j < 11; ++j) acc += c_win.w[j] * src[q][r][c + j];
      hbuf[q][r][c] = acc;
    }
  }
  __syncthreads();
  const int ly = threadIdx.x / kLB, lx = threadIdx.x % kLB;
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    float acc = 0.f;
#pragma unroll
    for (int i = 0; i < 11; ++i) acc += c_win.w[i] * hbuf[q][ly + i][lx];
    outv[q] = acc;
  }
}

__global__ void __launch_bounds__(256)
k_ssim_fwd(Win win, const float* __restrict__ x, const float* __restrict__ y, int H, int W, float lambda,
           float* __restrict__ dmu, float* __restrict__ dxx, float* __restrict__ dxy,
           float* __restrict__ part) {
  __shared__ float s_src[5][kLE][kLE];
  __shared__ float s_h[5][kLE][kLB];
  __shared__ float s_red[2][4];
  const int bx = blockIdx.x * kLB, by = blockIdx.y * kLB;
  const int ly = threadIdx.x / kLB, lx = threadIdx.x % kLB;
  const int px = bx + lx, py = by + ly;
  const bool inside = px < W && py < H;
  const int64_t P = (int64_t)H * W;
  const float n = 3.0f * (float)P;
  const float C1 = 0.01f * 0.01f, C2 = 0.03f * 0.03f;
  float ssum = 0.f, l1 = 0.f;
  for (int ch = 0; ch < 3; ++ch) {
    const float* xc = x + ch * P;
    const float* yc = y + ch * P;
    __syncthreads();
    for (int t = threadIdx.x; t < kLE * kLE; t += 256) {
      const int r = t / kLE, c = t % kLE;
      const int gy = by + r - kHalo, gx = bx + c - kHalo;
      float a = 0.f, b = 0.f;
      if (gx >= 0 && gx < W && gy >= 0 && gy < H) {
        a = xc[(int64_t)gy * W + gx];
        b = yc[(int64_t)gy * W + gx];
      }
      s_src[0][r][c] = a;
      s_src[1][r][c] = b;
      s_src[2][r][c] = a * a;
      s_src[3][r][c] = b * b;
      s_src[4][r][c] = a * b;
    }
    __syncthreads();
    float m[5];
    sep_blur<5>(win, s_src, s_h, m);
    if (inside) {
      const float mx = m[0], my = m[1];
      const float A1 = 2.f * mx * my + C1, A2 = 2.f * (m[4] - mx * my) + C2;
      const float B1 = mx * mx + my * my + C1, B2 = (m[2] - mx * mx) + (m[3] - my * my) + C2;
      const float num = A1 * A2, den = B1 * B2;
      const float S = num / den;
      ssum += S;
      const float s = -lambda / n;
      const float dnum = 2.f * my * A2 - 2.f * my * A1;
      const float dden = 2.f * mx * B2 - 2.f * mx * B1;
      const int64_t q = ch * P + (int64_t)py * W + px;
      dmu[q] = s * (dnum * den - num * dden) / (den * den);
      dxx[q] = s * (-num * B1 / (den * den));
      dxy[q] = s * (2.f * A1 / den);
      l1 += fabsf(s_src[0][ly + kHalo][lx + kHalo] - s_src[1][ly + kHalo][lx + kHalo]);
    }
  }
  ssum = wave_sum(ssum);
  l1 = wave_sum(l1);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) {
    s_red[0][wid] = ssum;
    s_red[1][wid] = l1;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const int64_t b = (int64_t)blockIdx.y * gridDim.x + blockIdx.x;
    part[2 * b] = s_red[0][0] + s_red[0][1] + s_red[0][2] + s_red[0][3];
    part[2 * b + 1] = s_red[1][0] + s_red[1][1] + s_red[1][2] + s_red[1][3];
  }
}

__global__ void __launch_bounds__(256)
k_ssim_bwd(Win win, const float* __restrict__ x, const float* __restrict__ y, int H, int W, float lambda,
           const float* __restrict__ dmu, const float* __restrict__ dxx, const float* __restrict__ dxy,
           float* __restrict__ gout) {
  __shared__ float s_src[3][kLE][kLE];
  __shared__ float s_h[3][kLE][kLB];
  const int bx = blockIdx.x * kLB, by = blockIdx.y * kLB;
  const int ly = threadIdx.x / kLB, lx = threadIdx.x % kLB;
  const int px = bx + lx, py = by + ly;
  const bool inside = px < W && py < H;
  const int64_t P = (int64_t)H * W;
  const float l1w = (1.0f - lambda) / (3.0f * (float)P);
  for (int ch = 0; ch < 3; ++ch) {
    __syncthreads();
    for (int t = threadIdx.x; t < kLE * kLE; t += 256) {
      const int r = t / kLE, c = t % kLE;
      const int gy = by + r - kHalo, gx = bx + c - kHalo;
      float a = 0.f, b = 0.f, d = 0.f;
      if (gx >= 0 && gx < W && gy >= 0 && gy < H) {
        const int64_t q = ch * P + (int64_t)gy * W + gx;
        a = dmu[q];
        b = dxx[q];
        d = dxy[q];
      }
      s_src[0][r][c] = a;
      s_src[1][r][c] = b;
      s_src[2][r][c] = d;
    }
    __syncthreads();
    float m[3];
    sep_blur<3>(win, s_src, s_h, m);
    if (inside) {
      const int64_t q = ch * P + (int64_t)py * W + px;
      const float xv = x[q], yv = y[q];
      const float d = xv - yv;
      const float sg = d > 0.f ? 1.f : (d < 0.f ? -1.f : 0.f);
      gout[q] = m[0] + 2.f * xv * m[1] + yv * m[2] + l1w * sg;
    }
  }
}

__global__ void __launch_bounds__(256)
k_loss_reduce(const float* __restrict__ part, int64_t nb, int64_t P, float lambda, float* __restrict__ loss) {
  __shared__ double s[2][256];
  double a = 0.0, b = 0.0;
  for (int64_t k = threadIdx.x; k < nb; k += 256) {
    a += part[2 * k];
    b += part[2 * k + 1];
  }
  s[0][threadIdx.x] = a;
  s[1][threadIdx.x] = b;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      s[0][threadIdx.x] += s[0][threadIdx.x + o];
      s[1][threadIdx.x] += s[1][threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double n = 3.0 * (double)P;
    loss[0] = (float)((1.0 - lambda) * s[1][0] / n + lambda * (1.0 - s[0][0] / n));
  }
}

int64_t loss_temp_floats(int H, int W) {
  const int64_t P = (int64_t)H * W;
  const int64_t nb = (int64_t)((W + kLB - 1) / kLB) * ((H + kLB - 1) / kLB);
  return 9 * P + 2 * nb + 64;
}

hipError_t ssim_loss(const float* out, const float* gt, int H, int W, float lambda, float* temp, float* loss,
                     float* gout, hipStream_t s) {
  const Win win = make_window();
  const int64_t P = (int64_t)H * W;
  float* dmu = temp;
  float* dxx = temp + 3 * P;
  float* dxy = temp + 6 * P;
  float* part = temp + 9 * P;
  const dim3 grid((W + kLB - 1) / kLB, (H + kLB - 1) / kLB);
  const int64_t nb = (int64_t)grid.x * grid.y;
  hipLaunchKernelGGL(k_ssim_fwd, grid, dim3(256), 0, s, win, out, gt, H, W, lambda, dmu, dxx, dxy, part);
  hipLaunchKernelGGL(k_ssim_bwd, grid, dim3(256), 0, s, win, out, gt, H, W, lambda, dmu, dxx, dxy, gout);
  hipLaunchKernelGGL(k_loss_reduce, dim3(1), dim3(256), 0, s, part, nb, P, lambda, loss);
  return hipGetLastError();
}

}  // namespace gs
