// Eq. 9 loss: L = (1 - lambda) mean|out - gt| + lambda (1 - mean SSIM(out, gt)) and its
// gradient. SSIM per channel with an 11x11 Gaussian window (sigma 1.5, separable),
// C1 = 0.01^2, C2 = 0.03^2, zero padding outside the image.
//
// One fused pass per 32x16 output tile (k_ssim_tile), channel by channel:
//   1. out and gt over the tile with a 10-pixel margin go to LDS (each lane loads the next
//      channel's share into registers while the current channel is processed);
//   2. the five local moments (mu_x, mu_y, E[x^2], E[y^2], E[xy]) over the tile with a
//      5-pixel margin: a horizontal then a vertical window pass, each lane producing a run
//      of outputs from values it holds in registers;
//   3. at those pixels (inside the image; zero outside) the partial derivatives of SSIM
//      with respect to mu_x, E[x^2] and E[xy], scaled by dL/dSSIM;
//   4. the same separable window applied to those three maps (the window is symmetric, so
//      the adjoint of the zero-padded correlation is the same correlation) gives
//      dL/dout = blur(d_mu) + 2 x blur(d_xx) + y blur(d_xy) + the L1 term on the tile.
// The moments of the 5-pixel margin are recomputed by the neighbouring tiles instead of
// going through HBM. A second launch adds the per-tile sums of SSIM and |out - gt| in a
// fixed order.
#include <cmath>

#include "gs_common.h"
#include "kernels.h"

namespace gs {

constexpr int kR = 5;                  // window radius
constexpr int kTW = 32, kTH = 16;      // output tile
constexpr int kBW = kTW + 2 * kR;      // 42: moments / derivative maps
constexpr int kBH = kTH + 2 * kR;      // 26
constexpr int kAW = kTW + 4 * kR;      // 52: inputs
constexpr int kAH = kTH + 4 * kR;      // 36
constexpr int kHRun = 6;               // horizontal moment pass: outputs per lane (42 = 7 x 6)
constexpr int kVRun = 5;               // vertical moment pass: rows per lane (26 = 5 x 5 + 1)
constexpr int kDRun = 4;               // horizontal derivative pass: outputs per lane (32 = 8 x 4)
constexpr int kGRun = 2;               // vertical derivative pass: rows per lane (16 = 8 x 2)
// every pass's lanes fit the 256-thread block
static_assert(kBW % kHRun == 0 && kAH * (kBW / kHRun) <= 256, "horizontal moment pass");
static_assert(kBW * ((kBH + kVRun - 1) / kVRun) <= 256, "vertical moment pass");
static_assert(kTW % kDRun == 0 && kBH * (kTW / kDRun) <= 256, "horizontal derivative pass");
static_assert(kTH % kGRun == 0 && kTW * (kTH / kGRun) == 256, "vertical derivative pass");

// Normalised 1-D Gaussian window (sigma 1.5), passed by value to the kernel.
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

struct SsimLds {
  float x[kAH][kAW + 1];
  float y[kAH][kAW + 1];
  union {
    float h[5][kAH][kBW];       // horizontal pass of the five moment maps
    float hd[3][kBH][kTW + 1];  // horizontal pass of the three derivative maps
  };
  float d[3][kBH][kBW + 1];     // derivative maps
  float red[2][4];
};

__global__ void __launch_bounds__(256)
k_ssim_tile(Win win, const float* __restrict__ x, const float* __restrict__ y, int H, int W, float lambda,
            float* __restrict__ gout, float* __restrict__ part) {
  __shared__ SsimLds L;
  const int bx = blockIdx.x * kTW, by = blockIdx.y * kTH;
  const int tid = threadIdx.x;
  const int64_t P = (int64_t)H * W;
  const float n = 3.0f * (float)P;
  const float C1 = 0.01f * 0.01f, C2 = 0.03f * 0.03f;
  const float s_ssim = -lambda / n;                    // dL/dSSIM per pixel and channel
  const float l1w = (1.0f - lambda) / n;
  float ssum = 0.f, l1 = 0.f;
  constexpr int kLoadPer = (kAH * kAW + 255) / 256;
  float pa[kLoadPer], pb[kLoadPer];
  auto fetch = [&](int ch) {
#pragma unroll
    for (int j = 0; j < kLoadPer; ++j) {
      const int t = tid + 256 * j;
      const int r = t / kAW, c = t % kAW;
      const int gy = by - 2 * kR + r, gx = bx - 2 * kR + c;
      pa[j] = pb[j] = 0.f;
      if (t < kAH * kAW && gx >= 0 && gx < W && gy >= 0 && gy < H) {
        pa[j] = x[ch * P + (int64_t)gy * W + gx];
        pb[j] = y[ch * P + (int64_t)gy * W + gx];
      }
    }
  };
  fetch(0);
  for (int ch = 0; ch < 3; ++ch) {
    __syncthreads();
    // 1. inputs with a 10-pixel margin (zero outside the image); the next channel's are
    // loaded into registers while this one is processed
#pragma unroll
    for (int j = 0; j < kLoadPer; ++j) {
      const int t = tid + 256 * j;
      if (t < kAH * kAW) {
        L.x[t / kAW][t % kAW] = pa[j];
        L.y[t / kAW][t % kAW] = pb[j];
      }
    }
    if (ch < 2) fetch(ch + 1);
    __syncthreads();
    // 2a. horizontal window pass of the five moments: rows of the input block, columns of
    // the moment block; lane = (row, run of kHRun columns)
    if (tid < kAH * (kBW / kHRun)) {
      const int r = tid / (kBW / kHRun), c0 = (tid % (kBW / kHRun)) * kHRun;
      float xv[kHRun + 10], yv[kHRun + 10];
#pragma unroll
      for (int j = 0; j < kHRun + 10; ++j) {
        xv[j] = L.x[r][c0 + j];
        yv[j] = L.y[r][c0 + j];
      }
#pragma unroll
      for (int o = 0; o < kHRun; ++o) {
        float m0 = 0.f, m1 = 0.f, m2 = 0.f, m3 = 0.f, m4 = 0.f;
#pragma unroll
        for (int j = 0; j < 11; ++j) {
          const float a = xv[o + j], b = yv[o + j], w = win.w[j];
          m0 += w * a;
          m1 += w * b;
          m2 += w * (a * a);
          m3 += w * (b * b);
          m4 += w * (a * b);
        }
        L.h[0][r][c0 + o] = m0;
        L.h[1][r][c0 + o] = m1;
        L.h[2][r][c0 + o] = m2;
        L.h[3][r][c0 + o] = m3;
        L.h[4][r][c0 + o] = m4;
      }
    }
    __syncthreads();
    // 2b. vertical pass and 3. the derivative maps; lane = (column, run of kVRun rows)
    constexpr int kVRuns = (kBH + kVRun - 1) / kVRun;
    if (tid < kBW * kVRuns) {
      const int c = tid % kBW, r0 = (tid / kBW) * kVRun;
      const int nr = min(kVRun, kBH - r0);
      float acc[5][kVRun];
#pragma unroll
      for (int k = 0; k < 5; ++k)
#pragma unroll
        for (int o = 0; o < kVRun; ++o) acc[k][o] = 0.f;
#pragma unroll
      for (int i = 0; i < kVRun + 10; ++i) {
        if (r0 + i >= kAH) break;
        float hv[5];
#pragma unroll
        for (int k = 0; k < 5; ++k) hv[k] = L.h[k][r0 + i][c];
#pragma unroll
        for (int o = 0; o < kVRun; ++o) {
          const int j = i - o;  // tap index of input row r0 + i for output row r0 + o
          if (j < 0 || j > 10) continue;
          const float w = win.w[j];
#pragma unroll
          for (int k = 0; k < 5; ++k) acc[k][o] += w * hv[k];
        }
      }
#pragma unroll
      for (int o = 0; o < kVRun; ++o) {
        if (o >= nr) break;
        const int rb = r0 + o;
        const int gy = by - kR + rb, gx = bx - kR + c;
        float dmu = 0.f, dxx = 0.f, dxy = 0.f;
        if (gx >= 0 && gx < W && gy >= 0 && gy < H) {
          const float mx = acc[0][o], my = acc[1][o];
          const float A1 = 2.f * mx * my + C1, A2 = 2.f * (acc[4][o] - mx * my) + C2;
          const float B1 = mx * mx + my * my + C1, B2 = (acc[2][o] - mx * mx) + (acc[3][o] - my * my) + C2;
          const float num = A1 * A2, den = B1 * B2;
          const float dnum = 2.f * my * A2 - 2.f * my * A1;
          const float dden = 2.f * mx * B2 - 2.f * mx * B1;
          // one division: with q = num / den (the SSIM value), d(q)/d. = (dnum - q dden) / den
          const float inv = 1.0f / den, q = num * inv, si = s_ssim * inv;
          dmu = si * (dnum - q * dden);
          dxx = -si * q * B1;
          dxy = 2.f * si * A1;
          // SSIM of the tile's own pixels (the margins belong to the neighbours)
          if (rb >= kR && rb < kR + kTH && c >= kR && c < kR + kTW) ssum += q;
        }
        L.d[0][rb][c] = dmu;
        L.d[1][rb][c] = dxx;
        L.d[2][rb][c] = dxy;
      }
    }
    __syncthreads();
    // 4a. horizontal window pass of the derivative maps; lane = (row, run of kDRun columns)
    if (tid < kBH * (kTW / kDRun)) {
      const int r = tid / (kTW / kDRun), c0 = (tid % (kTW / kDRun)) * kDRun;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        float dv[kDRun + 10];
#pragma unroll
        for (int j = 0; j < kDRun + 10; ++j) dv[j] = L.d[k][r][c0 + j];
#pragma unroll
        for (int o = 0; o < kDRun; ++o) {
          float a = 0.f;
#pragma unroll
          for (int j = 0; j < 11; ++j) a += win.w[j] * dv[o + j];
          L.hd[k][r][c0 + o] = a;
        }
      }
    }
    __syncthreads();
    // 4b. vertical pass and dL/dout on the tile; lane = (column, run of kGRun rows)
    {
      const int c = tid % kTW, r0 = (tid / kTW) * kGRun;
      float g[3][kGRun];
#pragma unroll
      for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int o = 0; o < kGRun; ++o) g[k][o] = 0.f;
#pragma unroll
      for (int i = 0; i < kGRun + 10; ++i) {
        float hv[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) hv[k] = L.hd[k][r0 + i][c];
#pragma unroll
        for (int o = 0; o < kGRun; ++o) {
          const int j = i - o;
          if (j < 0 || j > 10) continue;
#pragma unroll
          for (int k = 0; k < 3; ++k) g[k][o] += win.w[j] * hv[k];
        }
      }
#pragma unroll
      for (int o = 0; o < kGRun; ++o) {
        const int py = by + r0 + o, px = bx + c;
        if (px >= W || py >= H) continue;
        const float xv = L.x[r0 + o + 2 * kR][c + 2 * kR], yv = L.y[r0 + o + 2 * kR][c + 2 * kR];
        const float d = xv - yv;
        const float sg = d > 0.f ? 1.f : (d < 0.f ? -1.f : 0.f);
        gout[ch * P + (int64_t)py * W + px] = g[0][o] + 2.f * xv * g[1][o] + yv * g[2][o] + l1w * sg;
        l1 += fabsf(d);
      }
    }
  }
  ssum = wave_sum(ssum);
  l1 = wave_sum(l1);
  const int lane = tid & 63, wid = tid >> 6;
  __syncthreads();
  if (lane == 0) {
    L.red[0][wid] = ssum;
    L.red[1][wid] = l1;
  }
  __syncthreads();
  if (tid == 0) {
    const int64_t b = (int64_t)blockIdx.y * gridDim.x + blockIdx.x;
    part[2 * b] = L.red[0][0] + L.red[0][1] + L.red[0][2] + L.red[0][3];
    part[2 * b + 1] = L.red[1][0] + L.red[1][1] + L.red[1][2] + L.red[1][3];
  }
}

__global__ void __launch_bounds__(256)
k_loss_reduce(const float* __restrict__ part, int64_t nb, int64_t P, float lambda, float* __restrict__ loss,
              StepPrep prep) {
  __shared__ double s[2][256];
  if (prep.step && threadIdx.x == 0) {  // t += 1 and the bias corrections of step t
    const int64_t t = prep.step[0] + 1;
    prep.step[0] = t;
    prep.bc[0] = (float)(1.0 - pow((double)prep.beta1, (double)t));
    prep.bc[1] = (float)(1.0 - pow((double)prep.beta2, (double)t));
  }
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
  const int64_t nb = (int64_t)((W + kTW - 1) / kTW) * ((H + kTH - 1) / kTH);
  return 2 * nb + 64;
}

hipError_t ssim_loss(const float* out, const float* gt, int H, int W, float lambda, float* temp, float* loss,
                     float* gout, const StepPrep* prep, hipStream_t s) {
  const Win win = make_window();
  const int64_t P = (int64_t)H * W;
  float* part = temp;
  const dim3 grid((W + kTW - 1) / kTW, (H + kTH - 1) / kTH);
  const int64_t nb = (int64_t)grid.x * grid.y;
  hipLaunchKernelGGL(k_ssim_tile, grid, dim3(256), 0, s, win, out, gt, H, W, lambda, gout, part);
  hipLaunchKernelGGL(k_loss_reduce, dim3(1), dim3(256), 0, s, part, nb, P, lambda, loss,
                     prep ? *prep : StepPrep{nullptr, nullptr, 0.f, 0.f});
  return hipGetLastError();
}

}  // namespace gs
