// Eq. 9 loss: L = (1 - lambda) mean|out - gt| + lambda (1 - mean SSIM(out, gt)) and its
// gradient, for one or several images in one launch. SSIM per channel with an 11x11
// Gaussian window (sigma 1.5, separable), C1 = 0.01^2, C2 = 0.03^2, zero padding outside
// the image.
//
// One fused pass per 32x32 output tile (k_ssim_tile, 512 threads), channel by channel:
//   1. out and gt over the tile with a 10-pixel margin go to LDS as differences from the
//      tile's centre pixel (a = x - cx, b = y - cy; zero padding outside the image means
//      a = -cx there). The window sums are shift-covariant, so the local moments of a and b
//      give the variances and covariance without subtracting two nearly equal FP32
//      squares (E[x^2] - mu^2 cancels badly on smooth images); the means are cx + E[a].
//      Each lane loads the next channel's share into registers while this one runs;
//   2. the four local moments (E[a], E[b], E[a^2 + b^2], E[ab]) over the tile with a
//      5-pixel margin: a horizontal then a vertical window pass, each lane producing a run
//      of outputs from values it holds in registers. SSIM takes the two variances only as
//      their sum (its denominator's second factor), so one window of a^2 + b^2 serves;
//   3. at those pixels (inside the image; zero outside) the partial derivatives of SSIM
//      with respect to E[a], E[a^2] (= the derivative with respect to E[a^2 + b^2]) and
//      E[ab], scaled by dL/dSSIM;
//   4. the same separable window applied to those three maps (the window is symmetric, so
//      the adjoint of the zero-padded correlation is the same correlation) gives
//      dL/dout = blur(d_mu) + 2 a blur(d_aa) + b blur(d_ab) + the L1 term on the tile
//      (the L1 term from the unshifted values, so that sign(0) = 0 is exact).
// The moments of the 5-pixel margin are recomputed by the neighbouring tiles instead of
// going through HBM; a 32x32 tile recomputes 1.7x its pixels' moments (42 x 42 for 32 x 32)
// where a 32x16 tile recomputed 2.1x. Every block writes its sums of SSIM and |out - gt|; a
// second launch (one block per image) adds each image's sums in a fixed order and writes its
// loss. (A last-block ticket in the tile kernel would save that launch, but the
// device-scope release each block would then need writes back its XCD's L2 and cost more
// than the launch.)
#include <cmath>

#include "gs_common.h"
#include "kernels.h"

namespace gs {

constexpr int kR = 5;                  // window radius
constexpr int kTW = kLossTile, kTH = kLossTile;  // output tile (32 x 32)
constexpr int kBW = kTW + 2 * kR;      // 42: moments / derivative maps
constexpr int kBH = kTH + 2 * kR;      // 42
constexpr int kAW = kTW + 4 * kR;      // 52: inputs
constexpr int kAH = kTH + 4 * kR;      // 52
constexpr int kThreads = 512;
// Runs of outputs per lane. Each pass keeps the SIMDs' shares of the block's work even (a
// block's waves take the four SIMDs in turn): 8 waves for the horizontal passes and the
// last one, 4 for the vertical moment pass (its 8-wave form, runs of 4 rows, issues more
// instructions and measured slower). Where the run does not divide the width, the last run
// computes a few outputs more (from padding words) that nothing reads.
constexpr int kHRun = 5, kHRuns = 9;   // horizontal moment pass: 45 >= 42 columns
constexpr int kVRun = 7, kVRuns = 6;   // vertical moment pass: 42 rows
constexpr int kDRun = 3, kDRuns = 11;  // horizontal derivative pass: 33 >= 32 columns
constexpr int kGRun = 2;               // vertical derivative pass: 32 rows = 16 x 2
// LDS row strides in words: inputs, moments' horizontal pass, derivative maps and their
// horizontal pass (see the lane tables below)
constexpr int kSA = 61;
constexpr int kSB = 61;
constexpr int kSD = 43;
constexpr int kSE = 43;
constexpr int kHRows = kVRun * kVRuns + 10;  // rows of the moments' horizontal pass read
constexpr int kDRows = kVRun * kVRuns;       // rows of the derivative maps written
constexpr int kPartOffset = 64;        // temp: [64 ...) per-block partial sums
static_assert(kHRun * kHRuns >= kBW && kHRun * kHRuns <= kSB && kHRun * kHRuns + 10 <= kSA, "horizontal moment runs");
static_assert(kVRun * kVRuns >= kBH && kHRows >= kAH, "vertical moment runs");
static_assert(kDRun * kDRuns >= kTW && kDRun * kDRuns <= kSE && kDRun * kDRuns + 10 <= kSD, "horizontal derivative runs");
static_assert(kTW * (kTH / kGRun) == kThreads && kTH % kGRun == 0, "vertical derivative pass");

// Lane tables. LDS has 32 banks of 4 bytes and serves a wave's access as two halves of 32
// lanes; a half whose lanes touch 32 distinct banks takes one pass, a half with k words in
// one bank k passes. In the three passes below every lane reads a run of words at
// base(lane) + j for the same j, so a half is conflict-free exactly when its lanes' bases
// fall in distinct banks. Each pass's work items (row or column, run) are grouped by the
// bank of their base, and lane 32 h + u takes the h-th item whose base lies in bank u; the
// strides above make those groups small enough that the items fill 16, 8 and 16 halves (8,
// 4 and 8 waves), and make the horizontal passes' writes conflict-free as well (the
// vertical moment pass's writes are two-way). Entry: first index | run << 8; kNoItem for an
// idle lane.
constexpr uint16_t kNoItem = 0xFFFF;
struct LaneTable {
  uint16_t item[kThreads];
  int used;  // lanes up to the last busy one
};
// items (a, b), a < na, b < nb, enumerated with a outer; base bank = (a sa + b sb) mod 32
constexpr LaneTable pack_lanes(int na, int nb, int sa, int sb) {
  LaneTable t{};
  for (int i = 0; i < kThreads; ++i) t.item[i] = kNoItem;
  int cnt[32] = {};
  t.used = 0;
  for (int a = 0; a < na; ++a)
    for (int b = 0; b < nb; ++b) {
      const int u = (a * sa + b * sb) & 31;
      const int lane = 32 * cnt[u] + u;
      cnt[u] += 1;
      if (lane < kThreads) t.item[lane] = (uint16_t)(a | b << 8);
      if (lane + 1 > t.used) t.used = lane + 1;
    }
  return t;
}
// horizontal moment pass: (input row r, run k), base r kSA + k kHRun
constexpr LaneTable kLanesH = pack_lanes(kAH, kHRuns, kSA, kHRun);
// vertical moment pass: (column c, run q), base (q kVRun) kSB + c
constexpr LaneTable kLanesV = pack_lanes(kBW, kVRuns, 1, kVRun * kSB);
// horizontal derivative pass: (row r, run k), base r kSD + k kDRun
constexpr LaneTable kLanesD = pack_lanes(kBH, kDRuns, kSD, kDRun);
static_assert(kLanesH.used <= kThreads && kLanesV.used <= kThreads && kLanesD.used <= kThreads, "lane tables overflow");
struct LaneTables {
  uint16_t h[kThreads], v[kThreads], d[kThreads];
};
constexpr LaneTables make_lane_tables() {
  LaneTables t{};
  for (int i = 0; i < kThreads; ++i) {
    t.h[i] = kLanesH.item[i];
    t.v[i] = kLanesV.item[i];
    t.d[i] = kLanesD.item[i];
  }
  return t;
}
__constant__ LaneTables c_lanes = make_lane_tables();

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

// 76,192 bytes: two blocks fit a CU's 160 KiB of LDS. The inputs are dead once the
// horizontal moment pass has read them (the last pass takes a and b at its own pixels from
// the values it loads for the L1 term), so the derivative maps reuse their space; the
// moments' horizontal pass is dead once the vertical pass has read it.
struct SsimLds {
  union {
    struct {
      float x[kAH][kSA];        // a = x - cx (inputs with a 10-pixel margin)
      float y[kAH][kSA];        // b = y - cy
    };
    float d[3][kDRows][kSD];    // derivative maps
  };
  union {
    float h[4][kHRows][kSB];    // horizontal pass of the four moment maps
    float hd[3][kBH][kSE];      // horizontal pass of the three derivative maps
  };
  float wred[2][kThreads / 64];
};
static_assert(sizeof(SsimLds) == 76192 && sizeof(SsimLds) * 2 <= 160 * 1024, "two blocks per CU");

__device__ __forceinline__ int loss_view_of(const LossArg& la, int b) {
  int v = 0;
  while (v + 1 < la.n && b >= la.v[v + 1].tile_base) ++v;
  return v;
}

// two blocks per CU (as many as LDS allows): at most 128 VGPRs. With prep.step, block 0
// also advances the Adam step counter and its bias corrections (as adam_prepare), saving
// that launch in a fused step, or counts the step as skipped.
__global__ void __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(4)))
k_ssim_tile(Win win, LossArg la, float* __restrict__ part, StepPrep prep) {
  __shared__ SsimLds L;
  if (prep.step && blockIdx.x == 0 && threadIdx.x == 0) {
    if (prep.n_inst && (int64_t)prep.n_inst[0] > prep.inst_cap) {
      prep.skipped[0] += 1u;  // the step's render dropped instances: the step is skipped
    } else {
      const int64_t t = prep.step[0] + 1;
      prep.step[0] = t;
      prep.bc[0] = (float)(1.0 - pow((double)prep.beta1, (double)t));
      prep.bc[1] = (float)(1.0 - pow((double)prep.beta2, (double)t));
    }
  }
  const int view = loss_view_of(la, blockIdx.x);
  const LossView& V = la.v[view];
  const float* __restrict__ x = V.x;
  const float* __restrict__ y = V.y;
  float* __restrict__ gout = V.gout;
  const int H = V.H, W = V.W;
  const int lb = (int)blockIdx.x - V.tile_base;
  const int bx = (lb % V.tiles_x) * kTW, by = (lb / V.tiles_x) * kTH;
  const int tid = threadIdx.x;
  const int64_t P = (int64_t)H * W;
  const float n = 3.0f * (float)P;
  const float C1 = 0.01f * 0.01f, C2 = 0.03f * 0.03f;
  const float s_ssim = -la.lambda / n;                 // dL/dSSIM per pixel and channel
  const float l1w = (1.0f - la.lambda) / n;
  // this lane's work items in the table-driven passes
  const uint32_t item_h = c_lanes.h[tid], item_v = c_lanes.v[tid], item_d = c_lanes.d[tid];
  // centre pixel of the tile (inside the image)
  const int64_t cidx = (int64_t)min(by + kTH / 2, H - 1) * W + min(bx + kTW / 2, W - 1);
  float ssum = 0.f, l1 = 0.f;
  constexpr int kLoadPer = (kAH * kAW + kThreads - 1) / kThreads;
  float pa[kLoadPer], pb[kLoadPer];
  float ncx, ncy;
  // pixel index of each of the lane's input slots (-1: outside the image, zero padding).
  // Element indices stay 32-bit (images are at most 16384 x 16384, so 3 H W < 2^31) and
  // are formed per channel, so that no 64-bit addresses stay live across the channel loop.
  const int P32 = H * W;
  int off[kLoadPer];
#pragma unroll
  for (int j = 0; j < kLoadPer; ++j) {
    const int t = tid + kThreads * j;
    const int r = t / kAW, c = t % kAW;
    const int gy = by - 2 * kR + r, gx = bx - 2 * kR + c;
    off[j] = (t < kAH * kAW && gx >= 0 && gx < W && gy >= 0 && gy < H) ? gy * W + gx : -1;
  }
  auto fetch = [&](int ch) {
    const int base = ch * P32;
#pragma unroll
    for (int j = 0; j < kLoadPer; ++j) {
      pa[j] = off[j] >= 0 ? x[base + off[j]] : 0.f;
      pb[j] = off[j] >= 0 ? y[base + off[j]] : 0.f;
    }
    ncx = x[base + (int)cidx];
    ncy = y[base + (int)cidx];
  };
  fetch(0);
  for (int ch = 0; ch < 3; ++ch) {
    const float cx = ncx, cy = ncy;
    __syncthreads();
    // 1. inputs with a 10-pixel margin, shifted by the centre values; the next channel's
    // are loaded into registers while this one is processed
#pragma unroll
    for (int j = 0; j < kLoadPer; ++j) {
      const int t = tid + kThreads * j;
      if (t < kAH * kAW) {
        L.x[t / kAW][t % kAW] = pa[j] - cx;
        L.y[t / kAW][t % kAW] = pb[j] - cy;
      }
    }
    if (ch < 2) fetch(ch + 1);
    __syncthreads();
    // 2a. horizontal window pass of the four moments: rows of the input block, columns of
    // the moment block; a lane takes kHRun outputs of one row
    if (item_h != kNoItem) {
      const int r = item_h & 0xFF, c0 = (item_h >> 8) * kHRun;
      float xv[kHRun + 10], yv[kHRun + 10], ss[kHRun + 10], xy[kHRun + 10];
#pragma unroll
      for (int j = 0; j < kHRun + 10; ++j) {
        xv[j] = L.x[r][c0 + j];
        yv[j] = L.y[r][c0 + j];
        ss[j] = xv[j] * xv[j] + yv[j] * yv[j];
        xy[j] = xv[j] * yv[j];
      }
#pragma unroll
      for (int o = 0; o < kHRun; ++o) {
        float m0 = 0.f, m1 = 0.f, m2 = 0.f, m3 = 0.f;
#pragma unroll
        for (int j = 0; j < 11; ++j) {
          const float w = win.w[j];
          m0 += w * xv[o + j];
          m1 += w * yv[o + j];
          m2 += w * ss[o + j];
          m3 += w * xy[o + j];
        }
        L.h[0][r][c0 + o] = m0;
        L.h[1][r][c0 + o] = m1;
        L.h[2][r][c0 + o] = m2;
        L.h[3][r][c0 + o] = m3;
      }
    }
    __syncthreads();
    // 2b. vertical pass and 3. the derivative maps; a lane takes kVRun rows of one column
    if (item_v != kNoItem) {
      const int c = item_v & 0xFF, r0 = (item_v >> 8) * kVRun;
      float acc[4][kVRun];
#pragma unroll
      for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int o = 0; o < kVRun; ++o) acc[k][o] = 0.f;
#pragma unroll
      for (int i = 0; i < kVRun + 10; ++i) {
        float hv[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) hv[k] = L.h[k][r0 + i][c];
#pragma unroll
        for (int o = 0; o < kVRun; ++o) {
          const int j = i - o;  // tap index of input row r0 + i for output row r0 + o
          if (j < 0 || j > 10) continue;
          const float w = win.w[j];
#pragma unroll
          for (int k = 0; k < 4; ++k) acc[k][o] += w * hv[k];
        }
      }
#pragma unroll
      for (int o = 0; o < kVRun; ++o) {
        const int rb = r0 + o;
        const int gy = by - kR + rb, gx = bx - kR + c;
        float dmu = 0.f, dxx = 0.f, dxy = 0.f;
        if (gx >= 0 && gx < W && gy >= 0 && gy < H) {
          const float ea = acc[0][o], eb = acc[1][o];        // shifted means
          const float mx = cx + ea, my = cy + eb;            // means
          const float svv = acc[2][o] - ea * ea - eb * eb, sxy = acc[3][o] - ea * eb;  // sum of variances, covariance
          const float A1 = 2.f * mx * my + C1, A2 = 2.f * sxy + C2;
          const float B1 = mx * mx + my * my + C1, B2 = svv + C2;
          const float num = A1 * A2, den = B1 * B2;
          // derivatives with respect to E[a] at fixed E[a^2], E[ab]: mx moves with it, and
          // the variance and covariance through -E[a]^2 and -E[a] E[b]
          const float dnum = 2.f * my * A2 - 2.f * eb * A1;
          const float dden = 2.f * mx * B2 - 2.f * ea * B1;
          // one reciprocal (den >= C1 C2 - rounding, far from the denormal range): with
          // q = num / den (the SSIM value), d(q)/d. = (dnum - q dden) / den
          const float inv = __builtin_amdgcn_rcpf(den), q = num * inv, si = s_ssim * inv;
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
    // 4a. horizontal window pass of the derivative maps; a lane takes kDRun outputs of one
    // row
    if (item_d != kNoItem) {
      const int r = item_d & 0xFF, c0 = (item_d >> 8) * kDRun;
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
    // 4b. vertical pass and dL/dout on the tile; lane = (column, run of kGRun rows), a half
    // wave on 32 consecutive columns of one run
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
        const int64_t e = ch * P + (int64_t)py * W + px;
        const float xe = x[e], ye = y[e];
        const float av = xe - cx, bv = ye - cy;
        const float d = xe - ye;
        const float sg = d > 0.f ? 1.f : (d < 0.f ? -1.f : 0.f);
        gout[e] = g[0][o] + 2.f * av * g[1][o] + bv * g[2][o] + l1w * sg;
        l1 += fabsf(d);
      }
    }
  }
  ssum = wave_sum(ssum);
  l1 = wave_sum(l1);
  const int lane = tid & 63, wid = tid >> 6;
  __syncthreads();
  if (lane == 0) {
    L.wred[0][wid] = ssum;
    L.wred[1][wid] = l1;
  }
  __syncthreads();
  if (tid == 0) {
    const int64_t b = blockIdx.x;
    float s0 = 0.f, s1 = 0.f;
#pragma unroll
    for (int w = 0; w < kThreads / 64; ++w) {
      s0 += L.wred[0][w];
      s1 += L.wred[1][w];
    }
    part[2 * b] = s0;
    part[2 * b + 1] = s1;
  }
}

// Block v: the loss of image v from its tiles' partial sums, in a fixed order.
__global__ void __launch_bounds__(256)
k_loss_reduce(LossArg la, const float* __restrict__ part, int32_t nb) {
  __shared__ double s[2][256];
  const int v = blockIdx.x;
  const int b0 = la.v[v].tile_base;
  const int b1 = v + 1 < la.n ? la.v[v + 1].tile_base : nb;
  const float L = loss_from_partials(part, b0, b1, la.v[v].H, la.v[v].W, la.lambda, s);
  if (threadIdx.x == 0) la.v[v].loss[0] = L;
}

int64_t loss_tiles(int H, int W) { return (int64_t)((W + kTW - 1) / kTW) * ((H + kTH - 1) / kTH); }

hipError_t loss_finish_launch(const ViewsArg& va, const LossFinish& lf, hipStream_t s) {
  if (!lf.part || va.n <= 0) return hipSuccess;
  LossArg la{};
  la.n = va.n;
  la.lambda = lf.lambda;
  int64_t nb = 0;
  for (int v = 0; v < va.n; ++v) {
    la.v[v].H = va.v[v].H;
    la.v[v].W = va.v[v].W;
    la.v[v].loss = lf.loss + v;
    la.v[v].tile_base = (int32_t)nb;
    nb += loss_tiles(va.v[v].H, va.v[v].W);
  }
  hipLaunchKernelGGL(k_loss_reduce, dim3((unsigned)la.n), dim3(256), 0, s, la, lf.part, (int32_t)nb);
  return hipGetLastError();
}

int64_t loss_temp_floats(int H, int W) { return kPartOffset + 2 * loss_tiles(H, W); }

int64_t loss_part_offset() { return kPartOffset; }

int64_t loss_temp_floats_multi(const LossArg& la) {
  int64_t nb = 0;
  for (int v = 0; v < la.n; ++v) nb += loss_tiles(la.v[v].H, la.v[v].W);
  return kPartOffset + 2 * nb;
}

// la.v[*].tiles_x and tile_base are filled here. temp holds loss_temp_floats_multi(la)
// floats (nothing in it needs clearing: the reduction reads only what the tiles wrote).
hipError_t ssim_loss(LossArg la, float* temp, const StepPrep* prep, bool defer_finish, hipStream_t s) {
  const Win win = make_window();
  int64_t nb = 0;
  for (int v = 0; v < la.n; ++v) {
    la.v[v].tiles_x = (la.v[v].W + kTW - 1) / kTW;
    la.v[v].tile_base = (int32_t)nb;
    nb += loss_tiles(la.v[v].H, la.v[v].W);
  }
  if (nb <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_ssim_tile, dim3((unsigned)nb), dim3(kThreads), 0, s, win, la, temp + kPartOffset,
                     prep ? *prep : StepPrep{nullptr, nullptr, 0.f, 0.f, nullptr, 0, nullptr});
  if (!defer_finish)
    hipLaunchKernelGGL(k_loss_reduce, dim3((unsigned)la.n), dim3(256), 0, s, la, temp + kPartOffset, (int32_t)nb);
  return hipGetLastError();
}

}  // namespace gs
