// Internal definitions shared by the HIP kernels and the host code of libgslic.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/gslic.h"

namespace gs {

constexpr int kTile = GS_TILE;        // 16x16 pixel tiles
constexpr int kMaxViews = GS_MAX_VIEWS;
constexpr int kRecFloats = 16;        // per (view, Gaussian) projection record, 64 B
// per (view, Gaussian) 2D-gradient record, 48 B. With g = dL/dpower = dL/dalpha * alpha
// at each pixel the Gaussian reaches (dx, dy = pixel centre - 2D mean; none where alpha is
// clamped), sums over the pixels: [0] g dx  [1] g dy  [2] g dx^2  [3] g dx dy  [4] g dy^2
// [5] g, then [6..8] dL/dcolour, [9] dL/d(camera-frame depth) (depth-map gradient),
// [10..11] unused. Since power = -(A dx^2 + C dy^2) / 2 - B dx dy and alpha = o e^power,
// the projection backward forms dL/dmean2d = conic (g dx, g dy), dL/d(A, B, C) =
// (-[2] / 2, -[3], -[4] / 2) and dL/dlogit = [5] (1 - o): the blend keeps five products
// per pixel and leaves the per-Gaussian factors to one pass.
constexpr int kGradFloats = 12;  // 48 B: records packed back to back, read as 3 x float4

// Per-view constants, passed by value inside ViewsArg (so a captured graph keeps them).
struct ViewDev {
  float R[9];
  float t[3];
  float fx, fy, cx, cy;
  float limx, limy;         // 1.3 (W / 2) / fx and 1.3 (H / 2) / fy (FP32, IEEE division)
  float campos[3];          // camera centre in world coordinates (colour direction)
  float bg[3];
  int32_t W, H, tiles_x, tiles_y;
  int32_t tile_base;        // first global tile id of this view
  int32_t pad0;
  int64_t pix_base;         // first pixel of this view in the concatenated pixel arrays
  const float* exposure;    // 12 floats [A|b] or nullptr (identity)
  float* out_rgb;           // 3 x H x W
  float* out_T;             // H x W
  uint32_t* out_nc;         // H x W
  const float* dl_drgb;     // 3 x H x W (backward)
  float* dl_dexp;           // 12 (backward, may be nullptr)
  float* out_depth;         // H x W depth map (Eq. 6) or nullptr
  float* out_opac;          // H x W opacity map (Eq. 7) or nullptr
  const float* dl_ddepth;   // H x W (backward, may be nullptr)
  const float* dl_dopac;    // H x W (backward, may be nullptr)
};

struct ViewsArg {
  int32_t n;
  int32_t total_tiles;
  ViewDev v[kMaxViews];
  // the render's instance count (device) and the instance capacity: a render that needed
  // more dropped its instances, and its backward adds no gradient at all
  const uint32_t* n_inst;
  int64_t inst_cap;
};
__device__ __forceinline__ bool render_dropped(const ViewsArg& va) {
  return va.n_inst && (int64_t)va.n_inst[0] > va.inst_cap;
}
// passed by value to kernels: stays inside the 4 KiB kernel-argument space with room for
// the other arguments
static_assert(sizeof(ViewsArg) <= 3584, "ViewsArg too large for a kernel argument");

// Eq. 9 loss of an image from the loss kernel's per-tile partial sums (SSIM and |out - gt|
// of each 32 x 32 output tile, two floats per tile): the sums in a fixed order (thread t of
// a 256-thread block adds tiles b0 + t, b0 + t + 256, ... in FP64, then a tree in LDS), so
// every launch that finishes a loss gives the same value.
constexpr int kLossTile = 32;
__device__ __forceinline__ int loss_tiles_of(int H, int W) {
  return ((W + kLossTile - 1) / kLossTile) * ((H + kLossTile - 1) / kLossTile);
}
__device__ inline float loss_from_partials(const float* __restrict__ part, int b0, int b1, int H, int W,
                                           float lambda, double (&s)[2][256]) {
  const int tid = threadIdx.x;
  double a = 0.0, c = 0.0;
  for (int k = b0 + tid; k < b1; k += 256) {
    a += part[2 * k];
    c += part[2 * k + 1];
  }
  s[0][tid] = a;
  s[1][tid] = c;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (tid < o) {
      s[0][tid] += s[0][tid + o];
      s[1][tid] += s[1][tid + o];
    }
    __syncthreads();
  }
  const double nn = 3.0 * (double)H * (double)W;
  const float L = (float)((1.0 - lambda) * s[1][0] / nn + lambda * (1.0 - s[0][0] / nn));
  __syncthreads();  // s is reused by the next call
  return L;
}
// The losses of a fused step's views, left to the projection backward's first block (one
// launch fewer): part == nullptr for none; loss[v] for view v of the step's ViewsArg.
struct LossFinish {
  const float* part;
  float* loss;
  float lambda;
  int32_t pad;
};

// Projection record layout (floats), one per (view, Gaussian), view-major:
//   [0] mean2d x  [1] mean2d y  [2] conic A  [3] conic B
//   [4] conic C   [5] opacity   [6] red      [7] green
//   [8] blue      [9] depth     [10] unused  [11] thr = 2 ln(255 o)
//   [12] tile rect x0 | y0 << 16 (bits)   [13] x1 | y1 << 16 (bits)
//   [14..15] 64-bit mask of the tiles that pass the predicate, in row-major order inside
//            the rectangle (complete when the rectangle has at most 64 tiles)
// Only records whose tile count is > 0 are written.

__device__ __forceinline__ int view_of_tile(const ViewsArg& va, int tile) {
  int v = 0;
  for (int k = 1; k < va.n; ++k)
    if (tile >= va.v[k].tile_base) v = k;
  return v;
}

// ---------------------------------------------------------------------------------
// Key path. Every value that decides a tile key (visibility, depth, 2D mean, conic,
// opacity threshold, tile rectangle and tile predicate) is computed in FP32 in the fixed
// order below, with contraction off and correctly rounded division and square root, so
// that keys are reproducible bit for bit. The transcendentals (exp of a log-scale,
// sigmoid, ln(255 o)) are taken in FP64 and rounded once.
// ---------------------------------------------------------------------------------
struct KeyGeo {          // view-independent part: Sigma = (R S)(R S)^T, Eq. 1
  float S00, S01, S02, S11, S12, S22;
  bool ok;               // quaternion has non-zero norm
};

__device__ __forceinline__ KeyGeo key_geometry(float ls0, float ls1, float ls2, float qw, float qx,
                                               float qy, float qz) {
#pragma clang fp contract(off)
  KeyGeo g;
  const float n2 = ((qw * qw + qx * qx) + qy * qy) + qz * qz;
  const float qn = __fsqrt_rn(n2);
  g.ok = qn > 0.0f;
  const float w = __fdiv_rn(qw, qn), x = __fdiv_rn(qx, qn), y = __fdiv_rn(qy, qn),
              z = __fdiv_rn(qz, qn);
  const float R0 = 1.0f - 2.0f * (y * y + z * z), R1 = 2.0f * (x * y - w * z),
              R2 = 2.0f * (x * z + w * y);
  const float R3 = 2.0f * (x * y + w * z), R4 = 1.0f - 2.0f * (x * x + z * z),
              R5 = 2.0f * (y * z - w * x);
  const float R6 = 2.0f * (x * z - w * y), R7 = 2.0f * (y * z + w * x),
              R8 = 1.0f - 2.0f * (x * x + y * y);
  const float s0 = (float)exp((double)ls0), s1 = (float)exp((double)ls1),
              s2 = (float)exp((double)ls2);
  const float M0 = R0 * s0, M1 = R1 * s1, M2 = R2 * s2;
  const float M3 = R3 * s0, M4 = R4 * s1, M5 = R5 * s2;
  const float M6 = R6 * s0, M7 = R7 * s1, M8 = R8 * s2;
  g.S00 = (M0 * M0 + M1 * M1) + M2 * M2;
  g.S01 = (M0 * M3 + M1 * M4) + M2 * M5;
  g.S02 = (M0 * M6 + M1 * M7) + M2 * M8;
  g.S11 = (M3 * M3 + M4 * M4) + M5 * M5;
  g.S12 = (M3 * M6 + M4 * M7) + M5 * M8;
  g.S22 = (M6 * M6 + M7 * M7) + M8 * M8;
  return g;
}

struct KeyProj {
  bool visible;
  float zh, mx, my, A, B, C, o, thr;
  float a, c;            // diagonal of Sigma' (for the tile rectangle)
};

// Opacity o = sigmoid(logit) and thr = 2 ln(255 o) (for o >= 1/255; 0 otherwise), FP64
// then rounded: the same for every view, so computed once per Gaussian.
struct KeyOpacity {
  float o, thr;
};
__device__ __forceinline__ KeyOpacity key_opacity(float logit) {
  KeyOpacity k;
  k.o = (float)(1.0 / (1.0 + exp(-(double)logit)));
  k.thr = k.o < 1.0f / 255.0f ? 0.0f : (float)(2.0 * log(255.0 * (double)k.o));
  return k;
}

// Eq. 2-3 for one view; culls depth <= near_z, det <= 0 and opacity < 1/255.
__device__ __forceinline__ KeyProj key_project(const ViewDev& V, const KeyGeo& G, float m0, float m1,
                                               float m2, const KeyOpacity& op, float near_z) {
#pragma clang fp contract(off)
  KeyProj P;
  P.visible = false;
  const float* W = V.R;
  const float xh = ((W[0] * m0 + W[1] * m1) + W[2] * m2) + V.t[0];
  const float yh = ((W[3] * m0 + W[4] * m1) + W[5] * m2) + V.t[1];
  const float zh = ((W[6] * m0 + W[7] * m1) + W[8] * m2) + V.t[2];
  P.zh = zh;
  if (!(zh > near_z) || !G.ok) return P;
  const float limx = V.limx, limy = V.limy;
  float tx = __fdiv_rn(xh, zh), ty = __fdiv_rn(yh, zh);
  if (tx < -limx) tx = -limx;
  if (tx > limx) tx = limx;
  if (ty < -limy) ty = -limy;
  if (ty > limy) ty = limy;
  const float xc = tx * zh, yc = ty * zh;
  const float z2 = zh * zh;
  const float J00 = __fdiv_rn(V.fx, zh), J02 = -__fdiv_rn(V.fx * xc, z2);
  const float J11 = __fdiv_rn(V.fy, zh), J12 = -__fdiv_rn(V.fy * yc, z2);
  float T[6];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    T[k] = J00 * W[k] + J02 * W[6 + k];
    T[3 + k] = J11 * W[3 + k] + J12 * W[6 + k];
  }
  const float S[9] = {G.S00, G.S01, G.S02, G.S01, G.S11, G.S12, G.S02, G.S12, G.S22};
  float U[6];
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int k = 0; k < 3; ++k)
      U[3 * r + k] = (T[3 * r] * S[k] + T[3 * r + 1] * S[3 + k]) + T[3 * r + 2] * S[6 + k];
  const float a = ((U[0] * T[0] + U[1] * T[1]) + U[2] * T[2]) + 0.3f;
  const float b = (U[0] * T[3] + U[1] * T[4]) + U[2] * T[5];
  const float c = ((U[3] * T[3] + U[4] * T[4]) + U[5] * T[5]) + 0.3f;
  const float det = a * c - b * b;
  if (!(det > 0.0f)) return P;
  P.A = __fdiv_rn(c, det);
  P.B = __fdiv_rn(-b, det);
  P.C = __fdiv_rn(a, det);
  P.a = a;
  P.c = c;
  P.mx = V.fx * __fdiv_rn(xh, zh) + V.cx;
  P.my = V.fy * __fdiv_rn(yh, zh) + V.cy;
  P.o = op.o;
  if (P.o < 1.0f / 255.0f) return P;
  P.thr = op.thr;
  P.visible = true;
  return P;
}

// Candidate tile rectangle (inclusive) from the axis-aligned extent of {q <= thr}.
__device__ __forceinline__ bool key_rect(const KeyProj& P, int tiles_x, int tiles_y, int* r) {
#pragma clang fp contract(off)
  const float ex = __fsqrt_rn(P.thr * P.a), ey = __fsqrt_rn(P.thr * P.c);
  if (!isfinite(P.mx) || !isfinite(P.my) || !isfinite(ex) || !isfinite(ey)) return false;
  float fx0 = ceilf(((P.mx - ex) - 15.5f) / 16.0f);
  float fx1 = floorf(((P.mx + ex) - 0.5f) / 16.0f);
  float fy0 = ceilf(((P.my - ey) - 15.5f) / 16.0f);
  float fy1 = floorf(((P.my + ey) - 0.5f) / 16.0f);
  fx0 = (fx0 < 0.0f) ? 0.0f : fx0;
  fy0 = (fy0 < 0.0f) ? 0.0f : fy0;
  const float mxx = (float)(tiles_x - 1), mxy = (float)(tiles_y - 1);
  fx1 = (mxx < fx1) ? mxx : fx1;
  fy1 = (mxy < fy1) ? mxy : fy1;
  if (!(fx0 <= fx1) || !(fy0 <= fy1)) return false;
  r[0] = (int)fx0;
  r[1] = (int)fy0;
  r[2] = (int)fx1;
  r[3] = (int)fy1;
  return true;
}

// Tile predicate (Sec. III-D.2): min over the tile's pixel-centre rectangle of
// q = A dx^2 + 2B dx dy + C dy^2 is <= thr. The minimum is 0 with the mean inside, else it
// lies on an edge whose line separates the mean from the rectangle.
__device__ __forceinline__ bool key_tile_hit(float mx, float my, float A, float B, float C,
                                             float thr, int tx, int ty) {
#pragma clang fp contract(off)
  const float x0 = (float)(16 * tx) + 0.5f, x1 = (float)(16 * tx) + 15.5f;
  const float y0 = (float)(16 * ty) + 0.5f, y1 = (float)(16 * ty) + 15.5f;
  if (mx >= x0 && mx <= x1 && my >= y0 && my <= y1) return true;
  const float B2 = B + B;
  float qmin = __builtin_huge_valf();
  if (mx < x0 || mx > x1) {
    const float dx = ((mx < x0) ? x0 : x1) - mx;
    float dy = __fdiv_rn(-(B * dx), C);
    const float lo = y0 - my, hi = y1 - my;
    dy = (dy < lo) ? lo : dy;
    dy = (hi < dy) ? hi : dy;
    const float q = ((A * (dx * dx)) + (B2 * (dx * dy))) + (C * (dy * dy));
    qmin = (q < qmin) ? q : qmin;
  }
  if (my < y0 || my > y1) {
    const float dy = ((my < y0) ? y0 : y1) - my;
    float dx = __fdiv_rn(-(B * dy), A);
    const float lo = x0 - mx, hi = x1 - mx;
    dx = (dx < lo) ? lo : dx;
    dx = (hi < dx) ? hi : dx;
    const float q = ((A * (dx * dx)) + (B2 * (dx * dy))) + (C * (dy * dy));
    qmin = (q < qmin) ? q : qmin;
  }
  return qmin <= thr;
}

// ---------------------------------------------------------------------------------
// Blend arithmetic shared by the forward and the backward passes. Every blend kernel must
// take the same skip decisions, so the exponent is formed in one fixed sequence of
// explicitly rounded operations from the conic as the kernels stage it in LDS: with the
// exponent's -1/2 and the change to base 2 folded in, e^power = 2^(A2 dx^2 + B2 dx dy +
// C2 dy^2) for A2 = -A log2(e) / 2, B2 = -B log2(e), C2 = -C log2(e) / 2 (Eq. 4's Gaussian
// with the 2D covariance's inverse (A, B; B, C)).
// ---------------------------------------------------------------------------------
constexpr float kLog2e = 1.4426950408889634f;

// (mx, my, A, B) of a projection record -> (mx, my, A2, B2)
__device__ __forceinline__ float4 blend_stage_a(float4 r0) {
  return make_float4(r0.x, r0.y, __fmul_rn(-0.5f * kLog2e, r0.z), __fmul_rn(-kLog2e, r0.w));
}

// C -> C2
__device__ __forceinline__ float blend_stage_c(float C) { return __fmul_rn(-0.5f * kLog2e, C); }

// power in base 2 at pixel centre (px, py); dx, dy = pixel centre - 2D mean
__device__ __forceinline__ float blend_power2(float mx, float my, float A2, float B2, float C2, float px, float py,
                                              float& dx, float& dy) {
  dx = __fsub_rn(px, mx);
  dy = __fsub_rn(py, my);
  const float u = __fmaf_rn(B2, dy, __fmul_rn(A2, dx));  // A2 dx + B2 dy
  return __fmaf_rn(u, dx, __fmul_rn(__fmul_rn(C2, dy), dy));
}

// 2^x (the hardware's base-2 exponential)
__device__ __forceinline__ float blend_exp2(float x) { return __builtin_amdgcn_exp2f(x); }

constexpr float kAlphaMin = 1.0f / 255.0f;
constexpr float kAlphaMax = 0.99f;
constexpr float kTMin = 1e-4f;

// ---------------------------------------------------------------------------------
// Real spherical harmonics to degree 3 (Condon-Shortley phase, m = -l..l per band),
// written as polynomials in the unit direction (x, y, z). Constants:
//   c1 = sqrt(3/(4 pi)); band 2: sqrt(15/pi)/2, sqrt(5/pi)/4, sqrt(15/pi)/4;
//   band 3: sqrt(35/(2 pi))/4, sqrt(105/pi)/2, sqrt(21/(2 pi))/4, sqrt(7/pi)/4,
//           sqrt(105/pi)/4.
// ---------------------------------------------------------------------------------
constexpr float kSH0 = 0.28209479177387814f;   // 1/(2 sqrt(pi))
constexpr float kSH1 = 0.48860251190291992f;
constexpr float kSH2a = 1.0925484305920792f;
constexpr float kSH2b = 0.31539156525252005f;
constexpr float kSH2c = 0.54627421529603959f;
constexpr float kSH3a = 0.59004358992664352f;
constexpr float kSH3b = 2.8906114426405538f;
constexpr float kSH3c = 0.45704579946446572f;
constexpr float kSH3d = 0.37317633259011540f;
constexpr float kSH3e = 1.4453057213202769f;

template <int DEG>
__device__ __forceinline__ void sh_basis(float x, float y, float z, float* Y) {
  Y[0] = kSH0;
  if (DEG >= 1) {
    Y[1] = -kSH1 * y;
    Y[2] = kSH1 * z;
    Y[3] = -kSH1 * x;
  }
  if (DEG >= 2) {
    const float xx = x * x, yy = y * y, zz = z * z;
    Y[4] = kSH2a * x * y;
    Y[5] = -kSH2a * y * z;
    Y[6] = kSH2b * (2.0f * zz - xx - yy);
    Y[7] = -kSH2a * x * z;
    Y[8] = kSH2c * (xx - yy);
    if (DEG >= 3) {
      Y[9] = -kSH3a * y * (3.0f * xx - yy);
      Y[10] = kSH3b * x * y * z;
      Y[11] = -kSH3c * y * (4.0f * zz - xx - yy);
      Y[12] = kSH3d * z * (2.0f * zz - 3.0f * xx - 3.0f * yy);
      Y[13] = -kSH3c * x * (4.0f * zz - xx - yy);
      Y[14] = kSH3e * z * (xx - yy);
      Y[15] = -kSH3a * x * (xx - 3.0f * yy);
    }
  }
}

// Gradient of sum_k w[k] Y_k with respect to (x, y, z) of the polynomial forms above.
template <int DEG>
__device__ __forceinline__ void sh_basis_grad(float x, float y, float z, const float* w, float& gx,
                                              float& gy, float& gz) {
  gx = gy = gz = 0.0f;
  if (DEG >= 1) {
    gy += -kSH1 * w[1];
    gz += kSH1 * w[2];
    gx += -kSH1 * w[3];
  }
  if (DEG >= 2) {
    gx += kSH2a * y * w[4];
    gy += kSH2a * x * w[4];
    gy += -kSH2a * z * w[5];
    gz += -kSH2a * y * w[5];
    gx += -2.0f * kSH2b * x * w[6];
    gy += -2.0f * kSH2b * y * w[6];
    gz += 4.0f * kSH2b * z * w[6];
    gx += -kSH2a * z * w[7];
    gz += -kSH2a * x * w[7];
    gx += 2.0f * kSH2c * x * w[8];
    gy += -2.0f * kSH2c * y * w[8];
    if (DEG >= 3) {
      const float xx = x * x, yy = y * y, zz = z * z;
      gx += -kSH3a * 6.0f * x * y * w[9];
      gy += -kSH3a * 3.0f * (xx - yy) * w[9];
      gx += kSH3b * y * z * w[10];
      gy += kSH3b * x * z * w[10];
      gz += kSH3b * x * y * w[10];
      gx += -kSH3c * (-2.0f * x * y) * w[11];
      gy += -kSH3c * (4.0f * zz - xx - 3.0f * yy) * w[11];
      gz += -kSH3c * 8.0f * y * z * w[11];
      gx += kSH3d * (-6.0f * x * z) * w[12];
      gy += kSH3d * (-6.0f * y * z) * w[12];
      gz += kSH3d * (6.0f * zz - 3.0f * xx - 3.0f * yy) * w[12];
      gx += -kSH3c * (4.0f * zz - 3.0f * xx - yy) * w[13];
      gy += -kSH3c * (-2.0f * x * y) * w[13];
      gz += -kSH3c * 8.0f * x * z * w[13];
      gx += kSH3e * 2.0f * x * z * w[14];
      gy += kSH3e * (-2.0f * y * z) * w[14];
      gz += kSH3e * (xx - yy) * w[14];
      gx += -kSH3a * 3.0f * (xx - yy) * w[15];
      gy += -kSH3a * (-6.0f * x * y) * w[15];
    }
  }
}

// One Adam update of a parameter (Sec. III-D.2 sparse Adam, Sec. IV-A.1 rates). Shared by
// the Adam kernels; every operation is an explicitly rounded one (no contraction, IEEE
// division and square root), so that every path and kernel takes the same rounding steps.
__device__ __forceinline__ void adam_update(float& p, float& m, float& v, float g, float lr, float beta1,
                                            float beta2, float eps, float bc1, float bc2) {
  const float mm = __fadd_rn(__fmul_rn(beta1, m), __fmul_rn(__fsub_rn(1.0f, beta1), g));
  const float vv = __fadd_rn(__fmul_rn(beta2, v), __fmul_rn(__fsub_rn(1.0f, beta2), __fmul_rn(g, g)));
  m = mm;
  v = vv;
  const float den = __fadd_rn(__fsqrt_rn(__fdiv_rn(vv, bc2)), eps);
  p = __fsub_rn(p, __fdiv_rn(__fmul_rn(lr, __fdiv_rn(mm, bc1)), den));
}

__device__ __forceinline__ float wave_sum(float x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}

}  // namespace gs
