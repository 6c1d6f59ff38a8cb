// Plain CPU oracle for one optimisation step of a 3D Gaussian map.
//
// TEST INFRASTRUCTURE ONLY. The test suite, the smoke check and the CPU-baseline leg of
// the benchmark are the only callers. It shares no code, header, constant or helper with
// the HIP library, and the HIP library never loads it.
//
// What it follows (Gaussian-LIC, arXiv 2404.06926):
//   * Sec. III-A, Eq. 1      covariance from rotation and scale
//   * Sec. III-A, Eq. 2-3    camera transform, pinhole projection, EWA 2D covariance
//   * Sec. III-A, Eq. 4      Gaussian weight at a pixel
//   * Sec. III-A, Eq. 5, 7   depth-ordered front-to-back blending, opacity map
//   * Sec. III-C.3, Eq. 9    L1 + D-SSIM loss and the 3x4 exposure affine on the colour
//   * Sec. III-D.2           cull tiles a slim footprint barely touches; sparse Adam
//   * Sec. IV-A.1            lambda = 0.2, Adam learning rates of vanilla 3DGS
// The 3DGS conventions the paper inherits without stating them (opacity cut-off 1/255,
// transmittance stop 1e-4, alpha cap 0.99, 0.3 px^2 low-pass, near plane 0.2, off-screen
// clamp 1.3 tan(fov/2), log-scale / logit / unit-quaternion parameters) are written out
// here as plain math.
//
// Precision. Values are FP64. The "key path" (projection, culls, tile predicate and the
// depth key) is templated on the scalar: with float it runs a fixed FP32 operation order
// (this file is built with -ffp-contract=off) so that tile keys and sort order can be
// compared bit for bit; the three transcendentals on it (exp of a log-scale, sigmoid,
// ln(255 o)) are evaluated in FP64 and rounded. With a dual number it yields the exact
// Jacobian of the projection, which is how the adjoint reaches the parameters.
//
// Parameter row layout (double, F = 11 + 3K floats, K = (deg+1)^2):
//   [0:3] mean, [3:6] log-scale, [6:10] quaternion (w,x,y,z), [10] opacity logit,
//   [11 + 3k + c] SH coefficient k of colour channel c.
// Camera (double[16]): R_cw row-major (9), t_cw (3), fx, fy, cx, cy.
// Exposure (double[12]): 3x4 row-major [A | b]; out = A * colour + b.

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <limits>
#include <numeric>
#include <vector>

#include <omp.h>

namespace {

constexpr double kPi = 3.14159265358979323846;

// ---------------------------------------------------------------- dual numbers
// Forward-mode derivative with respect to ND inputs.
template <int ND>
struct Dual {
  double v;
  double d[ND];
  Dual() : v(0) { for (int i = 0; i < ND; ++i) d[i] = 0; }
  Dual(double x) : v(x) { for (int i = 0; i < ND; ++i) d[i] = 0; }  // NOLINT
};
template <int ND> Dual<ND> operator+(Dual<ND> a, Dual<ND> b) {
  Dual<ND> r(a.v + b.v); for (int i = 0; i < ND; ++i) r.d[i] = a.d[i] + b.d[i]; return r; }
template <int ND> Dual<ND> operator-(Dual<ND> a, Dual<ND> b) {
  Dual<ND> r(a.v - b.v); for (int i = 0; i < ND; ++i) r.d[i] = a.d[i] - b.d[i]; return r; }
template <int ND> Dual<ND> operator-(Dual<ND> a) {
  Dual<ND> r(-a.v); for (int i = 0; i < ND; ++i) r.d[i] = -a.d[i]; return r; }
template <int ND> Dual<ND> operator*(Dual<ND> a, Dual<ND> b) {
  Dual<ND> r(a.v * b.v); for (int i = 0; i < ND; ++i) r.d[i] = a.d[i] * b.v + a.v * b.d[i]; return r; }
template <int ND> Dual<ND> operator/(Dual<ND> a, Dual<ND> b) {
  Dual<ND> r(a.v / b.v);
  for (int i = 0; i < ND; ++i) r.d[i] = (a.d[i] * b.v - a.v * b.d[i]) / (b.v * b.v);
  return r; }
template <int ND> bool operator<(Dual<ND> a, Dual<ND> b) { return a.v < b.v; }
template <int ND> bool operator>(Dual<ND> a, Dual<ND> b) { return a.v > b.v; }
template <int ND> bool operator<=(Dual<ND> a, Dual<ND> b) { return a.v <= b.v; }

constexpr int kGeo = 11;  // mean 3, log-scale 3, quaternion 4, logit 1
using D11 = Dual<kGeo>;

inline double val(double x) { return x; }
inline double val(float x) { return x; }
template <int ND> double val(const Dual<ND>& x) { return x.v; }

// Transcendentals of the parameter transforms. For float they are taken in FP64 and
// rounded once (key-path rule); for double and duals they are exact FP64.
inline float t_exp(float x) { return (float)std::exp((double)x); }
inline double t_exp(double x) { return std::exp(x); }
template <int ND> Dual<ND> t_exp(Dual<ND> a) {
  Dual<ND> r(std::exp(a.v)); for (int i = 0; i < ND; ++i) r.d[i] = a.d[i] * r.v; return r; }
inline float t_sigmoid(float x) { return (float)(1.0 / (1.0 + std::exp(-(double)x))); }
inline double t_sigmoid(double x) { return 1.0 / (1.0 + std::exp(-x)); }
template <int ND> Dual<ND> t_sigmoid(Dual<ND> a) {
  double s = 1.0 / (1.0 + std::exp(-a.v));
  Dual<ND> r(s); for (int i = 0; i < ND; ++i) r.d[i] = a.d[i] * s * (1.0 - s); return r; }
inline float t_sqrt(float x) { return std::sqrt(x); }    // correctly rounded (IEEE)
inline double t_sqrt(double x) { return std::sqrt(x); }
template <int ND> Dual<ND> t_sqrt(Dual<ND> a) {
  double s = std::sqrt(a.v);
  Dual<ND> r(s); for (int i = 0; i < ND; ++i) r.d[i] = a.d[i] / (2.0 * s); return r; }

// ------------------------------------------------------- real spherical harmonics
// Orthonormal real SH with the Condon-Shortley phase, index k = l^2 + l + m, m = -l..l:
//   Y_l0   = N_l^0 P_l(z)
//   Y_lm   = sqrt2 N_l^m (-1)^m P_l^(m)(z) Re((x+iy)^m)        m > 0
//   Y_l,-m = sqrt2 N_l^m (-1)^m P_l^(m)(z) Im((x+iy)^m)        m > 0
// with N_l^m = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!) and P_l^(m) the m-th derivative of the
// Legendre polynomial P_l (the (1-z^2)^(m/2) factor of the associated function is the
// modulus of (x+iy)^m on the unit sphere). Coefficients come from Bonnet's recursion.
struct ShTables {
  double leg[4][4];      // leg[l][j]: coefficient of z^j in P_l
  double dleg[4][4][4];  // dleg[l][m][j]: coefficient of z^j in d^m/dz^m P_l
  double norm[4][4];     // N_l^m
  ShTables() {
    std::memset(leg, 0, sizeof(leg));
    leg[0][0] = 1.0;
    leg[1][1] = 1.0;
    for (int l = 1; l < 3; ++l)  // (l+1) P_{l+1} = (2l+1) z P_l - l P_{l-1}
      for (int j = 0; j < 4; ++j) {
        double a = (j > 0 ? leg[l][j - 1] : 0.0) * (2 * l + 1) - leg[l - 1][j] * l;
        leg[l + 1][j] = a / (l + 1);
      }
    std::memset(dleg, 0, sizeof(dleg));
    for (int l = 0; l < 4; ++l) {
      for (int j = 0; j < 4; ++j) dleg[l][0][j] = leg[l][j];
      for (int m = 1; m <= l; ++m)
        for (int j = 0; j + 1 < 4; ++j) dleg[l][m][j] = dleg[l][m - 1][j + 1] * (j + 1);
    }
    auto fact = [](int n) { double f = 1; for (int i = 2; i <= n; ++i) f *= i; return f; };
    for (int l = 0; l < 4; ++l)
      for (int m = 0; m <= l; ++m)
        norm[l][m] = std::sqrt((2 * l + 1) / (4 * kPi) * fact(l - m) / fact(l + m));
  }
};
const ShTables& sh_tables() { static ShTables t; return t; }

// Y[k] for k < (deg+1)^2 at the unit vector (x, y, z).
template <typename S>
void real_sh(int deg, S x, S y, S z, S* Y) {
  const ShTables& T = sh_tables();
  for (int l = 0; l <= deg; ++l) {
    S re = S(1.0), im = S(0.0);  // (x + i y)^m, starting at m = 0
    for (int m = 0; m <= l; ++m) {
      if (m > 0) { S nre = re * x - im * y; S nim = re * y + im * x; re = nre; im = nim; }
      S p = S(0.0), zp = S(1.0);
      for (int j = 0; j + m <= l; ++j) { p = p + S(T.dleg[l][m][j]) * zp; zp = zp * z; }
      if (m == 0) {
        Y[l * l + l] = S(T.norm[l][0]) * p;
      } else {
        double c = std::sqrt(2.0) * T.norm[l][m] * ((m & 1) ? -1.0 : 1.0);
        Y[l * l + l + m] = S(c) * p * re;
        Y[l * l + l - m] = S(c) * p * im;
      }
    }
  }
}

// ------------------------------------------------------------- projection
struct Cam {
  double R[9], t[3], fx, fy, cx, cy;
  int W, H;
};

template <typename S>
struct Proj {
  bool visible = false;
  S xh, yh, zh;          // camera-frame mean (Eq. 2)
  S mx, my;              // 2D mean in pixels
  S a, b, c;             // 2D covariance Sigma' = [[a, b], [b, c]] incl. low-pass (Eq. 3)
  S ca, cb, cc;          // conic = inverse of Sigma'
  S op;                  // opacity
};

// Eq. 1-3 for one Gaussian under one camera, in the scalar S. The operation order is
// fixed (each sum is left to right as parenthesised); with S = float this is the FP32
// key-path order. Culls: depth <= near, non-positive determinant, opacity < 1/255.
template <typename S>
Proj<S> project(const double* prm, const Cam& cam, double near_z, const S* geo_override) {
  Proj<S> P;
  S g[kGeo];
  for (int i = 0; i < kGeo; ++i) g[i] = geo_override ? geo_override[i] : S(prm[i]);
  S W[9];
  for (int i = 0; i < 9; ++i) W[i] = S(cam.R[i]);
  const S t0 = S(cam.t[0]), t1 = S(cam.t[1]), t2 = S(cam.t[2]);
  const S fx = S(cam.fx), fy = S(cam.fy), cx = S(cam.cx), cy = S(cam.cy);

  // camera-frame mean
  P.xh = ((W[0] * g[0] + W[1] * g[1]) + W[2] * g[2]) + t0;
  P.yh = ((W[3] * g[0] + W[4] * g[1]) + W[5] * g[2]) + t1;
  P.zh = ((W[6] * g[0] + W[7] * g[1]) + W[8] * g[2]) + t2;
  if (!(val(P.zh) > val(S(near_z)))) return P;

  // rotation from the normalised quaternion
  const S qn = t_sqrt(((g[6] * g[6] + g[7] * g[7]) + g[8] * g[8]) + g[9] * g[9]);
  if (!(val(qn) > 0.0)) return P;
  const S w = g[6] / qn, x = g[7] / qn, y = g[8] / qn, z = g[9] / qn;
  const S one = S(1.0), two = S(2.0);
  S Rq[9];
  Rq[0] = one - two * (y * y + z * z);
  Rq[1] = two * (x * y - w * z);
  Rq[2] = two * (x * z + w * y);
  Rq[3] = two * (x * y + w * z);
  Rq[4] = one - two * (x * x + z * z);
  Rq[5] = two * (y * z - w * x);
  Rq[6] = two * (x * z - w * y);
  Rq[7] = two * (y * z + w * x);
  Rq[8] = one - two * (x * x + y * y);

  // Sigma = (R S)(R S)^T  (Eq. 1)
  const S s0 = t_exp(g[3]), s1 = t_exp(g[4]), s2 = t_exp(g[5]);
  S M[9];
  for (int r = 0; r < 3; ++r) {
    M[3 * r + 0] = Rq[3 * r + 0] * s0;
    M[3 * r + 1] = Rq[3 * r + 1] * s1;
    M[3 * r + 2] = Rq[3 * r + 2] * s2;
  }
  S Sg[9];
  for (int r = 0; r < 3; ++r)
    for (int q = r; q < 3; ++q) {
      S v = (M[3 * r] * M[3 * q] + M[3 * r + 1] * M[3 * q + 1]) + M[3 * r + 2] * M[3 * q + 2];
      Sg[3 * r + q] = v;
      Sg[3 * q + r] = v;
    }

  // Jacobian of the pinhole projection at the (off-screen clamped) mean
  const S limx = S(1.3) * ((S(0.5) * S((double)cam.W)) / fx);
  const S limy = S(1.3) * ((S(0.5) * S((double)cam.H)) / fy);
  S tx = P.xh / P.zh, ty = P.yh / P.zh;
  if (tx < -limx) tx = -limx;
  if (tx > limx) tx = limx;
  if (ty < -limy) ty = -limy;
  if (ty > limy) ty = limy;
  const S xc = tx * P.zh, yc = ty * P.zh;
  const S z2 = P.zh * P.zh;
  const S J00 = fx / P.zh, J02 = -((fx * xc) / z2);
  const S J11 = fy / P.zh, J12 = -((fy * yc) / z2);

  // T = J R_cw (2x3), U = T Sigma, Sigma' = U T^T + 0.3 I  (Eq. 3)
  S T[6];
  for (int k = 0; k < 3; ++k) {
    T[k] = J00 * W[k] + J02 * W[6 + k];
    T[3 + k] = J11 * W[3 + k] + J12 * W[6 + k];
  }
  S U[6];
  for (int r = 0; r < 2; ++r)
    for (int k = 0; k < 3; ++k)
      U[3 * r + k] = (T[3 * r] * Sg[k] + T[3 * r + 1] * Sg[3 + k]) + T[3 * r + 2] * Sg[6 + k];
  P.a = ((U[0] * T[0] + U[1] * T[1]) + U[2] * T[2]) + S(0.3);
  P.b = (U[0] * T[3] + U[1] * T[4]) + U[2] * T[5];
  P.c = ((U[3] * T[3] + U[4] * T[4]) + U[5] * T[5]) + S(0.3);
  const S det = P.a * P.c - P.b * P.b;
  if (!(val(det) > 0.0)) return P;
  P.ca = P.c / det;
  P.cb = -P.b / det;
  P.cc = P.a / det;

  P.mx = fx * (P.xh / P.zh) + cx;
  P.my = fy * (P.yh / P.zh) + cy;

  P.op = t_sigmoid(g[10]);
  if (val(P.op) < val(S(1.0) / S(255.0))) return P;
  P.visible = true;
  return P;
}

// View-dependent colour from SH (value path, FP64 or duals over the mean):
// colour_c = max(0, sum_k sh[k][c] Y_k(dir) + 0.5), dir = (mean - camera centre) normalised.
template <typename S>
void sh_colour(int deg, const double* prm, const S* mean, const Cam& cam, S* col, bool* clamped,
               double* Yout) {
  const double cwx = -(cam.R[0] * cam.t[0] + cam.R[3] * cam.t[1] + cam.R[6] * cam.t[2]);
  const double cwy = -(cam.R[1] * cam.t[0] + cam.R[4] * cam.t[1] + cam.R[7] * cam.t[2]);
  const double cwz = -(cam.R[2] * cam.t[0] + cam.R[5] * cam.t[1] + cam.R[8] * cam.t[2]);
  S dx = mean[0] - S(cwx), dy = mean[1] - S(cwy), dz = mean[2] - S(cwz);
  S n = t_sqrt(dx * dx + dy * dy + dz * dz);
  dx = dx / n; dy = dy / n; dz = dz / n;
  const int K = (deg + 1) * (deg + 1);
  S Y[16];
  real_sh(deg, dx, dy, dz, Y);
  for (int ch = 0; ch < 3; ++ch) {
    S acc = S(0.5);
    for (int k = 0; k < K; ++k) acc = acc + S(prm[11 + 3 * k + ch]) * Y[k];
    clamped[ch] = val(acc) < 0.0;
    col[ch] = clamped[ch] ? S(0.0) : acc;
  }
  if (Yout)
    for (int k = 0; k < K; ++k) Yout[k] = val(Y[k]);
}

// Tile predicate (Sec. III-D.2): keep tile (tx, ty) iff the smallest value of the conic
// quadratic over the rectangle of its pixel centres is <= thr = 2 ln(255 o), i.e. some
// point of the tile can reach alpha >= 1/255. The minimum is 0 when the mean is inside;
// otherwise it lies on an edge whose supporting line separates the mean from the tile,
// and on each such edge it is a clamped 1-D quadratic minimum.
template <typename S>
bool tile_hit(S mx, S my, S A, S B, S C, S thr, int tx, int ty) {
  const S x0 = S((double)(16 * tx)) + S(0.5), x1 = S((double)(16 * tx)) + S(15.5);
  const S y0 = S((double)(16 * ty)) + S(0.5), y1 = S((double)(16 * ty)) + S(15.5);
  if (mx >= x0 && mx <= x1 && my >= y0 && my <= y1) return true;
  auto quad = [&](S dx, S dy) { return ((A * (dx * dx)) + ((B + B) * (dx * dy))) + (C * (dy * dy)); };
  S qmin = std::numeric_limits<S>::infinity();
  auto vert = [&](S X) {
    const S dx = X - mx;
    S dy = (-(B * dx)) / C;
    dy = std::min(std::max(dy, y0 - my), y1 - my);
    qmin = std::min(qmin, quad(dx, dy));
  };
  auto horz = [&](S Y) {
    const S dy = Y - my;
    S dx = (-(B * dy)) / A;
    dx = std::min(std::max(dx, x0 - mx), x1 - mx);
    qmin = std::min(qmin, quad(dx, dy));
  };
  if (mx < x0) vert(x0);
  if (mx > x1) vert(x1);
  if (my < y0) horz(y0);
  if (my > y1) horz(y1);
  return qmin <= thr;
}

// Candidate tile rectangle from the axis-aligned extent of {q <= thr}; returns false when
// it is empty.
template <typename S>
bool tile_rect(const Proj<S>& P, S thr, int tiles_x, int tiles_y, int* r) {
  const S ex = t_sqrt(thr * P.a), ey = t_sqrt(thr * P.c);
  if (!std::isfinite(val(P.mx)) || !std::isfinite(val(P.my)) || !std::isfinite(val(ex)) ||
      !std::isfinite(val(ey)))
    return false;
  S fx0 = std::ceil(((P.mx - ex) - S(15.5)) / S(16.0));
  S fx1 = std::floor(((P.mx + ex) - S(0.5)) / S(16.0));
  S fy0 = std::ceil(((P.my - ey) - S(15.5)) / S(16.0));
  S fy1 = std::floor(((P.my + ey) - S(0.5)) / S(16.0));
  fx0 = std::max(fx0, S(0.0));
  fy0 = std::max(fy0, S(0.0));
  fx1 = std::min(fx1, S((double)(tiles_x - 1)));
  fy1 = std::min(fy1, S((double)(tiles_y - 1)));
  if (!(fx0 <= fx1) || !(fy0 <= fy1)) return false;
  r[0] = (int)fx0; r[1] = (int)fy0; r[2] = (int)fx1; r[3] = (int)fy1;
  return true;
}

inline double ln255o_thr(float o) { return (double)(float)(2.0 * std::log(255.0 * (double)o)); }
inline double ln255o_thr(double o) { return 2.0 * std::log(255.0 * o); }

Cam make_cam(const double* c, int W, int H) {
  Cam cam;
  for (int i = 0; i < 9; ++i) cam.R[i] = c[i];
  for (int i = 0; i < 3; ++i) cam.t[i] = c[9 + i];
  cam.fx = c[12]; cam.fy = c[13]; cam.cx = c[14]; cam.cy = c[15];
  cam.W = W; cam.H = H;
  return cam;
}

template <typename S>
void project_all(int N, int deg, const double* params, const double* camv, int W, int H,
                 double near_z, uint8_t* visible, uint32_t* depth_bits, double* depth,
                 double* mean2d, double* conic, double* opac, double* thr, double* cov2d,
                 double* colour, int32_t* rect, int32_t* count) {
  const int F = 11 + 3 * (deg + 1) * (deg + 1);
  const Cam cam = make_cam(camv, W, H);
  const int tiles_x = (W + 15) / 16, tiles_y = (H + 15) / 16;
#pragma omp parallel for schedule(static)
  for (int i = 0; i < N; ++i) {
    const double* prm = params + (size_t)i * F;
    Proj<S> P = project<S>(prm, cam, near_z, nullptr);
    visible[i] = 0;
    count[i] = 0;
    depth[i] = val(P.zh);
    depth_bits[i] = 0;
    if (std::is_same<S, float>::value) {
      float zf = (float)val(P.zh);
      std::memcpy(&depth_bits[i], &zf, 4);
    }
    for (int k = 0; k < 4; ++k) rect[4 * i + k] = -1;
    if (!P.visible) continue;
    const S th = S(ln255o_thr(P.op));
    mean2d[2 * i] = val(P.mx); mean2d[2 * i + 1] = val(P.my);
    conic[3 * i] = val(P.ca); conic[3 * i + 1] = val(P.cb); conic[3 * i + 2] = val(P.cc);
    cov2d[3 * i] = val(P.a); cov2d[3 * i + 1] = val(P.b); cov2d[3 * i + 2] = val(P.c);
    opac[i] = val(P.op);
    thr[i] = val(th);
    double mean[3] = {prm[0], prm[1], prm[2]};
    bool cl[3];
    sh_colour<double>(deg, prm, mean, cam, colour + 3 * i, cl, nullptr);
    int r[4];
    if (!tile_rect(P, th, tiles_x, tiles_y, r)) continue;
    int n = 0;
    for (int ty = r[1]; ty <= r[3]; ++ty)
      for (int tx = r[0]; tx <= r[2]; ++tx)
        if (tile_hit<S>(P.mx, P.my, P.ca, P.cb, P.cc, th, tx, ty)) ++n;
    for (int k = 0; k < 4; ++k) rect[4 * i + k] = r[k];
    count[i] = n;
    visible[i] = n > 0 ? 1 : 0;
  }
}

// Emission order: Gaussian index ascending, then tiles row-major inside its rectangle.
template <typename S>
void emit_all(int N, int W, int H, int64_t tile_base, const int32_t* rect, const int32_t* count,
              const double* mean2d, const double* conic, const double* thr, const int64_t* offset,
              int64_t* tile_out, uint32_t* val_out) {
  const int tiles_x = (W + 15) / 16;
  (void)H;
#pragma omp parallel for schedule(dynamic, 256)
  for (int i = 0; i < N; ++i) {
    if (count[i] == 0) continue;
    int64_t o = offset[i];
    const S mx = S(mean2d[2 * i]), my = S(mean2d[2 * i + 1]);
    const S A = S(conic[3 * i]), B = S(conic[3 * i + 1]), C = S(conic[3 * i + 2]);
    const S th = S(thr[i]);
    for (int ty = rect[4 * i + 1]; ty <= rect[4 * i + 3]; ++ty)
      for (int tx = rect[4 * i]; tx <= rect[4 * i + 2]; ++tx)
        if (tile_hit<S>(mx, my, A, B, C, th, tx, ty)) {
          tile_out[o] = tile_base + (int64_t)ty * tiles_x + tx;
          val_out[o] = (uint32_t)i;
          ++o;
        }
  }
}

// ---------------------------------------------------------------- blending
constexpr double kAlphaMin = 1.0 / 255.0;
constexpr double kAlphaMax = 0.99;
constexpr double kTMin = 1e-4;

struct BlendIn {
  const double *mean2d, *conic, *opac, *colour, *depth;
  const double *E, *bg;
  double tie_alpha, tie_T;  // relative tie margins (0 disables tie marking)
};

struct PairRec {
  uint32_t g;
  int pos;
  double alpha, araw, expo, T, dx, dy;
};

// Front-to-back blend at one pixel over the ordered list ids[0..n) (Eq. 5). Returns the
// contributors in order; sets T_final, the list position after the last contributor and
// a tie flag when an alpha or transmittance decision sits within the stated margin.
int blend_pixel(const BlendIn& in, const uint32_t* ids, int n, double px, double py,
                std::vector<PairRec>* rec, double* Tfinal, int* ncontrib, int* tie) {
  double T = 1.0;
  int last = 0, ncon = 0;
  *tie = 0;
  for (int p = 0; p < n; ++p) {
    const uint32_t g = ids[p];
    const double dx = px - in.mean2d[2 * g], dy = py - in.mean2d[2 * g + 1];
    const double A = in.conic[3 * g], B = in.conic[3 * g + 1], C = in.conic[3 * g + 2];
    const double q = A * dx * dx + 2.0 * B * dx * dy + C * dy * dy;
    const double mag = A * dx * dx + 2.0 * std::fabs(B * dx * dy) + C * dy * dy;
    if (in.tie_alpha > 0 && std::fabs(q) <= 1e-6 * mag && mag > 0) *tie |= 1;
    const double power = -0.5 * q;
    if (power > 0.0) continue;
    const double expo = std::exp(power);
    const double araw = in.opac[g] * expo;
    if (in.tie_alpha > 0 && std::fabs(araw / kAlphaMin - 1.0) < in.tie_alpha) *tie |= 1;
    if (in.tie_alpha > 0 && std::fabs(araw / kAlphaMax - 1.0) < in.tie_alpha) *tie |= 2;
    const double alpha = std::min(kAlphaMax, araw);
    if (alpha < kAlphaMin) continue;
    const double Tn = T * (1.0 - alpha);
    if (in.tie_T > 0 && std::fabs(Tn / kTMin - 1.0) < in.tie_T * (1.0 + 0.2 * ncon)) *tie |= 1;
    if (Tn < kTMin) break;
    if (rec) rec->push_back(PairRec{g, p, alpha, araw, expo, T, dx, dy});
    T = Tn;
    last = p + 1;
    ++ncon;
  }
  *Tfinal = T;
  *ncontrib = last;
  return ncon;
}

// Colour (Eq. 5, background behind the last contributor, then the exposure affine), and
// optionally the depth map D = sum_i d_i a_i T_i (Eq. 6) and the opacity map
// O = sum_i a_i T_i (Eq. 7) as the plain sums over the contributors.
void finish_pixel(const BlendIn& in, const std::vector<PairRec>& rec, double Tf, double* pre,
                  double* out, double* D = nullptr, double* O = nullptr) {
  double Cc[3] = {0, 0, 0};
  for (const PairRec& r : rec)
    for (int ch = 0; ch < 3; ++ch) Cc[ch] += in.colour[3 * r.g + ch] * r.alpha * r.T;
  for (int ch = 0; ch < 3; ++ch) pre[ch] = Cc[ch] + Tf * in.bg[ch];
  for (int r = 0; r < 3; ++r)
    out[r] = in.E[4 * r] * pre[0] + in.E[4 * r + 1] * pre[1] + in.E[4 * r + 2] * pre[2] + in.E[4 * r + 3];
  if (D) {
    double s = 0.0;
    for (const PairRec& r : rec) s += in.depth[r.g] * r.alpha * r.T;
    *D = s;
  }
  if (O) {
    double s = 0.0;
    for (const PairRec& r : rec) s += r.alpha * r.T;
    *O = s;
  }
}

// Adjoint of Eq. 5 + exposure at one pixel, written with suffix sums:
//   pre = sum_i c_i a_i T_i + T_N bg,   T_i = prod_{j<i} (1 - a_j)
//   d pre / d c_i = a_i T_i,   d pre / d a_i = T_i c_i - S_i / (1 - a_i),
//   S_i = sum_{k>i} c_k a_k T_k + T_N bg.
// D (Eq. 6) and O (Eq. 7) are the same sums with c_i replaced by d_i and by 1 and no
// background term; gD and gO are dL/dD and dL/dO at this pixel (0 when not used).
// Per-Gaussian gradient rows (N x 10): mean2d x, y, conic A, B, C, opacity, colour r, g, b,
// camera-frame depth d.
void pixel_adjoint(const BlendIn& in, const std::vector<PairRec>& rec, double Tf, const double* pre,
                   const double* gout, double gD, double gO, double* g2d /*N x 10*/, double* gE) {
  double G[3];
  for (int c = 0; c < 3; ++c) G[c] = in.E[c] * gout[0] + in.E[4 + c] * gout[1] + in.E[8 + c] * gout[2];
  for (int r = 0; r < 3; ++r) {
    for (int c = 0; c < 3; ++c) gE[4 * r + c] += gout[r] * pre[c];
    gE[4 * r + 3] += gout[r];
  }
  const int n = (int)rec.size();
  std::vector<double> S(3 * (n + 1));
  for (int c = 0; c < 3; ++c) S[3 * n + c] = Tf * in.bg[c];  // S_{n-1} = T_N bg
  for (int i = n - 1; i >= 0; --i)
    for (int c = 0; c < 3; ++c)
      S[3 * i + c] = S[3 * (i + 1) + c] + (i + 1 < n ? in.colour[3 * rec[i + 1].g + c] * rec[i + 1].alpha * rec[i + 1].T : 0.0);
  // S[3*i + c] now holds S_i (contributions strictly behind i, plus background)
  std::vector<double> SD(n + 1, 0.0), SO(n + 1, 0.0);  // the same suffix sums for D and O
  for (int i = n - 2; i >= 0; --i) {
    const PairRec& b = rec[i + 1];
    SD[i] = SD[i + 1] + in.depth[b.g] * b.alpha * b.T;
    SO[i] = SO[i + 1] + b.alpha * b.T;
  }
  for (int i = 0; i < n; ++i) {
    const PairRec& r = rec[i];
    double* gg = g2d + 10 * (size_t)r.g;
    double da = 0.0;
    for (int c = 0; c < 3; ++c) {
      const double dc = r.alpha * r.T * G[c];
#pragma omp atomic
      gg[6 + c] += dc;
      da += G[c] * (r.T * in.colour[3 * r.g + c] - S[3 * i + c] / (1.0 - r.alpha));
    }
    if (gD != 0.0) {
      const double dd = r.alpha * r.T * gD;
#pragma omp atomic
      gg[9] += dd;
      da += gD * (r.T * in.depth[r.g] - SD[i] / (1.0 - r.alpha));
    }
    if (gO != 0.0) da += gO * (r.T - SO[i] / (1.0 - r.alpha));
    if (r.araw > kAlphaMax) continue;  // capped alpha: no gradient through it
    const double A = in.conic[3 * r.g], B = in.conic[3 * r.g + 1], C = in.conic[3 * r.g + 2];
    const double dpow = da * r.araw;  // d alpha / d power = alpha
    const double gmx = dpow * (A * r.dx + B * r.dy);
    const double gmy = dpow * (B * r.dx + C * r.dy);
    const double gA = dpow * (-0.5 * r.dx * r.dx);
    const double gB = dpow * (-r.dx * r.dy);
    const double gC = dpow * (-0.5 * r.dy * r.dy);
    const double go = da * r.expo;
#pragma omp atomic
    gg[0] += gmx;
#pragma omp atomic
    gg[1] += gmy;
#pragma omp atomic
    gg[2] += gA;
#pragma omp atomic
    gg[3] += gB;
#pragma omp atomic
    gg[4] += gC;
#pragma omp atomic
    gg[5] += go;
  }
}

// ------------------------------------------------------------- SSIM window
void gauss_window(double* w) {
  double g[11], s = 0;
  for (int i = 0; i < 11; ++i) { g[i] = std::exp(-((i - 5) * (i - 5)) / (2.0 * 1.5 * 1.5)); s += g[i]; }
  for (int i = 0; i < 11; ++i) g[i] /= s;
  for (int i = 0; i < 11; ++i)
    for (int j = 0; j < 11; ++j) w[11 * i + j] = g[i] * g[j];
}

}  // namespace

extern "C" {

int or_version() { return 4; }

// Host threads the oracle's parallel loops use (timing runs of the CPU baseline); returns
// the previous setting.
int or_set_threads(int n) {
  const int prev = omp_get_max_threads();
  if (n > 0) omp_set_num_threads(n);
  return prev;
}

// Per-Gaussian projection for one view. fp64 != 0 runs the key path in FP64, otherwise in
// the fixed FP32 order. Outputs are per Gaussian (double arrays hold the exact values of
// the chosen precision). visible[i] = passes every cull and hits >= 1 tile.
void or_project(int N, int deg, const double* params, const double* cam, int W, int H,
                double near_z, int fp64, uint8_t* visible, uint32_t* depth_bits, double* depth,
                double* mean2d, double* conic, double* opac, double* thr, double* cov2d,
                double* colour, int32_t* rect, int32_t* count) {
  if (fp64)
    project_all<double>(N, deg, params, cam, W, H, near_z, visible, depth_bits, depth, mean2d,
                        conic, opac, thr, cov2d, colour, rect, count);
  else
    project_all<float>(N, deg, params, cam, W, H, near_z, visible, depth_bits, depth, mean2d,
                       conic, opac, thr, cov2d, colour, rect, count);
}

// Emit (tile, Gaussian) instances for one view at the given exclusive offsets.
void or_emit(int N, int W, int H, int64_t tile_base, int fp64, const int32_t* rect,
             const int32_t* count, const double* mean2d, const double* conic, const double* thr,
             const int64_t* offset, int64_t* tile_out, uint32_t* val_out) {
  if (fp64)
    emit_all<double>(N, W, H, tile_base, rect, count, mean2d, conic, thr, offset, tile_out, val_out);
  else
    emit_all<float>(N, W, H, tile_base, rect, count, mean2d, conic, thr, offset, tile_out, val_out);
}

// Stable ascending sort of instances by (tile, depth); equal keys keep emission order
// (Sec. III-A: Gaussians are blended in depth order). Writes the permuted tile ids and
// values, and the 64-bit keys tile << 32 | float bits(depth) when depth_bits != NULL.
void or_sort(int64_t n, const int64_t* tile, const uint32_t* val, const double* depth_of_gauss,
             const uint32_t* depth_bits, int64_t* tile_sorted, uint32_t* val_sorted,
             uint64_t* key_sorted) {
  std::vector<int64_t> idx(n);
  std::iota(idx.begin(), idx.end(), 0);
  std::stable_sort(idx.begin(), idx.end(), [&](int64_t a, int64_t b) {
    if (tile[a] != tile[b]) return tile[a] < tile[b];
    return depth_of_gauss[val[a]] < depth_of_gauss[val[b]];
  });
  for (int64_t k = 0; k < n; ++k) {
    tile_sorted[k] = tile[idx[k]];
    val_sorted[k] = val[idx[k]];
    if (key_sorted && depth_bits)
      key_sorted[k] = ((uint64_t)tile[idx[k]] << 32) | (uint64_t)depth_bits[val[idx[k]]];
  }
}

// [start, end) of each tile in the sorted list (empty tiles: [0, 0)).
void or_ranges(int64_t n, const int64_t* tile_sorted, int64_t n_tiles, int64_t* ranges) {
  for (int64_t t = 0; t < 2 * n_tiles; ++t) ranges[t] = 0;
  for (int64_t k = 0; k < n; ++k) {
    const int64_t t = tile_sorted[k];
    if (k == 0 || tile_sorted[k - 1] != t) ranges[2 * t] = k;
    if (k == n - 1 || tile_sorted[k + 1] != t) ranges[2 * t + 1] = k + 1;
  }
}

// Tiled blend of one view: each pixel walks its tile's sorted list. Outputs the exposed
// colour (CHW), the pre-exposure colour incl. background (CHW), T_final, the list position
// after the last contributor, and tie flags.
void or_render_tiled(int W, int H, int64_t tile_base, const int64_t* ranges /*global tiles x 2*/,
                     const uint32_t* vals, const double* mean2d, const double* conic,
                     const double* opac, const double* colour, const double* E, const double* bg,
                     double tie_alpha, double tie_T, double* out, double* pre, double* Tfinal,
                     int32_t* ncontrib, int32_t* tie, int32_t* ncon, uint64_t* sig,
                     const double* depth, double* Dout, double* Oout) {
  const int tiles_x = (W + 15) / 16;
  BlendIn in{mean2d, conic, opac, colour, depth, E, bg, tie_alpha, tie_T};
  const int64_t P = (int64_t)W * H;
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t pix = 0; pix < P; ++pix) {
    const int x = (int)(pix % W), y = (int)(pix / W);
    const int64_t t = tile_base + (int64_t)(y / 16) * tiles_x + (x / 16);
    const int64_t s = ranges[2 * t], e = ranges[2 * t + 1];
    std::vector<PairRec> rec;
    double Tf;
    int nc, tf;
    const int k = blend_pixel(in, vals + s, (int)(e - s), x + 0.5, y + 0.5, &rec, &Tf, &nc, &tf);
    double pr[3], o[3];
    finish_pixel(in, rec, Tf, pr, o, (Dout && depth) ? Dout + pix : nullptr, Oout ? Oout + pix : nullptr);
    for (int c = 0; c < 3; ++c) { out[c * P + pix] = o[c]; pre[c * P + pix] = pr[c]; }
    Tfinal[pix] = Tf;
    ncontrib[pix] = nc;
    tie[pix] = tf;
    if (ncon) ncon[pix] = k;
    if (sig) {
      // order-independent signature of the contributor set and of which contributors have
      // a capped alpha (splitmix64 of id and cap bit): a finite-difference step that
      // changes either crosses a kink of the blend
      uint64_t h = 0;
      for (const PairRec& r : rec) {
        const uint64_t capped = r.araw > kAlphaMax ? (uint64_t(1) << 40) : 0;
        uint64_t z = ((uint64_t)r.g | capped) + 0x9E3779B97F4A7C15ull;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        h += z ^ (z >> 31);
      }
      sig[pix] = h;
    }
  }
}

// The tiled blend at a list of pixels only (sampled checks of large images).
void or_render_tiled_pixels(int W, int H, int64_t tile_base, const int64_t* ranges, const uint32_t* vals,
                            const double* mean2d, const double* conic, const double* opac,
                            const double* colour, const double* E, const double* bg, double tie_alpha,
                            double tie_T, int64_t npix, const int64_t* pix, double* out /*npix x 3*/,
                            double* Tfinal, int32_t* ncontrib, int32_t* tie, const double* depth,
                            double* Dout, double* Oout) {
  const int tiles_x = (W + 15) / 16;
  (void)H;
  BlendIn in{mean2d, conic, opac, colour, depth, E, bg, tie_alpha, tie_T};
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t k = 0; k < npix; ++k) {
    const int x = (int)(pix[k] % W), y = (int)(pix[k] / W);
    const int64_t t = tile_base + (int64_t)(y / 16) * tiles_x + (x / 16);
    const int64_t s = ranges[2 * t], e = ranges[2 * t + 1];
    std::vector<PairRec> rec;
    double Tf;
    int nc, tf;
    blend_pixel(in, vals + s, (int)(e - s), x + 0.5, y + 0.5, &rec, &Tf, &nc, &tf);
    double pr[3], o[3];
    finish_pixel(in, rec, Tf, pr, o, (Dout && depth) ? Dout + k : nullptr, Oout ? Oout + k : nullptr);
    for (int c = 0; c < 3; ++c) out[3 * k + c] = o[c];
    Tfinal[k] = Tf;
    ncontrib[k] = nc;
    tie[k] = tf;
  }
}

// Brute force, the plain definition: every pixel blends every visible Gaussian in
// (depth, index) order, with no tiles. ncon = number of contributors.
void or_render_brute(int N, int W, int H, const uint8_t* visible, const double* depth,
                     const double* mean2d, const double* conic, const double* opac,
                     const double* colour, const double* E, const double* bg, double* out,
                     double* Tfinal, int32_t* ncon, double* Dout, double* Oout) {
  std::vector<uint32_t> order;
  for (int i = 0; i < N; ++i)
    if (visible[i]) order.push_back((uint32_t)i);
  std::stable_sort(order.begin(), order.end(),
                   [&](uint32_t a, uint32_t b) { return depth[a] < depth[b]; });
  BlendIn in{mean2d, conic, opac, colour, depth, E, bg, 0.0, 0.0};
  const int64_t P = (int64_t)W * H;
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t pix = 0; pix < P; ++pix) {
    const int x = (int)(pix % W), y = (int)(pix / W);
    std::vector<PairRec> rec;
    double Tf;
    int nc, tf;
    int k = blend_pixel(in, order.data(), (int)order.size(), x + 0.5, y + 0.5, &rec, &Tf, &nc, &tf);
    double pr[3], o[3];
    finish_pixel(in, rec, Tf, pr, o, Dout ? Dout + pix : nullptr, Oout ? Oout + pix : nullptr);
    for (int c = 0; c < 3; ++c) out[c * P + pix] = o[c];
    Tfinal[pix] = Tf;
    ncon[pix] = k;
  }
}

// Adjoint of the tiled blend of one view: from dL/dout (CHW) and optionally dL/dD and
// dL/dO (H x W, may be NULL) to per-Gaussian gradients of (mean2d x, y, conic A, B, C,
// opacity, colour r, g, b, depth) accumulated into g2d (N x 10), and of the exposure into
// gE (12). Gaussians evaluated at a tie pixel are flagged in gtie.
void or_blend_backward(int W, int H, int64_t tile_base, const int64_t* ranges, const uint32_t* vals,
                       const double* mean2d, const double* conic, const double* opac,
                       const double* colour, const double* E, const double* bg,
                       double tie_alpha, double tie_T, const double* gout, double* g2d,
                       double* gE, uint8_t* gtie, const double* depth, const double* gDmap,
                       const double* gOmap) {
  const int tiles_x = (W + 15) / 16;
  BlendIn in{mean2d, conic, opac, colour, depth, E, bg, tie_alpha, tie_T};
  const int64_t P = (int64_t)W * H;
  double gEacc[12] = {0};
#pragma omp parallel
  {
    double gEl[12] = {0};
#pragma omp for schedule(dynamic, 64)
    for (int64_t pix = 0; pix < P; ++pix) {
      const int x = (int)(pix % W), y = (int)(pix / W);
      const int64_t t = tile_base + (int64_t)(y / 16) * tiles_x + (x / 16);
      const int64_t s = ranges[2 * t], e = ranges[2 * t + 1];
      std::vector<PairRec> rec;
      double Tf;
      int nc, tf;
      blend_pixel(in, vals + s, (int)(e - s), x + 0.5, y + 0.5, &rec, &Tf, &nc, &tf);
      if (tf && gtie) {
        // every Gaussian whose gradient sees this pixel: its contributors, and the entries
        // up to the first one past the last contributor (where a stop decision sits)
        const int64_t upto = std::min<int64_t>(e, s + (int64_t)nc + 1);
        for (int64_t k = s; k < upto; ++k) gtie[vals[k]] = 1;
      }
      double pr[3], o[3];
      finish_pixel(in, rec, Tf, pr, o);
      double go[3] = {gout[pix], gout[P + pix], gout[2 * P + pix]};
      pixel_adjoint(in, rec, Tf, pr, go, gDmap ? gDmap[pix] : 0.0, gOmap ? gOmap[pix] : 0.0, g2d, gEl);
    }
#pragma omp critical
    for (int k = 0; k < 12; ++k) gEacc[k] += gEl[k];
  }
  for (int k = 0; k < 12; ++k) gE[k] += gEacc[k];
}

// Chain rule from the per-Gaussian 2D gradients of one view to the parameters (N x F),
// accumulated into gparams. The Jacobian of (mean2d, conic, opacity, colour, camera-frame
// depth) with respect to (mean, log-scale, quaternion, logit) is evaluated exactly with dual
// numbers through the same projection as the forward pass (FP64); SH enters the colour
// linearly. g2d rows are N x 10 as written by or_blend_backward.
void or_project_backward(int N, int deg, const double* params, const double* camv, int W, int H,
                         double near_z, const uint8_t* visible, const double* g2d, double* gparams) {
  const int K = (deg + 1) * (deg + 1), F = 11 + 3 * K;
  const Cam cam = make_cam(camv, W, H);
#pragma omp parallel for schedule(static)
  for (int i = 0; i < N; ++i) {
    if (!visible[i]) continue;
    const double* prm = params + (size_t)i * F;
    const double* g = g2d + 10 * (size_t)i;
    D11 geo[kGeo];
    for (int k = 0; k < kGeo; ++k) { geo[k] = D11(prm[k]); geo[k].d[k] = 1.0; }
    Proj<D11> P = project<D11>(prm, cam, near_z, geo);
    if (!P.visible) continue;
    D11 col[3];
    bool cl[3];
    double Y[16];
    sh_colour<D11>(deg, prm, geo, cam, col, cl, Y);
    const D11* outs[10] = {&P.mx, &P.my, &P.ca, &P.cb, &P.cc, &P.op, &col[0], &col[1], &col[2], &P.zh};
    double* gp = gparams + (size_t)i * F;
    for (int k = 0; k < kGeo; ++k) {
      double s = 0.0;
      for (int o = 0; o < 10; ++o) s += g[o] * outs[o]->d[k];
      gp[k] += s;
    }
    for (int k = 0; k < K; ++k)
      for (int c = 0; c < 3; ++c)
        if (!cl[c]) gp[11 + 3 * k + c] += g[6 + c] * Y[k];
  }
}

// Real SH basis at unit vectors (for the basis pins).
void or_sh_basis(int deg, int n, const double* dirs, double* Y) {
  const int K = (deg + 1) * (deg + 1);
  for (int i = 0; i < n; ++i) {
    double y[16];
    real_sh<double>(deg, dirs[3 * i], dirs[3 * i + 1], dirs[3 * i + 2], y);
    for (int k = 0; k < K; ++k) Y[(size_t)i * K + k] = y[k];
  }
}

// L = (1 - lambda) mean|out - gt| + lambda (1 - mean SSIM(out, gt))   (Eq. 9)
// SSIM per channel with an 11x11 Gaussian window (sigma 1.5, normalised), C1 = 0.01^2,
// C2 = 0.03^2, windows zero-padded at the border; means over 3 H W. The gradient follows
// from SSIM as a function of the five local moments mu_x, mu_y, E[xx], E[yy], E[xy].
double or_loss(int H, int W, const double* out, const double* gt, double lambda, double* gout,
               double* ssim_mean_out) {
  const int64_t P = (int64_t)H * W;
  const double n = 3.0 * (double)P;
  double w[121];
  gauss_window(w);
  double l1 = 0.0;
  for (int64_t k = 0; k < 3 * P; ++k) {
    const double d = out[k] - gt[k];
    l1 += std::fabs(d);
    if (gout) gout[k] = (1.0 - lambda) / n * (d > 0 ? 1.0 : (d < 0 ? -1.0 : 0.0));
  }
  const double C1 = 0.01 * 0.01, C2 = 0.03 * 0.03;
  double ssim_sum = 0.0;
  std::vector<double> dmu(P), dxx(P), dxy(P);
  for (int ch = 0; ch < 3; ++ch) {
    const double* x = out + ch * P;
    const double* y = gt + ch * P;
    double chs = 0.0;
#pragma omp parallel for reduction(+ : chs) schedule(static)
    for (int64_t p = 0; p < P; ++p) {
      const int py = (int)(p / W), px = (int)(p % W);
      double mx = 0, my = 0, exx = 0, eyy = 0, exy = 0;
      for (int i = 0; i < 11; ++i) {
        const int yy = py + i - 5;
        if (yy < 0 || yy >= H) continue;
        for (int j = 0; j < 11; ++j) {
          const int xx = px + j - 5;
          if (xx < 0 || xx >= W) continue;
          const double ww = w[11 * i + j];
          const double a = x[(int64_t)yy * W + xx], b = y[(int64_t)yy * W + xx];
          mx += ww * a; my += ww * b; exx += ww * a * a; eyy += ww * b * b; exy += ww * a * b;
        }
      }
      const double A1 = 2 * mx * my + C1, A2 = 2 * (exy - mx * my) + C2;
      const double B1 = mx * mx + my * my + C1, B2 = (exx - mx * mx) + (eyy - my * my) + C2;
      const double num = A1 * A2, den = B1 * B2;
      const double S = num / den;
      chs += S;
      // partials of S w.r.t. the moments, scaled by dL/dS = -lambda / n
      const double dnum_dmx = 2 * my * A2 + A1 * (-2 * my);
      const double dden_dmx = 2 * mx * B2 + B1 * (-2 * mx);
      const double s = -lambda / n;
      dmu[p] = s * (dnum_dmx * den - num * dden_dmx) / (den * den);
      dxx[p] = s * (-num * B1 / (den * den));
      dxy[p] = s * (2 * A1 / den);
    }
    ssim_sum += chs;
    if (gout) {
#pragma omp parallel for schedule(static)
      for (int64_t p = 0; p < P; ++p) {
        const int py = (int)(p / W), px = (int)(p % W);
        double acc = 0.0;
        for (int i = 0; i < 11; ++i) {
          const int yy = py - (i - 5);  // moment at q = p - offset used x(p) with weight w
          if (yy < 0 || yy >= H) continue;
          for (int j = 0; j < 11; ++j) {
            const int xx = px - (j - 5);
            if (xx < 0 || xx >= W) continue;
            const int64_t q = (int64_t)yy * W + xx;
            const double ww = w[11 * i + j];
            acc += ww * (dmu[q] + dxx[q] * 2.0 * x[p] + dxy[q] * y[p]);
          }
        }
        gout[ch * P + p] += acc;
      }
    }
  }
  const double ssim_mean = ssim_sum / n;
  if (ssim_mean_out) *ssim_mean_out = ssim_mean;
  return (1.0 - lambda) * l1 / n + lambda * (1.0 - ssim_mean);
}

// Sparse Adam (Sec. III-D.2; Adam with vanilla-3DGS rates, Sec. IV-A.1): only rows with
// vis != 0 move; t is the step count after this step. Arrays are row-major N x F.
void or_adam(int64_t N, int F, double* p, double* g, double* m, double* v, const uint8_t* vis,
             const double* lr, double beta1, double beta2, double eps, int64_t t) {
  const double bc1 = 1.0 - std::pow(beta1, (double)t);
  const double bc2 = 1.0 - std::pow(beta2, (double)t);
  for (int64_t i = 0; i < N; ++i) {
    if (!vis[i]) continue;
    for (int f = 0; f < F; ++f) {
      const int64_t k = i * F + f;
      m[k] = beta1 * m[k] + (1.0 - beta1) * g[k];
      v[k] = beta2 * v[k] + (1.0 - beta2) * g[k] * g[k];
      const double mh = m[k] / bc1, vh = v[k] / bc2;
      p[k] -= lr[f] * mh / (std::sqrt(vh) + eps);
      g[k] = 0.0;
    }
  }
}

}  // extern "C"
