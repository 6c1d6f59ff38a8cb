// Per-Gaussian projection: forward (Sec. III-A Eq. 1-3, SH colour, culls, tile count of
// the footprint predicate of Sec. III-D.2) and its adjoint down to the parameters.
//
// One lane per Gaussian; the lane loops over the views of the batch so the parameters
// are read once and the view-independent covariance is formed once. Parameter planes
// are read coalesced; the per-(view, Gaussian) records are 64 B and written by the lane
// that owns them.
//
// No multiply-add contraction anywhere in this file (the pragma precedes the includes):
// the adjoint's kernels, fused with Adam or not, then round every gradient term the same
// way, and a step with the fused update gives bit for bit the parameters of a backward
// followed by the separate Adam kernel. These kernels are bound by memory traffic.
#pragma clang fp contract(off)
#include "gs_common.h"
#include "kernels.h"

namespace gs {

// Orders a wave's LDS accesses on either side (a wave executes its LDS instructions in
// order; the fences keep the compiler from moving accesses across and make it wait for
// the earlier ones).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Tile tests of a wave: the tests of all its rectangles of up to 64 tiles (the hit mask's
// width) are laid end to end, 64 (pair, tile) tests per step, so that the work per step
// does not depend on how unevenly the rectangle sizes fall over the lanes; larger
// rectangles are walked by the whole wave one at a time.
template <int DEG>
__global__ void __launch_bounds__(256)
k_project_fwd(const float* __restrict__ P, int64_t cap, int32_t N, ViewsArg va, float near_z,
              float4* __restrict__ rec, uint32_t* __restrict__ counts, uint32_t* __restrict__ dkey, ProjSide side) {
  __shared__ uint8_t s_own[4][64];  // per wave: the lane whose tile tests start at each position
  __shared__ float4 s_pair[4][64][2];  // per wave and lane: conic, mean, threshold, rectangle
  // lanes past the end stay (reading row N - 1) so that the whole wave takes part in the
  // cooperative tile counting below; they write nothing
  const int i0 = blockIdx.x * blockDim.x + threadIdx.x;
  if (side.nvn && i0 == 0) *side.nvn = side.nvn_value;
  for (int64_t z = i0; z < side.n_zero; z += (int64_t)gridDim.x * blockDim.x) side.zero[z] = 0u;
  const bool valid = i0 < N;
  const int i = valid ? i0 : N - 1;
  constexpr int K = (DEG + 1) * (DEG + 1);
  const float m0 = P[i], m1 = P[cap + i], m2 = P[2 * cap + i];
  const KeyGeo G = key_geometry(P[3 * cap + i], P[4 * cap + i], P[5 * cap + i], P[6 * cap + i],
                                P[7 * cap + i], P[8 * cap + i], P[9 * cap + i]);
  const KeyOpacity op = key_opacity(P[10 * cap + i]);
  float sh[3 * K];
#pragma unroll
  for (int f = 0; f < 3 * K; ++f) sh[f] = P[(11 + f) * cap + i];

  for (int v = 0; v < va.n; ++v) {
    const ViewDev& V = va.v[v];
    const size_t vi = (size_t)v * N + i;
    const KeyProj kp = key_project(V, G, m0, m1, m2, op, near_z);
    int r[4] = {0, 0, -1, -1};
    uint32_t cnt = 0;
    uint64_t hits = 0;  // passing tiles in row-major rectangle order (rectangles of <= 64 tiles)
    int area = 0;
    if (valid && kp.visible && key_rect(kp, V.tiles_x, V.tiles_y, r)) area = (r[2] - r[0] + 1) * (r[3] - r[1] + 1);
    // rectangles of up to 64 tiles: the tests of all of them in one list (lane order, each
    // rectangle row-major), 64 per step. In each step the lanes whose tests start in it
    // mark their start position in the wave's LDS row; a test's owner is the mark at or
    // before it, else the owner carried over from the step before.
    {
      const int lane = (int)(threadIdx.x & 63);
      uint8_t* const own_row = s_own[threadIdx.x >> 6];
      const int a = area <= 64 ? area : 0;
      int end = a;  // inclusive running sum: this lane's tests end before `end`
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const int t = __shfl_up(end, o, 64);
        if (lane >= o) end += t;
      }
      const int beg = end - a;
      const int total = __builtin_amdgcn_readfirstlane(__shfl(end, 63, 64));
      const uint64_t upto = ~0ull >> (63 - lane);  // lanes 0 .. lane
      // the lane's pair as its tests need it, read by the lanes that test it
      s_pair[threadIdx.x >> 6][lane][0] = make_float4(kp.mx, kp.my, kp.A, kp.B);
      s_pair[threadIdx.x >> 6][lane][1] =
          make_float4(kp.C, kp.thr, __uint_as_float((uint32_t)r[0] | ((uint32_t)r[1] << 16)),
                      __uint_as_float((uint32_t)beg | ((uint32_t)(r[2] - r[0] + 1) << 16)));
      int carry = 0;
      for (int base = 0; base < total; base += 64) {  // wave-uniform
        const int j = base + lane;
        own_row[lane] = 0xff;
        wave_lds_sync();
        if (a > 0 && beg >= base && beg < base + 64) own_row[beg - base] = (uint8_t)lane;
        wave_lds_sync();
        const int mark = own_row[lane];
        const uint64_t before = __ballot(mark != 0xff) & upto;
        const int own = before ? __shfl(mark, 63 - __clzll((long long)before), 64) : carry;
        carry = __builtin_amdgcn_readlane(own, 63);
        wave_lds_sync();  // the row is rewritten in the next step
        const float4 p0 = s_pair[threadIdx.x >> 6][own][0], p1 = s_pair[threadIdx.x >> 6][own][1];
        const float mx = p0.x, my = p0.y, A = p0.z, B = p0.w, C = p1.x, thr = p1.y;
        const uint32_t xy = __float_as_uint(p1.z), bw = __float_as_uint(p1.w);
        const int x0 = (int)(xy & 0xffffu), y0 = (int)(xy >> 16), rw = (int)(bw >> 16);
        const int t = j - (int)(bw & 0xffffu);
        // t < 64 and rw <= 64: the quotient t / rw exactly (as in the emission)
        const int qy = (int)fmaf((float)t, __builtin_amdgcn_rcpf((float)rw), 1.0f / 128.0f);
        const bool hit = j < total && key_tile_hit(mx, my, A, B, C, thr, x0 + (t - qy * rw), y0 + qy);
        const uint64_t m = __ballot(hit);
        // this lane's tests in the step: list positions [lo, hi), mask bits lo - beg on
        const int lo = max(beg, base), hi = min(end, base + 64);
        if (lo < hi) {
          const int n = hi - lo;
          const uint64_t seg = (m >> (lo - base)) & (n == 64 ? ~0ull : ((1ull << n) - 1ull));
          hits |= seg << (lo - beg);
        }
      }
      if (a > 0) cnt = (uint32_t)__popcll(hits);
      wave_lds_sync();  // the pair row is rewritten for the next view
    }
    // larger rectangles: the whole wave evaluates one lane's rectangle, 64 tiles per step,
    // so no lane loops over hundreds of tiles while the others wait
    uint64_t todo = __ballot(area > 64);
    while (todo) {
      const int src = __ffsll((long long)todo) - 1;
      todo &= todo - 1;
      const float mx = __shfl(kp.mx, src), my = __shfl(kp.my, src), A = __shfl(kp.A, src);
      const float B = __shfl(kp.B, src), C = __shfl(kp.C, src), thr = __shfl(kp.thr, src);
      const int x0 = __shfl(r[0], src), y0 = __shfl(r[1], src), rw = __shfl(r[2], src) - x0 + 1;
      const int a_src = __shfl(area, src);
      uint32_t c = 0;
      uint64_t first = 0;
      for (int t0 = 0; t0 < a_src; t0 += 64) {
        const int t = t0 + (int)(threadIdx.x & 63);
        const bool hit = t < a_src && key_tile_hit(mx, my, A, B, C, thr, x0 + t % rw, y0 + t / rw);
        const uint64_t m = __ballot(hit);
        if (t0 == 0) first = m;
        c += (uint32_t)__popcll(m);
      }
      if ((int)(threadIdx.x & 63) == src) {
        cnt = c;
        hits = a_src <= 64 ? first : 0ull;
      }
    }
    if (!valid) continue;
    counts[vi] = cnt;
    // depth-sort key of the pair: float bits of a positive depth, largest key when unused
    dkey[vi] = cnt ? __float_as_uint(kp.zh) : 0xffffffffu;
    if (cnt == 0) continue;
    // view-dependent colour: max(0, sum_k sh_k Y_k(dir) + 0.5)
    float dx = m0 - V.campos[0], dy = m1 - V.campos[1], dz = m2 - V.campos[2];
    const float inv = rsqrtf(dx * dx + dy * dy + dz * dz);
    dx *= inv;
    dy *= inv;
    dz *= inv;
    float Y[K];
    sh_basis<DEG>(dx, dy, dz, Y);
    float col[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      float acc = 0.5f;
#pragma unroll
      for (int k = 0; k < K; ++k) acc += sh[3 * k + c] * Y[k];
      col[c] = fmaxf(acc, 0.0f);
    }
    float4* o = rec + vi * 4;
    o[0] = make_float4(kp.mx, kp.my, kp.A, kp.B);
    o[1] = make_float4(kp.C, kp.o, col[0], col[1]);
    o[2] = make_float4(col[2], kp.zh, 0.0f, kp.thr);
    o[3] = make_float4(__uint_as_float((uint32_t)r[0] | ((uint32_t)r[1] << 16)),
                       __uint_as_float((uint32_t)r[2] | ((uint32_t)r[3] << 16)), __uint_as_float((uint32_t)hits),
                       __uint_as_float((uint32_t)(hits >> 32)));
  }
}

// Adjoint of the projection. Input: per (view, Gaussian) 2D-gradient records of 48 B (the
// moments of dL/dpower over the pixels, dL/dcolour and dL/d(camera-frame depth); consumed and
// reset to zero here, so the buffer is clean for the next backward), or, in deterministic
// mode, the sums of the pair's per-instance records in emission order. Output: gradients
// added to the parameter planes, summed over views; vis[i] = 1 for Gaussians with a tile
// in some view.
//
// Two phases keep register pressure low: first the colour (SH coefficients and the view
// direction), which needs only the mean; then the geometry (mean, scale, rotation,
// opacity), which needs the covariance.
//
// FUSED = true (one mapping step): instead of adding to the gradient planes, the kernel
// adds any gradient already accumulated there, applies the sparse Adam update to the row
// (same arithmetic as the separate Adam kernel), clears the accumulated gradient and the
// visibility flag. Rows that reached no tile in this batch but were marked by an earlier
// backward are updated from their accumulated gradient alone.
//
// The SH gradients of a single-view batch (MULTI = false) are emitted as soon as they are
// formed; with several views they are summed in per-lane LDS slots first.
__device__ __forceinline__ void pair_grad(size_t vi, const uint32_t* __restrict__ counts,
                                          const float4* __restrict__ g2d, const float4* __restrict__ inst_grad,
                                          const uint32_t* __restrict__ inst_off, float4& ga, float4& gb,
                                          float4& gc) {
  if (inst_grad) {
    ga = gb = gc = make_float4(0.f, 0.f, 0.f, 0.f);
    const uint32_t e0 = inst_off[vi], e1 = e0 + counts[vi];
    for (uint32_t e = e0; e < e1; ++e) {
      const float4 a = inst_grad[(size_t)e * 3], b = inst_grad[(size_t)e * 3 + 1], c = inst_grad[(size_t)e * 3 + 2];
      ga.x += a.x; ga.y += a.y; ga.z += a.z; ga.w += a.w;
      gb.x += b.x; gb.y += b.y; gb.z += b.z; gb.w += b.w;
      gc.x += c.x;
      gc.y += c.y;
    }
  } else {
    ga = g2d[vi * 3 + 0];
    gb = g2d[vi * 3 + 1];
    gc = g2d[vi * 3 + 2];
  }
}

// Element of one parameter plane at the row's 32-bit byte offset (capacity < 2^30 rows).
__device__ __forceinline__ float& plane_at(float* plane, uint32_t byte_off) {
  return *(float*)((char*)plane + byte_off);
}

// One Adam update of NB planes f0 + stride j of row i, parameter values p[j] already
// loaded: the moments (and any accumulated gradient) of all NB planes are loaded before
// any store, so a lane keeps 2 NB loads in flight; each value is read and written once per
// step and streamed past the caches.
template <int NB>
__device__ __forceinline__ void adam_rows(float* __restrict__ P, float* __restrict__ Mp, float* __restrict__ Vp,
                                          float* __restrict__ Gp, int64_t cap, uint32_t lo, int f0, int stride,
                                          const float* p, const float* g, const float* lr, const AdamArg& ad,
                                          float bc1, float bc2) {
  float m[NB], v[NB], acc[NB];
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    const int64_t f = (int64_t)(f0 + stride * j) * cap;
    m[j] = __builtin_nontemporal_load(&plane_at(Mp + f, lo));
    v[j] = __builtin_nontemporal_load(&plane_at(Vp + f, lo));
    // what the separate path reads: 0 + gradient, plus sums of earlier backward calls
    acc[j] = ad.grads_clean ? 0.0f : plane_at(Gp + f, lo);
  }
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    const int64_t f = (int64_t)(f0 + stride * j) * cap;
    float pp = p[j];
    // rounded sum (no contraction), as the separate path's += then load
    adam_update(pp, m[j], v[j], __fadd_rn(acc[j], g[j]), lr[j], ad.beta1, ad.beta2, ad.eps, bc1, bc2);
    __builtin_nontemporal_store(pp, &plane_at(P + f, lo));
    __builtin_nontemporal_store(m[j], &plane_at(Mp + f, lo));
    __builtin_nontemporal_store(v[j], &plane_at(Vp + f, lo));
    if (acc[j] != 0.0f) plane_at(Gp + f, lo) = 0.0f;
  }
}

// The K planes f0 + 3 k of one SH channel in batches of at most kAdamBatch (bounded
// registers).
constexpr int kAdamBatch = 4;
template <int K>
__device__ __forceinline__ void adam_sh(float* __restrict__ P, float* __restrict__ Mp, float* __restrict__ Vp,
                                        float* __restrict__ Gp, int64_t cap, uint32_t lo, int f0, const float* p,
                                        const float* g, const float* lr, const AdamArg& ad, float bc1, float bc2) {
  if constexpr (K <= kAdamBatch) {
    adam_rows<K>(P, Mp, Vp, Gp, cap, lo, f0, 3, p, g, lr, ad, bc1, bc2);
  } else {
    adam_rows<kAdamBatch>(P, Mp, Vp, Gp, cap, lo, f0, 3, p, g, lr, ad, bc1, bc2);
    adam_sh<K - kAdamBatch>(P, Mp, Vp, Gp, cap, lo, f0 + 3 * kAdamBatch, p + kAdamBatch, g + kAdamBatch,
                            lr + kAdamBatch, ad, bc1, bc2);
  }
}

template <int DEG, bool FUSED, bool MULTI>
__global__ void __launch_bounds__(256)
k_project_bwd(float* P, float* __restrict__ Gp, int64_t cap, int32_t N, ViewsArg va, float near_z,
              const uint32_t* __restrict__ counts, float4* __restrict__ g2d, const float4* __restrict__ inst_grad,
              const uint32_t* __restrict__ inst_off, uint8_t* __restrict__ vis, AdamArg ad, LossFinish lf) {
  constexpr int K = (DEG + 1) * (DEG + 1);
  __shared__ float s_gsh[MULTI ? 3 * K : 1][MULTI ? 256 : 1];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (FUSED && lf.part && blockIdx.x == 0) {
    // the step's losses (Eq. 9) from the loss kernel's per-tile sums, in place of a launch
    // of their own
    __shared__ double s_loss[2][256];
    int b0 = 0;
    for (int v = 0; v < va.n; ++v) {
      const int b1 = b0 + loss_tiles_of(va.v[v].H, va.v[v].W);
      const float L = loss_from_partials(lf.part, b0, b1, va.v[v].H, va.v[v].W, lf.lambda, s_loss);
      if (threadIdx.x == 0) lf.loss[v] = L;
      b0 = b1;
    }
  }
  // a render that dropped its instances (it needed more than the buffers hold) has no
  // gradient: nothing is added, and a fused step is skipped, leaving the map, its moments
  // and the exposures as they are (the same decision for every thread)
  if (render_dropped(va)) return;
  if (FUSED && blockIdx.x == 0 && (int)threadIdx.x < 12 * ad.n_exp) {
    // the views' exposures (their gradients are complete once the blend backward is done),
    // as the separate exposure update does, in place of a launch of its own
    float* st = const_cast<float*>(va.v[threadIdx.x / 12].exposure);
    const int k = (int)threadIdx.x % 12;
    float pp = st[k], mm = st[24 + k], vv = st[36 + k];
    adam_update(pp, mm, vv, st[12 + k], ad.lr_exp, ad.beta1, ad.beta2, ad.eps, ad.bc[0], ad.bc[1]);
    st[k] = pp;
    st[24 + k] = mm;
    st[36 + k] = vv;
    st[12 + k] = 0.0f;
  }
  if (i >= N) return;
  // non-fused: gradient g of plane f added to the gradient planes
  const uint32_t lo = (uint32_t)i * 4u;  // byte offset of the row in every plane (cap < 2^30)
  auto emit = [&](int f, float g) {
    float& d = plane_at(Gp + (int64_t)f * cap, lo);
    d = __fadd_rn(d, g);
  };
  auto ldp = [&](int f) { return plane_at(P + (int64_t)f * cap, lo); };
  float* __restrict__ Mp = ad.m;
  float* __restrict__ Vp = ad.v;
  const float bc1 = FUSED ? ad.bc[0] : 1.0f, bc2 = FUSED ? ad.bc[1] : 1.0f;
  // learning rates by plane (constant indices: a runtime index into the by-value table
  // would place it in scratch memory)
  float lr_sh[K];
#pragma unroll
  for (int k = 0; k < K; ++k) lr_sh[k] = ad.lr.lr[k == 0 ? 11 : 14];
  bool any = false;
  for (int v = 0; v < va.n; ++v) any |= counts[(size_t)v * N + i] > 0;
  if (!any && !(FUSED && vis[i])) return;

  const float mu0 = ldp(0), mu1 = ldp(1), mu2 = ldp(2);
  float gmu[3] = {0.f, 0.f, 0.f};

  // ---- phase 1: colour = max(0, sum_k sh_k Y_k(dir) + 0.5), dir = normalised (mu - campos)
  if (MULTI)
    for (int f = 0; f < 3 * K; ++f) s_gsh[f][threadIdx.x] = 0.0f;
  bool sh_done = false;  // single view: SH planes already emitted
  for (int v = 0; v < va.n; ++v) {
    const size_t vi = (size_t)v * N + i;
    if (counts[vi] == 0) continue;
    const ViewDev& V = va.v[v];
    float4 ga, gb, gc;
    pair_grad(vi, counts, g2d, inst_grad, inst_off, ga, gb, gc);
    const float g_col[3] = {gb.z, gb.w, gc.x};
    const float dv0 = mu0 - V.campos[0], dv1 = mu1 - V.campos[1], dv2 = mu2 - V.campos[2];
    const float inv = rsqrtf(dv0 * dv0 + dv1 * dv1 + dv2 * dv2);
    const float d0 = dv0 * inv, d1 = dv1 * inv, d2 = dv2 * inv;
    float Y[K];
    sh_basis<DEG>(d0, d1, d2, Y);
    float wsum[K];
#pragma unroll
    for (int k = 0; k < K; ++k) wsum[k] = 0.f;
#pragma unroll 1
    for (int ch = 0; ch < 3; ++ch) {
      float shc[K];
      float raw = 0.5f;
#pragma unroll
      for (int k = 0; k < K; ++k) {
        shc[k] = ldp(11 + 3 * k + ch);
        raw += shc[k] * Y[k];
      }
      const float gcol = raw < 0.0f ? 0.0f : g_col[ch];  // clamped channel: no gradient
      float gk[K];
#pragma unroll
      for (int k = 0; k < K; ++k) {
        wsum[k] += gcol * shc[k];
        gk[k] = __fmul_rn(gcol, Y[k]);  // rounded: both paths add exactly this value
      }
      if (MULTI) {
#pragma unroll
        for (int k = 0; k < K; ++k) s_gsh[3 * k + ch][threadIdx.x] += gk[k];
      } else if (FUSED) {
        adam_sh<K>(P, Mp, Vp, Gp, cap, lo, 11 + ch, shc, gk, lr_sh, ad, bc1, bc2);
      } else {
#pragma unroll 4
        for (int k = 0; k < K; ++k) emit(11 + 3 * k + ch, gk[k]);
      }
    }
    if (!MULTI) sh_done = true;
    if (DEG > 0) {
      float gdx, gdy, gdz;
      sh_basis_grad<DEG>(d0, d1, d2, wsum, gdx, gdy, gdz);
      const float dot = gdx * d0 + gdy * d1 + gdz * d2;
      gmu[0] += (gdx - dot * d0) * inv;
      gmu[1] += (gdy - dot * d1) * inv;
      gmu[2] += (gdz - dot * d2) * inv;
    }
  }
  if (MULTI || !sh_done) {
    // several views: the summed SH gradients; a single view without a tile in this batch
    // (fused path, row marked by an earlier backward): zero local part
#pragma unroll 1
    for (int ch = 0; ch < 3; ++ch) {
      float gk[K];
#pragma unroll
      for (int k = 0; k < K; ++k) gk[k] = MULTI ? s_gsh[3 * k + ch][threadIdx.x] : 0.0f;
      if (FUSED) {
        float pk[K];
#pragma unroll
        for (int k = 0; k < K; ++k) pk[k] = ldp(11 + 3 * k + ch);
        adam_sh<K>(P, Mp, Vp, Gp, cap, lo, 11 + ch, pk, gk, lr_sh, ad, bc1, bc2);
      } else {
#pragma unroll 4
        for (int k = 0; k < K; ++k) emit(11 + 3 * k + ch, gk[k]);
      }
    }
  }

  // ---- phase 2: geometry. Normalised quaternion, rotation, scales, M = R S, Sigma = M M^T
  const float q0 = ldp(6), q1 = ldp(7), q2 = ldp(8), q3 = ldp(9);
  const float qn = sqrtf(q0 * q0 + q1 * q1 + q2 * q2 + q3 * q3);
  const float iqn = qn > 0.f ? 1.0f / qn : 0.f;
  const float w = q0 * iqn, x = q1 * iqn, y = q2 * iqn, z = q3 * iqn;
  const float Rq[9] = {1.f - 2.f * (y * y + z * z), 2.f * (x * y - w * z), 2.f * (x * z + w * y),
                       2.f * (x * y + w * z), 1.f - 2.f * (x * x + z * z), 2.f * (y * z - w * x),
                       2.f * (x * z - w * y), 2.f * (y * z + w * x), 1.f - 2.f * (x * x + y * y)};
  const float ls0 = ldp(3), ls1 = ldp(4), ls2 = ldp(5);
  const float s[3] = {__expf(ls0), __expf(ls1), __expf(ls2)};
  float M[9];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int k = 0; k < 3; ++k) M[3 * r + k] = Rq[3 * r + k] * s[k];
  float Sg[6];  // 00 01 02 11 12 22
  Sg[0] = M[0] * M[0] + M[1] * M[1] + M[2] * M[2];
  Sg[1] = M[0] * M[3] + M[1] * M[4] + M[2] * M[5];
  Sg[2] = M[0] * M[6] + M[1] * M[7] + M[2] * M[8];
  Sg[3] = M[3] * M[3] + M[4] * M[4] + M[5] * M[5];
  Sg[4] = M[3] * M[6] + M[4] * M[7] + M[5] * M[8];
  Sg[5] = M[6] * M[6] + M[7] * M[7] + M[8] * M[8];
  const float logit = ldp(10);
  const float op = 1.0f / (1.0f + __expf(-logit));
  float gM[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  float glogit = 0.0f;

  for (int v = 0; v < va.n; ++v) {
    const size_t vi = (size_t)v * N + i;
    if (counts[vi] == 0) continue;
    const ViewDev& V = va.v[v];
    float4 ga, gb, gc;
    pair_grad(vi, counts, g2d, inst_grad, inst_off, ga, gb, gc);
    if (!inst_grad) {
      const float4 zero = make_float4(0.f, 0.f, 0.f, 0.f);
      g2d[vi * 3 + 0] = zero;
      g2d[vi * 3 + 1] = zero;
      g2d[vi * 3 + 2] = zero;
    }
    // moments of dL/dpower over the pixels (2D-gradient record): conic gradients now, the
    // 2D mean's once the conic is known
    const float s_x = ga.x, s_y = ga.y, s_p = gb.y;
    const float g_A = -0.5f * ga.z, g_B = -ga.w, g_C = -0.5f * gb.x;
    const float* W = V.R;
    const float xh = W[0] * mu0 + W[1] * mu1 + W[2] * mu2 + V.t[0];
    const float yh = W[3] * mu0 + W[4] * mu1 + W[5] * mu2 + V.t[1];
    const float zh = W[6] * mu0 + W[7] * mu1 + W[8] * mu2 + V.t[2];
    const float iz = 1.0f / zh, iz2 = iz * iz;
    const float limx = V.limx, limy = V.limy;
    const float rx = xh * iz, ry = yh * iz;
    const bool clx = rx < -limx || rx > limx, cly = ry < -limy || ry > limy;
    const float tx = fminf(limx, fmaxf(-limx, rx)), ty = fminf(limy, fmaxf(-limy, ry));
    const float J00 = V.fx * iz, J02 = -V.fx * tx * iz, J11 = V.fy * iz, J12 = -V.fy * ty * iz;
    float T0[3], T1[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      T0[k] = J00 * W[k] + J02 * W[6 + k];
      T1[k] = J11 * W[3 + k] + J12 * W[6 + k];
    }
    // Sigma T0, Sigma T1
    const float ST0[3] = {Sg[0] * T0[0] + Sg[1] * T0[1] + Sg[2] * T0[2], Sg[1] * T0[0] + Sg[3] * T0[1] + Sg[4] * T0[2],
                          Sg[2] * T0[0] + Sg[4] * T0[1] + Sg[5] * T0[2]};
    const float ST1[3] = {Sg[0] * T1[0] + Sg[1] * T1[1] + Sg[2] * T1[2], Sg[1] * T1[0] + Sg[3] * T1[1] + Sg[4] * T1[2],
                          Sg[2] * T1[0] + Sg[4] * T1[1] + Sg[5] * T1[2]};
    const float a = T0[0] * ST0[0] + T0[1] * ST0[1] + T0[2] * ST0[2] + 0.3f;
    const float b = T0[0] * ST1[0] + T0[1] * ST1[1] + T0[2] * ST1[2];
    const float c = T1[0] * ST1[0] + T1[1] * ST1[1] + T1[2] * ST1[2] + 0.3f;
    const float det = a * c - b * b;
    const float id2 = 1.0f / (det * det);
    const float idet = 1.0f / det;
    const float cA = c * idet, cB = -b * idet, cC = a * idet;  // the conic
    const float g_mx = cA * s_x + cB * s_y, g_my = cB * s_x + cC * s_y;
    // conic = inverse(Sigma'): gradients w.r.t. (a, b, c) of Sigma' = [[a, b], [b, c]]
    const float g_a = (-c * c * g_A + b * c * g_B - b * b * g_C) * id2;
    const float g_b = (2.f * b * c * g_A - (a * c + b * b) * g_B + 2.f * a * b * g_C) * id2;
    const float g_c = (-b * b * g_A + a * b * g_B - a * a * g_C) * id2;
    // Sigma' = T Sigma T^T: dL/dM = 2 Psym M with
    // Psym = g_a T0 T0^T + g_b (T0 T1^T + T1 T0^T) / 2 + g_c T1 T1^T
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      const float u = g_a * T0[r] + 0.5f * g_b * T1[r];   // row r of Psym = u T0^T + t T1^T
      const float t = 0.5f * g_b * T0[r] + g_c * T1[r];
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const float t0m = T0[0] * M[k] + T0[1] * M[3 + k] + T0[2] * M[6 + k];
        const float t1m = T1[0] * M[k] + T1[1] * M[3 + k] + T1[2] * M[6 + k];
        gM[3 * r + k] += 2.f * (u * t0m + t * t1m);
      }
    }
    float gT0[3], gT1[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      gT0[k] = 2.f * g_a * ST0[k] + g_b * ST1[k];
      gT1[k] = g_b * ST0[k] + 2.f * g_c * ST1[k];
    }
    const float gJ00 = gT0[0] * W[0] + gT0[1] * W[1] + gT0[2] * W[2];
    const float gJ02 = gT0[0] * W[6] + gT0[1] * W[7] + gT0[2] * W[8];
    const float gJ11 = gT1[0] * W[3] + gT1[1] * W[4] + gT1[2] * W[5];
    const float gJ12 = gT1[0] * W[6] + gT1[1] * W[7] + gT1[2] * W[8];
    // camera-frame mean: through J and the 2D mean
    float gx = 0.f, gy = 0.f, gz = gc.y;  // gc.y: gradient of the camera-frame depth (Eq. 6)
    gz += -V.fx * iz2 * gJ00 - V.fy * iz2 * gJ11;
    if (!clx) {
      gx += -V.fx * iz2 * gJ02;
      gz += 2.f * V.fx * xh * iz2 * iz * gJ02;
    } else {
      gz += V.fx * tx * iz2 * gJ02;
    }
    if (!cly) {
      gy += -V.fy * iz2 * gJ12;
      gz += 2.f * V.fy * yh * iz2 * iz * gJ12;
    } else {
      gz += V.fy * ty * iz2 * gJ12;
    }
    gx += g_mx * V.fx * iz;
    gz += -g_mx * V.fx * xh * iz2;
    gy += g_my * V.fy * iz;
    gz += -g_my * V.fy * yh * iz2;
    // world mean: R_cw^T
    gmu[0] += W[0] * gx + W[3] * gy + W[6] * gz;
    gmu[1] += W[1] * gx + W[4] * gy + W[7] * gz;
    gmu[2] += W[2] * gx + W[5] * gy + W[8] * gz;
    glogit += s_p * (1.0f - op);  // dL/do = s_p / o, do/dlogit = o (1 - o)
  }
  // M = R diag(s): scales and rotation
  float gls[3], gR[9];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const float gs_ = gM[k] * Rq[k] + gM[3 + k] * Rq[3 + k] + gM[6 + k] * Rq[6 + k];
    gls[k] = gs_ * s[k];
#pragma unroll
    for (int r = 0; r < 3; ++r) gR[3 * r + k] = gM[3 * r + k] * s[k];
  }
  // rotation from the unit quaternion, then through the normalisation
  float gq[4];
  gq[0] = 2.f * (-z * gR[1] + y * gR[2] + z * gR[3] - x * gR[5] - y * gR[6] + x * gR[7]);
  gq[1] = 2.f * (y * gR[1] + z * gR[2] + y * gR[3] - 2.f * x * gR[4] - w * gR[5] + z * gR[6] + w * gR[7] - 2.f * x * gR[8]);
  gq[2] = 2.f * (-2.f * y * gR[0] + x * gR[1] + w * gR[2] + x * gR[3] + z * gR[5] - w * gR[6] + z * gR[7] - 2.f * y * gR[8]);
  gq[3] = 2.f * (-2.f * z * gR[0] - w * gR[1] + x * gR[2] + w * gR[3] - 2.f * z * gR[4] + y * gR[5] + x * gR[6] + y * gR[7]);
  const float qd = gq[0] * w + gq[1] * x + gq[2] * y + gq[3] * z;
  const float unit[4] = {w, x, y, z};
  const float gg[11] = {gmu[0], gmu[1], gmu[2], gls[0], gls[1], gls[2], (gq[0] - qd * unit[0]) * iqn,
                        (gq[1] - qd * unit[1]) * iqn, (gq[2] - qd * unit[2]) * iqn, (gq[3] - qd * unit[3]) * iqn,
                        glogit};
  if (FUSED) {
    const float pg[11] = {mu0, mu1, mu2, ls0, ls1, ls2, q0, q1, q2, q3, logit};
    float lr_geo[11];
#pragma unroll
    for (int f = 0; f < 11; ++f) lr_geo[f] = ad.lr.lr[f];
    adam_rows<4>(P, Mp, Vp, Gp, cap, lo, 0, 1, pg, gg, lr_geo, ad, bc1, bc2);
    adam_rows<4>(P, Mp, Vp, Gp, cap, lo, 4, 1, pg + 4, gg + 4, lr_geo + 4, ad, bc1, bc2);
    adam_rows<3>(P, Mp, Vp, Gp, cap, lo, 8, 1, pg + 8, gg + 8, lr_geo + 8, ad, bc1, bc2);
  } else {
#pragma unroll
    for (int f = 0; f < 11; ++f) emit(f, gg[f]);
  }
  vis[i] = FUSED ? 0 : 1;
}

template <int DEG>
static hipError_t launch_fwd(const float* P, int64_t cap, int32_t N, const ViewsArg& va, float near_z,
                             float4* rec, uint32_t* counts, uint32_t* dkey, const ProjSide& side, hipStream_t s) {
  hipLaunchKernelGGL(k_project_fwd<DEG>, dim3((N + 255) / 256), dim3(256), 0, s, P, cap, N, va,
                     near_z, rec, counts, dkey, side);
  return hipGetLastError();
}

template <int DEG>
static hipError_t launch_bwd(float* P, float* G, int64_t cap, int32_t N, const ViewsArg& va, float near_z,
                             const uint32_t* counts, float4* g2d, const float* inst_grad, const uint32_t* inst_off,
                             uint8_t* vis, const AdamArg* ad, const LossFinish& lf, hipStream_t s) {
  const dim3 grid((N + 255) / 256), block(256);
  const float4* ig = (const float4*)inst_grad;
  const AdamArg a = ad ? *ad : AdamArg{};
  if (va.n == 1) {
    if (ad)
      hipLaunchKernelGGL((k_project_bwd<DEG, true, false>), grid, block, 0, s, P, G, cap, N, va, near_z, counts, g2d,
                         ig, inst_off, vis, a, lf);
    else
      hipLaunchKernelGGL((k_project_bwd<DEG, false, false>), grid, block, 0, s, P, G, cap, N, va, near_z, counts,
                         g2d, ig, inst_off, vis, a, lf);
  } else {
    if (ad)
      hipLaunchKernelGGL((k_project_bwd<DEG, true, true>), grid, block, 0, s, P, G, cap, N, va, near_z, counts, g2d,
                         ig, inst_off, vis, a, lf);
    else
      hipLaunchKernelGGL((k_project_bwd<DEG, false, true>), grid, block, 0, s, P, G, cap, N, va, near_z, counts,
                         g2d, ig, inst_off, vis, a, lf);
  }
  return hipGetLastError();
}

hipError_t project_forward(int deg, const float* P, int64_t cap, int32_t N, const ViewsArg& va,
                           float near_z, float4* rec, uint32_t* counts, uint32_t* dkey,
                           const ProjSide& side, hipStream_t s) {
  if (N <= 0) {  // no projection launch: the side writes get their own
    hipError_t e = hipSuccess;
    if (side.nvn) e = fill_u32(side.nvn, side.nvn_value, 1, s);
    if (e == hipSuccess && side.n_zero > 0) e = fill_u32(side.zero, 0u, side.n_zero, s);
    return e;
  }
  switch (deg) {
    case 0: return launch_fwd<0>(P, cap, N, va, near_z, rec, counts, dkey, side, s);
    case 1: return launch_fwd<1>(P, cap, N, va, near_z, rec, counts, dkey, side, s);
    case 2: return launch_fwd<2>(P, cap, N, va, near_z, rec, counts, dkey, side, s);
    default: return launch_fwd<3>(P, cap, N, va, near_z, rec, counts, dkey, side, s);
  }
}

hipError_t project_backward(int deg, float* P, float* G, int64_t cap, int32_t N, const ViewsArg& va, float near_z,
                            const uint32_t* counts, float4* g2d, const float* inst_grad, const uint32_t* inst_off,
                            uint8_t* vis, const AdamArg* adam, const LossFinish& lf, hipStream_t s) {
  if (N <= 0) {  // no projection launch: the losses and the exposures get launches of their own
    hipError_t e = loss_finish_launch(va, lf, s);
    if (e != hipSuccess || !adam || adam->n_exp <= 0) return e;
    ExpArg ea{};
    ea.n = adam->n_exp;
    for (int x = 0; x < ea.n; ++x) ea.p[x] = const_cast<float*>(va.v[x].exposure);
    return adam_exposures(ea, adam->bc, adam->lr_exp, adam->beta1, adam->beta2, adam->eps, s);
  }
  // only the fused kernel's first block finishes losses
  LossFinish lfk = lf;
  if (!adam) {
    hipError_t e = loss_finish_launch(va, lf, s);
    if (e != hipSuccess) return e;
    lfk = LossFinish{nullptr, nullptr, 0.f, 0};
  }
  switch (deg) {
    case 0: return launch_bwd<0>(P, G, cap, N, va, near_z, counts, g2d, inst_grad, inst_off, vis, adam, lfk, s);
    case 1: return launch_bwd<1>(P, G, cap, N, va, near_z, counts, g2d, inst_grad, inst_off, vis, adam, lfk, s);
    case 2: return launch_bwd<2>(P, G, cap, N, va, near_z, counts, g2d, inst_grad, inst_off, vis, adam, lfk, s);
    default: return launch_bwd<3>(P, G, cap, N, va, near_z, counts, g2d, inst_grad, inst_off, vis, adam, lfk, s);
  }
}

}  // namespace gs
