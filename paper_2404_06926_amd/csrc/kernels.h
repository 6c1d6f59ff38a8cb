// Host-side launchers of the HIP kernels (internal to libgslic).
#pragma once

#include "gs_common.h"

namespace gs {

constexpr int kMaxPlanes = 11 + 3 * 16;
constexpr int kMaxExposures = 64;

struct LrArg {
  float lr[kMaxPlanes];
};

struct ExpArg {
  int32_t n;
  float* p[kMaxExposures];
};

// Sparse Adam applied inside the projection backward (one mapping step).
struct AdamArg {
  LrArg lr;
  float* m;
  float* v;
  const float* bc;   // device bias corrections 1 - beta1^t, 1 - beta2^t
  float beta1, beta2, eps;
  int32_t grads_clean;  // the gradient planes are known to be zero: do not read them
  // the exposures of views 0 .. n_exp - 1 are updated too (by the first block); in a fused
  // step view e's exposure pointer is its 48-float state [E | gradient | m | v]
  int32_t n_exp;
  float lr_exp;
};

// projection (project.hip)
// Small writes the projection's threads make on the side, saving launches of their own:
// *nvn = nvn_value (if nvn is set) and zero[0 .. n_zero) = 0.
struct ProjSide {
  uint32_t* nvn;
  uint32_t nvn_value;
  uint32_t* zero;
  int64_t n_zero;
};
hipError_t project_forward(int deg, const float* P, int64_t cap, int32_t N, const ViewsArg& va, float near_z,
                           float4* rec, uint32_t* counts, uint32_t* dkey, const ProjSide& side, hipStream_t s);
// With inst_grad != nullptr the 2D gradients are the sums, in emission order, of the
// instance records [inst_off[vi], inst_off[vi] + counts[vi]); otherwise they come from g2d.
// With adam != nullptr the Adam update of each row is applied in the same kernel (one step).
// lf.part (fused steps only): the first block also writes the views' losses.
hipError_t project_backward(int deg, float* P, float* G, int64_t cap, int32_t N, const ViewsArg& va, float near_z,
                            const uint32_t* counts, float4* g2d, const float* inst_grad, const uint32_t* inst_off,
                            uint8_t* vis, const AdamArg* adam, const LossFinish& lf, hipStream_t s);

// binning (binning.hip)
int64_t scan_temp_elems(int64_t n);
hipError_t exclusive_scan(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* temp, hipStream_t s);
// offsets[k] = sum of counts[order[j]] for j < k; total = sum of all. With capacity > 0 it
// also writes block_start (block_start_elems(capacity) words) for duplicate_keys, as for
// that capacity.
hipError_t scan_counts(const uint32_t* counts, const uint32_t* order, uint32_t* offsets, int64_t n,
                       uint32_t* temp, uint32_t* total, uint32_t* block_start, int64_t capacity, hipStream_t s);
// Instances in depth order, one lane per instance (block_start: block_start_elems(capacity)
// words); a pair with more than 64 candidate tiles is emitted by one wave.
// overflow[0] |= 1 when the instances exceed the capacity; overflow[2] = max(overflow[2],
// instance count).
// With all_off, inst_off receives every pair's first emission index (the deterministic
// backward reads it). starts_marked: scan_counts wrote block_start for this capacity;
// otherwise a launch of its own writes it.
int64_t block_start_elems(int64_t capacity);
hipError_t duplicate_keys(const float4* rec, const uint32_t* counts, const uint32_t* order, const uint32_t* offsets,
                          const uint32_t* n_dev, int32_t N, const ViewsArg& va, uint32_t* tiles, uint32_t* emit_g,
                          uint32_t* inst_off,
                          bool all_off, uint32_t* block_start, bool starts_marked, int64_t capacity,
                          uint32_t* overflow, hipStream_t s);
hipError_t gather_gaussians(const uint32_t* vals, const uint32_t* emit_g, const uint32_t* n_dev, int64_t cap,
                            uint32_t* out, hipStream_t s);
int64_t sort_temp_elems(int64_t cap);
// vals_iota: the values are 0, 1, 2, ... and vals[0] is not read.
hipError_t radix_sort_u32(uint32_t* keys[2], uint32_t* vals[2], const uint32_t* n_dev, int64_t cap, int nbits,
                          uint32_t* temp, int* which, hipStream_t s, bool vals_iota);
hipError_t tile_ranges(const uint32_t* tiles, const uint32_t* n_dev, int64_t cap, uint2* ranges, int64_t n_tiles,
                       hipStream_t s);

// blending (blend.hip)
// Long tile lists are split into chunks that separate workgroups blend: a tile whose list
// is longer than `balance` times the mean list and than the chunk length L = max(min_len,
// ceil(instances / par)) (rounded up to a multiple of 64) is cut into ceil(n / L) chunks
// of near-equal length.
// With that L at most par tiles split, the chunks after the first number at most par and
// the chunks of all split tiles at most 2 par, which sizes every buffer below
// independently of the scene.
constexpr uint32_t kNoSlot = 0xFFFFFFFFu;
constexpr int kSplitFields = 7;   // per chunk and pixel: see blend.hip
struct SplitArg {
  uint32_t* tile_slot;      // per tile: first state slot of a split tile, kNoSlot otherwise
  uint2* extra;             // (tile, chunk) of every chunk >= 1 of a split tile, [0, counts[0])
  uint32_t* counts;         // [0] extra chunks, [1] slots taken; zero before split_items
  const uint32_t* n_inst;   // instance count of the render
  float* state;             // kSplitFields x 256 floats per slot (2 par slots)
  int32_t par;              // 0: no tile is split
  int32_t min_len;
  float balance;
};
hipError_t split_items(const uint2* ranges, int32_t n_tiles, const SplitArg& sp, hipStream_t s);

// vals: emission index of each instance in blend order; emit_g: Gaussian of each emission index.
// px: pixels per lane (1, 2 or 4), see blend.hip.
hipError_t blend_forward(const ViewsArg& va, const float4* rec, int32_t N, const uint32_t* vals,
                         const uint32_t* emit_g, const uint2* ranges, const SplitArg& sp, int px,
                         hipStream_t s);
// Gradients of (mean2d, conic, opacity, colour, depth) per (view, Gaussian): with inst_grad == nullptr
// they are added to g2d with wave-reduced atomics; otherwise every instance's gradient is
// written to inst_grad[emission index] (12 floats, fixed-order reduction, deterministic).
// sp: the split of the render whose lists and saved state this backward uses.
hipError_t blend_backward(const ViewsArg& va, const float4* rec, int32_t N, const uint32_t* vals,
                          const uint32_t* emit_g, const uint2* ranges, float* g2d, float* inst_grad,
                          float* exp_part, const SplitArg& sp, int px, hipStream_t s);

// Per-Gaussian form of blend_backward (blend_pg.hip): colour and exposure gradients only
// (no depth / opacity maps); the chunks of split tiles (sp, as in blend_backward) are
// separate work items.
hipError_t blend_backward_per_gaussian(const ViewsArg& va, const float4* rec, int32_t N, const uint32_t* vals,
                                       const uint32_t* emit_g, const uint2* ranges, float* g2d, float* inst_grad,
                                       float* exp_part, const SplitArg& sp, hipStream_t s);
// fixed-order reduction of the per-tile exposure partials of the deterministic backward
hipError_t exposure_reduce(const ViewsArg& va, const float* exp_part, hipStream_t s);

// loss (loss.hip)
// One image of a loss launch: out (x), target (y), dL/dout, where its loss goes, and its
// size; tiles_x and tile_base are filled by ssim_loss.
struct LossView {
  const float* x;
  const float* y;
  float* gout;
  float* loss;
  int32_t H, W, tiles_x, tile_base;
};
struct LossArg {
  int32_t n;
  float lambda;
  LossView v[kMaxViews];
};
// The Adam step counter advance of a fused step (by the loss kernel); a step whose render
// needed more than inst_cap instances is skipped instead and counted in *skipped.
struct StepPrep {
  int64_t* step;
  float* bc;
  float beta1, beta2;
  const uint32_t* n_inst;
  int64_t inst_cap;
  uint32_t* skipped;
};
int64_t loss_temp_floats(int H, int W);
int64_t loss_temp_floats_multi(const LossArg& la);
// defer_finish: the tile kernel only; the losses are left to the projection backward
// (LossFinish with part = temp + loss_part_offset()), or to loss_finish_launch.
hipError_t ssim_loss(LossArg la, float* temp, const StepPrep* prep, bool defer_finish, hipStream_t s);
int64_t loss_part_offset();
// the losses of va's views from the partial sums of a deferred loss launch
hipError_t loss_finish_launch(const ViewsArg& va, const LossFinish& lf, hipStream_t s);

// optimiser and map maintenance (adam.hip)
hipError_t adam_step(float* buf, int64_t cap, int32_t F, int32_t N, const uint8_t* vis, const LrArg& lr,
                     int64_t* step, float* bc, float beta1, float beta2, float eps, const ExpArg& ea,
                     float lr_exposure, hipStream_t s);
hipError_t adam_prepare(int64_t* step, float* bc, float beta1, float beta2, hipStream_t s);
hipError_t adam_exposures(const ExpArg& ea, const float* bc, float lr, float beta1, float beta2, float eps,
                          hipStream_t s);
hipError_t fill_u32(uint32_t* d, uint32_t val, int64_t n, hipStream_t s);
hipError_t append_rows(float* buf, int64_t cap, int32_t F, int32_t K, int64_t n0, int64_t n, const float* means,
                       const float* ls, const float* quats, const float* logits, const float* sh, uint8_t* vis,
                       hipStream_t s);
hipError_t init_points(float* buf, int64_t cap, int32_t F, int32_t K, int64_t n0, int64_t n, const float* xyz,
                       const float* rgb, const ViewDev& V, float near_z, float logit0, uint8_t* vis,
                       hipStream_t s);
// map growth (growth.hip): Eq. 8 selection of points by the opacity of their pixel, the
// selected points' rows, and sky rows from nearest-neighbour distances (d2: n floats).
hipError_t expand_flags(const float* xyz, int64_t n, const ViewDev& V, const float* T, float tau, float near_z,
                        uint32_t* flags, hipStream_t s);
hipError_t init_selected(float* buf, int64_t cap, int32_t F, int32_t K, int64_t n0, int64_t n, const float* xyz,
                         const float* rgb, const uint32_t* flags, const uint32_t* offsets, const ViewDev& V,
                         float near_z, float logit0, uint8_t* vis, hipStream_t s);
hipError_t init_sky(float* buf, int64_t cap, int32_t F, int32_t K, int64_t n0, int64_t n, const float* xyz,
                    float* d2, float logit0, uint8_t* vis, hipStream_t s);
hipError_t copy_planes(const float* src, int64_t cap0, float* dst, int64_t cap1, int64_t n, int nplanes,
                       hipStream_t s);

}  // namespace gs
