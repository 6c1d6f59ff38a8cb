// C ABI of libgslic: the map object, its device buffers and workspace, and the
// orchestration of the kernels for render, backward, loss, Adam and keyframe jobs.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "gs_common.h"
#include "kernels.h"

using namespace gs;

namespace {

thread_local std::string g_err;

constexpr int64_t kKeyframePeriod = 5;  // every fifth frame is a keyframe (Sec. III-C.2)

gs_status fail(gs_status code, const std::string& msg) {
  g_err = msg;
  return code;
}

#define GS_HIP(expr)                                                              \
  do {                                                                            \
    hipError_t _e = (expr);                                                       \
    if (_e != hipSuccess)                                                         \
      return fail(GS_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(_e)); \
  } while (0)

#define GS_TRY(expr)            \
  do {                          \
    gs_status _s = (expr);      \
    if (_s != GS_OK) return _s; \
  } while (0)

}  // namespace

// A device buffer that grows by reallocation (old contents are not kept).
struct DevBuf {
  void* ptr = nullptr;
  size_t bytes = 0;
};

struct KeyframeSlot {
  gs_view view{};
  float* image = nullptr;      // 3 x H x W (owned copy of the target)
  float* state = nullptr;      // exposure [E | grad | m | v] (48 floats)
  float* rgb = nullptr;        // render output
  float* T = nullptr;
  uint32_t* nc = nullptr;
  float* dl = nullptr;         // dL/d rgb
  size_t pix_bytes = 0;        // bytes of one float plane of this slot's buffers
};

// A keyframe kept for the whole session (the random-K schedule): pose, owned copy of the
// target image, exposure state [E | grad | m | v].
struct ArchivedKeyframe {
  gs_view view{};
  float* image = nullptr;
  float* state = nullptr;
  size_t pix_bytes = 0;
};

struct gs_map {
  gs_map_desc desc{};
  gs_allocator alloc{};
  bool has_alloc = false;
  int deg = 3, K = 16, F = 59;
  int64_t n = 0, cap = 0;
  float* buf = nullptr;        // params | grads | m | v, each F planes of cap floats
  uint8_t* vis = nullptr;      // cap bytes (rounded up to 4)
  int64_t* d_step = nullptr;   // Adam step t
  float* d_bc = nullptr;       // bias corrections
  uint32_t* d_ninst = nullptr; // instance count of the last render
  uint32_t* d_overflow = nullptr;
  float* d_loss = nullptr;     // loss values of keyframe jobs (64 floats)
  uint32_t* h_pinned = nullptr;
  int64_t h_step = 0;
  int64_t resident = 0;
  // workspace
  DevBuf rec, counts, offsets, scan_tmp, g2d, keys[2], vals[2], sort_tmp, ranges, pixT, pixN, loss_tmp;
  DevBuf dkey[2], dval[2];     // depth-sort keys / (view, Gaussian) ids, double-buffered
  DevBuf emit_g, inst_off;     // Gaussian of each emission index; first emission index per pair
  DevBuf block_start;           // instance-parallel binning: first pair per emission block
  DevBuf split_slot, split_extra, split_state;  // long lists cut into chunks (blend)
  DevBuf inst_grad, exp_part;  // deterministic backward: per-instance gradients, per-tile exposure sums
  DevBuf dbg_g;                // Gaussian index per instance in blend order (inspection only)
  DevBuf gr_rgb, gr_T, gr_flags, gr_off, gr_tmp, gr_d2;  // map growth: render, selection, scan, sky
  bool deterministic = false;
  bool fused_step = true;      // gs_step applies Adam inside the projection backward
  bool grads_dirty = false;    // gradient planes may hold non-zero values (a backward without Adam,
                               // or their pointer was handed out)
  bool step_assumed_clean = false;  // the last fused gs_step skipped reading the gradient planes
  bool dirty_step_since_check = false;  // a fused step read gradient planes since the last overflow check
  int64_t serve_peak = 0;   // largest instance count of the last keyframe job (gs_submit_keyframe)
  int serve_views = 0;      // its window size
  int fwd_px = 1, bwd_px = 1;  // pixels per lane of the blend kernels (fastest measured at 1280x720)
  int32_t split_par = 4096, split_min = 128;  // long-list split (SplitArg)
  float split_balance = 1.25f;
  SplitArg last_sp{};          // split of the last render, used by its backward
  int bwd_mode = 0;            // 0: pixel-order backward blend, 1: per-Gaussian (the forward keeps pre colour)
  uint32_t* d_nvn = nullptr;   // number of (view, Gaussian) pairs of the last render
  int64_t vn_cap = 0, inst_cap = 0, tiles_cap = 0, pix_cap = 0;
  bool sync_plan = true;
  // last render
  bool have_render = false;
  ViewsArg last_va{};
  int32_t last_N = 0;
  int sorted = 0;
  bool last_det = false;       // the last render wrote what the deterministic backward reads
  // keyframe window
  std::vector<KeyframeSlot> kf;
  int kf_next = 0;
  // all keyframes (random-K schedule) and the single-view buffers its steps share
  std::vector<ArchivedKeyframe> archive;
  // frame intake (gs_add_frame): frames seen, points of the frames since the last keyframe
  int64_t frames_seen = 0;
  DevBuf pend_xyz, pend_rgb;
  int64_t pend_n = 0;
  DevBuf ar_rgb, ar_T, ar_nc, ar_dl;
  // per-stage timing: event pairs recorded since the last query
  bool timing = false;
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  std::vector<std::pair<int, size_t>> ev_marks;  // (stage, index of its start event)
  bool capturing = false;      // inside gs_capture_step: no allocation, no timing, no host wait
  uint64_t epoch = 0;          // bumped whenever a device buffer of the map is reallocated
  int64_t render_gen = 0;      // renders so far (eager, inside steps and jobs, graph replays)
};

struct gs_step_graph {
  gs_map* map = nullptr;
  bool assumes_clean = false;  // captured with the gradient-plane read skipped
  uint64_t epoch = 0;          // the map's buffer epoch, row count and capacity at capture:
  int64_t n = 0, cap = 0;      // a replay after any of them changed would use stale pointers
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

void* dev_alloc(gs_map* m, size_t bytes, hipStream_t s) {
  if (bytes == 0) bytes = 256;
  bytes = (bytes + 255) & ~size_t(255);
  void* p = nullptr;
  if (m->has_alloc) {
    p = m->alloc.alloc(bytes, (void*)s, m->alloc.ctx);
  } else if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    p = nullptr;
  }
  if (p) m->resident += (int64_t)bytes;
  return p;
}

void dev_free(gs_map* m, void* p, size_t bytes, hipStream_t s) {
  if (!p) return;
  if (bytes == 0) bytes = 256;
  bytes = (bytes + 255) & ~size_t(255);
  m->resident -= (int64_t)bytes;
  if (m->has_alloc)
    m->alloc.free(p, (void*)s, m->alloc.ctx);
  else
    (void)hipFree(p);
}

// Grow `b` to at least `bytes` (contents dropped). zero: clear the new buffer.
gs_status ensure(gs_map* m, DevBuf& b, size_t bytes, hipStream_t s, bool zero = false) {
  if (b.bytes >= bytes && b.ptr) return GS_OK;
  if (m->capturing)
    return fail(GS_ERR_STATE, "capture would allocate: run an eager gs_step with the same views first");
  void* p = dev_alloc(m, bytes, s);
  if (!p) return fail(GS_ERR_OOM, "device allocation of " + std::to_string(bytes) + " bytes failed");
  dev_free(m, b.ptr, b.bytes, s);
  b.ptr = p;
  b.bytes = bytes;
  m->epoch += 1;
  if (zero) {
    hipError_t e = fill_u32((uint32_t*)p, 0u, (int64_t)((bytes + 3) / 4), s);
    if (e != hipSuccess) return fail(GS_ERR_HIP, hipGetErrorString(e));
  }
  return GS_OK;
}

float* params_of(gs_map* m) { return m->buf; }
float* grads_of(gs_map* m) { return m->buf + (int64_t)m->F * m->cap; }

gs_status grow_capacity(gs_map* m, int64_t need, hipStream_t s) {
  if (need <= m->cap) return GS_OK;
  // kernels address a row of a parameter plane with a 32-bit byte offset
  constexpr int64_t kMaxCapacity = int64_t(1) << 30;
  if (need > kMaxCapacity) return fail(GS_ERR_CAPACITY, "more than 2^30 Gaussians in one map");
  int64_t nc = std::min<int64_t>(kMaxCapacity, std::max<int64_t>(need, std::max<int64_t>(1024, 2 * m->cap)));
  const size_t fbytes = (size_t)4 * m->F * nc * sizeof(float);
  const size_t vbytes = (size_t)((nc + 3) / 4) * 4;
  float* nb = (float*)dev_alloc(m, fbytes, s);
  if (!nb) return fail(GS_ERR_OOM, "map growth to " + std::to_string(nc) + " Gaussians failed");
  uint8_t* nv = (uint8_t*)dev_alloc(m, vbytes, s);
  if (!nv) {
    dev_free(m, nb, fbytes, s);
    return fail(GS_ERR_OOM, "map growth (visibility) failed");
  }
  GS_HIP(fill_u32((uint32_t*)nv, 0u, (int64_t)(vbytes / 4), s));
  if (m->n > 0) {
    GS_HIP(copy_planes(m->buf, m->cap, nb, nc, m->n, 4 * m->F, s));
    GS_HIP(hipMemcpyAsync(nv, m->vis, (size_t)m->n, hipMemcpyDeviceToDevice, s));
  }
  if (m->buf) {
    // the old buffers may still be read by queued work on this stream
    GS_HIP(hipStreamSynchronize(s));
    dev_free(m, m->buf, (size_t)4 * m->F * m->cap * sizeof(float), s);
    dev_free(m, m->vis, (size_t)((m->cap + 3) / 4) * 4, s);
  }
  m->buf = nb;
  m->vis = nv;
  m->cap = nc;
  m->have_render = false;
  m->epoch += 1;
  return GS_OK;
}

gs_status ensure_instances(gs_map* m, int64_t nc, int64_t vn, hipStream_t s) {
  for (int b = 0; b < 2; ++b) {
    GS_TRY(ensure(m, m->keys[b], (size_t)nc * 4, s));
    GS_TRY(ensure(m, m->vals[b], (size_t)nc * 4, s));
  }
  GS_TRY(ensure(m, m->emit_g, (size_t)nc * 4, s));
  GS_TRY(ensure(m, m->block_start, (size_t)block_start_elems(nc) * 4, s));
  if (m->deterministic) GS_TRY(ensure(m, m->inst_grad, (size_t)nc * 12 * 4, s));
  GS_TRY(ensure(m, m->sort_tmp, (size_t)sort_temp_elems(std::max<int64_t>(nc, vn)) * 4, s));
  if (nc > m->inst_cap) m->inst_cap = nc;
  return GS_OK;
}

SplitArg split_arg(gs_map* m, int64_t tiles) {
  SplitArg sp{};
  sp.par = m->split_par;
  sp.min_len = m->split_min;
  sp.balance = m->split_balance;
  sp.tile_slot = (uint32_t*)m->split_slot.ptr;
  sp.extra = (uint2*)m->split_extra.ptr;
  sp.counts = (uint32_t*)m->ranges.ptr + 2 * tiles;
  sp.n_inst = m->d_ninst;
  sp.state = (float*)m->split_state.ptr;
  return sp;
}

LrArg lr_table(const gs_map* m) {
  LrArg lr{};
  const gs_map_desc& d = m->desc;
  for (int f = 0; f < m->F; ++f) {
    float r = d.lr_sh_rest;
    if (f < 3) r = d.lr_mean;
    else if (f < 6) r = d.lr_log_scale;
    else if (f < 10) r = d.lr_quat;
    else if (f < 11) r = d.lr_opacity;
    else if (f < 14) r = d.lr_sh_dc;
    lr.lr[f] = r;
  }
  return lr;
}

int bits_for(int64_t x) {
  int b = 0;
  while ((int64_t(1) << b) < x) ++b;
  return std::max(b, 1);
}

gs_status check_view(const gs_view& v, int idx) {
  if (v.width < 1 || v.height < 1 || v.width > 16384 || v.height > 16384)
    return fail(GS_ERR_INVALID, "view " + std::to_string(idx) + ": size out of range");
  const float vals[] = {v.fx, v.fy, v.cx, v.cy};
  for (float f : vals)
    if (!std::isfinite(f)) return fail(GS_ERR_INVALID, "view " + std::to_string(idx) + ": non-finite intrinsics");
  if (!(v.fx > 0.f) || !(v.fy > 0.f))
    return fail(GS_ERR_INVALID, "view " + std::to_string(idx) + ": focal length must be positive");
  for (int k = 0; k < 9; ++k)
    if (!std::isfinite(v.R_cw[k])) return fail(GS_ERR_INVALID, "view " + std::to_string(idx) + ": non-finite pose");
  for (int k = 0; k < 3; ++k)
    if (!std::isfinite(v.t_cw[k])) return fail(GS_ERR_INVALID, "view " + std::to_string(idx) + ": non-finite pose");
  return GS_OK;
}

void fill_viewdev(ViewDev& d, const gs_view& v) {
  std::memcpy(d.R, v.R_cw, sizeof(d.R));
  std::memcpy(d.t, v.t_cw, sizeof(d.t));
  d.fx = v.fx;
  d.fy = v.fy;
  d.cx = v.cx;
  d.cy = v.cy;
  // the projection's clamp of the view-space slope (FP32, as the kernels formed it)
  d.limx = 1.3f * ((0.5f * (float)v.width) / v.fx);
  d.limy = 1.3f * ((0.5f * (float)v.height) / v.fy);
  for (int k = 0; k < 3; ++k) {
    double c = 0.0;
    for (int r = 0; r < 3; ++r) c -= (double)v.R_cw[3 * r + k] * (double)v.t_cw[r];
    d.campos[k] = (float)c;
    d.bg[k] = v.bg[k];
  }
  d.W = v.width;
  d.H = v.height;
  d.tiles_x = (v.width + kTile - 1) / kTile;
  d.tiles_y = (v.height + kTile - 1) / kTile;
  d.exposure = v.exposure;
  d.dl_drgb = nullptr;
  d.dl_dexp = nullptr;
  d.out_depth = nullptr;
  d.out_opac = nullptr;
  d.dl_ddepth = nullptr;
  d.dl_dopac = nullptr;
}

// Records a start event for `stage` (when timing is on); stage_end records the stop.
struct StageTimer {
  gs_map* m;
  hipStream_t s;
  int stage;
  size_t idx = 0;
  bool on = false;
  StageTimer(gs_map* m_, hipStream_t s_, int st) : m(m_), s(s_), stage(st) {
    if (!m->timing || m->capturing) return;
    while (m->ev_pool.size() < m->ev_used + 2) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return;
      m->ev_pool.push_back(e);
    }
    idx = m->ev_used;
    m->ev_used += 2;
    on = hipEventRecord(m->ev_pool[idx], s) == hipSuccess;
  }
  ~StageTimer() {
    if (on && hipEventRecord(m->ev_pool[idx + 1], s) == hipSuccess) m->ev_marks.emplace_back(stage, idx);
  }
};

// Keeps a keyframe for the session (pose, a copy of its image, an identity exposure with
// zero gradient and moments) and reports its id.
gs_status archive_keyframe(gs_map* m, const gs_view* view, const float* image, int32_t* keyframe_id,
                           hipStream_t s) {
  ArchivedKeyframe a;
  a.pix_bytes = (size_t)view->width * view->height * sizeof(float);
  a.image = (float*)dev_alloc(m, 3 * a.pix_bytes, s);
  a.state = (float*)dev_alloc(m, GS_EXPOSURE_STATE_FLOATS * sizeof(float), s);
  if (!a.image || !a.state) {
    dev_free(m, a.image, 3 * a.pix_bytes, s);
    dev_free(m, a.state, GS_EXPOSURE_STATE_FLOATS * sizeof(float), s);
    return fail(GS_ERR_OOM, "keyframe buffers");
  }
  GS_HIP(hipMemcpyAsync(a.image, image, 3 * a.pix_bytes, hipMemcpyDeviceToDevice, s));
  GS_HIP(fill_u32((uint32_t*)a.state, 0u, GS_EXPOSURE_STATE_FLOATS, s));
  GS_HIP(fill_u32((uint32_t*)a.state + 0, 0x3f800000u, 1, s));
  GS_HIP(fill_u32((uint32_t*)a.state + 5, 0x3f800000u, 1, s));
  GS_HIP(fill_u32((uint32_t*)a.state + 10, 0x3f800000u, 1, s));
  a.view = *view;
  a.view.exposure = a.state;
  m->archive.push_back(a);
  if (keyframe_id) *keyframe_id = (int32_t)(m->archive.size() - 1);
  return GS_OK;
}

}  // namespace

extern "C" {

void gs_default_desc(gs_map_desc* d) {
  if (!d) return;
  std::memset(d, 0, sizeof(*d));
  d->sh_degree = 3;
  d->initial_capacity = 1 << 16;
  d->near_z = 0.2f;
  d->lr_mean = 1.6e-4f;
  d->lr_log_scale = 5e-3f;
  d->lr_quat = 1e-3f;
  d->lr_opacity = 5e-2f;
  d->lr_sh_dc = 2.5e-3f;
  d->lr_sh_rest = 2.5e-3f / 20.0f;
  d->lr_exposure = 1e-3f;
  d->beta1 = 0.9f;
  d->beta2 = 0.999f;
  d->eps = 1e-15f;
  d->expand_tau = 0.99f;
}

const char* gs_last_error(void) { return g_err.c_str(); }

gs_status gs_create_map(const gs_map_desc* desc, const gs_allocator* allocator, gs_map** out) {
  g_err.clear();
  if (!desc || !out) return fail(GS_ERR_INVALID, "desc and out must not be NULL");
  *out = nullptr;
  if (desc->sh_degree < 0 || desc->sh_degree > 3) return fail(GS_ERR_INVALID, "sh_degree must be 0..3");
  if (desc->initial_capacity < 0) return fail(GS_ERR_INVALID, "initial_capacity must be >= 0");
  if (!(desc->near_z > 0.f)) return fail(GS_ERR_INVALID, "near_z must be > 0");
  if (allocator && (!allocator->alloc || !allocator->free))
    return fail(GS_ERR_INVALID, "allocator needs both alloc and free");
  gs_map* m = new (std::nothrow) gs_map();
  if (!m) return fail(GS_ERR_OOM, "host allocation failed");
  m->desc = *desc;
  if (allocator) {
    m->alloc = *allocator;
    m->has_alloc = true;
  }
  m->deg = desc->sh_degree;
  m->K = (m->deg + 1) * (m->deg + 1);
  m->F = 11 + 3 * m->K;
  hipStream_t s = nullptr;
  m->d_step = (int64_t*)dev_alloc(m, 64, s);
  m->d_bc = (float*)dev_alloc(m, 64, s);
  m->d_ninst = (uint32_t*)dev_alloc(m, 64, s);
  m->d_overflow = (uint32_t*)dev_alloc(m, 64, s);
  m->d_loss = (float*)dev_alloc(m, 256, s);
  m->d_nvn = (uint32_t*)dev_alloc(m, 64, s);
  if (!m->d_step || !m->d_bc || !m->d_ninst || !m->d_overflow || !m->d_loss || !m->d_nvn) {
    gs_destroy_map(m);
    return fail(GS_ERR_OOM, "device allocation failed");
  }
  if (hipHostMalloc((void**)&m->h_pinned, 64, hipHostMallocDefault) != hipSuccess) {
    m->h_pinned = nullptr;
    gs_destroy_map(m);
    return fail(GS_ERR_HIP, "pinned host allocation failed");
  }
  hipError_t e = fill_u32((uint32_t*)m->d_step, 0u, 16, s);
  if (e == hipSuccess) e = fill_u32(m->d_overflow, 0u, 16, s);
  if (e == hipSuccess) e = fill_u32(m->d_ninst, 0u, 16, s);
  if (e != hipSuccess) {
    gs_destroy_map(m);
    return fail(GS_ERR_HIP, hipGetErrorString(e));
  }
  if (desc->initial_capacity > 0) {
    gs_status st = grow_capacity(m, desc->initial_capacity, s);
    if (st != GS_OK) {
      std::string msg = g_err;
      gs_destroy_map(m);
      return fail(st, msg);
    }
  }
  if (hipStreamSynchronize(s) != hipSuccess) {
    gs_destroy_map(m);
    return fail(GS_ERR_HIP, "initialisation failed");
  }
  *out = m;
  return GS_OK;
}

gs_status gs_destroy_map(gs_map* m) {
  if (!m) return GS_OK;
  (void)hipDeviceSynchronize();
  hipStream_t s = nullptr;
  dev_free(m, m->buf, (size_t)4 * m->F * m->cap * sizeof(float), s);
  dev_free(m, m->vis, (size_t)((m->cap + 3) / 4) * 4, s);
  dev_free(m, m->d_step, 64, s);
  dev_free(m, m->d_bc, 64, s);
  dev_free(m, m->d_ninst, 64, s);
  dev_free(m, m->d_overflow, 64, s);
  dev_free(m, m->d_loss, 256, s);
  dev_free(m, m->d_nvn, 64, s);
  DevBuf* bufs[] = {&m->rec, &m->counts, &m->offsets, &m->scan_tmp, &m->g2d, &m->keys[0], &m->keys[1],
                    &m->vals[0], &m->vals[1], &m->sort_tmp, &m->ranges, &m->pixT, &m->pixN, &m->loss_tmp,
                    &m->dkey[0], &m->dkey[1], &m->dval[0], &m->dval[1], &m->emit_g, &m->inst_off,
                    &m->block_start, &m->split_slot, &m->split_extra, &m->split_state,
                    &m->inst_grad, &m->exp_part, &m->dbg_g, &m->gr_rgb, &m->gr_T, &m->gr_flags,
                    &m->gr_off, &m->gr_tmp, &m->gr_d2, &m->ar_rgb, &m->ar_T, &m->ar_nc, &m->ar_dl,
                    &m->pend_xyz, &m->pend_rgb};
  for (DevBuf* b : bufs) dev_free(m, b->ptr, b->bytes, s);
  for (KeyframeSlot& k : m->kf) {
    dev_free(m, k.image, 3 * k.pix_bytes, s);
    dev_free(m, k.rgb, 3 * k.pix_bytes, s);
    dev_free(m, k.dl, 3 * k.pix_bytes, s);
    dev_free(m, k.T, k.pix_bytes, s);
    dev_free(m, k.nc, k.pix_bytes, s);
    dev_free(m, k.state, GS_EXPOSURE_STATE_FLOATS * sizeof(float), s);
  }
  for (ArchivedKeyframe& a : m->archive) {
    dev_free(m, a.image, 3 * a.pix_bytes, s);
    dev_free(m, a.state, GS_EXPOSURE_STATE_FLOATS * sizeof(float), s);
  }
  if (m->h_pinned) (void)hipHostFree(m->h_pinned);
  for (hipEvent_t e : m->ev_pool) (void)hipEventDestroy(e);
  delete m;
  return GS_OK;
}

gs_status gs_add_gaussians(gs_map* m, int64_t n, const float* means, const float* log_scales, const float* quats,
                           const float* opacity_logits, const float* sh, void* stream) {
  g_err.clear();
  if (!m) return fail(GS_ERR_INVALID, "map is NULL");
  if (n < 0) return fail(GS_ERR_INVALID, "n must be >= 0");
  if (n == 0) return GS_OK;
  if (!means || !log_scales || !quats || !opacity_logits || !sh)
    return fail(GS_ERR_INVALID, "input pointers must not be NULL");
  if (m->n + n > (int64_t)INT32_MAX) return fail(GS_ERR_CAPACITY, "more than 2^31-1 Gaussians");
  hipStream_t s = (hipStream_t)stream;
  GS_TRY(grow_capacity(m, m->n + n, s));
  GS_HIP(append_rows(m->buf, m->cap, m->F, m->K, m->n, n, means, log_scales, quats, opacity_logits, sh, m->vis, s));
  m->n += n;
  m->have_render = false;
  return GS_OK;
}

gs_status gs_add_points(gs_map* m, int64_t n, const float* xyz, const float* rgb, const gs_view* view, float o_init,
                        void* stream) {
  g_err.clear();
  if (!m || !view) return fail(GS_ERR_INVALID, "map and view must not be NULL");
  if (n < 0) return fail(GS_ERR_INVALID, "n must be >= 0");
  if (n == 0) return GS_OK;
  if (!xyz || !rgb) return fail(GS_ERR_INVALID, "xyz and rgb must not be NULL");
  if (!(o_init > 0.f && o_init < 1.f)) return fail(GS_ERR_INVALID, "o_init must be in (0, 1)");
  GS_TRY(check_view(*view, 0));
  if (m->n + n > (int64_t)INT32_MAX) return fail(GS_ERR_CAPACITY, "more than 2^31-1 Gaussians");
  hipStream_t s = (hipStream_t)stream;
  GS_TRY(grow_capacity(m, m->n + n, s));
  ViewDev V{};
  fill_viewdev(V, *view);
  const float logit0 = std::log(o_init / (1.0f - o_init));
  GS_HIP(init_points(m->buf, m->cap, m->F, m->K, m->n, n, xyz, rgb, V, m->desc.near_z, logit0, m->vis, s));
  m->n += n;
  m->have_render = false;
  return GS_OK;
}

gs_status gs_expand(gs_map* m, const gs_view* view, int64_t n, const float* xyz, const float* rgb, float tau,
                    float o_init, int64_t* n_added, void* stream) {
  g_err.clear();
  if (n_added) *n_added = 0;
  if (!m || !view) return fail(GS_ERR_INVALID, "map and view must not be NULL");
  if (n < 0) return fail(GS_ERR_INVALID, "n must be >= 0");
  if (!(tau > 0.f)) return fail(GS_ERR_INVALID, "tau must be > 0");
  if (!(o_init > 0.f && o_init < 1.f)) return fail(GS_ERR_INVALID, "o_init must be in (0, 1)");
  if (n == 0) return GS_OK;
  if (!xyz || !rgb) return fail(GS_ERR_INVALID, "xyz and rgb must not be NULL");
  if (m->capturing) return fail(GS_ERR_STATE, "expansion waits on the host and cannot be captured");
  GS_TRY(check_view(*view, 0));
  if (m->n + n > (int64_t)INT32_MAX) return fail(GS_ERR_CAPACITY, "more than 2^31-1 Gaussians");
  if (n > (int64_t)UINT32_MAX) return fail(GS_ERR_CAPACITY, "too many points");
  hipStream_t s = (hipStream_t)stream;
  // O = 1 - T_final of the current map at the keyframe view
  const int64_t P = (int64_t)view->width * view->height;
  GS_TRY(ensure(m, m->gr_rgb, (size_t)P * 3 * 4, s));
  GS_TRY(ensure(m, m->gr_T, (size_t)P * 4, s));
  gs_frame fr{(float*)m->gr_rgb.ptr, (float*)m->gr_T.ptr, nullptr, nullptr, nullptr};
  GS_TRY(gs_render(m, 1, view, &fr, stream));
  m->have_render = false;  // the map grows below; this render has no backward
  GS_TRY(ensure(m, m->gr_flags, (size_t)n * 4, s));
  GS_TRY(ensure(m, m->gr_off, (size_t)n * 4, s));
  GS_TRY(ensure(m, m->gr_tmp, (size_t)scan_temp_elems(n) * 4, s));
  uint32_t* flags = (uint32_t*)m->gr_flags.ptr;
  uint32_t* off = (uint32_t*)m->gr_off.ptr;
  ViewDev V{};
  fill_viewdev(V, *view);
  GS_HIP(expand_flags(xyz, n, V, (const float*)m->gr_T.ptr, tau, m->desc.near_z, flags, s));
  GS_HIP(exclusive_scan(flags, off, n, (uint32_t*)m->gr_tmp.ptr, s));
  GS_HIP(hipMemcpyAsync(m->h_pinned, off + (n - 1), 4, hipMemcpyDeviceToHost, s));
  GS_HIP(hipMemcpyAsync(m->h_pinned + 1, flags + (n - 1), 4, hipMemcpyDeviceToHost, s));
  GS_HIP(hipStreamSynchronize(s));
  const int64_t k = (int64_t)m->h_pinned[0] + (int64_t)m->h_pinned[1];
  if (k > 0) {
    GS_TRY(grow_capacity(m, m->n + k, s));
    const float logit0 = std::log(o_init / (1.0f - o_init));
    GS_HIP(init_selected(m->buf, m->cap, m->F, m->K, m->n, n, xyz, rgb, flags, off, V, m->desc.near_z, logit0,
                         m->vis, s));
    m->n += k;
  }
  if (n_added) *n_added = k;
  return GS_OK;
}

gs_status gs_add_sky(gs_map* m, int64_t n, const float* xyz, float o_sky, void* stream) {
  g_err.clear();
  if (!m) return fail(GS_ERR_INVALID, "map is NULL");
  if (n == 0) return GS_OK;
  if (n < 2) return fail(GS_ERR_INVALID, "sky initialisation needs n >= 2 (nearest-neighbour scale)");
  if (!xyz) return fail(GS_ERR_INVALID, "xyz must not be NULL");
  if (!(o_sky > 0.f && o_sky < 1.f)) return fail(GS_ERR_INVALID, "o_sky must be in (0, 1)");
  if (m->n + n > (int64_t)INT32_MAX) return fail(GS_ERR_CAPACITY, "more than 2^31-1 Gaussians");
  hipStream_t s = (hipStream_t)stream;
  GS_TRY(ensure(m, m->gr_d2, (size_t)n * 4, s));
  GS_TRY(grow_capacity(m, m->n + n, s));
  const float logit0 = std::log(o_sky / (1.0f - o_sky));
  GS_HIP(init_sky(m->buf, m->cap, m->F, m->K, m->n, n, xyz, (float*)m->gr_d2.ptr, logit0, m->vis, s));
  m->n += n;
  m->have_render = false;
  return GS_OK;
}

gs_status gs_render(gs_map* m, int32_t nv, const gs_view* views, const gs_frame* frames, void* stream) {
  g_err.clear();
  if (!m || !views || !frames) return fail(GS_ERR_INVALID, "map, views and frames must not be NULL");
  if (nv < 1 || nv > kMaxViews) return fail(GS_ERR_CAPACITY, "n_views must be in 1..16");
  hipStream_t s = (hipStream_t)stream;
  ViewsArg va{};
  va.n = nv;
  int64_t tiles = 0, pix = 0;
  for (int v = 0; v < nv; ++v) {
    GS_TRY(check_view(views[v], v));
    if (!frames[v].rgb) return fail(GS_ERR_INVALID, "frame " + std::to_string(v) + ": rgb must not be NULL");
    fill_viewdev(va.v[v], views[v]);
    va.v[v].tile_base = (int32_t)tiles;
    va.v[v].pix_base = pix;
    tiles += (int64_t)va.v[v].tiles_x * va.v[v].tiles_y;
    pix += (int64_t)views[v].width * views[v].height;
  }
  if (tiles >= (int64_t(1) << 31)) return fail(GS_ERR_CAPACITY, "too many tiles");
  va.total_tiles = (int32_t)tiles;
  const int32_t N = (int32_t)m->n;
  const int64_t vn = (int64_t)nv * N;
  // workspace
  GS_TRY(ensure(m, m->rec, (size_t)std::max<int64_t>(vn, 1) * kRecFloats * 4, s));
  GS_TRY(ensure(m, m->counts, (size_t)std::max<int64_t>(vn, 1) * 4, s));
  GS_TRY(ensure(m, m->offsets, (size_t)std::max<int64_t>(vn, 1) * 4, s));
  GS_TRY(ensure(m, m->scan_tmp, (size_t)scan_temp_elems(std::max<int64_t>(vn, 1)) * 4, s));
  GS_TRY(ensure(m, m->g2d, (size_t)std::max<int64_t>(vn, 1) * kGradFloats * 4, s, true));
  for (int b = 0; b < 2; ++b) {
    GS_TRY(ensure(m, m->dkey[b], (size_t)std::max<int64_t>(vn, 1) * 4, s));
    GS_TRY(ensure(m, m->dval[b], (size_t)std::max<int64_t>(vn, 1) * 4, s));
  }
  GS_TRY(ensure(m, m->inst_off, (size_t)std::max<int64_t>(vn, 1) * 4, s));
  GS_TRY(ensure(m, m->exp_part, (size_t)std::max<int64_t>(tiles, 1) * 12 * 4, s));
  GS_TRY(ensure(m, m->sort_tmp, (size_t)sort_temp_elems(std::max<int64_t>(std::max<int64_t>(vn, m->inst_cap), 1)) * 4,
                s));
  GS_TRY(ensure(m, m->ranges, (size_t)tiles * 8 + 16, s));  // + the split counters
  if (m->split_par > 0) {
    const size_t par = (size_t)m->split_par;
    GS_TRY(ensure(m, m->split_slot, (size_t)std::max<int64_t>(tiles, 1) * 4, s));
    GS_TRY(ensure(m, m->split_extra, par * 8, s));
    GS_TRY(ensure(m, m->split_state, 2 * par * kSplitFields * kTile * kTile * 4, s));
  }
  GS_TRY(ensure(m, m->pixT, (size_t)pix * 4, s));
  GS_TRY(ensure(m, m->pixN, (size_t)pix * 4, s));
  for (int v = 0; v < nv; ++v) {
    ViewDev& d = va.v[v];
    d.out_rgb = frames[v].rgb;
    d.out_T = frames[v].final_T ? frames[v].final_T : (float*)m->pixT.ptr + d.pix_base;
    d.out_nc = frames[v].n_contrib ? frames[v].n_contrib : (uint32_t*)m->pixN.ptr + d.pix_base;
    d.out_depth = frames[v].depth;
    d.out_opac = frames[v].opacity;
  }
  float4* rec = (float4*)m->rec.ptr;
  uint32_t* counts = (uint32_t*)m->counts.ptr;
  uint32_t* offsets = (uint32_t*)m->offsets.ptr;
  uint32_t* dkey[2] = {(uint32_t*)m->dkey[0].ptr, (uint32_t*)m->dkey[1].ptr};
  uint32_t* dval[2] = {(uint32_t*)m->dval[0].ptr, (uint32_t*)m->dval[1].ptr};
  {
    StageTimer t(m, s, GS_STAGE_PROJECT);
    // on the side: the pair count the depth sort reads, and the tile ranges (with the split
    // counters after them) zeroed for this render
    const ProjSide side{m->d_nvn, (uint32_t)vn, (uint32_t*)m->ranges.ptr, 2 * tiles + 2};
    GS_HIP(project_forward(m->deg, params_of(m), m->cap, N, va, m->desc.near_z, rec, counts, dkey[0], side, s));
  }
  int dwhich = 0;
  {
    StageTimer t(m, s, GS_STAGE_DEPTH_SORT);
    GS_HIP(radix_sort_u32(dkey, dval, m->d_nvn, vn, 32, (uint32_t*)m->sort_tmp.ptr, &dwhich, s, true));
  }
  const uint32_t* order = dval[dwhich];
  // the instance buffers of the current capacity exist before the scan of the counts, which
  // marks the emission blocks' first pairs for that capacity
  if (m->inst_cap > 0) GS_TRY(ensure_instances(m, m->inst_cap, vn, s));
  const int64_t marked_cap = m->inst_cap;
  {
    StageTimer t(m, s, GS_STAGE_SCAN);
    if (vn > 0)
      GS_HIP(scan_counts(counts, order, offsets, vn, (uint32_t*)m->scan_tmp.ptr, m->d_ninst,
                         (uint32_t*)m->block_start.ptr, marked_cap, s));
    else
      GS_HIP(fill_u32(m->d_ninst, 0u, 1, s));
  }
  if (m->sync_plan && m->capturing) return fail(GS_ERR_STATE, "capture needs sync_plan = 0");
  if (m->sync_plan) {
    GS_HIP(hipMemcpyAsync(m->h_pinned, m->d_ninst, 4, hipMemcpyDeviceToHost, s));
    GS_HIP(hipStreamSynchronize(s));
    const int64_t need = m->h_pinned[0];
    if (need > m->inst_cap) GS_TRY(ensure_instances(m, std::max<int64_t>(need + need / 4, 1 << 16), vn, s));
  } else if (m->inst_cap == 0) {
    return fail(GS_ERR_STATE, "sync_plan = 0 needs an instance capacity (gs_set_instance_policy)");
  }
  GS_TRY(ensure_instances(m, m->inst_cap, vn, s));
  // the backward of this render checks these: a render that dropped its instances has none
  va.n_inst = m->d_ninst;
  va.inst_cap = m->inst_cap;
  uint32_t* keys[2] = {(uint32_t*)m->keys[0].ptr, (uint32_t*)m->keys[1].ptr};
  uint32_t* vals[2] = {(uint32_t*)m->vals[0].ptr, (uint32_t*)m->vals[1].ptr};
  {
    StageTimer t(m, s, GS_STAGE_DUPLICATE);
    GS_HIP(duplicate_keys(rec, counts, order, offsets, m->d_ninst, N, va, keys[0], (uint32_t*)m->emit_g.ptr, (uint32_t*)m->inst_off.ptr, m->deterministic,
                          (uint32_t*)m->block_start.ptr, marked_cap > 0 && marked_cap == m->inst_cap, m->inst_cap,
                          m->d_overflow, s));
  }
  int which = 0;
  {
    // stable sort by tile id; one extra bit keeps the sentinel id above every real tile
    StageTimer t(m, s, GS_STAGE_SORT);
    GS_HIP(radix_sort_u32(keys, vals, m->d_ninst, m->inst_cap, bits_for(tiles + 1), (uint32_t*)m->sort_tmp.ptr,
                          &which, s, true));
  }
  uint2* ranges = (uint2*)m->ranges.ptr;
  {
    StageTimer t(m, s, GS_STAGE_RANGES);
    GS_HIP(tile_ranges(keys[which], m->d_ninst, m->inst_cap, ranges, tiles, s));
    m->last_sp = split_arg(m, tiles);
    GS_HIP(split_items(ranges, (int32_t)tiles, m->last_sp, s));
  }
  {
    StageTimer t(m, s, GS_STAGE_BLEND);
    GS_HIP(blend_forward(va, rec, N, vals[which], (const uint32_t*)m->emit_g.ptr, ranges, m->last_sp, m->fwd_px,
                         s));
  }
  m->have_render = true;
  m->last_va = va;
  m->last_N = N;
  m->sorted = which;
  m->last_det = m->deterministic;
  if (!m->capturing) m->render_gen += 1;
  return GS_OK;
}

static gs_status backward_impl(gs_map* m, int32_t nv, const float* const* dL_drgb, const float* const* dL_ddepth,
                               const float* const* dL_dopacity, float* const* dL_dexposure, const AdamArg* fused,
                               const LossFinish& lf, hipStream_t s);
static const LossFinish kNoLossFinish{nullptr, nullptr, 0.f, 0};

gs_status gs_render_backward(gs_map* m, int32_t nv, const float* const* dL_drgb, const float* const* dL_ddepth,
                             const float* const* dL_dopacity, float* const* dL_dexposure, void* stream) {
  g_err.clear();
  if (m) m->grads_dirty = true;
  return backward_impl(m, nv, dL_drgb, dL_ddepth, dL_dopacity, dL_dexposure, nullptr, kNoLossFinish,
                       (hipStream_t)stream);
}

static gs_status backward_impl(gs_map* m, int32_t nv, const float* const* dL_drgb, const float* const* dL_ddepth,
                               const float* const* dL_dopacity, float* const* dL_dexposure, const AdamArg* fused,
                               const LossFinish& lf, hipStream_t stream) {
  if (!m || !dL_drgb) return fail(GS_ERR_INVALID, "map and dL_drgb must not be NULL");
  if (!m->have_render) return fail(GS_ERR_STATE, "render_backward needs a preceding render of the same map");
  if (nv != m->last_va.n) return fail(GS_ERR_STATE, "n_views differs from the preceding render");
  if (m->last_N != (int32_t)m->n) return fail(GS_ERR_STATE, "map changed since the render");
  for (int v = 0; v < nv; ++v)
    if (!dL_drgb[v]) return fail(GS_ERR_INVALID, "dL_drgb[" + std::to_string(v) + "] is NULL");
  hipStream_t s = (hipStream_t)stream;
  ViewsArg va = m->last_va;
  for (int v = 0; v < nv; ++v) {
    va.v[v].dl_drgb = dL_drgb[v];
    va.v[v].dl_dexp = dL_dexposure ? dL_dexposure[v] : nullptr;
    va.v[v].dl_ddepth = dL_ddepth ? dL_ddepth[v] : nullptr;
    va.v[v].dl_dopac = dL_dopacity ? dL_dopacity[v] : nullptr;
  }
  const int32_t N = m->last_N;
  float4* rec = (float4*)m->rec.ptr;
  float* g2d = (float*)m->g2d.ptr;
  bool maps = false;
  for (int v = 0; v < nv; ++v) maps = maps || va.v[v].dl_ddepth || va.v[v].dl_dopac;
  {
    StageTimer t(m, s, GS_STAGE_BLEND_BACKWARD);
    // deterministic when the render was (it wrote every pair's first emission index)
    float* ig = m->last_det ? (float*)m->inst_grad.ptr : nullptr;
    if (m->bwd_mode == 1 && !maps)
      GS_HIP(blend_backward_per_gaussian(va, rec, N, (const uint32_t*)m->vals[m->sorted].ptr,
                                         (const uint32_t*)m->emit_g.ptr, (const uint2*)m->ranges.ptr, g2d, ig,
                                         (float*)m->exp_part.ptr, m->last_sp, s));
    else
      GS_HIP(blend_backward(va, rec, N, (const uint32_t*)m->vals[m->sorted].ptr, (const uint32_t*)m->emit_g.ptr,
                            (const uint2*)m->ranges.ptr, g2d, ig, (float*)m->exp_part.ptr, m->last_sp,
                            m->bwd_px, s));
  }
  {
    StageTimer t(m, s, GS_STAGE_PROJECT_BACKWARD);
    GS_HIP(project_backward(m->deg, params_of(m), grads_of(m), m->cap, N, va, m->desc.near_z,
                            (const uint32_t*)m->counts.ptr, (float4*)g2d,
                            m->last_det ? (const float*)m->inst_grad.ptr : nullptr,
                            (const uint32_t*)m->inst_off.ptr, m->vis, fused, lf, s));
  }
  return GS_OK;
}

gs_status gs_adam_step(gs_map* m, int32_t ne, float* const* exposure_states, void* stream) {
  g_err.clear();
  if (!m) return fail(GS_ERR_INVALID, "map is NULL");
  if (ne < 0 || ne > kMaxExposures) return fail(GS_ERR_CAPACITY, "n_exposures must be in 0..64");
  if (ne > 0 && !exposure_states) return fail(GS_ERR_INVALID, "exposure_states is NULL");
  ExpArg ea{};
  ea.n = ne;
  for (int e = 0; e < ne; ++e) {
    if (!exposure_states[e]) return fail(GS_ERR_INVALID, "exposure_states[" + std::to_string(e) + "] is NULL");
    ea.p[e] = exposure_states[e];
  }
  const LrArg lr = lr_table(m);
  const gs_map_desc& d = m->desc;
  hipStream_t s = (hipStream_t)stream;
  StageTimer t(m, s, GS_STAGE_ADAM);
  GS_HIP(adam_step(m->buf, m->cap, m->F, (int32_t)m->n, m->vis, lr, m->d_step, m->d_bc, d.beta1, d.beta2, d.eps,
                   ea, d.lr_exposure, s));
  if (m->n > 0) GS_HIP(fill_u32((uint32_t*)m->vis, 0u, (m->n + 3) / 4, s));
  m->grads_dirty = false;  // every row with a gradient was visible and had it cleared
  m->h_step += 1;
  return GS_OK;
}

static gs_status check_loss_view(const float* out, const float* gt, int32_t H, int32_t W, const float* loss_dev,
                                 const float* dL_dout) {
  if (!out || !gt || !loss_dev || !dL_dout) return fail(GS_ERR_INVALID, "NULL argument");
  if (H < 1 || W < 1 || H > 16384 || W > 16384) return fail(GS_ERR_INVALID, "image size out of range");
  return GS_OK;
}

// One loss launch over la.n images (their sizes and pointers already checked), the
// partial sums in the map's workspace.
// defer_finish: the losses are left to a later launch (LossFinish on loss_tmp).
static gs_status loss_impl(gs_map* m, const LossArg& la, const StepPrep* prep, bool defer_finish, hipStream_t s) {
  if (!(la.lambda >= 0.f && la.lambda <= 1.f)) return fail(GS_ERR_INVALID, "lambda must be in [0, 1]");
  GS_TRY(ensure(m, m->loss_tmp, (size_t)loss_temp_floats_multi(la) * 4, s));
  StageTimer t(m, s, GS_STAGE_LOSS);
  GS_HIP(ssim_loss(la, (float*)m->loss_tmp.ptr, prep, defer_finish, s));
  return GS_OK;
}

static LossArg one_loss_view(const float* out, const float* gt, int32_t H, int32_t W, float lambda, float* loss_dev,
                             float* dL_dout) {
  LossArg la{};
  la.n = 1;
  la.lambda = lambda;
  la.v[0] = LossView{out, gt, dL_dout, loss_dev, H, W, 0, 0};
  return la;
}

gs_status gs_loss(gs_map* m, const float* out, const float* gt, int32_t H, int32_t W, float lambda, float* loss_dev,
                  float* dL_dout, void* stream) {
  g_err.clear();
  if (!m) return fail(GS_ERR_INVALID, "NULL argument");
  GS_TRY(check_loss_view(out, gt, H, W, loss_dev, dL_dout));
  return loss_impl(m, one_loss_view(out, gt, H, W, lambda, loss_dev, dL_dout), nullptr, false, (hipStream_t)stream);
}

// ------------------------------------------------------- loss without allocation
// The loss's per-tile partial sums live in a fixed device array instead of a map's
// workspace. Each GPU holds its own copy; its address is looked up once per device (with
// that device current) and kept, and only that address is handed to kernels.
static __device__ __align__(256) float scratch[GS_LOSS_NOALLOC_SCRATCH_FLOATS];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

gs_status gs_loss_noalloc(const float* out, const float* gt, int32_t H, int32_t W, float lambda, float* loss_dev,
                          float* dL_dout, void* stream) {
  g_err.clear();
  GS_TRY(check_loss_view(out, gt, H, W, loss_dev, dL_dout));
  if (!(lambda >= 0.f && lambda <= 1.f)) return fail(GS_ERR_INVALID, "lambda must be in [0, 1]");
  if (loss_temp_floats(H, W) > GS_LOSS_NOALLOC_SCRATCH_FLOATS)
    return fail(GS_ERR_CAPACITY, "image too large for the fixed loss scratch (" +
                                     std::to_string(loss_temp_floats(H, W)) + " > " +
                                     std::to_string(GS_LOSS_NOALLOC_SCRATCH_FLOATS) + " floats)");
  int dev = -1;
  GS_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(GS_ERR_INVALID, "device ordinal out of range");
  float* part = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
      void* p = nullptr;
      GS_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
      if (!p) return fail(GS_ERR_HIP, "hipGetSymbolAddress returned NULL for the loss scratch");
      g_scratch_ptr[dev] = (float*)p;
    }
    part = g_scratch_ptr[dev];
  }
  // every partial sum the reduction reads is written by the tile kernel first: nothing to clear
  GS_HIP(ssim_loss(one_loss_view(out, gt, H, W, lambda, loss_dev, dL_dout), part, nullptr, false, (hipStream_t)stream));
  return GS_OK;
}

static gs_status read_overflow(gs_map* m, hipStream_t s, uint32_t* flag, uint32_t* skipped, uint32_t* peak);

gs_status gs_submit_keyframe(gs_map* m, const gs_view* view, const float* image, int64_t n_points, const float* xyz,
                             const float* rgb, int32_t iters, int32_t window, float lambda, float o_init,
                             void* done_event, void* stream) {
  g_err.clear();
  if (!m || !view || !image) return fail(GS_ERR_INVALID, "map, view and image must not be NULL");
  if (iters < 0) return fail(GS_ERR_INVALID, "iters must be >= 0");
  if (window < 1 || window > kMaxViews) return fail(GS_ERR_INVALID, "window must be in 1..16");
  if (n_points < 0 || (n_points > 0 && (!xyz || !rgb))) return fail(GS_ERR_INVALID, "bad point arguments");
  GS_TRY(check_view(*view, 0));
  hipStream_t s = (hipStream_t)stream;
  if (n_points > 0) {
    if (m->desc.expand_tau > 0.f)
      GS_TRY(gs_expand(m, view, n_points, xyz, rgb, m->desc.expand_tau, o_init, nullptr, stream));
    else
      GS_TRY(gs_add_points(m, n_points, xyz, rgb, view, o_init, stream));
  }
  // keyframe slot (ring of `window`)
  if ((int)m->kf.size() > window) {
    for (size_t k = window; k < m->kf.size(); ++k) {
      KeyframeSlot& q = m->kf[k];
      dev_free(m, q.image, 3 * q.pix_bytes, s);
      dev_free(m, q.rgb, 3 * q.pix_bytes, s);
      dev_free(m, q.dl, 3 * q.pix_bytes, s);
      dev_free(m, q.T, q.pix_bytes, s);
      dev_free(m, q.nc, q.pix_bytes, s);
      dev_free(m, q.state, GS_EXPOSURE_STATE_FLOATS * sizeof(float), s);
    }
    m->kf.resize(window);
    m->kf_next %= window;
  }
  int slot;
  if ((int)m->kf.size() < window) {
    m->kf.push_back(KeyframeSlot{});
    slot = (int)m->kf.size() - 1;
  } else {
    slot = m->kf_next;
  }
  m->kf_next = (slot + 1) % window;
  KeyframeSlot& k = m->kf[slot];
  const size_t pb = (size_t)view->width * view->height * sizeof(float);
  if (k.pix_bytes != pb) {
    GS_HIP(hipStreamSynchronize(s));
    dev_free(m, k.image, 3 * k.pix_bytes, s);
    dev_free(m, k.rgb, 3 * k.pix_bytes, s);
    dev_free(m, k.dl, 3 * k.pix_bytes, s);
    dev_free(m, k.T, k.pix_bytes, s);
    dev_free(m, k.nc, k.pix_bytes, s);
    k.image = (float*)dev_alloc(m, 3 * pb, s);
    k.rgb = (float*)dev_alloc(m, 3 * pb, s);
    k.dl = (float*)dev_alloc(m, 3 * pb, s);
    k.T = (float*)dev_alloc(m, pb, s);
    k.nc = (uint32_t*)dev_alloc(m, pb, s);
    k.pix_bytes = pb;
    if (!k.image || !k.rgb || !k.dl || !k.T || !k.nc) {
      // leave the slot empty-sized so a later call reallocates it
      dev_free(m, k.image, 3 * pb, s);
      dev_free(m, k.rgb, 3 * pb, s);
      dev_free(m, k.dl, 3 * pb, s);
      dev_free(m, k.T, pb, s);
      dev_free(m, k.nc, pb, s);
      k = KeyframeSlot{};
      m->kf.erase(m->kf.begin() + slot);
      m->kf_next = m->kf.empty() ? 0 : (int)(slot % m->kf.size());
      return fail(GS_ERR_OOM, "keyframe buffers");
    }
  }
  if (!k.state) {
    k.state = (float*)dev_alloc(m, GS_EXPOSURE_STATE_FLOATS * sizeof(float), s);
    if (!k.state) return fail(GS_ERR_OOM, "exposure state");
  }
  GS_HIP(hipMemcpyAsync(k.image, image, 3 * pb, hipMemcpyDeviceToDevice, s));
  // identity exposure, zero gradient and moments
  {
    GS_HIP(fill_u32((uint32_t*)k.state, 0u, GS_EXPOSURE_STATE_FLOATS, s));
    GS_HIP(fill_u32((uint32_t*)k.state + 0, 0x3f800000u, 1, s));
    GS_HIP(fill_u32((uint32_t*)k.state + 5, 0x3f800000u, 1, s));
    GS_HIP(fill_u32((uint32_t*)k.state + 10, 0x3f800000u, 1, s));
  }
  k.view = *view;
  k.view.exposure = k.state;
  const int nk = (int)m->kf.size();
  std::vector<gs_view> vv(nk);
  std::vector<gs_frame> ff(nk);
  std::vector<const float*> tg(nk);
  std::vector<float*> dl(nk), es(nk);
  for (int j = 0; j < nk; ++j) {
    KeyframeSlot& q = m->kf[j];
    vv[j] = q.view;
    ff[j] = gs_frame{q.rgb, q.T, q.nc, nullptr, nullptr};
    tg[j] = q.image;
    dl[j] = q.dl;
    es[j] = q.state;
  }
  // The iterations run without host waits: the instance buffers are sized from the map's
  // previous job (its largest render, scaled to this window, with a quarter to spare; a
  // map's first job plans its first render with a wait). A fused step whose render needs
  // more is skipped on the device (nothing applied) and counted; the job's end reads the
  // counters once, grows the buffers to the largest need and runs the skipped iterations
  // again with planning, so every job applies `iters` steps.
  if (iters > 0) {
    const bool plan_before = m->sync_plan;
    const int64_t vn = (int64_t)nk * m->n;
    int it = 0;
    auto restore = [&](gs_status st) {
      m->sync_plan = plan_before;
      return st;
    };
    if (m->serve_peak == 0 || !m->fused_step) {
      m->sync_plan = true;
      gs_status st = gs_step(m, nk, vv.data(), ff.data(), tg.data(), lambda, es.data(), dl.data(), m->d_loss, stream);
      if (st != GS_OK) return restore(st);
      it = 1;
    }
    if (it < iters) {
      if (!m->fused_step) {
        // the separate update has no skip: plan every render
        for (; it < iters; ++it) {
          gs_status st =
              gs_step(m, nk, vv.data(), ff.data(), tg.data(), lambda, es.data(), dl.data(), m->d_loss, stream);
          if (st != GS_OK) return restore(st);
        }
      } else {
        int64_t est = m->inst_cap;
        if (m->serve_peak > 0 && m->serve_views > 0) {
          const int64_t scaled = m->serve_peak * nk / m->serve_views;
          est = std::max<int64_t>(est, scaled + scaled / 4 + (1 << 16));
        }
        gs_status st = ensure_instances(m, est, vn, s);
        if (st != GS_OK) return restore(st);
        m->sync_plan = false;
        for (; it < iters; ++it) {
          st = gs_step(m, nk, vv.data(), ff.data(), tg.data(), lambda, es.data(), dl.data(), m->d_loss, stream);
          if (st != GS_OK) return restore(st);
        }
      }
    }
    uint32_t flag = 0, skipped = 0, peak = 0;
    gs_status st = read_overflow(m, s, &flag, &skipped, &peak);
    if (st != GS_OK) return restore(st);
    if (skipped > 0) {
      m->sync_plan = true;  // plans (and grows) each render
      for (uint32_t k = 0; k < skipped; ++k) {
        st = gs_step(m, nk, vv.data(), ff.data(), tg.data(), lambda, es.data(), dl.data(), m->d_loss, stream);
        if (st != GS_OK) return restore(st);
      }
      uint32_t f2, s2, p2;
      st = read_overflow(m, s, &f2, &s2, &p2);
      if (st != GS_OK) return restore(st);
      peak = std::max(peak, p2);
    }
    m->serve_peak = std::max<int64_t>(peak, 1);
    m->serve_views = nk;
    m->sync_plan = plan_before;
  }
  if (done_event) GS_HIP(hipEventRecord((hipEvent_t)done_event, s));
  return GS_OK;
}

gs_status gs_add_keyframe(gs_map* m, const gs_view* view, const float* image, int64_t n_points, const float* xyz,
                          const float* rgb, float o_init, int32_t* keyframe_id, void* stream) {
  g_err.clear();
  if (keyframe_id) *keyframe_id = -1;
  if (!m || !view || !image) return fail(GS_ERR_INVALID, "map, view and image must not be NULL");
  if (n_points < 0 || (n_points > 0 && (!xyz || !rgb))) return fail(GS_ERR_INVALID, "bad point arguments");
  if (m->archive.size() >= (size_t)INT32_MAX) return fail(GS_ERR_CAPACITY, "too many keyframes");
  GS_TRY(check_view(*view, 0));
  hipStream_t s = (hipStream_t)stream;
  if (n_points > 0) {
    if (m->desc.expand_tau > 0.f)
      GS_TRY(gs_expand(m, view, n_points, xyz, rgb, m->desc.expand_tau, o_init, nullptr, stream));
    else
      GS_TRY(gs_add_points(m, n_points, xyz, rgb, view, o_init, stream));
  }
  return archive_keyframe(m, view, image, keyframe_id, s);
}

gs_status gs_add_frame(gs_map* m, const gs_view* view, const float* image, int64_t n_points, const float* xyz,
                       const float* rgb, float o_init, int32_t* keyframe_id, void* stream) {
  g_err.clear();
  if (keyframe_id) *keyframe_id = -1;
  if (!m || !view) return fail(GS_ERR_INVALID, "map and view must not be NULL");
  if (n_points < 0 || (n_points > 0 && (!xyz || !rgb))) return fail(GS_ERR_INVALID, "bad point arguments");
  if (!(o_init > 0.f && o_init < 1.f)) return fail(GS_ERR_INVALID, "o_init must be in (0, 1)");
  if (m->capturing) return fail(GS_ERR_STATE, "frame intake cannot be captured");
  GS_TRY(check_view(*view, 0));
  const bool key = m->frames_seen % kKeyframePeriod == 0;
  if (key && !image) return fail(GS_ERR_INVALID, "a keyframe needs its image");
  if (key && m->archive.size() >= (size_t)INT32_MAX) return fail(GS_ERR_CAPACITY, "too many keyframes");
  hipStream_t s = (hipStream_t)stream;
  if (m->frames_seen == 0) {
    // the first frame bootstraps the map with all of its points (Sec. III-C.1)
    if (n_points > 0) GS_TRY(gs_add_points(m, n_points, xyz, rgb, view, o_init, stream));
  } else if (n_points > 0) {
    // keep the frame's points until the next keyframe merges them (contents kept on growth)
    const int64_t need = m->pend_n + n_points;
    if ((size_t)need * 12 > m->pend_xyz.bytes) {
      const size_t nb = (size_t)std::max<int64_t>(need, 2 * m->pend_n) * 12;
      void* px = dev_alloc(m, nb, s);
      void* pr = dev_alloc(m, nb, s);
      if (!px || !pr) {
        dev_free(m, px, nb, s);
        dev_free(m, pr, nb, s);
        return fail(GS_ERR_OOM, "pending points of the frames since the last keyframe");
      }
      if (m->pend_n > 0) {
        GS_HIP(hipMemcpyAsync(px, m->pend_xyz.ptr, (size_t)m->pend_n * 12, hipMemcpyDeviceToDevice, s));
        GS_HIP(hipMemcpyAsync(pr, m->pend_rgb.ptr, (size_t)m->pend_n * 12, hipMemcpyDeviceToDevice, s));
      }
      GS_HIP(hipStreamSynchronize(s));  // queued copies read the old buffers
      dev_free(m, m->pend_xyz.ptr, m->pend_xyz.bytes, s);
      dev_free(m, m->pend_rgb.ptr, m->pend_rgb.bytes, s);
      m->pend_xyz = DevBuf{px, nb};
      m->pend_rgb = DevBuf{pr, nb};
    }
    GS_HIP(hipMemcpyAsync((char*)m->pend_xyz.ptr + (size_t)m->pend_n * 12, xyz, (size_t)n_points * 12,
                          hipMemcpyDeviceToDevice, s));
    GS_HIP(hipMemcpyAsync((char*)m->pend_rgb.ptr + (size_t)m->pend_n * 12, rgb, (size_t)n_points * 12,
                          hipMemcpyDeviceToDevice, s));
    m->pend_n = need;
  }
  if (key && m->frames_seen > 0 && m->pend_n > 0) {
    // Sec. III-C.2: the points of the five frames up to this keyframe, merged in arrival
    // order, go through the opacity mask of this keyframe's view (Eq. 8)
    const float* px = (const float*)m->pend_xyz.ptr;
    const float* pr = (const float*)m->pend_rgb.ptr;
    if (m->desc.expand_tau > 0.f)
      GS_TRY(gs_expand(m, view, m->pend_n, px, pr, m->desc.expand_tau, o_init, nullptr, stream));
    else
      GS_TRY(gs_add_points(m, m->pend_n, px, pr, view, o_init, stream));
    m->pend_n = 0;
  }
  m->frames_seen += 1;
  if (!key) return GS_OK;
  return archive_keyframe(m, view, image, keyframe_id, s);
}

gs_status gs_optimize_keyframes(gs_map* m, int32_t n, const int32_t* ids, float lambda, void* done_event,
                                void* stream) {
  g_err.clear();
  if (!m) return fail(GS_ERR_INVALID, "map is NULL");
  if (n < 0 || (n > 0 && !ids)) return fail(GS_ERR_INVALID, "bad keyframe list");
  for (int32_t k = 0; k < n; ++k)
    if (ids[k] < 0 || (size_t)ids[k] >= m->archive.size())
      return fail(GS_ERR_INVALID, "keyframe id " + std::to_string(ids[k]) + " out of range");
  hipStream_t s = (hipStream_t)stream;
  size_t pb = 0;
  for (int32_t k = 0; k < n; ++k) pb = std::max(pb, m->archive[ids[k]].pix_bytes);
  if (n > 0) {
    GS_TRY(ensure(m, m->ar_rgb, 3 * pb, s));
    GS_TRY(ensure(m, m->ar_dl, 3 * pb, s));
    GS_TRY(ensure(m, m->ar_T, pb, s));
    GS_TRY(ensure(m, m->ar_nc, pb, s));
  }
  for (int32_t k = 0; k < n; ++k) {
    ArchivedKeyframe& a = m->archive[ids[k]];
    gs_frame fr{(float*)m->ar_rgb.ptr, (float*)m->ar_T.ptr, (uint32_t*)m->ar_nc.ptr, nullptr, nullptr};
    const float* tg = a.image;
    float* es = a.state;
    float* dl = (float*)m->ar_dl.ptr;
    GS_TRY(gs_step(m, 1, &a.view, &fr, &tg, lambda, &es, &dl, m->d_loss, stream));
  }
  if (done_event) GS_HIP(hipEventRecord((hipEvent_t)done_event, s));
  return GS_OK;
}

gs_status gs_keyframe_count(gs_map* m, int32_t* count) {
  if (!m || !count) return fail(GS_ERR_INVALID, "NULL argument");
  *count = (int32_t)m->archive.size();
  return GS_OK;
}

gs_status gs_keyframe_state(gs_map* m, int32_t id, float** state) {
  if (!m || !state) return fail(GS_ERR_INVALID, "NULL argument");
  if (id < 0 || (size_t)id >= m->archive.size())
    return fail(GS_ERR_INVALID, "keyframe id " + std::to_string(id) + " out of range");
  *state = m->archive[id].state;
  return GS_OK;
}

gs_status gs_step(gs_map* m, int32_t nv, const gs_view* views, const gs_frame* frames, const float* const* targets,
                  float lambda, float* const* exposure_states, float* const* dl_drgb, float* loss_dev, void* stream) {
  g_err.clear();
  if (!m || !views || !frames || !targets || !exposure_states || !dl_drgb || !loss_dev)
    return fail(GS_ERR_INVALID, "NULL argument");
  if (nv < 1 || nv > kMaxViews) return fail(GS_ERR_CAPACITY, "n_views must be in 1..16");
  for (int v = 0; v < nv; ++v)
    if (!targets[v] || !exposure_states[v] || !dl_drgb[v] || !frames[v].rgb)
      return fail(GS_ERR_INVALID, "NULL entry in view " + std::to_string(v));
  gs_view vv[kMaxViews];
  const float* dl[kMaxViews];
  float* eg[kMaxViews];
  for (int v = 0; v < nv; ++v) {
    vv[v] = views[v];
    vv[v].exposure = exposure_states[v];
    dl[v] = dl_drgb[v];
    eg[v] = exposure_states[v] + 12;
  }
  GS_TRY(gs_render(m, nv, vv, frames, stream));
  hipStream_t s = (hipStream_t)stream;
  const gs_map_desc& d = m->desc;
  // one loss launch over all views; in a fused step its first block also advances the Adam
  // step counter (or counts the step as skipped when its render dropped instances), and the
  // losses are finished by the projection backward's first block
  const StepPrep prep{m->d_step, m->d_bc, d.beta1, d.beta2, m->d_ninst, m->inst_cap, m->d_overflow + 1};
  LossArg la{};
  la.n = nv;
  la.lambda = lambda;
  for (int v = 0; v < nv; ++v)
    la.v[v] = LossView{frames[v].rgb, targets[v], dl_drgb[v], loss_dev + v, vv[v].height, vv[v].width, 0, 0};
  GS_TRY(loss_impl(m, la, m->fused_step ? &prep : nullptr, m->fused_step, s));
  if (!m->fused_step) {
    GS_TRY(gs_render_backward(m, nv, dl, nullptr, nullptr, eg, stream));
    GS_TRY(gs_adam_step(m, nv, exposure_states, stream));
    return GS_OK;
  }
  // one step: the gradient is complete after this backward, so Adam runs inside the
  // projection backward (no gradient planes written and read back)
  AdamArg ad{};
  ad.lr = lr_table(m);
  ad.m = m->buf + 2 * (int64_t)m->F * m->cap;
  ad.v = m->buf + 3 * (int64_t)m->F * m->cap;
  ad.bc = m->d_bc;
  ad.beta1 = d.beta1;
  ad.beta2 = d.beta2;
  ad.eps = d.eps;
  ad.grads_clean = m->grads_dirty ? 0 : 1;
  // the views' exposures (each view's exposure is its state) are updated by the same kernel
  ad.n_exp = nv;
  ad.lr_exp = d.lr_exposure;
  m->step_assumed_clean = ad.grads_clean != 0;
  if (!ad.grads_clean) m->dirty_step_since_check = true;
  const LossFinish lf{(const float*)m->loss_tmp.ptr + loss_part_offset(), loss_dev, lambda, 0};
  GS_TRY(backward_impl(m, nv, dl, nullptr, nullptr, eg, &ad, lf, s));
  m->grads_dirty = false;  // the fused update cleared every accumulated gradient it read
  m->h_step += 1;
  return GS_OK;
}

gs_status gs_set_fused_step(gs_map* m, int32_t enable) {
  if (!m) return fail(GS_ERR_INVALID, "map is NULL");
  m->fused_step = enable != 0;
  return GS_OK;
}

gs_status gs_capture_step(gs_map* m, int32_t nv, const gs_view* views, const gs_frame* frames,
                          const float* const* targets, float lambda, float* const* exposure_states,
                          float* const* dl_drgb, float* loss_dev, void* stream, gs_step_graph** out) {
  g_err.clear();
  if (!m || !out) return fail(GS_ERR_INVALID, "NULL argument");
  *out = nullptr;
  if (m->sync_plan) return fail(GS_ERR_STATE, "capture needs sync_plan = 0 (gs_set_instance_policy)");
  hipStream_t s = (hipStream_t)stream;
  if (!s) return fail(GS_ERR_INVALID, "capture needs a non-default stream");
  GS_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
  m->capturing = true;
  const int64_t step_before = m->h_step;
  const bool dirty_before = m->grads_dirty;
  m->step_assumed_clean = false;
  gs_status st = gs_step(m, nv, views, frames, targets, lambda, exposure_states, dl_drgb, loss_dev, stream);
  m->capturing = false;
  m->h_step = step_before;  // nothing ran yet
  m->grads_dirty = dirty_before;
  const bool assumes_clean = m->step_assumed_clean;
  std::string msg = g_err;
  hipGraph_t graph = nullptr;
  hipError_t e = hipStreamEndCapture(s, &graph);
  if (st != GS_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return fail(st, msg);
  }
  if (e != hipSuccess) return fail(GS_ERR_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
  hipGraphExec_t exec = nullptr;
  e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(graph);
    return fail(GS_ERR_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
  }
  gs_step_graph* g = new (std::nothrow) gs_step_graph();
  if (!g) {
    (void)hipGraphExecDestroy(exec);
    (void)hipGraphDestroy(graph);
    return fail(GS_ERR_OOM, "host allocation failed");
  }
  g->map = m;
  g->graph = graph;
  g->exec = exec;
  g->assumes_clean = assumes_clean;
  g->epoch = m->epoch;
  g->n = m->n;
  g->cap = m->cap;
  *out = g;
  return GS_OK;
}

gs_status gs_launch_step(gs_step_graph* g, void* stream) {
  if (!g) return fail(GS_ERR_INVALID, "graph is NULL");
  if (g->epoch != g->map->epoch || g->n != g->map->n || g->cap != g->map->cap)
    return fail(GS_ERR_STATE,
                "the map grew or its workspace was reallocated since the capture: capture the step again");
  if (g->assumes_clean && g->map->grads_dirty)
    return fail(GS_ERR_STATE,
                "the gradient planes may hold values (gs_render_backward or gs_map_params since the capture): "
                "run gs_adam_step first, or capture again");
  GS_HIP(hipGraphLaunch(g->exec, (hipStream_t)stream));
  g->map->h_step += 1;
  if (!g->assumes_clean) g->map->dirty_step_since_check = true;
  g->map->grads_dirty = false;
  g->map->render_gen += 1;
  return GS_OK;
}

gs_status gs_destroy_step(gs_step_graph* g) {
  if (!g) return GS_OK;
  (void)hipGraphExecDestroy(g->exec);
  (void)hipGraphDestroy(g->graph);
  delete g;
  return GS_OK;
}

gs_status gs_map_info(const gs_map* m, int64_t* n, int64_t* capacity, int64_t* resident_bytes) {
  if (!m) return fail(GS_ERR_INVALID, "map is NULL");
  if (n) *n = m->n;
  if (capacity) *capacity = m->cap;
  if (resident_bytes) *resident_bytes = m->resident;
  return GS_OK;
}

gs_status gs_map_params(gs_map* m, float** params, float** grads, float** am, float** av, int64_t* stride) {
  if (!m) return fail(GS_ERR_INVALID, "map is NULL");
  const int64_t pl = (int64_t)m->F * m->cap;
  if (params) *params = m->buf;
  if (grads) {
    *grads = m->buf ? m->buf + pl : nullptr;
    m->grads_dirty = true;  // the caller may write them
  }
  if (am) *am = m->buf ? m->buf + 2 * pl : nullptr;
  if (av) *av = m->buf ? m->buf + 3 * pl : nullptr;
  if (stride) *stride = m->cap;
  return GS_OK;
}

gs_status gs_map_visibility(gs_map* m, uint8_t** vis) {
  if (!m || !vis) return fail(GS_ERR_INVALID, "NULL argument");
  *vis = m->vis;
  return GS_OK;
}

gs_status gs_map_render_generation(const gs_map* m, int64_t* gen) {
  if (!m || !gen) return fail(GS_ERR_INVALID, "NULL argument");
  *gen = m->render_gen;
  return GS_OK;
}

gs_status gs_map_step_count(const gs_map* m, int64_t* t) {
  if (!m || !t) return fail(GS_ERR_INVALID, "NULL argument");
  *t = m->h_step;
  return GS_OK;
}

gs_status gs_map_set_step_count(gs_map* m, int64_t t, void* stream) {
  g_err.clear();
  if (!m) return fail(GS_ERR_INVALID, "map is NULL");
  if (t < 0) return fail(GS_ERR_INVALID, "step count must be >= 0");
  hipStream_t s = (hipStream_t)stream;
  const uint64_t u = (uint64_t)t;
  GS_HIP(fill_u32((uint32_t*)m->d_step, (uint32_t)u, 1, s));
  GS_HIP(fill_u32((uint32_t*)m->d_step + 1, (uint32_t)(u >> 32), 1, s));
  m->h_step = t;
  return GS_OK;
}

gs_status gs_debug_last_render(gs_map* m, void* stream, const uint32_t** keys, const uint32_t** vals,
                               int64_t* n_inst, const uint32_t** ranges, int64_t* n_tiles, const float** proj,
                               const uint32_t** counts) {
  if (!m) return fail(GS_ERR_INVALID, "map is NULL");
  if (!m->have_render) return fail(GS_ERR_STATE, "no render yet");
  hipStream_t s = (hipStream_t)stream;
  GS_HIP(hipMemcpyAsync(m->h_pinned, m->d_ninst, 4, hipMemcpyDeviceToHost, s));
  GS_HIP(hipStreamSynchronize(s));
  if (keys) *keys = (const uint32_t*)m->keys[m->sorted].ptr;
  if (vals) {
    GS_TRY(ensure(m, m->dbg_g, (size_t)std::max<int64_t>(m->inst_cap, 1) * 4, s));
    GS_HIP(gather_gaussians((const uint32_t*)m->vals[m->sorted].ptr, (const uint32_t*)m->emit_g.ptr, m->d_ninst,
                            m->inst_cap, (uint32_t*)m->dbg_g.ptr, s));
    GS_HIP(hipStreamSynchronize(s));
    *vals = (const uint32_t*)m->dbg_g.ptr;
  }
  if (n_inst) *n_inst = m->h_pinned[0];
  if (ranges) *ranges = (const uint32_t*)m->ranges.ptr;
  if (n_tiles) *n_tiles = m->last_va.total_tiles;
  if (proj) *proj = (const float*)m->rec.ptr;
  if (counts) *counts = (const uint32_t*)m->counts.ptr;
  return GS_OK;
}

gs_status gs_set_instance_policy(gs_map* m, int32_t sync_plan, int64_t capacity) {
  if (!m) return fail(GS_ERR_INVALID, "map is NULL");
  if (capacity < 0 || capacity > (int64_t)UINT32_MAX) return fail(GS_ERR_INVALID, "capacity out of range");
  if (capacity > m->inst_cap) {
    hipStream_t s = nullptr;
    GS_TRY(ensure_instances(m, capacity, 0, s));
    GS_HIP(hipStreamSynchronize(s));
  }
  m->sync_plan = sync_plan != 0;
  return GS_OK;
}

// Reads and clears the overflow words: [0] a render dropped instances, [1] fused steps
// skipped for it, [2] the largest instance count needed. After skipped steps the host's
// step count follows the device's, and gradient planes a skipped step would have consumed
// are marked as holding values again.
static gs_status read_overflow(gs_map* m, hipStream_t s, uint32_t* flag, uint32_t* skipped, uint32_t* peak) {
  GS_HIP(hipMemcpyAsync(m->h_pinned, m->d_overflow, 12, hipMemcpyDeviceToHost, s));
  GS_HIP(hipMemcpyAsync(m->h_pinned + 4, m->d_step, 8, hipMemcpyDeviceToHost, s));
  GS_HIP(hipStreamSynchronize(s));
  *flag = m->h_pinned[0];
  *skipped = m->h_pinned[1];
  *peak = m->h_pinned[2];
  if (*skipped) {
    m->h_step = (int64_t)((uint64_t)m->h_pinned[4] | ((uint64_t)m->h_pinned[5] << 32));
    if (m->dirty_step_since_check) m->grads_dirty = true;
  }
  m->dirty_step_since_check = false;
  GS_HIP(fill_u32(m->d_overflow, 0u, 3, s));
  return GS_OK;
}

gs_status gs_check_overflow(gs_map* m, void* stream, int32_t* overflow) {
  if (!m || !overflow) return fail(GS_ERR_INVALID, "NULL argument");
  uint32_t flag, skipped, peak;
  GS_TRY(read_overflow(m, (hipStream_t)stream, &flag, &skipped, &peak));
  *overflow = flag ? 1 : 0;
  return GS_OK;
}

gs_status gs_set_stage_timing(gs_map* m, int32_t enable) {
  if (!m) return fail(GS_ERR_INVALID, "map is NULL");
  m->timing = enable != 0;
  return GS_OK;
}

gs_status gs_stage_times(gs_map* m, void* stream, double* ms, int64_t* count) {
  if (!m || !ms || !count) return fail(GS_ERR_INVALID, "NULL argument");
  GS_HIP(hipStreamSynchronize((hipStream_t)stream));
  for (int k = 0; k < GS_NUM_STAGES; ++k) {
    ms[k] = 0.0;
    count[k] = 0;
  }
  for (const auto& mk : m->ev_marks) {
    float t = 0.f;
    GS_HIP(hipEventElapsedTime(&t, m->ev_pool[mk.second], m->ev_pool[mk.second + 1]));
    ms[mk.first] += t;
    count[mk.first] += 1;
  }
  m->ev_marks.clear();
  m->ev_used = 0;
  return GS_OK;
}

gs_status gs_set_deterministic(gs_map* m, int32_t enable) {
  if (!m) return fail(GS_ERR_INVALID, "map is NULL");
  m->deterministic = enable != 0;
  m->have_render = false;  // the next render sizes the per-instance buffers
  return GS_OK;
}

gs_status gs_set_backward_mode(gs_map* m, int32_t mode) {
  if (!m) return fail(GS_ERR_INVALID, "map is NULL");
  if (mode != 0 && mode != 1) return fail(GS_ERR_INVALID, "backward mode must be 0 (pixel order) or 1 (per Gaussian)");
  if (m->capturing) return fail(GS_ERR_STATE, "cannot change the backward mode while capturing");
  m->bwd_mode = mode;
  m->have_render = false;  // the next render saves what the backward needs
  return GS_OK;
}

gs_status gs_set_tile_split(gs_map* m, int32_t parallel, int32_t min_chunk, float balance) {
  if (!m) return fail(GS_ERR_INVALID, "map is NULL");
  if (parallel < 0 || parallel > (1 << 16)) return fail(GS_ERR_INVALID, "parallel must be in [0, 65536]");
  if (min_chunk < 1 || min_chunk > (1 << 24)) return fail(GS_ERR_INVALID, "min_chunk must be in [1, 2^24]");
  if (!(balance >= 0.0f && balance <= 1e6f)) return fail(GS_ERR_INVALID, "balance must be in [0, 1e6]");
  if (m->capturing) return fail(GS_ERR_STATE, "cannot change the tile split while capturing");
  m->split_par = parallel;
  m->split_min = min_chunk;
  m->split_balance = balance;
  m->have_render = false;  // a backward needs the split of its own render
  return GS_OK;
}

gs_status gs_set_blend_config(gs_map* m, int32_t fwd, int32_t bwd) {
  if (!m) return fail(GS_ERR_INVALID, "map is NULL");
  auto ok = [](int32_t px) { return px == 1 || px == 2 || px == 4; };
  if (!ok(fwd) || !ok(bwd)) return fail(GS_ERR_INVALID, "pixels per lane must be 1, 2 or 4");
  if (m->capturing) return fail(GS_ERR_STATE, "cannot change the blend configuration while capturing");
  m->fwd_px = fwd;
  m->bwd_px = bwd;
  return GS_OK;
}

}  // extern "C"
