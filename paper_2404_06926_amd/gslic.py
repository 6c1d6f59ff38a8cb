"""ctypes binding of libgslic (include/gslic.h).

Argument marshalling only: every step of the mapping iteration runs in the HIP library.
PyTorch supplies device memory (the library's allocator callbacks hand out torch
tensors) and streams (the current torch stream is passed to every call). A missing
library raises; there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgslic.so")

GS_OK = 0
GS_ERR_INVALID = -1
GS_ERR_OOM = -2
GS_ERR_HIP = -3
GS_ERR_CAPACITY = -4
GS_ERR_STATE = -6
GS_ERR_UNIMPLEMENTED = -7
GS_MAX_VIEWS = 16
GS_EXPOSURE_STATE_FLOATS = 48

_ERR_NAMES = {GS_ERR_INVALID: "GS_ERR_INVALID", GS_ERR_OOM: "GS_ERR_OOM", GS_ERR_HIP: "GS_ERR_HIP",
              GS_ERR_CAPACITY: "GS_ERR_CAPACITY", GS_ERR_STATE: "GS_ERR_STATE",
              GS_ERR_UNIMPLEMENTED: "GS_ERR_UNIMPLEMENTED"}


class GsError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_ERR_NAMES.get(code, code)}: {msg}")
        self.code = code


_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)


class GsAllocator(ctypes.Structure):
    _fields_ = [("alloc", _ALLOC_FN), ("free", _FREE_FN), ("ctx", ctypes.c_void_p)]


class GsMapDesc(ctypes.Structure):
    _fields_ = [("sh_degree", ctypes.c_int32), ("initial_capacity", ctypes.c_int64),
                ("near_z", ctypes.c_float), ("lr_mean", ctypes.c_float),
                ("lr_log_scale", ctypes.c_float), ("lr_quat", ctypes.c_float),
                ("lr_opacity", ctypes.c_float), ("lr_sh_dc", ctypes.c_float),
                ("lr_sh_rest", ctypes.c_float), ("lr_exposure", ctypes.c_float),
                ("beta1", ctypes.c_float), ("beta2", ctypes.c_float), ("eps", ctypes.c_float),
                ("expand_tau", ctypes.c_float)]


class GsView(ctypes.Structure):
    _fields_ = [("R_cw", ctypes.c_float * 9), ("t_cw", ctypes.c_float * 3), ("fx", ctypes.c_float),
                ("fy", ctypes.c_float), ("cx", ctypes.c_float), ("cy", ctypes.c_float),
                ("width", ctypes.c_int32), ("height", ctypes.c_int32), ("bg", ctypes.c_float * 3),
                ("exposure", ctypes.c_void_p)]


class GsFrame(ctypes.Structure):
    _fields_ = [("rgb", ctypes.c_void_p), ("final_T", ctypes.c_void_p), ("n_contrib", ctypes.c_void_p),
                ("depth", ctypes.c_void_p), ("opacity", ctypes.c_void_p)]


_P = ctypes.c_void_p
_I32, _I64, _F = ctypes.c_int32, ctypes.c_int64, ctypes.c_float
_SIGS = {
    "gs_default_desc": (None, [ctypes.POINTER(GsMapDesc)]),
    "gs_create_map": (_I32, [ctypes.POINTER(GsMapDesc), ctypes.POINTER(GsAllocator), ctypes.POINTER(_P)]),
    "gs_destroy_map": (_I32, [_P]),
    "gs_add_gaussians": (_I32, [_P, _I64, _P, _P, _P, _P, _P, _P]),
    "gs_add_points": (_I32, [_P, _I64, _P, _P, ctypes.POINTER(GsView), _F, _P]),
    "gs_expand": (_I32, [_P, ctypes.POINTER(GsView), _I64, _P, _P, _F, _F, ctypes.POINTER(_I64), _P]),
    "gs_add_sky": (_I32, [_P, _I64, _P, _F, _P]),
    "gs_add_keyframe": (_I32, [_P, ctypes.POINTER(GsView), _P, _I64, _P, _P, _F, ctypes.POINTER(_I32), _P]),
    "gs_add_frame": (_I32, [_P, ctypes.POINTER(GsView), _P, _I64, _P, _P, _F, ctypes.POINTER(_I32), _P]),
    "gs_optimize_keyframes": (_I32, [_P, _I32, ctypes.POINTER(_I32), _F, _P, _P]),
    "gs_keyframe_count": (_I32, [_P, ctypes.POINTER(_I32)]),
    "gs_keyframe_state": (_I32, [_P, _I32, ctypes.POINTER(_P)]),
    "gs_render": (_I32, [_P, _I32, ctypes.POINTER(GsView), ctypes.POINTER(GsFrame), _P]),
    "gs_render_backward": (_I32, [_P, _I32, ctypes.POINTER(_P), ctypes.POINTER(_P), ctypes.POINTER(_P),
                                  ctypes.POINTER(_P), _P]),
    "gs_adam_step": (_I32, [_P, _I32, ctypes.POINTER(_P), _P]),
    "gs_loss": (_I32, [_P, _P, _P, _I32, _I32, _F, _P, _P, _P]),
    "gs_loss_noalloc": (_I32, [_P, _P, _I32, _I32, _F, _P, _P, _P]),
    "gs_submit_keyframe": (_I32, [_P, ctypes.POINTER(GsView), _P, _I64, _P, _P, _I32, _I32, _F, _F, _P, _P]),
    "gs_last_error": (ctypes.c_char_p, []),
    "gs_map_info": (_I32, [_P, ctypes.POINTER(_I64), ctypes.POINTER(_I64), ctypes.POINTER(_I64)]),
    "gs_map_params": (_I32, [_P, ctypes.POINTER(_P), ctypes.POINTER(_P), ctypes.POINTER(_P), ctypes.POINTER(_P),
                             ctypes.POINTER(_I64)]),
    "gs_map_visibility": (_I32, [_P, ctypes.POINTER(_P)]),
    "gs_map_step_count": (_I32, [_P, ctypes.POINTER(_I64)]),
    "gs_map_render_generation": (_I32, [_P, ctypes.POINTER(_I64)]),
    "gs_map_set_step_count": (_I32, [_P, _I64, _P]),
    "gs_debug_last_render": (_I32, [_P, _P, ctypes.POINTER(_P), ctypes.POINTER(_P), ctypes.POINTER(_I64),
                                    ctypes.POINTER(_P), ctypes.POINTER(_I64), ctypes.POINTER(_P),
                                    ctypes.POINTER(_P)]),
    "gs_set_instance_policy": (_I32, [_P, _I32, _I64]),
    "gs_check_overflow": (_I32, [_P, _P, ctypes.POINTER(_I32)]),
    "gs_set_blend_config": (_I32, [_P, _I32, _I32]),
    "gs_set_tile_split": (_I32, [_P, _I32, _I32, _F]),
    "gs_set_backward_mode": (_I32, [_P, _I32]),
    "gs_set_stage_timing": (_I32, [_P, _I32]),
    "gs_set_deterministic": (_I32, [_P, _I32]),
    "gs_set_fused_step": (_I32, [_P, _I32]),
    "gs_step": (_I32, [_P, _I32, ctypes.POINTER(GsView), ctypes.POINTER(GsFrame), ctypes.POINTER(_P), _F,
                       ctypes.POINTER(_P), ctypes.POINTER(_P), _P, _P]),
    "gs_capture_step": (_I32, [_P, _I32, ctypes.POINTER(GsView), ctypes.POINTER(GsFrame), ctypes.POINTER(_P), _F,
                               ctypes.POINTER(_P), ctypes.POINTER(_P), _P, _P, ctypes.POINTER(_P)]),
    "gs_launch_step": (_I32, [_P, _P]),
    "gs_destroy_step": (_I32, [_P]),
    "gs_stage_times": (_I32, [_P, _P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_I64)]),
}

STAGES = ["project", "scan", "duplicate", "sort", "ranges", "blend", "loss", "blend_backward",
          "project_backward", "adam", "depth_sort"]

_lib = None


def lib():
    """Load libgslic.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built (python -m paper_2404_06926_amd.build)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(code):
    if code != GS_OK:
        raise GsError(code, lib().gs_last_error().decode())


def _torch():
    import torch
    return torch


def _stream(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


class TorchAllocator:
    """Device memory for the library from torch's caching allocator."""

    def __init__(self, device):
        self.device = device
        self.live = {}
        self._alloc = _ALLOC_FN(self._do_alloc)
        self._free = _FREE_FN(self._do_free)
        self.struct = GsAllocator(self._alloc, self._free, None)

    def _do_alloc(self, nbytes, stream, ctx):
        try:
            t = _torch().empty(int(nbytes), dtype=_torch().uint8, device=self.device)
        except Exception:  # out of memory: the library reports GS_ERR_OOM
            return None
        self.live[t.data_ptr()] = t
        return t.data_ptr()

    def _do_free(self, ptr, stream, ctx):
        self.live.pop(ptr, None)

    def view(self, ptr, nbytes):
        """uint8 tensor aliasing [ptr, ptr + nbytes) inside a live allocation."""
        for base, t in self.live.items():
            if base <= ptr and ptr + nbytes <= base + t.numel():
                return t[ptr - base: ptr - base + nbytes]
        raise KeyError("pointer not owned by this allocator")


def loss_noalloc(out, gt, lam, loss_out, grad_out, stream=None):
    """gs_loss_noalloc: the Eq. 9 loss into caller-provided loss_out (float[1]) and grad_out
    (shape of out), with no map and no device allocation inside the library."""
    _, H, W = out.shape
    _check(lib().gs_loss_noalloc(_ptr(out), _ptr(gt), H, W, float(lam), _ptr(loss_out), _ptr(grad_out),
                                 _stream(stream)))
    return loss_out, grad_out


def identity_exposure_state(device="cuda"):
    """[E | grad | m | v] with E = [I | 0]."""
    torch = _torch()
    s = torch.zeros(GS_EXPOSURE_STATE_FLOATS, dtype=torch.float32, device=device)
    s[0] = s[5] = s[10] = 1.0
    return s


@dataclass
class Frame:
    rgb: "object"
    final_T: "object"
    n_contrib: "object"
    depth: "object" = None      # depth map (Eq. 6), when asked for
    opacity: "object" = None    # opacity map (Eq. 7), when asked for


def _frame_struct(f) -> "GsFrame":
    return GsFrame(f.rgb.data_ptr(), f.final_T.data_ptr(), f.n_contrib.data_ptr(),
                   f.depth.data_ptr() if f.depth is not None else None,
                   f.opacity.data_ptr() if f.opacity is not None else None)


def make_view(cam, exposure=None) -> GsView:
    """GsView from any object with R, t, fx, fy, cx, cy, width, height and optional bg;
    exposure: device tensor of 12 (or a 48-float state whose first 12 are E) or None."""
    v = GsView()
    R = np.asarray(cam.R, np.float32).reshape(9)
    t = np.asarray(cam.t, np.float32).reshape(3)
    for k in range(9):
        v.R_cw[k] = float(R[k])
    for k in range(3):
        v.t_cw[k] = float(t[k])
    v.fx, v.fy, v.cx, v.cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    v.width, v.height = int(cam.width), int(cam.height)
    bg = np.asarray(getattr(cam, "bg", np.zeros(3)), np.float32).reshape(3)
    for k in range(3):
        v.bg[k] = float(bg[k])
    v.exposure = exposure.data_ptr() if exposure is not None else None
    return v


class GaussianMap:
    """A Gaussian map on one GPU with the mapping-step operations of libgslic."""

    def __init__(self, sh_degree=3, capacity=1 << 16, device="cuda", **desc_overrides):
        torch = _torch()
        self.device = torch.device(device)
        d = GsMapDesc()
        lib().gs_default_desc(ctypes.byref(d))
        d.sh_degree = sh_degree
        d.initial_capacity = capacity
        for k, val in desc_overrides.items():
            setattr(d, k, val)
        self.desc = d
        self.allocator = TorchAllocator(self.device)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(lib().gs_create_map(ctypes.byref(d), ctypes.byref(self.allocator.struct), ctypes.byref(h)))
        self.handle = h
        self.sh_degree = sh_degree
        self.K = (sh_degree + 1) ** 2
        self.F = 11 + 3 * self.K
        self._keep = []

    def close(self):
        if getattr(self, "handle", None):
            lib().gs_destroy_map(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ----------------------------------------------------------------- info
    def info(self):
        n, c, r = _I64(), _I64(), _I64()
        _check(lib().gs_map_info(self.handle, ctypes.byref(n), ctypes.byref(c), ctypes.byref(r)))
        return n.value, c.value, r.value

    @property
    def n(self):
        return self.info()[0]

    @property
    def step_count(self):
        t = _I64()
        _check(lib().gs_map_step_count(self.handle, ctypes.byref(t)))
        return t.value

    @property
    def render_generation(self):
        """Renders of this map so far (eager, inside steps and jobs, graph replays)."""
        g = _I64()
        _check(lib().gs_map_render_generation(self.handle, ctypes.byref(g)))
        return g.value

    def set_step_count(self, t: int, stream=None):
        """Restores the Adam step counter (with the parameters and moments of a checkpoint)."""
        _check(lib().gs_map_set_step_count(self.handle, int(t), _stream(stream)))

    def _planes(self, which):
        torch = _torch()
        p = [_P(), _P(), _P(), _P()]
        stride = _I64()
        # ask only for the plane wanted: handing out the gradient pointer marks the
        # gradient planes as possibly written
        args = [ctypes.byref(x) if k == which else None for k, x in enumerate(p)]
        _check(lib().gs_map_params(self.handle, *args, ctypes.byref(stride)))
        ptr = p[which].value
        cap = stride.value
        raw = self.allocator.view(ptr, self.F * cap * 4)
        return raw.view(torch.float32).view(self.F, cap)[:, : self.n]

    def params(self):
        """[F, n] float32 view of the parameter planes (aliases map memory)."""
        return self._planes(0)

    def grads(self):
        return self._planes(1)

    def adam_moments(self):
        return self._planes(2), self._planes(3)

    def visibility(self):
        torch = _torch()
        p = _P()
        _check(lib().gs_map_visibility(self.handle, ctypes.byref(p)))
        return self.allocator.view(p.value, max(self.n, 1))[: self.n]

    # ------------------------------------------------------------- building
    def add_gaussians(self, rows, stream=None):
        """rows: [n, F] float32 (mean 3, log-scale 3, quat 4, logit 1, SH [k][c])."""
        torch = _torch()
        rows = torch.as_tensor(rows, dtype=torch.float32, device=self.device)
        assert rows.ndim == 2 and rows.shape[1] == self.F, rows.shape
        n = rows.shape[0]
        parts = [rows[:, 0:3].contiguous(), rows[:, 3:6].contiguous(), rows[:, 6:10].contiguous(),
                 rows[:, 10].contiguous(), rows[:, 11:].contiguous()]
        _check(lib().gs_add_gaussians(self.handle, n, *[_ptr(p) for p in parts], _stream(stream)))
        self._keep = parts  # inputs stay alive until the stream has consumed them

    def add_points(self, xyz, rgb, cam, o_init=0.1, stream=None):
        torch = _torch()
        xyz = torch.as_tensor(xyz, dtype=torch.float32, device=self.device).contiguous()
        rgb = torch.as_tensor(rgb, dtype=torch.float32, device=self.device).contiguous()
        v = make_view(cam)
        _check(lib().gs_add_points(self.handle, xyz.shape[0], _ptr(xyz), _ptr(rgb), ctypes.byref(v),
                                   float(o_init), _stream(stream)))
        self._keep = [xyz, rgb]

    def expand(self, cam, xyz, rgb, tau=0.99, o_init=0.1, stream=None) -> int:
        """Eq. 8 expansion at a keyframe view; returns the number of Gaussians appended."""
        torch = _torch()
        xyz = torch.as_tensor(xyz, dtype=torch.float32, device=self.device).contiguous()
        rgb = torch.as_tensor(rgb, dtype=torch.float32, device=self.device).contiguous()
        v = make_view(cam)
        k = _I64()
        _check(lib().gs_expand(self.handle, ctypes.byref(v), xyz.shape[0], _ptr(xyz), _ptr(rgb), float(tau),
                               float(o_init), ctypes.byref(k), _stream(stream)))
        self._keep = [xyz, rgb]
        return int(k.value)

    def add_sky(self, xyz, o_sky=0.7, stream=None):
        """Sky Gaussians at the given positions (scale = nearest-neighbour distance)."""
        torch = _torch()
        xyz = torch.as_tensor(xyz, dtype=torch.float32, device=self.device).contiguous()
        _check(lib().gs_add_sky(self.handle, xyz.shape[0], _ptr(xyz), float(o_sky), _stream(stream)))
        self._keep = [xyz]

    def add_keyframe(self, cam, image, xyz=None, rgb=None, o_init=0.1, stream=None) -> int:
        """Keep a keyframe for the random-K schedule (after expanding the map with its
        points); returns its id."""
        n = 0 if xyz is None else int(xyz.shape[0])
        v = make_view(cam)
        kid = _I32()
        _check(lib().gs_add_keyframe(self.handle, ctypes.byref(v), _ptr(image), n, _ptr(xyz), _ptr(rgb),
                                     float(o_init), ctypes.byref(kid), _stream(stream)))
        self._keep = [image, xyz, rgb]
        return int(kid.value)

    def add_frame(self, cam, image=None, xyz=None, rgb=None, o_init=0.1, stream=None) -> int:
        """Frame intake of Sec. III-C.2 (every fifth frame a keyframe, the five frames' points
        merged at it); returns the keyframe id, or -1 for a frame that is not a keyframe."""
        n = 0 if xyz is None else int(xyz.shape[0])
        v = make_view(cam)
        kid = _I32()
        _check(lib().gs_add_frame(self.handle, ctypes.byref(v), _ptr(image), n, _ptr(xyz), _ptr(rgb),
                                  float(o_init), ctypes.byref(kid), _stream(stream)))
        self._keep = [image, xyz, rgb]
        return int(kid.value)

    def optimize_keyframes(self, ids, lam=0.2, done_event=None, stream=None):
        """One single-view mapping step per id, in the given order."""
        arr = (_I32 * max(len(ids), 1))(*[int(i) for i in ids])
        ev = ctypes.c_void_p(done_event.cuda_event) if done_event is not None else None
        _check(lib().gs_optimize_keyframes(self.handle, len(ids), arr, float(lam), ev, _stream(stream)))

    def keyframe_count(self) -> int:
        c = _I32()
        _check(lib().gs_keyframe_count(self.handle, ctypes.byref(c)))
        return int(c.value)

    def keyframe_state(self, kid: int):
        """float32[48] view of kept keyframe `kid`'s exposure state [E | grad | m | v]."""
        torch = _torch()
        p = _P()
        _check(lib().gs_keyframe_state(self.handle, int(kid), ctypes.byref(p)))
        return self.allocator.view(p.value, 4 * 48).view(torch.float32)

    # ------------------------------------------------------------- the step
    def render(self, cams: Sequence, exposures: Optional[Sequence] = None, frames=None, stream=None,
               depth: bool = False, opacity: bool = False) -> List[Frame]:
        """Batched forward over the views; depth / opacity also return the depth and opacity
        maps (Eq. 6-7) in frames allocated here."""
        torch = _torch()
        nv = len(cams)
        views = (GsView * nv)()
        fr = (GsFrame * nv)()
        out = []
        for k, c in enumerate(cams):
            e = exposures[k] if exposures is not None else None
            views[k] = make_view(c, e)
            if frames is not None:
                f = frames[k]
            else:
                f = Frame(torch.empty(3, c.height, c.width, device=self.device),
                          torch.empty(c.height, c.width, device=self.device),
                          torch.empty(c.height, c.width, dtype=torch.int32, device=self.device),
                          torch.empty(c.height, c.width, device=self.device) if depth else None,
                          torch.empty(c.height, c.width, device=self.device) if opacity else None)
            fr[k] = _frame_struct(f)
            out.append(f)
        _check(lib().gs_render(self.handle, nv, views, fr, _stream(stream)))
        # the kernels of this render and of render_backward read these buffers
        self._last_frames = out
        self._last_exposures = list(exposures) if exposures is not None else None
        self._last_nv = nv
        return out

    def render_backward(self, dl_drgb: Sequence, dl_dexposure: Optional[Sequence] = None, stream=None,
                        dl_ddepth: Optional[Sequence] = None, dl_dopacity: Optional[Sequence] = None):
        nv = len(dl_drgb)
        dl = (_P * nv)(*[t.data_ptr() for t in dl_drgb])

        def arr(ts):
            if ts is None:
                return None
            return (_P * nv)(*[(t.data_ptr() if t is not None else None) for t in ts])

        _check(lib().gs_render_backward(self.handle, nv, dl, arr(dl_ddepth), arr(dl_dopacity), arr(dl_dexposure),
                                        _stream(stream)))

    def adam_step(self, exposure_states: Sequence = (), stream=None):
        ne = len(exposure_states)
        arr = (_P * max(ne, 1))(*[t.data_ptr() for t in exposure_states])
        _check(lib().gs_adam_step(self.handle, ne, arr, _stream(stream)))

    def loss(self, out, gt, lam, loss_out=None, grad_out=None, stream=None):
        torch = _torch()
        _, H, W = out.shape
        lo = loss_out if loss_out is not None else torch.empty(1, device=self.device)
        g = grad_out if grad_out is not None else torch.empty_like(out)
        _check(lib().gs_loss(self.handle, _ptr(out), _ptr(gt), H, W, float(lam), _ptr(lo), _ptr(g),
                             _stream(stream)))
        return lo, g

    def submit_keyframe(self, cam, image, xyz=None, rgb=None, iters=10, window=8, lam=0.2, o_init=0.1,
                        done_event=None, stream=None):
        n = 0 if xyz is None else int(xyz.shape[0])
        v = make_view(cam)
        ev = ctypes.c_void_p(done_event.cuda_event) if done_event is not None else None
        _check(lib().gs_submit_keyframe(self.handle, ctypes.byref(v), _ptr(image), n, _ptr(xyz), _ptr(rgb),
                                        iters, window, float(lam), float(o_init), ev, _stream(stream)))
        self._keep = [image, xyz, rgb]

    def _step_args(self, cams, frames, targets, exposure_states, grads, loss_out):
        nv = len(cams)
        views = (GsView * nv)(*[make_view(c) for c in cams])
        fr = (GsFrame * nv)(*[_frame_struct(f)
                              for f in frames])
        tg = (_P * nv)(*[t.data_ptr() for t in targets])
        es = (_P * nv)(*[e.data_ptr() for e in exposure_states])
        gr = (_P * nv)(*[g.data_ptr() for g in grads])
        return nv, views, fr, tg, es, gr, _ptr(loss_out)

    def step(self, cams, frames, targets, exposure_states, grads, loss_out, lam=0.2, stream=None):
        """One mapping step (render, loss, backward, Adam) over the views in one batch."""
        nv, views, fr, tg, es, gr, lo = self._step_args(cams, frames, targets, exposure_states, grads, loss_out)
        _check(lib().gs_step(self.handle, nv, views, fr, tg, float(lam), es, gr, lo, _stream(stream)))
        self._last_frames = frames
        self._last_exposures = exposure_states
        self._last_nv = nv

    def capture_step(self, cams, frames, targets, exposure_states, grads, loss_out, lam=0.2, stream=None):
        """A StepGraph replaying the same step; all tensors passed must stay alive."""
        nv, views, fr, tg, es, gr, lo = self._step_args(cams, frames, targets, exposure_states, grads, loss_out)
        h = _P()
        _check(lib().gs_capture_step(self.handle, nv, views, fr, tg, float(lam), es, gr, lo, _stream(stream),
                                     ctypes.byref(h)))
        self._last_nv = nv
        return StepGraph(h, keep=(frames, targets, exposure_states, grads, loss_out))

    # ------------------------------------------------------------- control
    def set_instance_policy(self, sync_plan: bool, capacity: int = 0):
        _check(lib().gs_set_instance_policy(self.handle, 1 if sync_plan else 0, int(capacity)))

    def check_overflow(self, stream=None) -> bool:
        o = _I32()
        _check(lib().gs_check_overflow(self.handle, _stream(stream), ctypes.byref(o)))
        return bool(o.value)

    def set_fused_step(self, enable: bool):
        _check(lib().gs_set_fused_step(self.handle, 1 if enable else 0))

    def set_deterministic(self, enable: bool):
        _check(lib().gs_set_deterministic(self.handle, 1 if enable else 0))

    def set_backward_mode(self, mode: int):
        """0: pixel-order backward blend; 1: per-Gaussian (lanes own list entries)."""
        _check(lib().gs_set_backward_mode(self.handle, int(mode)))

    def set_blend_config(self, fwd_px_per_lane: int, bwd_px_per_lane: int):
        """Pixels per lane (1, 2 or 4) of the forward and backward blend kernels."""
        _check(lib().gs_set_blend_config(self.handle, int(fwd_px_per_lane), int(bwd_px_per_lane)))

    def set_tile_split(self, parallel: int = 4096, min_chunk: int = 128, balance: float = 1.25):
        """Blend tiles whose lists exceed `balance` times the mean list and max(min_chunk,
        instances / parallel) entries in chunks on separate workgroups; parallel = 0
        keeps every tile in one workgroup."""
        _check(lib().gs_set_tile_split(self.handle, int(parallel), int(min_chunk), float(balance)))

    def set_stage_timing(self, enable: bool):
        _check(lib().gs_set_stage_timing(self.handle, 1 if enable else 0))

    def stage_times(self, stream=None):
        """{stage: (total ms, launches)} since the previous query (synchronises)."""
        ms = (ctypes.c_double * len(STAGES))()
        cnt = (_I64 * len(STAGES))()
        _check(lib().gs_stage_times(self.handle, _stream(stream), ms, cnt))
        return {name: (ms[k], cnt[k]) for k, name in enumerate(STAGES)}

    def debug_last_render(self, stream=None):
        """Copies of the last render's instance tiles and Gaussian indices (blend order),
        tile ranges, per-(view, Gaussian) projection records and tile counts."""
        torch = _torch()
        k, v, r, p, c = _P(), _P(), _P(), _P(), _P()
        ni, nt = _I64(), _I64()
        _check(lib().gs_debug_last_render(self.handle, _stream(stream), ctypes.byref(k), ctypes.byref(v),
                                          ctypes.byref(ni), ctypes.byref(r), ctypes.byref(nt), ctypes.byref(p),
                                          ctypes.byref(c)))
        n, T = ni.value, nt.value
        nv = self._last_nv
        out = dict(n_inst=n, n_tiles=T)
        if n > 0:
            out["tiles"] = self.allocator.view(k.value, 4 * n).view(torch.int32)[:n].clone()
            out["vals"] = self.allocator.view(v.value, 4 * n).view(torch.int32)[:n].clone()
        else:
            out["tiles"] = torch.zeros(0, dtype=torch.int32, device=self.device)
            out["vals"] = torch.zeros(0, dtype=torch.int32, device=self.device)
        out["ranges"] = self.allocator.view(r.value, 8 * T).view(torch.int32).view(T, 2).clone()
        out["proj"] = self.allocator.view(p.value, 64 * nv * max(self.n, 1)).view(torch.float32).view(
            nv, max(self.n, 1), 16)[:, : self.n].clone()
        out["counts"] = self.allocator.view(c.value, 4 * nv * max(self.n, 1)).view(torch.int32).view(
            nv, max(self.n, 1))[:, : self.n].clone()
        return out


class StepGraph:
    """A captured mapping step (gs_capture_step); launch() replays it on a stream."""

    def __init__(self, handle, keep=()):
        self.handle = handle
        self.keep = keep

    def launch(self, stream=None):
        _check(lib().gs_launch_step(self.handle, _stream(stream)))

    def close(self):
        if self.handle:
            lib().gs_destroy_step(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class RenderFunction:
    """torch.autograd.Function over gs_render / gs_render_backward: inputs are the map's
    parameter planes ([F, n] view) and one exposure tensor (12) per view; outputs are the
    rendered images. Parameter gradients are returned as a [F, n] tensor."""

    _fn = None

    @classmethod
    def get(cls):
        if cls._fn is None:
            torch = _torch()

            class _Render(torch.autograd.Function):
                @staticmethod
                def forward(ctx, gmap, cams, params, *exposures):
                    frames = gmap.render(cams, list(exposures) if exposures else None)
                    ctx.gmap = gmap
                    ctx.n_exp = len(exposures)
                    # the backward consumes the map's saved state of its most recent render
                    ctx.generation = gmap.render_generation
                    return tuple(f.rgb for f in frames)

                @staticmethod
                def backward(ctx, *grads):
                    gmap = ctx.gmap
                    if gmap.render_generation != ctx.generation:
                        raise RuntimeError("the map rendered again after this forward; its backward would "
                                           "use the newer render's state: render_autograd again")
                    g = gmap.grads()
                    g.zero_()
                    gexp = [torch.zeros(12, device=gmap.device) for _ in range(len(grads))]
                    gmap.render_backward([x.contiguous() for x in grads], gexp)
                    gp = g.clone()
                    g.zero_()
                    gmap.visibility().zero_()
                    return (None, None, gp, *(gexp[: ctx.n_exp]))

            cls._fn = _Render
        return cls._fn


def render_autograd(gmap: GaussianMap, cams, exposures=None):
    """Differentiable render of several views; returns a tuple of [3, H, W] images."""
    params = gmap.params()
    if not params.requires_grad:
        params = params.detach().requires_grad_(True)
    ex = list(exposures) if exposures is not None else []
    return RenderFunction.get().apply(gmap, cams, params, *ex), params
