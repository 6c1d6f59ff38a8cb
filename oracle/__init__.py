"""Plain CPU oracle for one optimisation step of a 3D Gaussian map.

TEST INFRASTRUCTURE ONLY: the test suite, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` are its only users. It shares no code with the HIP
library and never loads it; the product path never imports this package.

The arithmetic lives in ``gs_oracle.cpp`` (FP64, with an FP32 key path for the
bit-exact tile keys); this module only marshals numpy arrays through ctypes and
composes the per-view steps in the paper's order:

    project (Sec. III-A, Eq. 1-3) -> emit (tile, Gaussian) pairs for tiles the footprint
    reaches (Sec. III-D.2) -> stable sort by (tile, depth) (Sec. III-A) -> per-tile ranges
    -> blend front to back with exposure (Eq. 5, Sec. III-C.3), depth and opacity maps
    (Eq. 6-7) -> loss (Eq. 9)
    -> adjoint -> sparse Adam (Sec. III-D.2, Sec. IV-A.1).

Cameras are ``float64[16]`` = R_cw row-major (9), t_cw (3), fx, fy, cx, cy. Parameter rows
are ``float64[N, 11 + 3K]`` = mean (3), log-scale (3), quaternion wxyz (4), opacity logit
(1), SH [k][channel] (3K), K = (deg + 1)^2.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gs_oracle.cpp")
_LIB = os.path.join(_HERE, "libgs_oracle.so")

NEAR_Z = 0.2
TILE = 16


def build(force: bool = False) -> str:
    """Compile the oracle with g++ (FP32 key path needs -ffp-contract=off)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        cmd = ["g++", "-O2", "-std=c++17", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
               "-shared", "-fPIC", "-o", _LIB + ".tmp", _SRC]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        _lib = ctypes.CDLL(_LIB)
        _lib.or_loss.restype = ctypes.c_double
    return _lib


def set_threads(n: int) -> int:
    """Host threads of the oracle's OpenMP loops from now on; returns the previous count."""
    return int(lib().or_set_threads(ctypes.c_int(int(n))))


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def n_sh(deg: int) -> int:
    return (deg + 1) * (deg + 1)


def n_floats(deg: int) -> int:
    return 11 + 3 * n_sh(deg)


@dataclass
class OView:
    """One camera of a step: pose, intrinsics, size, exposure [A|b] (3x4) and background."""
    cam: np.ndarray          # float64[16]
    W: int
    H: int
    E: np.ndarray = field(default_factory=lambda: np.concatenate(
        [np.eye(3), np.zeros((3, 1))], axis=1).reshape(12))
    bg: np.ndarray = field(default_factory=lambda: np.zeros(3))

    @property
    def tiles_x(self):
        return (self.W + TILE - 1) // TILE

    @property
    def tiles_y(self):
        return (self.H + TILE - 1) // TILE

    @property
    def n_tiles(self):
        return self.tiles_x * self.tiles_y


def project(params, deg, view: OView, fp64=False, near=NEAR_Z):
    """Per-Gaussian projection (Eq. 1-3), culls and tile counts for one view."""
    params = np.ascontiguousarray(params, dtype=np.float64)
    N = params.shape[0]
    assert params.shape[1] == n_floats(deg)
    cam = np.ascontiguousarray(view.cam, dtype=np.float64)
    out = dict(
        visible=np.zeros(N, np.uint8), depth_bits=np.zeros(N, np.uint32),
        depth=np.zeros(N), mean2d=np.zeros((N, 2)), conic=np.zeros((N, 3)),
        opacity=np.zeros(N), thr=np.zeros(N), cov2d=np.zeros((N, 3)),
        colour=np.zeros((N, 3)), rect=np.zeros((N, 4), np.int32), count=np.zeros(N, np.int32))
    lib().or_project(ctypes.c_int(N), ctypes.c_int(deg), _p(params), _p(cam),
                     ctypes.c_int(view.W), ctypes.c_int(view.H), ctypes.c_double(near),
                     ctypes.c_int(1 if fp64 else 0),
                     _p(out["visible"]), _p(out["depth_bits"]), _p(out["depth"]),
                     _p(out["mean2d"]), _p(out["conic"]), _p(out["opacity"]), _p(out["thr"]),
                     _p(out["cov2d"]), _p(out["colour"]), _p(out["rect"]), _p(out["count"]))
    return out


def bin_views(projs, views, fp64=False):
    """Emit, stable-sort and range the (tile, Gaussian) instances of several views whose
    tiles are numbered consecutively (view 0's tiles first)."""
    tile_chunks, val_chunks, depth_cat, bits_cat = [], [], [], []
    base, n_total_g = 0, 0
    for pr, v in zip(projs, views):
        N = pr["count"].shape[0]
        counts = pr["count"].astype(np.int64)
        offs = np.zeros(N, np.int64)
        if N > 1:
            offs[1:] = np.cumsum(counts)[:-1]
        n = int(counts.sum())
        tiles = np.zeros(n, np.int64)
        vals = np.zeros(n, np.uint32)
        lib().or_emit(ctypes.c_int(N), ctypes.c_int(v.W), ctypes.c_int(v.H), ctypes.c_int64(base),
                      ctypes.c_int(1 if fp64 else 0), _p(pr["rect"]), _p(pr["count"]),
                      _p(pr["mean2d"]), _p(pr["conic"]), _p(pr["thr"]), _p(offs), _p(tiles),
                      _p(vals))
        tile_chunks.append(tiles)
        # values index the concatenation of all views' per-Gaussian arrays
        val_chunks.append(vals.astype(np.uint64) + n_total_g)
        depth_cat.append(pr["depth"])
        bits_cat.append(pr["depth_bits"])
        base += v.n_tiles
        n_total_g += N
    tiles = np.concatenate(tile_chunks) if tile_chunks else np.zeros(0, np.int64)
    vals_g = np.concatenate(val_chunks).astype(np.uint32) if val_chunks else np.zeros(0, np.uint32)
    depth = np.ascontiguousarray(np.concatenate(depth_cat))
    bits = np.ascontiguousarray(np.concatenate(bits_cat))
    n = tiles.shape[0]
    ts = np.zeros(n, np.int64)
    vs = np.zeros(n, np.uint32)
    ks = np.zeros(n, np.uint64)
    lib().or_sort(ctypes.c_int64(n), _p(tiles), _p(vals_g), _p(depth), _p(bits), _p(ts), _p(vs),
                  _p(ks) if not fp64 else None)
    ranges = np.zeros((base, 2), np.int64)
    lib().or_ranges(ctypes.c_int64(n), _p(ts), ctypes.c_int64(base), _p(ranges))
    # local Gaussian index (the product path stores the Gaussian index, not the view's)
    Ns = [pr["count"].shape[0] for pr in projs]
    view_of = np.repeat(np.arange(len(views)), [v.n_tiles for v in views])
    starts = np.concatenate([[0], np.cumsum(Ns)[:-1]]).astype(np.int64)
    local = (vs.astype(np.int64) - starts[view_of[ts]]).astype(np.uint32) if n else vs
    return dict(tile=ts, val=vs, local_val=local, key=ks if not fp64 else None, ranges=ranges,
                n_tiles=base)


def _cat(projs, name):
    return np.ascontiguousarray(np.concatenate([p[name] for p in projs]))


def render(projs, views, bins, tie_alpha=0.0, tie_T=0.0):
    """Tiled blend of every view. Returns per-view dicts with out (3,H,W), pre, T_final,
    n_contrib, tie flags, the depth map D and the opacity map O (H,W)."""
    mean2d, conic = _cat(projs, "mean2d"), _cat(projs, "conic")
    opac, colour = _cat(projs, "opacity"), _cat(projs, "colour")
    depth = _cat(projs, "depth")
    res, base = [], 0
    for v in views:
        P = v.W * v.H
        D, O = np.zeros(P), np.zeros(P)
        out, pre = np.zeros(3 * P), np.zeros(3 * P)
        Tf, nc, tie = np.zeros(P), np.zeros(P, np.int32), np.zeros(P, np.int32)
        ncon, sig = np.zeros(P, np.int32), np.zeros(P, np.uint64)
        E = np.ascontiguousarray(v.E, dtype=np.float64)
        bg = np.ascontiguousarray(v.bg, dtype=np.float64)
        lib().or_render_tiled(ctypes.c_int(v.W), ctypes.c_int(v.H), ctypes.c_int64(base),
                              _p(bins["ranges"]), _p(bins["val"]), _p(mean2d), _p(conic),
                              _p(opac), _p(colour), _p(E), _p(bg), ctypes.c_double(tie_alpha),
                              ctypes.c_double(tie_T), _p(out), _p(pre), _p(Tf), _p(nc), _p(tie),
                              _p(ncon), _p(sig), _p(depth), _p(D), _p(O))
        res.append(dict(out=out.reshape(3, v.H, v.W), pre=pre.reshape(3, v.H, v.W),
                        T_final=Tf.reshape(v.H, v.W), n_contrib=nc.reshape(v.H, v.W),
                        tie=tie.reshape(v.H, v.W), n_contributors=ncon.reshape(v.H, v.W),
                        signature=sig.reshape(v.H, v.W), depth=D.reshape(v.H, v.W),
                        opacity=O.reshape(v.H, v.W)))
        base += v.n_tiles
    return res


def render_pixels(projs, views, bins, view_index, pix, tie_alpha=0.0, tie_T=0.0):
    """Tiled blend of one view at the flat pixel indices `pix` only."""
    mean2d, conic = _cat(projs, "mean2d"), _cat(projs, "conic")
    opac, colour = _cat(projs, "opacity"), _cat(projs, "colour")
    depth = _cat(projs, "depth")
    base = sum(v.n_tiles for v in views[:view_index])
    v = views[view_index]
    pix = np.ascontiguousarray(pix, dtype=np.int64)
    n = pix.shape[0]
    D, O = np.zeros(n), np.zeros(n)
    out, Tf = np.zeros((n, 3)), np.zeros(n)
    nc, tie = np.zeros(n, np.int32), np.zeros(n, np.int32)
    E = np.ascontiguousarray(v.E, dtype=np.float64)
    bg = np.ascontiguousarray(v.bg, dtype=np.float64)
    lib().or_render_tiled_pixels(ctypes.c_int(v.W), ctypes.c_int(v.H), ctypes.c_int64(base),
                                 _p(bins["ranges"]), _p(bins["val"]), _p(mean2d), _p(conic), _p(opac),
                                 _p(colour), _p(E), _p(bg), ctypes.c_double(tie_alpha),
                                 ctypes.c_double(tie_T), ctypes.c_int64(n), _p(pix), _p(out), _p(Tf),
                                 _p(nc), _p(tie), _p(depth), _p(D), _p(O))
    return dict(out=out, T_final=Tf, n_contrib=nc, tie=tie, depth=D, opacity=O)


def render_brute(proj, view: OView):
    """Per-pixel blend over all visible Gaussians in (depth, index) order; no tiles."""
    N = proj["count"].shape[0]
    P = view.W * view.H
    out, Tf, nc = np.zeros(3 * P), np.zeros(P), np.zeros(P, np.int32)
    D, O = np.zeros(P), np.zeros(P)
    E = np.ascontiguousarray(view.E, dtype=np.float64)
    bg = np.ascontiguousarray(view.bg, dtype=np.float64)
    lib().or_render_brute(ctypes.c_int(N), ctypes.c_int(view.W), ctypes.c_int(view.H),
                          _p(proj["visible"]), _p(proj["depth"]), _p(proj["mean2d"]),
                          _p(proj["conic"]), _p(proj["opacity"]), _p(proj["colour"]), _p(E),
                          _p(bg), _p(out), _p(Tf), _p(nc), _p(D), _p(O))
    return dict(out=out.reshape(3, view.H, view.W), T_final=Tf.reshape(view.H, view.W),
                n_contributors=nc.reshape(view.H, view.W), depth=D.reshape(view.H, view.W),
                opacity=O.reshape(view.H, view.W))


def loss(out, gt, lam):
    """Eq. 9: (1 - lam) mean|out - gt| + lam (1 - mean SSIM); returns (L, dL/dout, ssim)."""
    out = np.ascontiguousarray(out, dtype=np.float64)
    gt = np.ascontiguousarray(gt, dtype=np.float64)
    _, H, W = out.shape
    g = np.zeros_like(out)
    ss = ctypes.c_double(0.0)
    L = lib().or_loss(ctypes.c_int(H), ctypes.c_int(W), _p(out), _p(gt), ctypes.c_double(lam),
                      _p(g), ctypes.byref(ss))
    return float(L), g, float(ss.value)


def blend_backward(projs, views, bins, gouts, tie_alpha=0.0, tie_T=0.0, gdepths=None, gopacs=None):
    """Adjoint of the blend: per view, per Gaussian (mean2d 2, conic 3, opacity, colour 3,
    depth) gradients, exposure gradients (12) and tie flags. gdepths / gopacs: optional
    per-view dL/dD and dL/dO maps (H, W)."""
    mean2d, conic = _cat(projs, "mean2d"), _cat(projs, "conic")
    opac, colour = _cat(projs, "opacity"), _cat(projs, "colour")
    depth = _cat(projs, "depth")
    Ntot = mean2d.shape[0]
    g2d = np.zeros((Ntot, 10))
    gtie = np.zeros(Ntot, np.uint8)
    gEs, base = [], 0
    for k, (v, go) in enumerate(zip(views, gouts)):
        gE = np.zeros(12)
        E = np.ascontiguousarray(v.E, dtype=np.float64)
        bg = np.ascontiguousarray(v.bg, dtype=np.float64)
        go = np.ascontiguousarray(go, dtype=np.float64).reshape(-1)
        gD = None if gdepths is None or gdepths[k] is None else \
            np.ascontiguousarray(gdepths[k], dtype=np.float64).reshape(-1)
        gO = None if gopacs is None or gopacs[k] is None else \
            np.ascontiguousarray(gopacs[k], dtype=np.float64).reshape(-1)
        lib().or_blend_backward(ctypes.c_int(v.W), ctypes.c_int(v.H), ctypes.c_int64(base),
                                _p(bins["ranges"]), _p(bins["val"]), _p(mean2d), _p(conic),
                                _p(opac), _p(colour), _p(E), _p(bg), ctypes.c_double(tie_alpha),
                                ctypes.c_double(tie_T), _p(go), _p(g2d), _p(gE), _p(gtie), _p(depth),
                                _p(gD) if gD is not None else None, _p(gO) if gO is not None else None)
        gEs.append(gE)
        base += v.n_tiles
    Ns = [p["count"].shape[0] for p in projs]
    splits = np.cumsum(Ns)[:-1]
    return np.split(g2d, splits), gEs, np.split(gtie, splits)


def project_backward(params, deg, view: OView, visible, g2d, near=NEAR_Z):
    """Chain rule from one view's 2D gradients to the parameter rows (FP64)."""
    params = np.ascontiguousarray(params, dtype=np.float64)
    N = params.shape[0]
    gp = np.zeros_like(params)
    cam = np.ascontiguousarray(view.cam, dtype=np.float64)
    g2d = np.ascontiguousarray(g2d, dtype=np.float64)
    vis = np.ascontiguousarray(visible, dtype=np.uint8)
    lib().or_project_backward(ctypes.c_int(N), ctypes.c_int(deg), _p(params), _p(cam),
                              ctypes.c_int(view.W), ctypes.c_int(view.H), ctypes.c_double(near),
                              _p(vis), _p(g2d), _p(gp))
    return gp


def sh_basis(deg, dirs):
    dirs = np.ascontiguousarray(dirs, dtype=np.float64)
    Y = np.zeros((dirs.shape[0], n_sh(deg)))
    lib().or_sh_basis(ctypes.c_int(deg), ctypes.c_int(dirs.shape[0]), _p(dirs), _p(Y))
    return Y


def adam(p, g, m, v, vis, lr, beta1, beta2, eps, t):
    """Sparse Adam on row-major (N, F) arrays; returns updated copies (p, g, m, v)."""
    p, g, m, v = (np.array(a, dtype=np.float64, order="C") for a in (p, g, m, v))
    N, F = p.shape
    lr = np.ascontiguousarray(np.broadcast_to(np.asarray(lr, np.float64), (F,)))
    vis = np.ascontiguousarray(vis, dtype=np.uint8)
    lib().or_adam(ctypes.c_int64(N), ctypes.c_int(F), _p(p), _p(g), _p(m), _p(v), _p(vis), _p(lr),
                  ctypes.c_double(beta1), ctypes.c_double(beta2), ctypes.c_double(eps),
                  ctypes.c_int64(t))
    return p, g, m, v


def forward(params, deg, views, fp64=False, tie_alpha=0.0, tie_T=0.0):
    """Project, bin and blend every view; returns (projs, bins, renders)."""
    projs = [project(params, deg, v, fp64=fp64) for v in views]
    bins = bin_views(projs, views, fp64=fp64)
    rend = render(projs, views, bins, tie_alpha=tie_alpha, tie_T=tie_T)
    return projs, bins, rend


def backward(params, deg, views, projs, bins, gouts, tie_alpha=0.0, tie_T=0.0, gdepths=None, gopacs=None):
    """Full adjoint: parameter-row gradients summed over views, exposure gradients per view,
    per-Gaussian tie flags (OR over views). gdepths / gopacs: optional dL/dD and dL/dO."""
    g2ds, gEs, gties = blend_backward(projs, views, bins, gouts, tie_alpha, tie_T, gdepths, gopacs)
    gp = np.zeros_like(np.asarray(params, dtype=np.float64))
    tie = np.zeros(gp.shape[0], np.uint8)
    for v, pr, g2d, gt in zip(views, projs, g2ds, gties):
        gp += project_backward(params, deg, v, pr["visible"], g2d)
        tie |= gt
    return gp, gEs, tie


# ------------------------------------------------------------------ map growth
# Sec. III-C.1 (initialisation from points, sky) and Sec. III-C.2 (expansion, Eq. 8).
# Plain numpy; the pixel a point falls on is an integer decision and is taken in the FP32
# order of the key path (x_c = ((R00 x + R01 y) + R02 z) + t0, u = f_x (x_c / z_c) + c_x).

SH_C0 = 0.28209479177387814   # Y_00 = 1 / (2 sqrt(pi))


def point_pixels(xyz, view: OView, near=NEAR_Z):
    """(inside, px, py, z) of each point under the view: camera-frame z > near and the
    projection (u, v) within [0, W) x [0, H); px = floor(u), py = floor(v)."""
    f32 = np.float32
    c = np.asarray(view.cam, np.float64).astype(f32)
    p = np.asarray(xyz, np.float64).astype(f32)
    x, y, z = p[:, 0], p[:, 1], p[:, 2]
    xc = ((c[0] * x + c[1] * y) + c[2] * z) + c[9]
    yc = ((c[3] * x + c[4] * y) + c[5] * z) + c[10]
    zc = ((c[6] * x + c[7] * y) + c[8] * z) + c[11]
    with np.errstate(divide="ignore", invalid="ignore"):
        u = c[12] * (xc / zc) + c[14]
        v = c[13] * (yc / zc) + c[15]
    inside = (zc > f32(near)) & (u >= 0) & (u < f32(view.W)) & (v >= 0) & (v < f32(view.H))
    px = np.where(inside, np.floor(np.where(inside, u, 0)), -1).astype(np.int64)
    py = np.where(inside, np.floor(np.where(inside, v, 0)), -1).astype(np.int64)
    return inside, px, py, zc.astype(np.float64)


def init_points(xyz, rgb, view: OView, o_init, deg, near=NEAR_Z):
    """Sec. III-C.1: one Gaussian per point, centred on it, SH DC so that it renders as the
    point's colour (colour = Y00 dc + 0.5), other SH 0, opacity o_init, identity rotation,
    isotropic scale d / f_x with d the point's depth in the view (clamped below at near)."""
    xyz = np.asarray(xyz, np.float64)
    rgb = np.asarray(rgb, np.float64)
    n = xyz.shape[0]
    R = np.asarray(view.cam[:9], np.float64).reshape(3, 3)
    d = xyz @ R[2] + view.cam[11]
    ls = np.log(np.maximum(d, near) / view.cam[12])
    K = n_sh(deg)
    rows = np.zeros((n, 11 + 3 * K))
    rows[:, 0:3] = xyz
    rows[:, 3:6] = ls[:, None]
    rows[:, 6] = 1.0
    rows[:, 10] = np.log(o_init / (1.0 - o_init))
    rows[:, 11:14] = (rgb - 0.5) / SH_C0
    return rows


def expansion_select(xyz, view: OView, opacity, tau, near=NEAR_Z, tie=0.0):
    """Eq. 8: M = O < tau over the keyframe's opacity map; a point is kept when it
    projects inside the image onto a pixel of M. Returns (keep, tie_flags): tie_flags marks
    points whose pixel has |O - tau| <= tie (a decision the FP32 path may take the other way)."""
    inside, px, py, _ = point_pixels(xyz, view, near)
    O = np.asarray(opacity, np.float64)
    o = np.where(inside, O[np.maximum(py, 0), np.maximum(px, 0)], np.inf)
    keep = inside & (o < tau)
    ties = inside & (np.abs(o - tau) <= tie)
    return keep, ties


def keyframe_merges(n_frames, period=5):
    """Sec. III-C.2 frame rule: every fifth frame (0, 5, 10, ...) is a keyframe. Frame 0
    bootstraps the map with its own points; a later keyframe f merges the points of the
    frames since the previous keyframe, f - 4 .. f, in arrival order. Returns
    [(keyframe, [frames whose points it uses])] for the keyframes among n_frames frames."""
    out = []
    for f in range(0, n_frames, period):
        out.append((f, [0] if f == 0 else list(range(f - period + 1, f + 1))))
    return out


def nearest_neighbour_distance(xyz):
    """Distance from every point to its closest other point (brute force)."""
    p = np.asarray(xyz, np.float64)
    n = p.shape[0]
    out = np.full(n, np.inf)
    for s in range(0, n, 1024):
        d2 = ((p[s:s + 1024, None, :] - p[None, :, :]) ** 2).sum(-1)
        idx = np.arange(s, min(s + 1024, n))
        d2[idx - s, idx] = np.inf
        out[s:s + 1024] = np.sqrt(d2.min(axis=1))
    return out


def init_sky(xyz, o_sky, deg):
    """Sec. III-C.1 sky Gaussians at the given positions: white SH DC (colour 1), opacity
    o_sky, identity rotation, isotropic scale = distance to the closest other sky Gaussian."""
    xyz = np.asarray(xyz, np.float64)
    n = xyz.shape[0]
    K = n_sh(deg)
    rows = np.zeros((n, 11 + 3 * K))
    rows[:, 0:3] = xyz
    rows[:, 3:6] = np.log(nearest_neighbour_distance(xyz))[:, None]
    rows[:, 6] = 1.0
    rows[:, 10] = np.log(o_sky / (1.0 - o_sky))
    rows[:, 11:14] = (1.0 - 0.5) / SH_C0
    return rows
