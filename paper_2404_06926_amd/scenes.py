"""Seeded synthetic inputs: Gaussian maps, cameras and exposures.

This module only draws random numbers and lays out geometry for inputs. It holds none of
the rendering or optimisation arithmetic, so both the HIP path and the CPU oracle can take
their inputs from it. Every array is drawn from its own stream keyed by (seed, name).

Shapes follow the paper's workloads: outdoor LiDAR-shaped scenes (Sec. IV-A.2 uses
640x512 / 640x480 driving and campus sequences that are not available here), Gaussians
initialised from points with scale d/f (Sec. III-C.1), SH of degree 3 (Sec. III-A).

Parameter rows are float32 ``(N, 11 + 3K)``: mean (3), log-scale (3), quaternion w,x,y,z
(4), opacity logit (1), SH coefficients [k][channel] (3K), K = (deg + 1)^2.
"""
from __future__ import annotations

import zlib
from dataclasses import dataclass, field

import numpy as np


def n_sh(deg: int) -> int:
    return (deg + 1) * (deg + 1)


def n_floats(deg: int) -> int:
    return 11 + 3 * n_sh(deg)


def rng(seed: int, name: str) -> np.random.Generator:
    """Independent stream for (seed, tensor name)."""
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, zlib.crc32(name.encode())])))


@dataclass
class Camera:
    """Pinhole camera: world->camera rotation R (3x3), translation t, intrinsics, size."""
    R: np.ndarray
    t: np.ndarray
    fx: float
    fy: float
    cx: float
    cy: float
    width: int
    height: int
    exposure: np.ndarray = field(default_factory=lambda: identity_exposure())
    bg: np.ndarray = field(default_factory=lambda: np.zeros(3, np.float32))

    def __post_init__(self):
        self.R = np.asarray(self.R, np.float32).reshape(3, 3)
        self.t = np.asarray(self.t, np.float32).reshape(3)
        self.fx, self.fy = float(np.float32(self.fx)), float(np.float32(self.fy))
        self.cx, self.cy = float(np.float32(self.cx)), float(np.float32(self.cy))
        self.exposure = np.asarray(self.exposure, np.float32).reshape(12)
        self.bg = np.asarray(self.bg, np.float32).reshape(3)

    def cam16(self) -> np.ndarray:
        """float64[16] of the float32 values: R row-major, t, fx, fy, cx, cy."""
        return np.concatenate([self.R.reshape(9), self.t,
                               np.array([self.fx, self.fy, self.cx, self.cy], np.float32)]).astype(np.float64)


def identity_exposure() -> np.ndarray:
    """3x4 [A | b] with A = I, b = 0, row-major."""
    return np.concatenate([np.eye(3), np.zeros((3, 1))], axis=1).reshape(12).astype(np.float32)


def random_exposure(seed: int, name: str = "exposure") -> np.ndarray:
    """A = I + N(0, 0.05) entries, b = N(0, 0.02)."""
    r = rng(seed, name)
    A = np.eye(3) + r.normal(0.0, 0.05, (3, 3))
    b = r.normal(0.0, 0.02, (3, 1))
    return np.concatenate([A, b], axis=1).reshape(12).astype(np.float32)


def pinhole(width: int, height: int, f: float, R=None, t=None, cx=None, cy=None) -> Camera:
    return Camera(R=np.eye(3) if R is None else R, t=np.zeros(3) if t is None else t,
                  fx=f, fy=f, cx=width / 2 if cx is None else cx, cy=height / 2 if cy is None else cy,
                  width=width, height=height)


def axis_angle(v) -> np.ndarray:
    """Rotation matrix of the rotation vector v (Rodrigues)."""
    v = np.asarray(v, np.float64)
    th = np.linalg.norm(v)
    if th < 1e-15:
        return np.eye(3)
    k = v / th
    K = np.array([[0, -k[2], k[1]], [k[2], 0, -k[0]], [-k[1], k[0], 0]])
    return np.eye(3) + np.sin(th) * K + (1 - np.cos(th)) * K @ K


def random_quats(r: np.random.Generator, n: int) -> np.ndarray:
    q = r.normal(size=(n, 4))
    return q / np.linalg.norm(q, axis=1, keepdims=True)


def _assemble(means, log_scales, quats, logits, sh) -> np.ndarray:
    n = means.shape[0]
    return np.concatenate([means, log_scales, quats, logits.reshape(n, 1), sh.reshape(n, sh.shape[1] * sh.shape[2])],
                          axis=1).astype(np.float32)


def frustum_gaussians(n: int, deg: int, cam: Camera, seed: int, zmin: float = 2.0,
                      zmax: float = 20.0, log_scale_mean: float = -3.0) -> np.ndarray:
    """Means volume-uniform in the camera frustum between zmin and zmax (camera at the
    origin looking +z), log-scales N(mu, 0.5), random unit quaternions, logits N(0, 1),
    SH DC N(0.5, 0.2), higher SH N(0, 0.05)."""
    r = rng(seed, "means")
    z = np.cbrt(zmin ** 3 + r.random(n) * (zmax ** 3 - zmin ** 3))
    u = r.random(n) * cam.width
    v = r.random(n) * cam.height
    pc = np.stack([(u - cam.cx) * z / cam.fx, (v - cam.cy) * z / cam.fy, z], axis=1)
    # camera -> world
    means = (pc - cam.t[None, :]) @ cam.R
    log_scales = rng(seed, "log_scales").normal(log_scale_mean, 0.5, (n, 3))
    quats = random_quats(rng(seed, "quats"), n)
    logits = rng(seed, "logits").normal(0.0, 1.0, n)
    K = n_sh(deg)
    sh = np.zeros((n, K, 3))
    sh[:, 0, :] = rng(seed, "sh_dc").normal(0.5, 0.2, (n, 3))
    if K > 1:
        sh[:, 1:, :] = rng(seed, "sh_rest").normal(0.0, 0.05, (n, K - 1, 3))
    return _assemble(means, log_scales, quats, logits, sh)


def jitter_means(params: np.ndarray, sigma: float, seed: int) -> np.ndarray:
    out = params.copy()
    out[:, 0:3] += rng(seed, "jitter").normal(0.0, sigma, (params.shape[0], 3)).astype(np.float32)
    return out


def look_camera(width, height, f, position, forward, up=(0.0, 0.0, 1.0)) -> Camera:
    """Camera at `position` looking along `forward` in a z-up world; camera axes are
    x right, y down, z forward."""
    fwd = np.asarray(forward, np.float64)
    fwd /= np.linalg.norm(fwd)
    right = np.cross(fwd, np.asarray(up, np.float64))
    right /= np.linalg.norm(right)
    down = np.cross(fwd, right)
    R = np.stack([right, down, fwd])
    t = -R @ np.asarray(position, np.float64)
    return Camera(R=R, t=t, fx=f, fy=f, cx=width / 2, cy=height / 2, width=width, height=height)


def outdoor_scene(seed: int, deg: int = 3, n_ground=273_000, n_facade=182_000, n_tri=25_000,
                  n_sky=20_000, cam_x: float = 20.0):
    """LiDAR-shaped street scene along a 100 m straight ego path (world z-up): ground plane,
    facade segments at y = +-12 m, sparse far points at 30-80 m, and a sky shell of radius
    500 m. Returns (params, camera at x = cam_x, height 1.8 m, looking +x)."""
    cam = look_camera(1280, 720, 1000.0, (cam_x, 0.0, 1.8), (1.0, 0.0, 0.0))
    r = rng(seed, "outdoor_points")
    ground = np.stack([r.uniform(0, 100, n_ground), r.uniform(-15, 15, n_ground), np.zeros(n_ground)], 1)
    fac = []
    side = 0
    while sum(len(f) for f in fac) < n_facade:
        x = r.uniform(0, 5)
        while x < 100:
            length = r.uniform(10, 25)
            height = r.uniform(6, 15)
            m = int(1400 * length * height / 150)
            fx_ = r.uniform(x, min(x + length, 100), m)
            fz = r.uniform(0, height, m)
            fac.append(np.stack([fx_, np.full(m, 12.0 if side % 2 == 0 else -12.0), fz], 1))
            x += length + r.uniform(3, 8)
        side += 1
    facade = np.concatenate(fac)[:n_facade]
    rr = r.uniform(30, 80, n_tri)
    az = r.uniform(-np.pi / 2, np.pi / 2, n_tri)
    tri = np.stack([cam_x + rr * np.cos(az), rr * np.sin(az), r.uniform(0, 25, n_tri)], 1)
    pts = np.concatenate([ground, facade, tri])
    pts += r.normal(0, 0.02, pts.shape)
    # sky: area-uniform on the upper hemisphere around (50, 0, 0)
    cz = r.uniform(0, 1, n_sky)
    ph = r.uniform(0, 2 * np.pi, n_sky)
    sr = np.sqrt(1 - cz ** 2)
    sky = np.stack([50 + 500 * sr * np.cos(ph), 500 * sr * np.sin(ph), 500 * cz], 1)
    n_fg = pts.shape[0]
    means = np.concatenate([pts, sky])
    n = means.shape[0]
    d = np.linalg.norm(means - np.array([cam_x, 0.0, 1.8]), axis=1)
    ls = np.log(np.maximum(d, 0.5) / 1000.0)[:, None] + rng(seed, "log_scales").normal(0, 0.3, (n, 3))
    # sky spacing: mean nearest-neighbour distance of n_sky points on the hemisphere
    spacing = np.sqrt(2 * np.pi * 500.0 ** 2 / n_sky)
    ls[n_fg:] = np.log(spacing) + rng(seed, "sky_log_scales").normal(0, 0.3, (n - n_fg, 3))
    quats = random_quats(rng(seed, "quats"), n)
    logits = rng(seed, "logits").normal(0.0, 1.0, n)
    K = n_sh(deg)
    sh = np.zeros((n, K, 3))
    sh[:, 0, :] = rng(seed, "sh_dc").normal(0.5, 0.2, (n, 3))
    if K > 1:
        sh[:, 1:, :] = rng(seed, "sh_rest").normal(0.0, 0.05, (n, K - 1, 3))
    return _assemble(means, ls, quats, logits, sh), cam


BATCH_SIZES = [(640, 400), (960, 600), (1280, 720), (1440, 1080)]


def batch_views(seed: int, n_views: int = 8):
    """Uneven keyframes around the reference camera at the origin looking +z: sizes from
    BATCH_SIZES (each twice, shuffled), f = 200 W / 256, c = image centre, position noise
    N(0, 0.3 m), rotation noise N(0, 3 deg) axis-angle."""
    r = rng(seed, "batch_views")
    sizes = [BATCH_SIZES[i % len(BATCH_SIZES)] for i in range(n_views)]
    order = r.permutation(n_views)
    cams = []
    for k in order:
        w, h = sizes[k]
        Rn = axis_angle(r.normal(0, np.deg2rad(3.0), 3))
        pos = r.normal(0, 0.3, 3)
        # world->camera: x_c = Rn (x_w - pos)
        cams.append(Camera(R=Rn, t=-Rn @ pos, fx=200.0 * w / 256, fy=200.0 * w / 256,
                           cx=w / 2, cy=h / 2, width=w, height=h))
    return cams


def smooth_image(seed: int, H: int, W: int, name: str = "image") -> np.ndarray:
    """A smooth random RGB image in [0, 1] (3, H, W) used as a stand-in target."""
    r = rng(seed, name)
    yy, xx = np.mgrid[0:H, 0:W] / max(H, W)
    img = np.zeros((3, H, W))
    for c in range(3):
        for _ in range(4):
            a, fx_, fy_, ph = r.uniform(0.05, 0.2), r.uniform(1, 8), r.uniform(1, 8), r.uniform(0, 6.3)
            img[c] += a * np.sin(2 * np.pi * (fx_ * xx + fy_ * yy) + ph)
    img += 0.5 + r.normal(0, 0.02, img.shape)
    return np.clip(img, 0, 1).astype(np.float32)


# ---------------------------------------------------------------------------------------
# Streaming street scene: a straight ego path along +x (world z-up), LiDAR-like points
# arriving with the keyframes.

STREET_MIX = (273, 182, 25)   # ground : facade : far-point proportions of outdoor_scene


def street_layout(seed: int, length: float = 500.0) -> np.ndarray:
    """Facade segments along both sides of the path: rows (x_start, x_end, y, height),
    segments 10-25 m long with 3-8 m gaps, heights 6-15 m, at y = +-12 m."""
    r = rng(seed, "street_layout")
    segs = []
    for y in (12.0, -12.0):
        x = r.uniform(0, 5)
        while x < length:
            seg_len = r.uniform(10, 25)
            segs.append((x, min(x + seg_len, length), y, r.uniform(6, 15)))
            x += seg_len + r.uniform(3, 8)
    return np.array(segs)


def street_points(seed: int, layout: np.ndarray, x0: float, x1: float, n: int, key: str):
    """n points of the slab x in [x0, x1] in the outdoor_scene proportions: ground
    (|y| <= 15 m), facade segments of `layout`, sparse far points 30-80 m ahead of x0;
    +-2 cm noise. Colours: grey ground, one colour per facade segment, random far points,
    all with N(0, 0.03) noise. Returns (xyz (n, 3), rgb (n, 3)) float32."""
    r = rng(seed, "street_points/" + key)
    tot = sum(STREET_MIX)
    n_g = int(round(n * STREET_MIX[0] / tot))
    n_f = int(round(n * STREET_MIX[1] / tot))
    n_t = n - n_g - n_f
    ground = np.stack([r.uniform(x0, x1, n_g), r.uniform(-15, 15, n_g), np.zeros(n_g)], 1)
    g_rgb = np.full((n_g, 3), 0.4)
    ov0 = np.maximum(layout[:, 0], x0)
    ov1 = np.minimum(layout[:, 1], x1)
    w = np.maximum(ov1 - ov0, 0.0) * layout[:, 3]
    if n_f and w.sum() > 0:
        seg = r.choice(len(layout), n_f, p=w / w.sum())
        fac = np.stack([r.uniform(ov0[seg], ov1[seg]), layout[seg, 2], r.uniform(0, layout[seg, 3])], 1)
        seg_col = rng(seed, "street_facade_colours").uniform(0.2, 0.9, (len(layout), 3))
        f_rgb = seg_col[seg]
    else:  # no facade in the slab: those points go to the ground
        fac = np.stack([r.uniform(x0, x1, n_f), r.uniform(-15, 15, n_f), np.zeros(n_f)], 1)
        f_rgb = np.full((n_f, 3), 0.4)
    rr = r.uniform(30, 80, n_t)
    az = r.uniform(-np.pi / 2, np.pi / 2, n_t)
    far = np.stack([x0 + rr * np.cos(az), rr * np.sin(az), r.uniform(0, 25, n_t)], 1)
    t_rgb = r.uniform(0.1, 0.9, (n_t, 3))
    xyz = np.concatenate([ground, fac, far]) + r.normal(0, 0.02, (n, 3))
    rgb = np.clip(np.concatenate([g_rgb, f_rgb, t_rgb]) + r.normal(0, 0.03, (n, 3)), 0, 1)
    return xyz.astype(np.float32), rgb.astype(np.float32)


def street_gaussians(seed: int, xyz: np.ndarray, rgb: np.ndarray, deg: int, ref=None) -> np.ndarray:
    """Gaussians on points: log-scales ln(d / 1000) + N(0, 0.3) with d the distance to the
    point `ref` (or, with ref None, to the ego path: the line y = 0, z = 1.8 m), random unit
    quaternions, logits N(0, 1), SH DC from the colour plus N(0, 0.05), higher SH N(0, 0.05)."""
    n = xyz.shape[0]
    if ref is None:
        d = np.hypot(xyz[:, 1], xyz[:, 2] - 1.8)
    else:
        d = np.linalg.norm(xyz - np.asarray(ref, np.float64)[None, :], axis=1)
    ls = np.log(np.maximum(d, 0.5) / 1000.0)[:, None] + rng(seed, "street_log_scales").normal(0, 0.3, (n, 3))
    quats = random_quats(rng(seed, "street_quats"), n)
    logits = rng(seed, "street_logits").normal(0.0, 1.0, n)
    K = n_sh(deg)
    sh = np.zeros((n, K, 3))
    sh[:, 0, :] = (rgb - 0.5) / 0.28209479177387814 + rng(seed, "street_dc").normal(0, 0.05, (n, 3))
    if K > 1:
        sh[:, 1:, :] = rng(seed, "street_sh_rest").normal(0.0, 0.05, (n, K - 1, 3))
    return _assemble(xyz, ls, quats, logits, sh)


def stream_schedule(seed: int, duration_s: float, rate_hz: float = 10.0, length: float = 500.0):
    """Keyframe arrival times (Poisson, rate_hz) and the ego position at each: speed
    re-drawn from U[5, 15] m/s every 5 s, camera yaw = heading + N(0, 5 deg).
    Returns (arrivals, x, yaw) arrays."""
    r = rng(seed, "stream_schedule")
    arrivals = []
    t = 0.0
    while True:
        t += r.exponential(1.0 / rate_hz)
        if t >= duration_s:
            break
        arrivals.append(t)
    arrivals = np.array(arrivals)
    n_seg = int(np.ceil(max(duration_s, 1e-9) / 5.0)) + 1
    speeds = r.uniform(5, 15, n_seg)
    seg_start = np.concatenate([[0.0], np.cumsum(speeds * 5.0)])

    def pos(tt):
        k = min(int(tt // 5.0), n_seg - 1)
        return seg_start[k] + speeds[k] * (tt - 5.0 * k)

    x = np.array([min(pos(a), length - 60.0) for a in arrivals])
    yaw = r.normal(0, np.deg2rad(5.0), len(arrivals))
    return arrivals, x, yaw


def street_camera(x: float, yaw: float, width: int = 1280, height: int = 720, f: float = 1000.0) -> Camera:
    """Camera 1.8 m above the path at x looking along heading +x rotated by yaw."""
    return look_camera(width, height, f, (x, 0.0, 1.8), (np.cos(yaw), np.sin(yaw), 0.0))


def sky_gaussians(seed: int, n: int, centre, radius: float, deg: int) -> np.ndarray:
    """Sky shell: n Gaussians area-uniform on the upper hemisphere of `radius` around
    `centre`, log-scales ln(mean point spacing) + N(0, 0.3), light-blue DC colour."""
    r = rng(seed, "sky_points")
    cz = r.uniform(0, 1, n)
    ph = r.uniform(0, 2 * np.pi, n)
    sr = np.sqrt(1 - cz ** 2)
    c = np.asarray(centre, np.float64)
    xyz = np.stack([c[0] + radius * sr * np.cos(ph), c[1] + radius * sr * np.sin(ph), c[2] + radius * cz], 1)
    spacing = np.sqrt(2 * np.pi * radius ** 2 / max(n, 1))
    ls = np.log(spacing) + rng(seed, "sky_log_scales").normal(0, 0.3, (n, 3))
    quats = random_quats(rng(seed, "sky_quats"), n)
    logits = rng(seed, "sky_logits").normal(0.0, 1.0, n)
    K = n_sh(deg)
    sh = np.zeros((n, K, 3))
    sh[:, 0, :] = (np.array([0.6, 0.75, 0.9]) - 0.5) / 0.28209479177387814
    sh[:, 0, :] += rng(seed, "sky_dc").normal(0, 0.05, (n, 3))
    return _assemble(xyz, ls, quats, logits, sh)
