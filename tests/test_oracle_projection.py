"""Pins of the oracle's projection (Sec. III-A, Eq. 1-3), culls, tile predicate
(Sec. III-D.2) and SH basis against closed forms, textbook special cases, an independent
numerical optimiser and brute force. No GPU."""
import numpy as np
import pytest
from scipy.optimize import minimize

import oracle
from helpers import Y00, dc_for_colour, gauss_row, logit, oview
from paper_2404_06926_amd import scenes


def cam64():
    return scenes.pinhole(64, 48, 50.0)


def proj_one(row, cam, deg=0, fp64=True):
    return oracle.project(row[None, :], deg, oview(cam), fp64=fp64)


def cov_from_conic(c):
    A, B, C = c
    return np.linalg.inv(np.array([[A, B], [B, C]]))


def test_isotropic_on_axis_closed_form():
    # Isotropic scale s at depth Z on the optical axis: Sigma' = (f s / Z)^2 I + 0.3 I.
    s, Z, f = 0.1, 5.0, 50.0
    pr = proj_one(gauss_row([0, 0, Z], np.log(s), logit=logit(0.8)), cam64())
    assert pr["visible"][0] == 1
    np.testing.assert_allclose(pr["mean2d"][0], [32.0, 24.0], atol=1e-12)
    expect = ((f * s / Z) ** 2 + 0.3) * np.eye(2)
    np.testing.assert_allclose(cov_from_conic(pr["conic"][0]), expect, rtol=1e-12)
    np.testing.assert_allclose(pr["depth"][0], Z)
    np.testing.assert_allclose(pr["opacity"][0], 0.8, rtol=1e-12)
    np.testing.assert_allclose(pr["thr"][0], 2 * np.log(255 * 0.8), rtol=1e-12)


def test_isotropic_off_axis_closed_form():
    # Isotropic: R_cw Sigma R_cw^T = s^2 I, so Sigma' = s^2 J J^T + 0.3 I with the pinhole
    # Jacobian J = [[f/Z, 0, -f X/Z^2], [0, f/Z, -f Y/Z^2]].
    s, f = 0.07, 50.0
    X, Y, Z = 1.0, -0.5, 5.0
    pr = proj_one(gauss_row([X, Y, Z], np.log(s), quat=[0.3, -0.2, 0.9, 0.1]), cam64())
    J = np.array([[f / Z, 0, -f * X / Z ** 2], [0, f / Z, -f * Y / Z ** 2]])
    np.testing.assert_allclose(cov_from_conic(pr["conic"][0]), s * s * J @ J.T + 0.3 * np.eye(2),
                               rtol=1e-12)
    np.testing.assert_allclose(pr["mean2d"][0], [f * X / Z + 32, f * Y / Z + 24], rtol=1e-14)


def test_offscreen_jacobian_clamp():
    # Beyond 1.3 tan(half fov) the Jacobian is taken at the clamped point X_c = 1.3 tanx Z.
    s, f, Z = 0.05, 50.0, 4.0
    lim = 1.3 * 32.0 / f
    X = 2.0 * Z  # X/Z = 2 > lim
    pr = proj_one(gauss_row([X, 0.0, Z], np.log(s)), cam64())
    J = np.array([[f / Z, 0, -f * lim * Z / Z ** 2], [0, f / Z, 0.0]])
    np.testing.assert_allclose(cov_from_conic(pr["conic"][0]), s * s * J @ J.T + 0.3 * np.eye(2),
                               rtol=1e-12)


@pytest.mark.parametrize("theta", [0.3, -1.1, 2.0])
def test_anisotropic_rotation_about_optical_axis(theta):
    # q = (cos th/2, 0, 0, sin th/2) rotates by +th about z: on axis,
    # Sigma' = (f/Z)^2 R_th diag(s1^2, s2^2) R_th^T + 0.3 I.
    s1, s2, s3, Z, f = 0.2, 0.05, 0.1, 5.0, 50.0
    q = [np.cos(theta / 2), 0, 0, np.sin(theta / 2)]
    pr = proj_one(gauss_row([0, 0, Z], np.log([s1, s2, s3]), quat=q), cam64())
    R = np.array([[np.cos(theta), -np.sin(theta)], [np.sin(theta), np.cos(theta)]])
    expect = (f / Z) ** 2 * R @ np.diag([s1 ** 2, s2 ** 2]) @ R.T + 0.3 * np.eye(2)
    np.testing.assert_allclose(cov_from_conic(pr["conic"][0]), expect, rtol=1e-11)


def test_quarter_turns_about_x_and_y():
    s = np.array([0.2, 0.05, 0.1])
    Z, f = 5.0, 50.0
    c45 = np.sqrt(0.5)
    # about x by 90 deg: camera-y sees the third scale
    pr = proj_one(gauss_row([0, 0, Z], np.log(s), quat=[c45, c45, 0, 0]), cam64())
    np.testing.assert_allclose(cov_from_conic(pr["conic"][0]),
                               (f / Z) ** 2 * np.diag([s[0] ** 2, s[2] ** 2]) + 0.3 * np.eye(2),
                               rtol=1e-11, atol=1e-12)
    # about y by 90 deg: camera-x sees the third scale
    pr = proj_one(gauss_row([0, 0, Z], np.log(s), quat=[c45, 0, c45, 0]), cam64())
    np.testing.assert_allclose(cov_from_conic(pr["conic"][0]),
                               (f / Z) ** 2 * np.diag([s[2] ** 2, s[1] ** 2]) + 0.3 * np.eye(2),
                               rtol=1e-11, atol=1e-12)


def test_quaternion_scale_invariance():
    # only the direction of q matters
    row = gauss_row([0.3, 0.2, 4.0], np.log([0.1, 0.03, 0.2]), quat=[0.5, -0.1, 0.7, 0.2])
    row2 = row.copy()
    row2[6:10] *= 3.7
    a, b = proj_one(row, cam64()), proj_one(row2, cam64())
    np.testing.assert_allclose(a["conic"], b["conic"], rtol=1e-12)


def qmul(a, b):
    w1, x1, y1, z1 = a
    w2, x2, y2, z2 = b
    return np.array([w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2, w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
                     w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2, w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2])


def test_rigid_motion_invariance():
    # Moving world and camera together leaves every 2D quantity unchanged.
    cam = scenes.pinhole(256, 192, 200.0)
    params = scenes.frustum_gaussians(300, 0, cam, seed=7).astype(np.float64)
    ax = np.array([0.3, -0.5, 0.8])
    ang = 0.7
    Q = scenes.axis_angle(ax / np.linalg.norm(ax) * ang)
    qQ = np.concatenate([[np.cos(ang / 2)], np.sin(ang / 2) * ax / np.linalg.norm(ax)])
    d = np.array([3.0, -1.0, 2.0])
    moved = params.copy()
    moved[:, 0:3] = params[:, 0:3] @ Q.T + d
    moved[:, 6:10] = np.stack([qmul(qQ, q) for q in params[:, 6:10]])
    v0 = oview(cam)
    v1 = oracle.OView(cam=np.concatenate([(cam.R @ Q.T).reshape(9), cam.t - cam.R @ Q.T @ d,
                                          [cam.fx, cam.fy, cam.cx, cam.cy]]), W=256, H=192)
    a = oracle.project(params, 0, v0, fp64=True)
    b = oracle.project(moved, 0, v1, fp64=True)
    np.testing.assert_array_equal(a["visible"], b["visible"])
    vis = a["visible"] == 1
    for k in ("mean2d", "conic", "depth", "colour"):
        np.testing.assert_allclose(a[k][vis], b[k][vis], rtol=1e-8, atol=1e-9)


def test_culls():
    cam = cam64()
    assert proj_one(gauss_row([0, 0, 0.15], np.log(0.1)), cam)["visible"][0] == 0  # near plane
    assert proj_one(gauss_row([0, 0, -3.0], np.log(0.1)), cam)["visible"][0] == 0  # behind
    assert proj_one(gauss_row([0, 0, 5.0], np.log(0.1), logit=-10.0), cam)["visible"][0] == 0
    assert proj_one(gauss_row([0, 0, 5.0], np.log(0.1), logit=logit(0.0045)), cam)["visible"][0] == 1
    # far off screen: no tile reached
    assert proj_one(gauss_row([100.0, 0, 5.0], np.log(0.01)), cam)["visible"][0] == 0


def test_sh0_colour_and_clamp():
    cam = cam64()
    c = np.array([0.2, 0.7, 0.9])
    pr = proj_one(gauss_row([0.2, 0.1, 5.0], np.log(0.1), dc=dc_for_colour(c)), cam)
    np.testing.assert_allclose(pr["colour"][0], c, rtol=1e-12)
    pr = proj_one(gauss_row([0.2, 0.1, 5.0], np.log(0.1), dc=[-3.0, 0.0, 1.0]), cam)
    np.testing.assert_allclose(pr["colour"][0], [0.0, 0.5, 0.5 + Y00], rtol=1e-12)


def test_fp32_key_path_tracks_fp64():
    cam = scenes.pinhole(256, 192, 200.0)
    params = scenes.frustum_gaussians(5000, 0, cam, seed=1000)
    a = oracle.project(params, 0, oview(cam), fp64=False)
    b = oracle.project(params, 0, oview(cam), fp64=True)
    both = (a["visible"] == 1) & (b["visible"] == 1)
    assert both.sum() > 0.9 * max(a["visible"].sum(), b["visible"].sum())
    np.testing.assert_allclose(a["mean2d"][both], b["mean2d"][both], rtol=1e-5, atol=1e-4)
    np.testing.assert_allclose(a["conic"][both], b["conic"][both], rtol=2e-3,
                               atol=1e-5 * np.abs(b["conic"][both]).max())
    assert (a["count"][both] == b["count"][both]).mean() > 0.999
    # depth key bits are the float32 depth
    np.testing.assert_array_equal(a["depth_bits"][both],
                                  a["depth"][both].astype(np.float32).view(np.uint32))


def _tiles_of(bins, g):
    return set(bins["tile"][bins["val"] == g].tolist())


def test_tile_predicate_against_optimiser_and_pixels():
    # Each kept tile must have min over its pixel-centre rectangle of the conic quadratic
    # <= thr (found here by a bounded quasi-Newton search); each dropped candidate must
    # not; and every pixel centre with q <= thr lies in a kept tile (conservative).
    cam = scenes.pinhole(256, 192, 200.0)
    params = scenes.frustum_gaussians(400, 0, cam, seed=3, log_scale_mean=-2.5)
    # make some Gaussians slim so the ellipse clips tile corners
    params[::3, 3] -= 2.0
    v = oview(cam)
    pr = oracle.project(params, 0, v, fp64=True)
    bins = oracle.bin_views([pr], [v], fp64=True)
    ys, xs = np.mgrid[0:192, 0:256]
    pcx, pcy = xs + 0.5, ys + 0.5
    checked = 0
    for g in np.nonzero(pr["visible"])[0][:120]:
        mx, my = pr["mean2d"][g]
        A, B, C = pr["conic"][g]
        thr = pr["thr"][g]
        kept = _tiles_of(bins, g)
        dx, dy = pcx - mx, pcy - my
        q = A * dx * dx + 2 * B * dx * dy + C * dy * dy
        need = set(((ys[q <= thr] // 16) * 16 + xs[q <= thr] // 16).tolist())
        assert need <= kept, (g, need - kept)
        x0, y0, x1, y1 = pr["rect"][g]
        for ty in range(max(0, y0 - 1), min(11, y1 + 1) + 1):
            for tx in range(max(0, x0 - 1), min(15, x1 + 1) + 1):
                lo = [16 * tx + 0.5 - mx, 16 * ty + 0.5 - my]
                hi = [16 * tx + 15.5 - mx, 16 * ty + 15.5 - my]
                fun = lambda d: A * d[0] ** 2 + 2 * B * d[0] * d[1] + C * d[1] ** 2
                best = np.inf
                for st in ([lo[0], lo[1]], [hi[0], hi[1]], [lo[0], hi[1]], [hi[0], lo[1]],
                           [(lo[0] + hi[0]) / 2, (lo[1] + hi[1]) / 2]):
                    r = minimize(fun, st, bounds=list(zip(lo, hi)), method="L-BFGS-B",
                                 options=dict(ftol=1e-15, gtol=1e-12))
                    best = min(best, r.fun)
                t = ty * 16 + tx
                if abs(best - thr) < 1e-6 * max(1.0, thr):
                    continue
                assert (t in kept) == (best <= thr), (g, tx, ty, best, thr)
                checked += 1
    assert checked > 300


def test_sh_basis_orthonormal_and_textbook_band1():
    deg = 3
    xg, wg = np.polynomial.legendre.leggauss(16)
    phi = np.arange(32) * 2 * np.pi / 32
    ct, ph = np.meshgrid(xg, phi, indexing="ij")
    wts = (wg[:, None] * np.full(32, 2 * np.pi / 32)[None, :]).reshape(-1)
    st = np.sqrt(1 - ct ** 2)
    dirs = np.stack([st * np.cos(ph), st * np.sin(ph), ct], -1).reshape(-1, 3)
    Y = oracle.sh_basis(deg, dirs)
    G = (Y * wts[:, None]).T @ Y
    np.testing.assert_allclose(G, np.eye(16), atol=1e-12)
    # addition theorem: sum_m Y_lm^2 = (2l+1) / (4 pi) at every direction
    for l in range(4):
        np.testing.assert_allclose((Y[:, l * l:(l + 1) ** 2] ** 2).sum(1), (2 * l + 1) / (4 * np.pi),
                                   rtol=1e-12)
    # parity Y(-d) = (-1)^l Y(d)
    Yn = oracle.sh_basis(deg, -dirs)
    for l in range(4):
        np.testing.assert_allclose(Yn[:, l * l:(l + 1) ** 2], (-1) ** l * Y[:, l * l:(l + 1) ** 2],
                                   atol=1e-13)
    # degree 0 and 1 with the Condon-Shortley phase: Y00 = 1/(2 sqrt pi),
    # (Y1-1, Y10, Y11) = sqrt(3/(4 pi)) (-y, z, -x)
    np.testing.assert_allclose(Y[:, 0], Y00, rtol=1e-14)
    c1 = np.sqrt(3 / (4 * np.pi))
    np.testing.assert_allclose(Y[:, 1:4], c1 * np.stack([-dirs[:, 1], dirs[:, 2], -dirs[:, 0]], 1),
                               atol=1e-14)
    # Y20 = sqrt(5/(16 pi)) (3 z^2 - 1)
    np.testing.assert_allclose(Y[:, 6], np.sqrt(5 / (16 * np.pi)) * (3 * dirs[:, 2] ** 2 - 1),
                               atol=1e-14)
