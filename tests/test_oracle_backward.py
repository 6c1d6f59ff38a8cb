"""Pins of the oracle's adjoint, loss (Eq. 9) and sparse Adam (Sec. III-D.2): FP64 central
finite differences, closed forms of SSIM, and hand-computed Adam steps. No GPU."""
import numpy as np
import pytest

import oracle
from helpers import Y00, dc_for_colour, gauss_row, logit, oview
from paper_2404_06926_amd import scenes


def _fwd(params, deg, v):
    projs, bins, rend = oracle.forward(params, deg, [v], fp64=True)
    return projs, bins, rend[0]


def _fd_check(params, deg, v, coords, h=1e-4, skip_frac=0.05, tol=2e-5, maps=False, colour=True):
    """L = sum w * out (+ sum wD * D + sum wO * O with maps): the adjoint against central
    differences of L, skipping coordinates whose step changes a contributor set."""
    rng = np.random.default_rng(1)
    projs, bins, r0 = _fwd(params, deg, v)
    w = rng.normal(size=r0["out"].shape) * (1.0 if colour else 0.0)
    wD = rng.normal(size=r0["depth"].shape) if maps else None
    wO = rng.normal(size=r0["opacity"].shape) if maps else None

    def L(r):
        val = (w * r["out"]).sum()
        if maps:
            val += (wD * r["depth"]).sum() + (wO * r["opacity"]).sum()
        return val

    gp, gE, _ = oracle.backward(params, deg, [v], projs, bins, [w],
                                gdepths=[wD] if maps else None, gopacs=[wO] if maps else None)
    scale = np.abs(gp).max()
    skipped, checked, worst = 0, 0, 0.0
    for (i, f) in coords:
        vals = []
        same = True
        for sgn in (+1, -1):
            p = params.copy()
            p[i, f] += sgn * h
            pr, bn, r = _fwd(p, deg, v)
            same &= np.array_equal(r["signature"], r0["signature"]) and np.array_equal(bn["val"], bins["val"])
            vals.append(L(r))
        if not same:
            skipped += 1
            continue
        fd = (vals[0] - vals[1]) / (2 * h)
        err = abs(fd - gp[i, f]) / (abs(gp[i, f]) + 1e-3 * scale)
        worst = max(worst, err)
        checked += 1
        assert err < tol, (i, f, fd, gp[i, f])
    assert skipped <= skip_frac * len(coords), (skipped, len(coords))
    return checked, worst, gE, r0, w


def test_adjoint_matches_finite_differences_sh3():
    # 64x48 view, SH degree 3, random exposure and background (config-3a shape, fewer
    # Gaussians so the CPU suite stays short; the full 2k-Gaussian sweep is the slow test).
    cam = scenes.pinhole(64, 48, 50.0)
    cam.exposure = scenes.random_exposure(3000)
    cam.bg = np.array([0.1, 0.05, 0.2], np.float32)
    params = scenes.frustum_gaussians(250, 3, cam, seed=3000).astype(np.float64)
    v = oview(cam)
    F = params.shape[1]
    rng = np.random.default_rng(0)
    proj = oracle.project(params, 3, v, fp64=True)
    vis = np.nonzero(proj["visible"])[0]
    coords = [(int(rng.choice(vis)), f) for f in range(F) for _ in range(3)]
    checked, worst, gE, r0, w = _fd_check(params, 3, v, coords)
    assert checked >= 0.95 * len(coords)
    # exposure: out = A pre + b, so dL/dA = sum w pre^T and dL/db = sum w
    pre = r0["pre"].reshape(3, -1)
    wf = w.reshape(3, -1)
    expect = np.concatenate([wf @ pre.T, wf.sum(1, keepdims=True)], axis=1).reshape(12)
    np.testing.assert_allclose(gE[0], expect, rtol=1e-10)


def test_capped_alpha_gradient_closed_form():
    # A capped alpha (0.99, reading of Eq. 5) is constant in the Gaussian's geometry and
    # opacity: at a capped pixel dL/dalpha reaches no parameter except through the colour
    # term alpha T. One on-axis Gaussian with o = 0.995 and Sigma' = 100.3 I px^2, SH0,
    # identity exposure; L = out_0 at one pixel.
    #   capped pixel (32, 24): d out_0/d dc_0 = 0.99 Y00 and every geometric and opacity
    #   gradient is exactly 0;
    #   free pixel (35, 24): a = o e^power, d out_0/d logit = (c_0 - bg_0) e^power o (1 - o).
    cam = scenes.pinhole(64, 48, 50.0)
    cam.bg = np.array([0.1, 0.2, 0.05], np.float32)
    s, Z, o = 1.0, 5.0, 0.995
    c = np.array([0.9, 0.3, 0.6])
    row = gauss_row([0, 0, Z], np.log(s), logit=logit(o), dc=dc_for_colour(c))[None]
    v = oview(cam)
    projs, bins, r0 = _fwd(row, 0, v)
    var = (50.0 * s / Z) ** 2 + 0.3
    bg0 = float(cam.bg[0])
    for (x, y) in [(32, 24), (35, 24)]:
        w = np.zeros((3, 48, 64))
        w[0, y, x] = 1.0
        gp, gE, _ = oracle.backward(row, 0, [v], projs, bins, [w])
        e = np.exp(-0.5 * ((x + 0.5 - 32) ** 2 + (y + 0.5 - 24) ** 2) / var)
        if o * e > 0.99:
            assert np.all(gp[0, 0:11] == 0.0), gp[0, 0:11]
            np.testing.assert_allclose(gp[0, 11], 0.99 * Y00, rtol=1e-12)
        else:
            np.testing.assert_allclose(gp[0, 10], (c[0] - bg0) * e * o * (1 - o), rtol=1e-10)
            np.testing.assert_allclose(gp[0, 11], o * e * Y00, rtol=1e-12)
            assert abs(gp[0, 0]) > 0


def test_adjoint_matches_finite_differences_with_capped_alphas():
    # A map where a tenth of the Gaussians have logits in [5, 9] (o > 0.993) and wide
    # footprints, so that pairs with a capped alpha occur among the contributors; every
    # coordinate of the capped Gaussians and random coordinates of the others, against
    # FP64 central differences (steps that move a pair across the cap are skipped).
    cam = scenes.pinhole(48, 40, 40.0)
    cam.exposure = scenes.random_exposure(31)
    cam.bg = np.array([0.2, 0.1, 0.3], np.float32)
    params = scenes.frustum_gaussians(150, 1, cam, seed=31, log_scale_mean=-0.8).astype(np.float64)
    rng = np.random.default_rng(31)
    hi = rng.choice(150, 15, replace=False)
    params[hi, 10] = rng.uniform(5.0, 9.0, 15)
    v = oview(cam)
    proj = oracle.project(params, 1, v, fp64=True)
    # pixels where a high-opacity Gaussian's alpha is capped (before occlusion)
    ys, xs = np.mgrid[0:40, 0:48]
    capped_g = []
    for g in hi:
        if not proj["visible"][g]:
            continue
        mx, my = proj["mean2d"][g]
        A, B, C = proj["conic"][g]
        dx, dy = xs + 0.5 - mx, ys + 0.5 - my
        araw = proj["opacity"][g] * np.exp(-0.5 * (A * dx * dx + 2 * B * dx * dy + C * dy * dy))
        if (araw > 0.99).any():
            capped_g.append(int(g))
    assert len(capped_g) >= 3, capped_g
    vis = np.nonzero(proj["visible"])[0]
    F = params.shape[1]
    coords = [(g, f) for g in capped_g for f in range(F)]
    coords += [(int(rng.choice(vis)), f) for f in range(F) for _ in range(2)]
    checked, worst, _, _, _ = _fd_check(params, 1, v, coords)
    assert checked >= 0.95 * len(coords)


@pytest.mark.parametrize("colour", [False, True])
def test_depth_and_opacity_map_adjoint_matches_finite_differences(colour):
    # Eq. 6-7: L = sum wD D + sum wO O (+ sum w out), D = sum d_i a_i T_i with d_i the
    # camera-frame depth, O = sum a_i T_i. Every geometric coordinate of sampled Gaussians.
    cam = scenes.pinhole(48, 40, 40.0)
    cam.R = scenes.axis_angle([0.1, -0.2, 0.05]).astype(np.float32)
    cam.t = np.array([0.3, -0.2, 0.5], np.float32)
    cam.exposure = scenes.random_exposure(21)
    params = scenes.frustum_gaussians(200, 1, scenes.pinhole(48, 40, 40.0), seed=21).astype(np.float64)
    v = oview(cam)
    proj = oracle.project(params, 1, v, fp64=True)
    vis = np.nonzero(proj["visible"])[0]
    rng = np.random.default_rng(3)
    coords = [(int(rng.choice(vis)), f) for f in range(params.shape[1]) for _ in range(3)]
    checked, worst, _, _, _ = _fd_check(params, 1, v, coords, maps=True, colour=colour)
    assert checked >= 0.95 * len(coords)


def test_depth_map_gradient_reaches_only_geometry():
    # D and O do not depend on SH or on the exposure: with L = sum wD D + sum wO O the SH
    # columns and dL/dE are exactly zero, and the mean gradient is non-zero.
    cam = scenes.pinhole(40, 32, 30.0)
    cam.exposure = scenes.random_exposure(4)
    params = scenes.frustum_gaussians(100, 2, cam, seed=4).astype(np.float64)
    v = oview(cam)
    projs, bins, r0 = _fwd(params, 2, v)
    rng = np.random.default_rng(5)
    gp, gE, _ = oracle.backward(params, 2, [v], projs, bins, [np.zeros((3, 32, 40))],
                                gdepths=[rng.normal(size=(32, 40))], gopacs=[rng.normal(size=(32, 40))])
    assert np.all(gp[:, 11:] == 0.0)
    assert np.all(gE[0] == 0.0)
    assert np.abs(gp[:, 0:3]).max() > 0


def test_exposure_gradient_finite_differences():
    cam = scenes.pinhole(48, 32, 40.0)
    cam.exposure = scenes.random_exposure(5)
    params = scenes.frustum_gaussians(150, 1, cam, seed=8).astype(np.float64)
    v = oview(cam)
    projs, bins, r0 = _fwd(params, 1, v)
    w = np.random.default_rng(2).normal(size=r0["out"].shape)
    _, gE, _ = oracle.backward(params, 1, [v], projs, bins, [w])
    h = 1e-5
    for k in range(12):
        Lp, Lm = 0.0, 0.0
        for sgn in (+1, -1):
            vv = oview(cam)
            vv.E = v.E.copy()
            vv.E[k] += sgn * h
            out = oracle.forward(params, 1, [vv], fp64=True)[2][0]["out"]
            if sgn > 0:
                Lp = (w * out).sum()
            else:
                Lm = (w * out).sum()
        np.testing.assert_allclose((Lp - Lm) / (2 * h), gE[0][k], rtol=1e-7, atol=1e-9)


@pytest.mark.slow
def test_adjoint_full_fd_sweep_config3a():
    # Every coordinate of a 2k-Gaussian SH3 map at 64x48 (FP64, h = 1e-4).
    cam = scenes.pinhole(64, 48, 50.0)
    cam.exposure = scenes.random_exposure(3000)
    params = scenes.frustum_gaussians(2000, 3, cam, seed=3000).astype(np.float64)
    v = oview(cam)
    proj = oracle.project(params, 3, v, fp64=True)
    coords = [(int(i), f) for i in np.nonzero(proj["visible"])[0] for f in range(params.shape[1])]
    _fd_check(params, 3, v, coords)


def test_loss_gradient_finite_differences():
    rng = np.random.default_rng(4)
    out = rng.random((3, 13, 17))
    gt = rng.random((3, 13, 17))
    L, g, _ = oracle.loss(out, gt, 0.2)
    h = 1e-6
    for _ in range(60):
        c, y, x = rng.integers(3), rng.integers(13), rng.integers(17)
        if abs(out[c, y, x] - gt[c, y, x]) < 10 * h:
            continue
        o1, o2 = out.copy(), out.copy()
        o1[c, y, x] += h
        o2[c, y, x] -= h
        fd = (oracle.loss(o1, gt, 0.2)[0] - oracle.loss(o2, gt, 0.2)[0]) / (2 * h)
        np.testing.assert_allclose(fd, g[c, y, x], rtol=1e-6, atol=1e-10)


def test_ssim_constant_images_closed_form():
    # Constant images a, b with zero padding: at a pixel whose window keeps mass m inside
    # the image, mu_x = a m, E[x^2] = a^2 m, so
    # S = ((2ab m^2 + C1)(2ab (m - m^2) + C2)) / (((a^2+b^2) m^2 + C1)((a^2+b^2)(m - m^2) + C2)).
    H, W, a, b = 9, 14, 0.7, 0.3
    g = np.exp(-((np.arange(11) - 5) ** 2) / (2 * 1.5 ** 2))
    g /= g.sum()
    def mass_1d(n):
        return np.array([sum(g[j] for j in range(11) if 0 <= p + j - 5 < n) for p in range(n)])
    m = np.outer(mass_1d(H), mass_1d(W))
    C1, C2 = 0.01 ** 2, 0.03 ** 2
    S = ((2 * a * b * m * m + C1) * (2 * a * b * (m - m * m) + C2)) / (
        ((a * a + b * b) * m * m + C1) * ((a * a + b * b) * (m - m * m) + C2))
    _, _, ssim = oracle.loss(np.full((3, H, W), a), np.full((3, H, W), b), 1.0)
    np.testing.assert_allclose(ssim, S.mean(), rtol=1e-12)
    L1, _, _ = oracle.loss(np.full((3, H, W), a), np.full((3, H, W), b), 0.0)
    np.testing.assert_allclose(L1, abs(a - b), rtol=1e-14)


def test_ssim_of_identical_images():
    x = np.random.default_rng(5).random((3, 20, 23))
    L, g, ssim = oracle.loss(x, x, 1.0)
    np.testing.assert_allclose(ssim, 1.0, atol=1e-14)
    np.testing.assert_allclose(L, 0.0, atol=1e-14)
    np.testing.assert_allclose(g, 0.0, atol=1e-14)


def test_sparse_adam_closed_form_steps():
    b1, b2, eps = 0.9, 0.999, 1e-15
    lr = np.array([0.1, 0.01, 1.0])
    p = np.array([[1.0, -2.0, 0.5], [3.0, 4.0, 5.0]])
    g = np.array([[0.5, -0.25, 2.0], [0.0, 0.0, 0.0]])
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    vis = np.array([1, 0], np.uint8)
    p1, g1, m1, v1 = oracle.adam(p, g, m, v, vis, lr, b1, b2, eps, 1)
    # first step from zero moments: dp = -lr g / (|g| + eps) = -lr sign(g)
    np.testing.assert_allclose(p1[0], p[0] - lr * np.sign(g[0]), rtol=1e-12)
    np.testing.assert_array_equal(p1[1], p[1])        # invisible row untouched
    np.testing.assert_array_equal(m1[1], 0.0)
    np.testing.assert_array_equal(g1[0], 0.0)         # gradients cleared
    # second step with g2: m = .9 m1 + .1 g2, v = .999 v1 + .001 g2^2, t = 2
    g2 = np.array([[1.0, 0.5, -1.0], [0.0, 0.0, 0.0]])
    p2, _, m2, v2 = oracle.adam(p1, g2, m1, v1, vis, lr, b1, b2, eps, 2)
    mm = 0.9 * (0.1 * g[0]) + 0.1 * g2[0]
    vv = 0.999 * (0.001 * g[0] ** 2) + 0.001 * g2[0] ** 2
    step = lr * (mm / (1 - 0.81)) / (np.sqrt(vv / (1 - 0.999 ** 2)) + eps)
    np.testing.assert_allclose(p2[0], p1[0] - step, rtol=1e-12)
    np.testing.assert_allclose(m2[0], mm, rtol=1e-14)
    np.testing.assert_allclose(v2[0], vv, rtol=1e-14)
