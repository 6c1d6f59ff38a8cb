"""Pins of the oracle's blend (Sec. III-A, Eq. 4-5, 7), exposure (Sec. III-C.3), binning
and sort: closed forms, invariants and brute force against the tiled path. No GPU."""
import numpy as np

import oracle
from helpers import Y00, dc_for_colour, gauss_row, logit, oview
from paper_2404_06926_amd import scenes

AMIN = 1.0 / 255.0


def render_rows(rows, cam, deg=0, fp64=True, E=None, bg=None):
    v = oview(cam)
    if E is not None:
        v.E = np.asarray(E, np.float64)
    if bg is not None:
        v.bg = np.asarray(bg, np.float64)
    projs, bins, rend = oracle.forward(np.atleast_2d(rows), deg, [v], fp64=fp64)
    return projs[0], bins, rend[0], v


def test_single_isotropic_gaussian_image_closed_form():
    # Sigma' = (f s/Z)^2 + 0.3 on axis; out = c a + (1 - a) bg where a = min(.99, o e^{-q/2})
    # is >= 1/255, else bg.
    cam = scenes.pinhole(64, 48, 50.0)
    s, Z, o, f = 0.1, 5.0, 0.8, 50.0
    c = np.array([0.9, 0.3, 0.6])
    bg = np.array([0.1, 0.2, 0.05])
    _, _, r, _ = render_rows(gauss_row([0, 0, Z], np.log(s), logit=logit(o), dc=dc_for_colour(c)),
                             cam, bg=bg)
    var = (f * s / Z) ** 2 + 0.3
    ys, xs = np.mgrid[0:48, 0:64]
    q = ((xs + 0.5 - 32) ** 2 + (ys + 0.5 - 24) ** 2) / var
    a = np.minimum(0.99, o * np.exp(-0.5 * q))
    inside = a >= AMIN
    tie = np.abs(a * 255 - 1) < 1e-9
    expect = np.where(inside[None], c[:, None, None] * a[None] + (1 - a[None]) * bg[:, None, None],
                      bg[:, None, None])
    np.testing.assert_allclose(r["out"][:, ~tie], expect[:, ~tie], atol=1e-12)
    np.testing.assert_allclose(r["T_final"][~tie], np.where(inside, 1 - a, 1.0)[~tie], atol=1e-12)
    # footprint {a >= 1/255} is the ellipse q <= 2 ln(255 o), area 2 pi ln(255 o) sqrt(det)
    area = 2 * np.pi * np.log(255 * o) * var
    assert abs(inside.sum() - area) <= 2 * np.pi * np.sqrt(2 * np.log(255 * o) * var) + 4


def test_alpha_cap_closed_form():
    # Reading of Eq. 5 (alpha capped at 0.99): one on-axis Gaussian with o = 0.995 and
    # Sigma' = 100.3 I px^2. The four pixels around the mean (offset (0.5, 0.5) px) have
    # o e^power = 0.9925 > 0.99, so they composite with alpha = 0.99 exactly:
    # out = 0.99 c + 0.01 bg and T_final = 0.01. Every other pixel has o e^power < 0.99
    # and stays unclamped.
    cam = scenes.pinhole(64, 48, 50.0)
    s, Z, o = 1.0, 5.0, 0.995
    c = np.array([0.9, 0.3, 0.6])
    bg = np.array([0.1, 0.2, 0.05])
    _, _, r, _ = render_rows(gauss_row([0, 0, Z], np.log(s), logit=logit(o), dc=dc_for_colour(c)),
                             cam, bg=bg)
    var = (50.0 * s / Z) ** 2 + 0.3
    ys, xs = np.mgrid[0:48, 0:64]
    araw = o * np.exp(-0.5 * ((xs + 0.5 - 32) ** 2 + (ys + 0.5 - 24) ** 2) / var)
    capped = araw > 0.99
    assert capped.sum() == 4 and capped[23:25, 31:33].all()
    np.testing.assert_allclose(r["T_final"][capped], 0.01, rtol=0, atol=1e-14)
    np.testing.assert_allclose(r["out"][:, capped], (0.99 * c + 0.01 * bg)[:, None] * np.ones((1, 4)),
                               rtol=0, atol=1e-14)
    # unclamped elsewhere: out = c a + (1 - a) bg with a = o e^power
    free = ~capped & (araw >= AMIN) & (np.abs(araw * 255 - 1) > 1e-9)
    assert free.sum() > 1000
    expect = c[:, None] * araw[free] + (1 - araw[free]) * bg[:, None]
    np.testing.assert_allclose(r["out"][:, free], expect, rtol=0, atol=1e-12)
    np.testing.assert_allclose(r["T_final"][free], 1 - araw[free], rtol=0, atol=1e-12)


def test_single_gaussian_depth_and_opacity_maps_closed_form():
    # Eq. 6-7 for one Gaussian on the axis at depth Z: D = Z a and O = a where a >= 1/255.
    cam = scenes.pinhole(64, 48, 50.0)
    s, Z, o, f = 0.1, 5.0, 0.8, 50.0
    _, _, r, _ = render_rows(gauss_row([0, 0, Z], np.log(s), logit=logit(o)), cam)
    var = (f * s / Z) ** 2 + 0.3
    ys, xs = np.mgrid[0:48, 0:64]
    a = np.minimum(0.99, o * np.exp(-0.5 * ((xs + 0.5 - 32) ** 2 + (ys + 0.5 - 24) ** 2) / var))
    a = np.where(a >= AMIN, a, 0.0)
    tie = np.abs(a * 255 - 1) < 1e-9
    np.testing.assert_allclose(r["depth"][~tie], (Z * a)[~tie], atol=1e-12)
    np.testing.assert_allclose(r["opacity"][~tie], a[~tie], atol=1e-12)


def test_two_gaussians_depth_and_opacity_maps():
    # D = d1 a1 + d2 a2 (1 - a1), O = a1 + a2 (1 - a1), with d the camera-frame depth of a
    # camera that is rotated and translated (depth is z in the camera frame, not |x|).
    cam = scenes.pinhole(64, 48, 50.0)
    cam.R = scenes.axis_angle([0.0, 0.15, 0.0]).astype(np.float32)
    cam.t = np.array([0.1, 0.0, 0.4], np.float32)
    g1 = gauss_row([0.6, 0.0, 4.0], np.log(0.09), logit=logit(0.6))
    g2 = gauss_row([0.7, 0.03, 6.5], np.log(0.14), logit=logit(0.7))
    pr, _, r, _ = render_rows(np.stack([g1, g2]), cam)
    Rm = cam.R.astype(np.float64)
    d = [(Rm @ g[0:3] + cam.t)[2] for g in (g1, g2)]
    np.testing.assert_allclose(pr["depth"], d, rtol=1e-12)
    ys, xs = np.mgrid[0:48, 0:64]

    def alpha(k):
        mx, my = pr["mean2d"][k]
        A, B, C = pr["conic"][k]
        dx, dy = xs + 0.5 - mx, ys + 0.5 - my
        a = np.minimum(0.99, pr["opacity"][k] * np.exp(-0.5 * (A * dx * dx + 2 * B * dx * dy + C * dy * dy)))
        return np.where(a >= AMIN, a, 0.0)

    a1, a2 = alpha(0), alpha(1)
    np.testing.assert_allclose(r["depth"], d[0] * a1 + d[1] * a2 * (1 - a1), atol=1e-12)
    np.testing.assert_allclose(r["opacity"], a1 + a2 * (1 - a1), atol=1e-12)


def test_opacity_map_equals_one_minus_final_transmittance():
    # O = sum a_i prod_{j<i}(1 - a_j) telescopes to 1 - prod_i (1 - a_i) = 1 - T_final, and
    # D lies within [min d, max d] * O of the pixel's contributors (a weighted mean times O).
    cam = scenes.pinhole(96, 64, 80.0)
    params = scenes.frustum_gaussians(3000, 0, cam, seed=17, log_scale_mean=-2.5).astype(np.float64)
    pr, _, r, _ = render_rows(params, cam)
    np.testing.assert_allclose(r["opacity"], 1.0 - r["T_final"], atol=1e-12)
    vis = pr["visible"] > 0
    dmin, dmax = pr["depth"][vis].min(), pr["depth"][vis].max()
    assert np.all(r["depth"] >= dmin * r["opacity"] - 1e-9)
    assert np.all(r["depth"] <= dmax * r["opacity"] + 1e-9)


def test_depth_and_opacity_maps_tiled_equal_brute_force():
    cam = scenes.pinhole(80, 56, 60.0)
    params = scenes.frustum_gaussians(1500, 0, cam, seed=23, log_scale_mean=-2.7).astype(np.float64)
    pr, _, r, v = render_rows(params, cam)
    b = oracle.render_brute(pr, v)
    np.testing.assert_allclose(r["depth"], b["depth"], rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(r["opacity"], b["opacity"], rtol=1e-12, atol=1e-12)


def test_opacity_integral_of_wide_gaussian():
    # sum over pixels of alpha -> 2 pi o sqrt(det Sigma') (1 - 1/(255 o)) for wide footprints
    cam = scenes.pinhole(256, 192, 200.0)
    s, Z, o = 0.2, 4.0, 0.6
    _, _, r, _ = render_rows(gauss_row([0, 0, Z], np.log(s), logit=logit(o), dc=dc_for_colour([1, 1, 1])),
                             cam)
    var = (200 * s / Z) ** 2 + 0.3
    integral = 2 * np.pi * o * var * (1 - 1 / (255 * o))
    np.testing.assert_allclose((1 - r["T_final"]).sum(), integral, rtol=2e-3)


def test_two_gaussians_composite_and_depth_swap():
    cam = scenes.pinhole(64, 48, 50.0)
    c1, c2 = np.array([1.0, 0.0, 0.0]), np.array([0.0, 0.0, 1.0])
    g1 = gauss_row([0.0, 0.0, 4.0], np.log(0.08), logit=logit(0.6), dc=dc_for_colour(c1))
    g2 = gauss_row([0.02, 0.01, 6.0], np.log(0.12), logit=logit(0.7), dc=dc_for_colour(c2))
    bg = np.array([0.0, 0.3, 0.0])
    pr, _, r, _ = render_rows(np.stack([g1, g2]), cam, bg=bg)
    ys, xs = np.mgrid[0:48, 0:64]

    def alpha(k):
        mx, my = pr["mean2d"][k]
        A, B, C = pr["conic"][k]
        dx, dy = xs + 0.5 - mx, ys + 0.5 - my
        a = np.minimum(0.99, pr["opacity"][k] * np.exp(-0.5 * (A * dx * dx + 2 * B * dx * dy + C * dy * dy)))
        return np.where(a >= AMIN, a, 0.0)

    a1, a2 = alpha(0), alpha(1)
    expect = (c1[:, None, None] * a1 + c2[:, None, None] * a2 * (1 - a1)
              + bg[:, None, None] * (1 - a1) * (1 - a2))
    np.testing.assert_allclose(r["out"], expect, atol=1e-12)
    # swap depths: the blue one is now in front
    g1b, g2b = g1.copy(), g2.copy()
    g1b[0:3] *= 6.0 / 4.0
    g2b[0:3] *= 4.0 / 6.0
    pr2, _, r2, _ = render_rows(np.stack([g1b, g2b]), cam, bg=bg)
    a1, a2 = alpha(0), alpha(1)  # 2D footprints unchanged (same rays, scale ratio differs)
    b1 = _alpha_from(pr2, 0, xs, ys)
    b2 = _alpha_from(pr2, 1, xs, ys)
    expect2 = (c2[:, None, None] * b2 + c1[:, None, None] * b1 * (1 - b2)
               + bg[:, None, None] * (1 - b1) * (1 - b2))
    np.testing.assert_allclose(r2["out"], expect2, atol=1e-12)


def _alpha_from(pr, k, xs, ys):
    mx, my = pr["mean2d"][k]
    A, B, C = pr["conic"][k]
    dx, dy = xs + 0.5 - mx, ys + 0.5 - my
    a = np.minimum(0.99, pr["opacity"][k] * np.exp(-0.5 * (A * dx * dx + 2 * B * dx * dy + C * dy * dy)))
    return np.where(a >= AMIN, a, 0.0)


def test_early_termination_stack():
    # 20 Gaussians centred on one pixel centre with o = 0.5: T halves per layer and the
    # blend stops before T(1 - a) < 1e-4, i.e. after 13 layers (2^-13 >= 1e-4 > 2^-14).
    cam = scenes.pinhole(64, 48, 50.0)
    rows = []
    for k in range(20):
        Z = 3.0 + 0.25 * k
        rows.append(gauss_row([0.5 * Z / 50.0, 0.5 * Z / 50.0, Z], np.log(0.05), logit=0.0,
                              dc=dc_for_colour([0.8, 0.4, 0.2])))
    _, bins, r, _ = render_rows(np.stack(rows), cam)
    y, x = 24, 32
    assert r["n_contributors"][y, x] == 13
    np.testing.assert_allclose(r["T_final"][y, x], 2.0 ** -13, rtol=1e-6)
    np.testing.assert_allclose(r["out"][:, y, x], np.array([0.8, 0.4, 0.2]) * (1 - 2.0 ** -13), rtol=1e-6)
    assert (r["T_final"] >= 1e-4).all()


def test_exposure_is_affine_on_colour():
    cam = scenes.pinhole(64, 48, 50.0)
    params = scenes.frustum_gaussians(300, 2, cam, seed=5)
    E = scenes.random_exposure(11).astype(np.float64)
    bg = np.array([0.2, 0.1, 0.4])
    _, _, r0, _ = render_rows(params, cam, deg=2, bg=bg)
    _, _, r1, _ = render_rows(params, cam, deg=2, E=E, bg=bg)
    A, b = E.reshape(3, 4)[:, :3], E.reshape(3, 4)[:, 3]
    np.testing.assert_allclose(r1["out"], np.einsum("rc,chw->rhw", A, r0["out"]) + b[:, None, None],
                               atol=1e-12)
    np.testing.assert_allclose(r1["pre"], r0["out"], atol=1e-12)


def test_zero_opacity_gives_background():
    cam = scenes.pinhole(64, 48, 50.0)
    params = scenes.frustum_gaussians(200, 0, cam, seed=9).astype(np.float64)
    params[:, 10] = -30.0
    E = scenes.random_exposure(3).astype(np.float64)
    bg = np.array([0.25, 0.5, 0.75])
    _, bins, r, _ = render_rows(params, cam, E=E, bg=bg)
    A, b = E.reshape(3, 4)[:, :3], E.reshape(3, 4)[:, 3]
    assert bins["tile"].size == 0
    np.testing.assert_array_equal(r["out"], np.broadcast_to((A @ bg + b)[:, None, None], r["out"].shape))
    np.testing.assert_array_equal(r["T_final"], 1.0)


def test_invariants_config1():
    cam = scenes.pinhole(256, 192, 200.0)
    params = scenes.frustum_gaussians(10_000, 0, cam, seed=1000)
    projs, bins, rend = oracle.forward(params, 0, [oview(cam)], fp64=False)
    r = rend[0]
    assert (r["T_final"] >= 1e-4).all() and (r["T_final"] <= 1.0).all()
    opac_map = 1 - r["T_final"]
    assert opac_map.min() >= 0 and opac_map.max() <= 1 - 1e-4
    lens = np.diff(bins["ranges"], axis=1)[:, 0]
    tile_of_px = (np.arange(192)[:, None] // 16) * 16 + np.arange(256)[None, :] // 16
    assert (r["n_contrib"] <= lens[tile_of_px]).all()
    assert (r["n_contributors"] <= r["n_contrib"]).all()


def test_permutation_invariance():
    cam = scenes.pinhole(96, 64, 75.0)
    params = scenes.frustum_gaussians(2000, 1, cam, seed=21)
    _, _, r0, _ = render_rows(params.astype(np.float64), cam, deg=1)
    perm = np.random.default_rng(0).permutation(2000)
    _, _, r1, _ = render_rows(params[perm].astype(np.float64), cam, deg=1)
    np.testing.assert_array_equal(r0["out"], r1["out"])


def test_brute_force_equals_tiled():
    # The plain definition (every pixel over every Gaussian in depth order) equals the
    # tiled path with the footprint predicate, in both key-path precisions.
    for (W, H, f, n, deg, seed) in [(64, 48, 50.0, 2000, 3, 3000), (256, 192, 200.0, 10_000, 0, 1000)]:
        cam = scenes.pinhole(W, H, f)
        cam.bg = np.array([0.1, 0.2, 0.3], np.float32)
        params = scenes.frustum_gaussians(n, deg, cam, seed=seed)
        for fp64 in (False, True):
            v = oview(cam)
            projs, bins, rend = oracle.forward(params, deg, [v], fp64=fp64)
            b = oracle.render_brute(projs[0], v)
            np.testing.assert_allclose(rend[0]["out"], b["out"], atol=1e-12)
            np.testing.assert_allclose(rend[0]["T_final"], b["T_final"], atol=1e-12)
            np.testing.assert_array_equal(rend[0]["n_contributors"], b["n_contributors"])


def test_keys_sorted_stable_and_ranges():
    cam = scenes.pinhole(256, 192, 200.0)
    params = scenes.frustum_gaussians(3000, 0, cam, seed=1000)
    # force equal depths on some Gaussians to exercise the index tie-break
    params[100:140, 0:3] = params[100, 0:3]
    v = oview(cam)
    pr = oracle.project(params, 0, v)
    bins = oracle.bin_views([pr], [v])
    # rebuild the emission order independently and sort with Python's sorted
    emitted = []
    for g in range(3000):
        for t in sorted(set(bins["tile"][bins["val"] == g].tolist())):
            emitted.append((t, int(pr["depth_bits"][g]), g))
    # emission within a Gaussian is row-major = ascending tile id
    ref = sorted(range(len(emitted)), key=lambda k: (emitted[k][0], emitted[k][1], k))
    np.testing.assert_array_equal(bins["val"], [emitted[k][2] for k in ref])
    keys = np.array([(emitted[k][0] << 32) | emitted[k][1] for k in ref], np.uint64)
    np.testing.assert_array_equal(bins["key"], keys)
    # ranges: first/last+1 of each tile, empty tiles [0, 0)
    for t in range(v.n_tiles):
        idx = np.nonzero(bins["tile"] == t)[0]
        if idx.size:
            assert tuple(bins["ranges"][t]) == (idx[0], idx[-1] + 1)
        else:
            assert tuple(bins["ranges"][t]) == (0, 0)


def test_multi_view_tiles_are_consecutive():
    cams = [scenes.pinhole(64, 48, 50.0), scenes.pinhole(96, 40, 60.0)]
    params = scenes.frustum_gaussians(500, 0, cams[0], seed=4)
    views = [oview(c) for c in cams]
    projs, bins, rend = oracle.forward(params, 0, views)
    single = [oracle.forward(params, 0, [v])[2][0] for v in views]
    for a, b in zip(rend, single):
        np.testing.assert_array_equal(a["out"], b["out"])
    assert bins["n_tiles"] == views[0].n_tiles + views[1].n_tiles


def test_sampled_pixels_equal_full_render():
    cam = scenes.pinhole(96, 64, 75.0)
    params = scenes.frustum_gaussians(1500, 1, cam, seed=12)
    v = oview(cam)
    projs, bins, rend = oracle.forward(params, 1, [v])
    pix = np.random.default_rng(0).choice(96 * 64, 300, replace=False)
    s = oracle.render_pixels(projs, [v], bins, 0, pix)
    np.testing.assert_array_equal(s["out"], rend[0]["out"].reshape(3, -1)[:, pix].T)
    np.testing.assert_array_equal(s["T_final"], rend[0]["T_final"].reshape(-1)[pix])
    np.testing.assert_array_equal(s["n_contrib"], rend[0]["n_contrib"].reshape(-1)[pix])
