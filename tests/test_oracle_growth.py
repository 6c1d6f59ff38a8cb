"""Pins of the oracle's map growth: initialisation from points and sky Gaussians
(Sec. III-C.1) and expansion by the opacity mask (Sec. III-C.2, Eq. 8). No GPU."""
import numpy as np

import oracle
from helpers import gauss_row, logit, oview
from paper_2404_06926_amd import scenes


def test_init_point_renders_its_colour_with_one_pixel_footprint():
    # scale d / f makes the projected standard deviation exactly one pixel on the axis:
    # Sigma' = (f (d / f) / d)^2 + 0.3 = 1.3 px^2; colour = the point's colour; o = o_a.
    cam = scenes.pinhole(64, 48, 50.0)
    v = oview(cam)
    rgb = np.array([[0.2, 0.7, 0.4]])
    rows = oracle.init_points([[0.0, 0.0, 7.0]], rgb, v, 0.1, deg=2)
    pr = oracle.project(rows, 2, v, fp64=True)
    np.testing.assert_allclose(pr["cov2d"][0], [1.3, 0.0, 1.3], atol=1e-12)
    np.testing.assert_allclose(pr["colour"][0], rgb[0], atol=1e-12)
    np.testing.assert_allclose(pr["opacity"][0], 0.1, rtol=1e-12)
    assert np.all(rows[0, 14:] == 0.0) and np.all(rows[0, 6:10] == [1, 0, 0, 0])


def test_init_scale_uses_camera_frame_depth():
    # d is the depth in the current camera frame (z), not the distance to the centre; the
    # camera is rotated and moved so that the two differ.
    cam = scenes.pinhole(64, 48, 40.0)
    cam.R = scenes.axis_angle([0.0, 0.3, 0.0]).astype(np.float32)
    cam.t = np.array([0.5, 0.0, 1.0], np.float32)
    v = oview(cam)
    p = np.array([[1.0, 0.5, 6.0], [-2.0, 0.0, 3.0]])
    rows = oracle.init_points(p, np.full((2, 3), 0.5), v, 0.3, deg=0)
    z = (p @ cam.R.astype(np.float64).T + cam.t)[:, 2]
    np.testing.assert_allclose(rows[:, 3], np.log(z / 40.0), rtol=1e-12)
    np.testing.assert_allclose(rows[:, 3:6], np.repeat(rows[:, 3:4], 3, axis=1))


def test_expansion_on_empty_map_keeps_exactly_the_points_in_view():
    cam = scenes.pinhole(80, 60, 60.0)
    v = oview(cam)
    rng = np.random.default_rng(0)
    p = rng.uniform([-3, -3, -1], [3, 3, 10], (5000, 3))
    keep, _ = oracle.expansion_select(p, v, np.zeros((60, 80)), 0.99)
    u = 60.0 * p[:, 0] / p[:, 2] + 40.0
    w = 60.0 * p[:, 1] / p[:, 2] + 30.0
    expect = (p[:, 2] > 0.2) & (u >= 0) & (u < 80) & (w >= 0) & (w < 60)
    margin = (np.abs(u) < 1e-4) | (np.abs(u - 80) < 1e-4) | (np.abs(w) < 1e-4) | (np.abs(w - 60) < 1e-4)
    np.testing.assert_array_equal(keep[~margin], expect[~margin])
    assert 0 < keep.sum() < len(p)


def test_expansion_drops_points_behind_an_opaque_layer():
    # Five stacked wide Gaussians cover the left part of the image (O > 0.99 there); the
    # right half stays empty (O = 0). Points over the left half are dropped, the rest kept.
    cam = scenes.pinhole(64, 48, 50.0)
    v = oview(cam)
    wall = [gauss_row([-3.0, 0.0, 4.0 + 0.1 * k], [np.log(1.5), np.log(4.0), np.log(0.1)], logit=logit(0.999))
            for k in range(5)]
    _, _, rend = oracle.forward(np.stack(wall), 0, [v], fp64=True)
    O = rend[0]["opacity"]
    assert O[:, :8].min() > 0.99 and O[:, 60:].max() < 1e-6
    rng = np.random.default_rng(1)
    px = rng.uniform(0, 64, 400)
    py = rng.uniform(0, 48, 400)
    z = rng.uniform(2, 12, 400)
    p = np.stack([(px - 32) * z / 50, (py - 24) * z / 50, z], 1)
    keep, ties = oracle.expansion_select(p, v, O, 0.99)
    cols = np.floor(px).astype(int)
    rows = np.floor(py).astype(int)
    clear = ~ties & (np.abs(px - np.round(px)) > 1e-3) & (np.abs(py - np.round(py)) > 1e-3)
    np.testing.assert_array_equal(keep[clear], (O[rows, cols] < 0.99)[clear])
    assert keep[cols < 8].sum() == 0 and keep[cols >= 60].all()


def test_point_on_a_pixel_boundary_goes_to_the_right_and_lower_pixel():
    cam = scenes.pinhole(32, 32, 16.0)
    v = oview(cam)
    # u = 16 (x / z) + 16 lands exactly on 20.0 and 8.0
    inside, px, py, _ = oracle.point_pixels(np.array([[1.0, -1.0, 4.0]]), v)
    assert inside[0] and px[0] == 20 and py[0] == 12


def test_nearest_neighbour_distance_matches_kd_tree_and_grid():
    from scipy.spatial import cKDTree
    rng = np.random.default_rng(2)
    p = rng.normal(size=(3000, 3))
    d, _ = cKDTree(p).query(p, k=2)
    np.testing.assert_allclose(oracle.nearest_neighbour_distance(p), d[:, 1], rtol=1e-12)
    g = np.stack(np.meshgrid(np.arange(5), np.arange(4), np.arange(3), indexing="ij"), -1).reshape(-1, 3) * 0.7
    np.testing.assert_allclose(oracle.nearest_neighbour_distance(g), 0.7, rtol=1e-12)


def test_sky_init_rows():
    rng = np.random.default_rng(3)
    p = rng.normal(size=(500, 3)) * 100
    rows = oracle.init_sky(p, 0.7, deg=3)
    Y00 = 0.28209479177387814
    np.testing.assert_allclose(rows[:, 11:14] * Y00 + 0.5, 1.0, rtol=1e-12)   # white
    np.testing.assert_allclose(1 / (1 + np.exp(-rows[:, 10])), 0.7, rtol=1e-12)
    np.testing.assert_allclose(np.exp(rows[:, 3]), oracle.nearest_neighbour_distance(p), rtol=1e-12)
    assert np.all(rows[:, 14:] == 0)


def test_keyframe_rule_merges_the_five_frames_since_the_last_keyframe():
    # Sec. III-C.2: frames 0, 5, 10 are keyframes; frame 0 bootstraps with its own points,
    # keyframe 5 merges frames 1-5, keyframe 10 frames 6-10; frames 11-13 wait for keyframe 15
    got = oracle.keyframe_merges(14)
    assert got == [(0, [0]), (5, [1, 2, 3, 4, 5]), (10, [6, 7, 8, 9, 10])]
    assert oracle.keyframe_merges(1) == [(0, [0])]
    # every frame's points are used exactly once by the time its keyframe has arrived
    used = [f for _, fs in oracle.keyframe_merges(16) for f in fs]
    assert sorted(used) == list(range(16))
