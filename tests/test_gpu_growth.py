"""GPU parity of map growth through the C ABI: initialisation from points and sky
Gaussians (Sec. III-C.1), expansion by the opacity mask (Sec. III-C.2, Eq. 8), against the
oracle on the same seeded inputs."""
import numpy as np
import pytest

import oracle
from gpu_common import gpu_map, torch_mod
from helpers import oview
from paper_2404_06926_amd import scenes

pytestmark = pytest.mark.gpu


def _points(cam, n, seed, zmin=1.0, zmax=15.0, margin=0.2):
    """Points around the frustum (some outside it, some behind the near plane) and colours."""
    r = np.random.default_rng(seed)
    z = r.uniform(zmin, zmax, n)
    u = r.uniform(-margin * cam.width, (1 + margin) * cam.width, n)
    v = r.uniform(-margin * cam.height, (1 + margin) * cam.height, n)
    pc = np.stack([(u - cam.cx) * z / cam.fx, (v - cam.cy) * z / cam.fy, z], 1)
    xyz = (pc - cam.t[None, :]) @ cam.R.astype(np.float64)
    xyz[: n // 20, 2] = -xyz[: n // 20, 2]          # a few behind the camera
    return xyz.astype(np.float32), r.random((n, 3)).astype(np.float32)


def _cam():
    cam = scenes.pinhole(120, 88, 90.0)
    cam.R = scenes.axis_angle([0.05, -0.1, 0.02]).astype(np.float32)
    cam.t = np.array([0.1, -0.05, 0.3], np.float32)
    return cam


def test_add_points_matches_oracle_init():
    torch = torch_mod()
    cam = _cam()
    xyz, rgb = _points(cam, 3000, 1)
    m = gpu_map(np.zeros((0, 11 + 3 * 4), np.float32), 1, cap=1024)
    m.add_points(torch.tensor(xyz).cuda(), torch.tensor(rgb).cuda(), cam, o_init=0.1)
    torch.cuda.synchronize()
    got = m.params().cpu().numpy().T.astype(np.float64)
    ref = oracle.init_points(xyz, rgb, oview(cam), 0.1, 1)
    assert got.shape == ref.shape
    np.testing.assert_array_equal(got[:, 0:3], xyz)
    np.testing.assert_allclose(got[:, 3:6], ref[:, 3:6], rtol=1e-6, atol=1e-6)
    np.testing.assert_allclose(got[:, 6:], ref[:, 6:], rtol=1e-6, atol=1e-6)


@pytest.mark.parametrize("n_map", [0, 4000])
def test_expansion_selects_the_oracle_points(n_map):
    torch = torch_mod()
    cam = _cam()
    params = scenes.frustum_gaussians(n_map, 1, scenes.pinhole(120, 88, 90.0), seed=5, log_scale_mean=-2.2)
    xyz, rgb = _points(cam, 6000, 2)
    # points exactly on pixel boundaries (u = 40.0, v = 30.0 in the camera frame)
    zb = np.array([3.0, 5.0, 7.5])
    pb = np.stack([(40.0 - cam.cx) * zb / cam.fx, (30.0 - cam.cy) * zb / cam.fy, zb], 1)
    xyz = np.concatenate([xyz, ((pb - cam.t[None, :]) @ cam.R.astype(np.float64)).astype(np.float32)])
    rgb = np.concatenate([rgb, np.full((3, 3), 0.5, np.float32)])
    m = gpu_map(params, 1, cap=max(1024, n_map))
    k = m.expand(cam, torch.tensor(xyz).cuda(), torch.tensor(rgb).cuda(), tau=0.99, o_init=0.1)
    torch.cuda.synchronize()
    v = oview(cam)
    if n_map:
        _, _, rend = oracle.forward(params, 1, [v], fp64=True)
        O = rend[0]["opacity"]
    else:
        O = np.zeros((cam.height, cam.width))
    keep, ties = oracle.expansion_select(xyz, v, O, 0.99, tie=1e-5)
    print(f"map {n_map}: kept {k} of {len(xyz)}, oracle {keep.sum()}, ties {ties.sum()}", flush=True)
    got = m.params().cpu().numpy().T.astype(np.float64)[n_map:]
    assert got.shape[0] == k == m.n - n_map
    # rows appended in input order: match them to the points by position
    kept_gpu = np.zeros(len(xyz), bool)
    index = {tuple(p): i for i, p in enumerate(xyz.tolist())}
    for row in got:
        kept_gpu[index[tuple(row[0:3].astype(np.float32).tolist())]] = True
    np.testing.assert_array_equal(kept_gpu[~ties], keep[~ties])
    assert 0 < keep.sum() < len(xyz)
    ref = oracle.init_points(xyz[kept_gpu], rgb[kept_gpu], v, 0.1, 1)
    np.testing.assert_allclose(got[:, 3:], ref[:, 3:], rtol=1e-6, atol=1e-6)


def test_sky_rows_match_oracle():
    torch = torch_mod()
    r = np.random.default_rng(9)
    n = 3000
    cz = r.uniform(0, 1, n)
    ph = r.uniform(0, 2 * np.pi, n)
    sr = np.sqrt(1 - cz ** 2)
    xyz = (np.stack([sr * np.cos(ph), sr * np.sin(ph), cz], 1) * 500.0).astype(np.float32)
    m = gpu_map(np.zeros((0, 11 + 3 * 16), np.float32), 3, cap=1024)
    m.add_sky(torch.tensor(xyz).cuda(), o_sky=0.7)
    torch.cuda.synchronize()
    got = m.params().cpu().numpy().T.astype(np.float64)
    ref = oracle.init_sky(xyz, 0.7, 3)
    np.testing.assert_array_equal(got[:, 0:3], xyz)
    np.testing.assert_allclose(got[:, 3:6], ref[:, 3:6], atol=1e-4)
    np.testing.assert_allclose(got[:, 6:], ref[:, 6:], rtol=1e-6, atol=1e-6)


def test_keyframe_job_expands_by_the_mask():
    # gs_submit_keyframe appends what gs_expand would append on the same map state.
    torch = torch_mod()
    cam = _cam()
    params = scenes.frustum_gaussians(3000, 1, scenes.pinhole(120, 88, 90.0), seed=6, log_scale_mean=-2.2)
    xyz, rgb = _points(cam, 2000, 3)
    a = gpu_map(params, 1)
    k = a.expand(cam, torch.tensor(xyz).cuda(), torch.tensor(rgb).cuda(), tau=0.99, o_init=0.1)
    b = gpu_map(params, 1)
    img = torch.tensor(scenes.smooth_image(1, cam.height, cam.width)).cuda()
    b.submit_keyframe(cam, img, torch.tensor(xyz).cuda(), torch.tensor(rgb).cuda(), iters=1, window=2)
    torch.cuda.synchronize()
    assert b.n == a.n == 3000 + k
    # one Adam step moves a mean by at most lr_mean (1.6e-4) per coordinate
    np.testing.assert_allclose(b.params()[0:3, 3000:].cpu().numpy(), a.params()[0:3, 3000:].cpu().numpy(),
                               atol=2e-4)


def test_frame_rule_merges_five_frames_at_each_keyframe():
    # Sec. III-C.2 through gs_add_frame: frame 0 bootstraps the map with all of its points;
    # frames 5 and 10 are keyframes whose expansion takes the merged points of the five
    # frames up to them through the Eq. 8 mask of the keyframe's view. After each keyframe
    # the appended rows are the oracle's selection on the merged points (in arrival order)
    # initialised by the Sec. III-C.1 rule; other frames append nothing.
    torch = torch_mod()
    base = _cam()
    frames = []
    for f in range(11):
        cam = scenes.pinhole(120, 88, 90.0)
        cam.R = base.R
        cam.t = (base.t + np.array([0.02 * f, 0.0, -0.05 * f])).astype(np.float32)
        xyz, rgb = _points(cam, 700 + 37 * f, 100 + f, margin=0.1)
        frames.append((cam, xyz, rgb, scenes.smooth_image(200 + f, cam.height, cam.width)))
    m = gpu_map(np.zeros((0, 11 + 3 * 4), np.float32), 1, cap=1024)
    merges = dict(oracle.keyframe_merges(len(frames)))
    n_before = 0
    for f, (cam, xyz, rgb, img) in enumerate(frames):
        prev = m.params().cpu().numpy().T.astype(np.float64).copy()
        kid = m.add_frame(cam, torch.tensor(img).cuda(), torch.tensor(xyz).cuda(), torch.tensor(rgb).cuda(), 0.1)
        torch.cuda.synchronize()
        got = m.params().cpu().numpy().T.astype(np.float64)
        if f not in merges:
            assert kid == -1 and got.shape[0] == n_before
            continue
        assert kid == len([k for k in merges if k < f])
        v = oview(cam)
        mxyz = np.concatenate([frames[j][1] for j in merges[f]])
        mrgb = np.concatenate([frames[j][2] for j in merges[f]])
        if f == 0:
            keep, ties = np.ones(len(mxyz), bool), np.zeros(len(mxyz), bool)
        else:
            _, _, rend = oracle.forward(prev, 1, [v], fp64=True)
            keep, ties = oracle.expansion_select(mxyz, v, rend[0]["opacity"], 0.99, tie=1e-5)
        new = got[n_before:]
        index = {tuple(p): i for i, p in enumerate(mxyz.tolist())}
        kept_gpu = np.zeros(len(mxyz), bool)
        order = []
        for row in new:
            i = index[tuple(row[0:3].astype(np.float32).tolist())]
            kept_gpu[i] = True
            order.append(i)
        print(f"keyframe {f}: merged {len(mxyz)} points of frames {merges[f]}, kept {len(new)}, "
              f"oracle {keep.sum()}, ties {ties.sum()}", flush=True)
        assert order == sorted(order)                          # arrival order
        np.testing.assert_array_equal(kept_gpu[~ties], keep[~ties])
        assert 0 < len(new) < len(mxyz) or f == 0
        ref = oracle.init_points(mxyz[kept_gpu], mrgb[kept_gpu], v, 0.1, 1)
        np.testing.assert_allclose(new[:, 3:], ref[:, 3:], rtol=1e-6, atol=1e-6)
        n_before = got.shape[0]
    assert m.keyframe_count() == 3
