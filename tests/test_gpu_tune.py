"""The launch-shape autotuner: it times candidates on the caller's map without changing
the map, and leaves a configuration whose render matches the default one."""
import numpy as np
import pytest

from gpu_common import IMG_TOL, case, exposures, gpu_map, torch_mod
from paper_2404_06926_amd import scenes, tune

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name", ["c3a", "dense"])
def test_autotune_leaves_the_map_unchanged(name):
    torch = torch_mod()
    params, deg, cams = case(name)
    print(f"case {name}", flush=True)
    m = gpu_map(params, deg)
    tg = [torch.tensor(scenes.smooth_image(3, c.height, c.width), device="cuda") for c in cams]
    ex = exposures(cams)
    p0 = m.params().clone()
    m0 = [t.clone() for t in m.adam_moments()]
    best, times = tune.autotune(m, cams, tg, ex, iters=1, rounds=2, warmup=1)
    torch.cuda.synchronize()
    assert len(times) == len(tune.candidates()) and best in times
    assert all(np.isfinite(v) and v > 0 for v in times.values())
    assert torch.equal(m.params(), p0)
    for a, b in zip(m.adam_moments(), m0):
        assert torch.equal(a, b)
    assert m.step_count == 0
    assert float(m.grads().abs().max()) == 0.0
    assert int(m.visibility().sum()) == 0
    # the chosen shapes change summation order only
    f_best = m.render(cams, ex)
    f_ref = gpu_map(params, deg).render(cams, ex)
    torch.cuda.synchronize()
    for a, b in zip(f_best, f_ref):
        assert float((a.rgb - b.rgb).abs().max()) <= IMG_TOL


def test_autotune_step_restores_the_state():
    # Deterministic backward: a map that tuned and was restored takes the next step
    # bit-identically to one that never tuned, which needs the step counter restored too
    # (it sets the bias corrections); a map with a different counter does not.
    torch = torch_mod()
    from paper_2404_06926_amd import gslic
    params, deg, cams = case("multi")
    print("case multi", flush=True)
    tg = [torch.tensor(scenes.smooth_image(k, c.height, c.width), device="cuda") for k, c in enumerate(cams)]
    frames = [gslic.Frame(torch.empty(3, c.height, c.width, device="cuda"), torch.empty(c.height, c.width, device="cuda"),
                          torch.empty(c.height, c.width, dtype=torch.int32, device="cuda")) for c in cams]
    grads = [torch.empty(3, c.height, c.width, device="cuda") for c in cams]
    loss = torch.empty(len(cams), device="cuda")
    maps, states = [], []
    for _ in range(3):
        m = gpu_map(params, deg)
        m.set_deterministic(True)
        es = [gslic.identity_exposure_state() for _ in cams]
        for _ in range(3):
            m.step(cams, frames, tg, es, grads, loss)
        maps.append(m)
        states.append(es)
    torch.cuda.synchronize()
    m, es = maps[0], states[0]
    p0, m0, e0 = m.params().clone(), [t.clone() for t in m.adam_moments()], [e.clone() for e in es]
    t0 = m.step_count
    configs = tune.candidates(pxs=(1, 2), splits=[(4096, 128, 1.25), (65536, 64, 0.0)])
    best, times = tune.autotune_step(m, cams, frames, tg, es, grads, loss, steps=2, rounds=2, warmup=1,
                                     configs=configs)
    torch.cuda.synchronize()
    assert best in configs and set(times) == set(configs)
    assert all(np.isfinite(v) and v > 0 for v in times.values())
    assert torch.equal(m.params(), p0) and m.step_count == t0
    for a, b in zip(m.adam_moments(), m0):
        assert torch.equal(a, b)
    for a, b in zip(es, e0):
        assert torch.equal(a, b)
    tune.apply(m, (1, 1, 0, (4096, 128, 1.25)))
    maps[2].set_step_count(t0 + 100)
    for mm, ee in zip(maps, states):
        mm.step(cams, frames, tg, ee, grads, loss)
    torch.cuda.synchronize()
    assert maps[0].step_count == maps[1].step_count == t0 + 1 and maps[2].step_count == t0 + 101
    assert torch.equal(maps[0].params(), maps[1].params())
    for a, b in zip(maps[0].adam_moments(), maps[1].adam_moments()):
        assert torch.equal(a, b)
    assert not torch.equal(maps[0].params(), maps[2].params())
