"""Launch-shape autotuner for the blend kernels of one map and one set of views.

The forward and backward blends have tunable shapes that leave results unchanged beyond
FP32 summation order: pixels per lane (1, 2 or 4; gs_set_blend_config), the backward's
parallelisation (pixel order or per Gaussian; gs_set_backward_mode) and the long-list
split (gs_set_tile_split). Which is fastest depends on the scene (list lengths, how soon
pixels saturate) and on the views (sizes, how many per batch). `autotune` times each
candidate on the caller's own map and views and keeps the fastest.

Two tuners:
- `autotune` times the parts the shapes affect, render, loss and render_backward of the
  views (with the exposure gradient when exposures are given, as a mapping step has it),
  at the map's current state. No Adam step is taken, so parameters, moments and the step
  count are untouched; the gradient planes and visibility marks the timing leaves are
  cleared afterwards.
- `autotune_step` times runs of consecutive mapping steps (gs_step) from the map's
  current state, restoring parameters, moments, exposure states and the step counter
  before each run and at the end. Blend cost changes as Adam moves the map (opacities and
  scales drift, so pixels saturate sooner or later), and which shape wins can change with
  it; a run of steps sees that drift where a single state does not.
"""
import itertools
import statistics
from typing import Dict, List, Optional, Sequence, Tuple

# (forward px, backward px, backward mode, (parallel, min_chunk, balance))
Config = Tuple[int, int, int, Tuple[int, int, float]]

DEFAULT_SPLITS = [(4096, 128, 1.25), (4096, 128, 2.0), (0, 256, 1.25)]


def candidates(pxs=(1, 2, 4), modes=(0, 1), splits=None) -> List[Config]:
    """Every combination of forward px, backward px, backward mode and split setting; the
    per-Gaussian backward has a fixed shape, so it is paired with one backward px only."""
    out = []
    for fpx, bpx, mode, sp in itertools.product(pxs, pxs, modes, splits or DEFAULT_SPLITS):
        if mode == 1 and bpx != pxs[0]:
            continue
        out.append((fpx, bpx, mode, sp))
    return out


def apply(m, cfg: Config):
    fpx, bpx, mode, sp = cfg
    m.set_blend_config(fpx, bpx)
    m.set_backward_mode(mode)
    m.set_tile_split(*sp)


def autotune(m, cams: Sequence, targets: Sequence, exposures: Optional[Sequence] = None, lam: float = 0.2,
             iters: int = 3, rounds: int = 3, warmup: int = 10,
             configs: Optional[Sequence[Config]] = None) -> Tuple[Config, Dict[Config, float]]:
    """Time render + loss + backward of `cams` for every configuration in `configs`
    (default: `candidates()`), leave the map set to the fastest and return it with the
    measured milliseconds per iteration of every configuration.

    Clocks and caches settle over the first iterations, so `warmup` untimed iterations
    come first, and each of `rounds` rounds visits the configurations in a different
    order (rotated, and reversed every other round); a configuration's time is its
    median over the rounds, each round timing `iters` iterations."""
    from . import gslic
    torch = gslic._torch()
    stream = torch.cuda.current_stream()
    cands = list(configs or candidates())
    if not cands or iters < 1 or rounds < 1:
        raise ValueError("autotune needs at least one configuration, iteration and round")
    grads = [torch.empty(3, c.height, c.width, device=m.device) for c in cams]
    # with exposures the step also differentiates them, which changes the blend backward
    dexp = [torch.zeros(12, device=m.device) for _ in cams] if exposures is not None else None
    frames = None

    def one():
        nonlocal frames
        frames = m.render(cams, exposures, frames=frames)
        for k in range(len(cams)):
            m.loss(frames[k].rgb, targets[k], lam, grad_out=grads[k])
        m.render_backward(grads, dexp)

    apply(m, cands[0])
    for _ in range(warmup):
        one()
    samples: Dict[Config, List[float]] = {c: [] for c in cands}
    n = len(cands)
    for r in range(rounds):
        order = cands[r % n:] + cands[:r % n]
        if r % 2:
            order.reverse()
        for cfg in order:
            apply(m, cfg)
            one()  # sizes the workspaces of this configuration
            start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            start.record(stream)
            for _ in range(iters):
                one()
            stop.record(stream)
            stop.synchronize()
            samples[cfg].append(start.elapsed_time(stop) / iters)
    times = {c: statistics.median(v) for c, v in samples.items()}
    best = min(times, key=times.get)
    apply(m, best)
    m.grads().zero_()
    m.visibility().zero_()
    torch.cuda.synchronize()
    return best, times


def autotune_step(m, cams: Sequence, frames: Sequence, targets: Sequence, exposure_states: Sequence, grads: Sequence,
                  loss_out, lam: float = 0.2, steps: int = 50, rounds: int = 2, warmup: int = 5,
                  configs: Optional[Sequence[Config]] = None) -> Tuple[Config, Dict[Config, float]]:
    """Time `steps` consecutive mapping steps (the arguments of GaussianMap.step) from the
    map's current state for every configuration, leave the map set to the fastest and in
    the state it had on entry, and return the fastest with every configuration's median
    milliseconds per step over `rounds` rounds (orders as in `autotune`)."""
    from . import gslic
    torch = gslic._torch()
    stream = torch.cuda.current_stream()
    cands = list(configs or candidates())
    if not cands or steps < 1 or rounds < 1:
        raise ValueError("autotune_step needs at least one configuration, step and round")
    t0 = m.step_count
    snap = [m.params().clone(), *(t.clone() for t in m.adam_moments()), *(e.clone() for e in exposure_states)]

    def restore():
        m.params().copy_(snap[0])
        mm, vv = m.adam_moments()
        mm.copy_(snap[1])
        vv.copy_(snap[2])
        for e, sv in zip(exposure_states, snap[3:]):
            e.copy_(sv)
        m.set_step_count(t0, stream)
        m.grads().zero_()
        m.visibility().zero_()

    def one():
        m.step(cams, frames, targets, exposure_states, grads, loss_out, lam=lam)

    apply(m, cands[0])
    for _ in range(warmup):
        one()
    samples: Dict[Config, List[float]] = {c: [] for c in cands}
    n = len(cands)
    for r in range(rounds):
        order = cands[r % n:] + cands[:r % n]
        if r % 2:
            order.reverse()
        for cfg in order:
            apply(m, cfg)
            restore()
            one()  # sizes the workspaces of this configuration
            restore()
            start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            start.record(stream)
            for _ in range(steps):
                one()
            stop.record(stream)
            stop.synchronize()
            samples[cfg].append(start.elapsed_time(stop) / steps)
    times = {c: statistics.median(v) for c, v in samples.items()}
    best = min(times, key=times.get)
    apply(m, best)
    restore()
    torch.cuda.synchronize()
    return best, times
