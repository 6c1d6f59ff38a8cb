"""Mapping-iteration throughput on one MI355X.

One step = one optimisation iteration of the Gaussian map: project, bin, sort, blend (with
exposure), L1 + D-SSIM loss, backward, sparse Adam (Gaussians and exposures).

Default workload (the headline metric): 1M Gaussians volume-uniform at 2-20 m in the
frustum of a 1280x720 pinhole camera (f = 1000), SH degree 3, one keyframe per step,
target = render of the same map with means jittered by N(0, 5 cm). The step is captured
as a HIP graph and replayed; a second timed region runs the same steps eagerly with HIP
events around every stage for the per-kernel durations.

--workload batch8: 1M Gaussians (SH0) and 8 keyframes of uneven size (640x400, 960x600,
1280x720, 1440x1080, each twice) per step, batched in one launch sequence and captured,
against the plain path that launches the same sequence once per view and takes one Adam
step over the summed gradients.

--workload stream: one map session fed by a street drive (keyframes at Poisson 10 Hz,
speed U[5, 15] m/s re-drawn every 5 s, 1280x720, 200k initial Gaussians, 20k-80k new points
per keyframe from 10-60 m ahead, appended with the point initialisation up to 3M); every
keyframe runs 10 iterations over the 8 most recent keyframes. Reports iterations/s and the
p50/p99 keyframe latency (completion of the 10th iteration minus arrival; the upload of the
keyframe's image and points is inside it).

--workload multi: 16 sessions with static maps of exp(U[ln 1e5, ln 6e6]) Gaussians (SH3),
resolutions from {640x480, 960x600, 1280x720, 1440x1080, 1920x1200}, Poisson keyframe
arrivals at U[5, 20] Hz each, the same 10-iteration / 8-keyframe jobs, admission under an
HBM budget (32 GiB). Reports aggregate iterations/s and p50/p99 per session and overall.

Inputs are synthetic and resident in HBM before timing (serving workloads: targets and
points in pinned host memory, uploaded inside each job). Prints one JSON line.
`--gpus N` with N > 1 exits: this build runs on one GPU.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "mapping iters/s (fwd+bwd+Adam) @1M Gaussians 1280×720; p50/p99 keyframe latency"
HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3          # 256 CU x 128 FP32 lanes x 2 (FMA) x 2.4 GHz
# FLOPs per (pixel, list entry) pair, counted from the blend arithmetic up to the pixel's
# last contributor. Forward: offset 2, quadratic 6, exp 1, alpha 2, cut-off and stop
# tests 3, T (1 - alpha) 2, colour 4. Backward: the forward's 9 for alpha, T recovery 2,
# colour gradient 4, dL/dalpha 9, colour-behind update 6, dL/dpower and its five moments
# 6, share of the wave reduction 10.
FWD_FLOPS_PER_PAIR = 20
BWD_FLOPS_PER_PAIR = 46


def split_config(args):
    par, mn, bal = args.split.split(",")
    return int(par), int(mn), float(bal)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def recorded_traffic(kernel, workload_tag):
    """HBM bytes per launch of `kernel` from the committed counter summary of this workload
    (profiles/hbm_traffic_<tag>.md), or None when there is none or the kernel's source file
    changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"hbm_traffic_{workload_tag}.md")
    if not os.path.exists(path):
        return None
    for line in open(path):
        if not line.startswith("kernel="):
            continue
        f = dict(kv.split("=", 1) for kv in line.split())
        if f["kernel"] != kernel:
            continue
        src = os.path.join(ROOT, f["source"])
        if not os.path.exists(src) or hashlib.sha256(open(src, "rb").read()).hexdigest() != f["sha256"]:
            return None
        return float(f["bytes_per_launch"])
    return None


def recorded_valu(kernel, workload_tag):
    """VALU wave-instructions per launch of `kernel` from the committed SQ counter summary
    (profiles/sq_counters_<tag>.md), or None (no summary, or the source changed since)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"sq_counters_{workload_tag}.md")
    if not os.path.exists(path):
        return None
    for line in open(path):
        if not line.startswith("kernel="):
            continue
        f = dict(kv.split("=", 1) for kv in line.split())
        if f["kernel"] != kernel:
            continue
        src = os.path.join(ROOT, f["source"])
        if not os.path.exists(src) or hashlib.sha256(open(src, "rb").read()).hexdigest() != f["sha256"]:
            return None
        return float(f["valu_insts"])
    return None


# wave64 VALU instructions the device can issue per second: 256 CUs x 4 SIMDs, one every
# 4 cycles, 2.4 GHz
VALU_ISSUE_PER_S = 256 * 4 * 2.4e9 / 4


def headline_workload(n, deg, W, H, seed=2024):
    from paper_2404_06926_amd import scenes
    cam = scenes.pinhole(W, H, 1000.0 * W / 1280.0)
    params = scenes.frustum_gaussians(n, deg, cam, seed=seed)
    target_params = scenes.jitter_means(params, 0.05, seed)
    return [cam], params, target_params


def batch_workload(n, seed=3003):
    from paper_2404_06926_amd import scenes
    ref = scenes.pinhole(1280, 720, 1000.0)
    params = scenes.frustum_gaussians(n, 0, ref, seed=seed)
    target_params = scenes.jitter_means(params, 0.05, seed)
    return scenes.batch_views(seed, 8), params, target_params


def cpu_baseline(params, target_params, deg, cam, lam):
    """The oracle's full step (FP64 blend, loss, adjoint, sparse Adam) on the same
    workload, timed once on this host."""
    import oracle
    v = oracle.OView(cam=cam.cam16(), W=cam.width, H=cam.height, E=cam.exposure.astype(np.float64),
                     bg=cam.bg.astype(np.float64))
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    t0 = time.perf_counter()
    _, _, tgt = oracle.forward(target_params, deg, [v])
    t_target = time.perf_counter() - t0
    t0 = time.perf_counter()
    projs, bins, rend = oracle.forward(params, deg, [v])
    L, g, _ = oracle.loss(rend[0]["out"], tgt[0]["out"], lam)
    gp, gE, _ = oracle.backward(params, deg, [v], projs, bins, [g])
    vis = (projs[0]["count"] > 0).astype(np.uint8)
    F = params.shape[1]
    oracle.adam(params, gp, np.zeros_like(gp), np.zeros_like(gp), vis, np.full(F, 1e-3), 0.9, 0.999, 1e-15, 1)
    dt = time.perf_counter() - t0
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return dict(value=1.0 / dt, unit="iters/s", cores=threads, kind="oracle", cpu_model=model,
                nproc=os.cpu_count(),
                sample=f"one full step of the same workload (FP64 oracle, {dt:.1f} s; target render "
                       f"{t_target:.1f} s not counted)")


class StepBuffers:
    def __init__(self, torch, gslic, cams, dev):
        self.frames = [gslic.Frame(torch.empty(3, c.height, c.width, device=dev), torch.empty(c.height, c.width, device=dev),
                                   torch.empty(c.height, c.width, dtype=torch.int32, device=dev)) for c in cams]
        self.expo = [gslic.identity_exposure_state(dev) for _ in cams]
        self.grads = [torch.empty(3, c.height, c.width, device=dev) for c in cams]
        self.loss = torch.empty(len(cams), device=dev)


def timed(torch, fn, steps):
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record()
    for _ in range(steps):
        fn()
    stop.record()
    torch.cuda.synchronize()
    return start.elapsed_time(stop) / steps


def _pinned(torch, a):
    t = torch.empty(a.shape, dtype=torch.float32, pin_memory=True)
    t.copy_(torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)))
    return t


def _render_targets(torch, gslic, params, deg, cams, dev):
    """Renders of a hidden map at the given cameras, copied to pinned host memory."""
    gt = gslic.GaussianMap(sh_degree=deg, capacity=max(1024, params.shape[0]))
    gt.add_gaussians(torch.from_numpy(params).to(dev))
    out = []
    for c in cams:
        img = gt.render([c])[0].rgb
        h = torch.empty(img.shape, dtype=torch.float32, pin_memory=True)
        h.copy_(img)
        out.append(h)
    torch.cuda.synchronize()
    gt.close()
    return out


def stream_specs(args, torch, gslic, dev):
    """Config of the street drive: one session whose jobs carry targets and new points."""
    from paper_2404_06926_amd import scenes, serve
    seed, deg, cap = 4000, args.sh, 3_000_000
    dur = args.duration if args.duration is not None else 5.0
    lay = scenes.street_layout(seed)
    arrivals, xs, yaws = scenes.stream_schedule(seed, dur)
    cams = [scenes.street_camera(x, y) for x, y in zip(xs, yaws)]
    centre = (250.0, 0.0, 0.0)
    # hidden ground-truth map over the driven stretch (3000 points per metre) and the sky
    x_hi = (float(xs.max()) if len(xs) else 0.0) + 100.0
    gxyz, grgb = scenes.street_points(seed, lay, -5.0, x_hi, int(3000 * (x_hi + 5.0)), "ground_truth")
    gt = np.concatenate([scenes.street_gaussians(seed + 1, gxyz, grgb, deg),
                         scenes.sky_gaussians(seed + 1, 20_000, centre, 500.0, deg)])
    log(f"stream: {len(arrivals)} keyframes over {dur} s, x up to {x_hi - 100:.1f} m, GT map {gt.shape[0]}")
    targets = _render_targets(torch, gslic, gt, deg, cams, dev)
    del gt
    # the map at the start: first 20 m and the sky
    xyz0, rgb0 = scenes.street_points(seed, lay, 0.0, 20.0, 200_000, "initial")
    init = np.concatenate([scenes.street_gaussians(seed + 2, xyz0, rgb0, deg, ref=(0.0, 0.0, 1.8)),
                           scenes.sky_gaussians(seed + 2, 20_000, centre, 500.0, deg)])
    r = scenes.rng(seed, "stream_counts")
    n = init.shape[0]
    jobs = []
    for k, (a, x) in enumerate(zip(arrivals, xs)):
        cnt = int(r.integers(20_000, 80_001))
        xyz = rgb = None
        if n + cnt <= cap:
            pxyz, prgb = scenes.street_points(seed, lay, x + 10.0, x + 60.0, cnt, f"keyframe{k}")
            xyz, rgb = _pinned(torch, pxyz), _pinned(torch, prgb)
            n += cnt
        jobs.append(serve.Job(arrival=float(a), cam=cams[k], image=targets[k], xyz=xyz, rgb=rgb))
    est = serve.estimate_bytes(n, deg, 8, 1280, 720)
    return [serve.SessionSpec(sid=0, jobs=jobs, est_bytes=est, init=init, sh_degree=deg)], n


def multi_specs(args, torch, gslic, dev):
    """16 sessions with static maps, poses around each session's reference camera."""
    from paper_2404_06926_amd import scenes, serve
    seed, deg = 5000, 3
    dur = args.duration if args.duration is not None else 2.0
    r = scenes.rng(seed, "sessions")
    sizes = [(640, 480), (960, 600), (1280, 720), (1440, 1080), (1920, 1200)]
    specs = []
    for sid in range(16):
        n = int(np.exp(r.uniform(np.log(1e5), np.log(6e6))))
        W, H = sizes[int(r.integers(0, len(sizes)))]
        rate = float(r.uniform(5, 20))
        ref = scenes.pinhole(W, H, 200.0 * W / 256)
        params = scenes.frustum_gaussians(n, deg, ref, seed=seed + sid)
        poses = scenes.batch_views(seed + sid, 8)
        cams = [scenes.pinhole(W, H, 200.0 * W / 256, R=c.R, t=c.t) for c in poses]
        targets = _render_targets(torch, gslic, scenes.jitter_means(params, 0.05, seed + sid), deg, cams, dev)
        arr = serve.poisson_arrivals(scenes.rng(seed + sid, "arrivals"), rate, dur)
        jobs = [serve.Job(arrival=a, cam=cams[k % 8], image=targets[k % 8]) for k, a in enumerate(arr)]
        specs.append(serve.SessionSpec(sid=sid, jobs=jobs, est_bytes=serve.estimate_bytes(n, deg, 8, W, H),
                                       init=params, sh_degree=deg))
        log(f"session {sid}: N={n} {W}x{H} {rate:.1f} Hz, {len(jobs)} keyframes")
    return specs


def run_serving(args, torch, gslic):
    from paper_2404_06926_amd import serve
    dev = torch.device("cuda:0")
    if args.workload == "stream":
        specs, n_final = stream_specs(args, torch, gslic, dev)
        budget = 256 << 30
        be = serve.GpuBackend(device=dev, iters=10, window=8, lam=args.lam, o_init=0.1, capacity=n_final)
    else:
        specs = multi_specs(args, torch, gslic, dev)
        budget = int(args.budget_gib * (1 << 30))
        be = serve.GpuBackend(device=dev, iters=10, window=8, lam=args.lam, o_init=0.1)
    sch = serve.Scheduler(be, budget_bytes=budget, slots=4, poll_s=2e-4)
    for sp in specs:
        sch.add(sp)
    torch.cuda.synchronize()
    log(f"serving run: {sum(len(sp.jobs) for sp in specs)} keyframes")
    res = sch.run(max_wall_s=900)
    iters = 10 * res["jobs"]
    views = sum(min(k + 1, 8) * 10 for sp in specs for k in range(len(sp.jobs)))
    dur = max(j.arrival for sp in specs for j in sp.jobs) if res["jobs"] else 0.0
    out = {
        "metric": METRIC,
        "value": iters / res["wall_s"],
        "unit": "iters/s",
        "n_gpus": 1,
        "steps": iters,
        "warmup": 0,
        "ms_per_step": res["wall_s"] * 1e3 / max(iters, 1),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": ("street drive, 1 session, 1280x720, 10 iterations over the 8 latest keyframes "
                                "per keyframe" if args.workload == "stream" else
                                "16 sessions, static maps 1e5-6e6 Gaussians SH3, 10 iterations over the 8 latest "
                                "keyframes per keyframe, HBM budget %.0f GiB" % args.budget_gib),
                   "arrivals_s": dur, "keyframes": res["jobs"], "view_iterations": views},
        "latency_ms": {"p50": res["p50_ms"], "p99": res["p99_ms"]},
        "wall_s": res["wall_s"],
        "view_iterations_per_s": views / res["wall_s"],
        "peak_resident_bytes": res["peak_resident_bytes"],
    }
    if args.workload == "multi":
        out["sessions"] = res["sessions"]
    else:
        out["final_gaussians"] = n_final
    return out


def run_schedule(args, torch, gslic):
    """The paper's keyframe schedule against batched windows, from the same starting map
    over the same number of view-iterations: every keyframe is kept; each round of the
    paper's schedule draws K = min(100, keyframes) of them without replacement in random
    order and takes one single-view Adam step per keyframe (Sec. III-C.3); a batched step
    takes 8 keyframes drawn the same way in one launch sequence. Reports view-iterations/s
    of both and the PSNR of every keyframe's render against its target at the start and
    after each run, the batched run continued to as many Adam steps as the paper's takes
    (400k Gaussians SH3; 40 uneven keyframes around a reference camera; the targets render
    the map with jittered means)."""
    from paper_2404_06926_amd import scenes
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream(device=dev)
    torch.cuda.set_stream(stream)
    seed, n, n_kf, deg, budget = 4040, 400_000, 40, 3, 1600
    ref = scenes.pinhole(1280, 720, 1000.0)
    params = scenes.frustum_gaussians(n, deg, ref, seed=seed)
    target_params = scenes.jitter_means(params, 0.05, seed)
    cams = scenes.batch_views(seed, n_kf)
    targets = [t.to(dev) for t in _render_targets(torch, gslic, target_params, deg, cams, dev)]
    rng = np.random.default_rng(seed)

    def new_map(views_per_step):
        m = gslic.GaussianMap(sh_degree=deg, capacity=n)
        m.add_gaussians(torch.from_numpy(params).to(dev))
        cap = 0
        for c in cams:  # instance buffers sized once, from every keyframe's render
            m.render([c])
            torch.cuda.synchronize()
            cap = max(cap, m.debug_last_render()["n_inst"])
        m.set_instance_policy(False, int(cap * 1.5) * views_per_step + 65536)
        return m

    def psnr(m):
        vals = []
        for c, t in zip(cams, targets):
            f = m.render([c])[0]
            mse = float(((f.rgb - t) ** 2).mean())
            vals.append(10.0 * np.log10(1.0 / max(mse, 1e-12)))
        return float(np.mean(vals))

    # paper's schedule
    mp = new_map(1)
    psnr0 = psnr(mp)
    for c, t in zip(cams, targets):
        mp.add_keyframe(c, t)
    K = min(100, n_kf)
    rounds = [rng.permutation(n_kf)[:K].tolist() for _ in range(budget // K)]
    mp.optimize_keyframes(rounds[0][:4], lam=args.lam)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for ids in rounds:
        mp.optimize_keyframes(ids, lam=args.lam)
    torch.cuda.synchronize()
    t_paper = time.perf_counter() - t0
    psnr_paper = psnr(mp)
    overflow = mp.check_overflow()
    mp.close()

    # batched windows of 8 keyframes
    mb = new_map(8)
    B = StepBuffers(torch, gslic, cams, dev)
    win = 8
    # as many view-iterations as the paper's schedule, then on to as many Adam steps
    draws = [rng.permutation(n_kf)[:win].tolist() for _ in range(budget)]

    def bstep(ids):
        mb.step([cams[i] for i in ids], [B.frames[i] for i in ids], [targets[i] for i in ids],
                [B.expo[i] for i in ids], [B.grads[i] for i in ids], B.loss[:len(ids)], lam=args.lam)

    bstep(draws[0][:2])  # warm-up
    torch.cuda.synchronize()
    n_eq = budget // win
    t0 = time.perf_counter()
    for ids in draws[:n_eq]:
        bstep(ids)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    psnr_batch = psnr(mb)
    t0 = time.perf_counter()
    for ids in draws[n_eq:]:
        bstep(ids)
    torch.cuda.synchronize()
    t_batch2 = t_batch + time.perf_counter() - t0
    psnr_batch2 = psnr(mb)
    overflow = overflow or mb.check_overflow()
    mb.close()
    if overflow:
        raise RuntimeError("instance capacity exceeded in the schedule comparison")
    views = K * len(rounds)
    return {
        "metric": "view-iterations/s, paper's random-K keyframe schedule vs batched windows of 8",
        "value": views / t_paper,
        "unit": "view-iterations/s",
        "n_gpus": 1,
        "steps": len(rounds) * K,
        "warmup": 4,
        "ms_per_step": t_paper * 1e3 / views,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "%d Gaussians SH%d, %d uneven keyframes (640x400 to 1440x1080), K = %d per round, "
                               "%d view-iterations per schedule; PSNR of identity-exposure renders" % (n, deg, n_kf, K, views)},
        "paper_schedule": {"view_iterations_per_s": views / t_paper, "wall_s": t_paper, "psnr_db": psnr_paper},
        "batched_window": {"view_iterations_per_s": n_eq * win / t_batch, "wall_s": t_batch,
                           "steps": n_eq, "psnr_db": psnr_batch},
        "batched_window_equal_steps": {"view_iterations_per_s": budget * win / t_batch2, "wall_s": t_batch2,
                                       "steps": budget, "psnr_db": psnr_batch2},
        "psnr_start_db": psnr0,
    }


def measure_copy(torch, dev, nbytes=1 << 30, reps=20):
    """Achievable HBM bandwidth: a device-to-device copy of `nbytes` (torch's copy kernel),
    counted as nbytes read + nbytes written per copy, averaged over `reps` copies."""
    src = torch.ones(nbytes // 4, device=dev)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    ms = timed(torch, lambda: dst.copy_(src), reps)
    del src, dst
    torch.cuda.empty_cache()
    return {"GBs": 2.0 * nbytes / (ms * 1e-3) / 1e9, "bytes_per_copy": 2 * nbytes, "ms_per_copy": ms,
            "frac_of_peak": 2.0 * nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, "kernel": "torch copy_ (device to device)"}


def cpu_config1(lam=0.0):
    """The oracle's config-1 step (10k Gaussians SH0 at 256x192, L1 only, one forward and
    backward) with one host thread and with every host thread."""
    import oracle
    from paper_2404_06926_amd import scenes
    cam = scenes.pinhole(256, 192, 200.0)
    params = scenes.frustum_gaussians(10_000, 0, cam, seed=1000)
    target = scenes.jitter_means(params, 0.05, 1000)
    v = oracle.OView(cam=cam.cam16(), W=cam.width, H=cam.height)
    tgt = oracle.forward(target, 0, [v])[2][0]["out"]

    def one():
        t0 = time.perf_counter()
        projs, bins, rend = oracle.forward(params, 0, [v])
        _, g, _ = oracle.loss(rend[0]["out"], tgt, lam)
        oracle.backward(params, 0, [v], projs, bins, [g])
        return time.perf_counter() - t0

    all_threads = oracle.set_threads(1)
    try:
        t1 = min(one() for _ in range(2))
    finally:
        oracle.set_threads(all_threads)
    tn = min(one() for _ in range(2))
    return {"workload": "10k Gaussians SH0, 256x192, L1, one forward + backward (best of 2)",
            "threads_1": {"iters_per_s": 1.0 / t1, "s": t1},
            f"threads_{all_threads}": {"iters_per_s": 1.0 / tn, "s": tn}, "host_threads": all_threads}


def bench_step(torch, gslic, args, dev, workload, steps, warmup, with_plain=False, with_cpu=False):
    """Graph-replayed mapping steps of one workload (headline, outdoor or batch8) from a
    restored state, eager steps with per-stage HIP events, the roofline of the dominant
    stage; batch8 also times the plain path (one view per launch)."""
    sh = 0 if workload == "batch8" else args.sh
    n = args.n
    if workload == "batch8":
        cams, params, target_params = batch_workload(n)
    elif workload == "outdoor":
        from paper_2404_06926_amd import scenes
        params, cam = scenes.outdoor_scene(2000, deg=3)
        target_params = scenes.jitter_means(params, 0.05, 2000)
        cams = [cam]
        n, sh = params.shape[0], 3
    else:
        cams, params, target_params = headline_workload(n, sh, args.width, args.height)
    log(f"workload {workload}: n={n} sh={sh} views={[(c.width, c.height) for c in cams]}")

    # targets: renders of the jittered map (outside the timed regions)
    tmap = gslic.GaussianMap(sh_degree=sh, capacity=n)
    tmap.add_gaussians(torch.from_numpy(target_params).to(dev))
    targets = [f.rgb.clone() for f in tmap.render(cams)]
    tmap.close()
    del tmap

    m = gslic.GaussianMap(sh_degree=sh, capacity=n)
    m.add_gaussians(torch.from_numpy(params).to(dev))
    fpx, bpx = (int(x) for x in args.blend_px.split(","))
    m.set_blend_config(fpx, bpx)
    m.set_backward_mode(args.bwd_mode)
    m.set_tile_split(*split_config(args))
    B = StepBuffers(torch, gslic, cams, dev)

    def step():
        m.step(cams, B.frames, targets, B.expo, B.grads, B.loss, lam=args.lam)

    step()  # plans the instance buffers
    torch.cuda.synchronize()
    n_inst0 = m.debug_last_render()["n_inst"]
    m.set_instance_policy(False, int(n_inst0 * 1.5) + 65536)
    tuned = None
    if args.autotune and workload == args.workload:
        from paper_2404_06926_amd import tune
        best, times = tune.autotune_step(m, cams, B.frames, targets, B.expo, B.grads, B.loss, lam=args.lam,
                                         steps=min(steps, 50))
        fpx, bpx, args.bwd_mode, sp = best
        args.split = ",".join(str(x) for x in sp)
        tuned = {"chosen": {"blend_px_per_lane": [fpx, bpx], "backward_mode": args.bwd_mode, "tile_split": list(sp)},
                 "configs_tried": len(times), "ms_best": times[best],
                 "ms_defaults": times.get((1, 1, 0, (4096, 128, 1.25)))}
        log(f"autotune: {tuned}")
        log("autotune times: " + "; ".join(f"{k}: {v:.3f}" for k, v in sorted(times.items(), key=lambda kv: kv[1])))
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()

    # Every timed region starts from this state: the map's cost changes as Adam moves it
    # (opacities and scales drift), so regions are made comparable by restoring parameters,
    # Adam moments and exposure states before each (outside the timed regions).
    snap = [m.params().clone(), *(t.clone() for t in m.adam_moments()), *(e.clone() for e in B.expo)]

    def restore():
        m.params().copy_(snap[0])
        mm, vv = m.adam_moments()
        mm.copy_(snap[1])
        vv.copy_(snap[2])
        for e, sv in zip(B.expo, snap[3:]):
            e.copy_(sv)
        torch.cuda.synchronize()

    def work_counts():
        dbg = m.debug_last_render()
        return dict(n_inst=dbg["n_inst"], n_vis=int((dbg["counts"] > 0).sum().item()),
                    pairs=sum(int(f.n_contrib.to(torch.int64).sum().item()) for f in B.frames),
                    n_tiles=dbg["n_tiles"])

    # work of the first step of a region (untimed), for the average with the last one
    restore()
    step()
    torch.cuda.synchronize()
    wc_first = work_counts()

    # eager timed region with per-stage HIP events
    restore()
    m.set_stage_timing(True)
    m.stage_times()
    log(f"instances {n_inst0}; eager timed region ({steps} steps)")
    ms_eager = timed(torch, step, steps)
    stages = m.stage_times()
    m.set_stage_timing(False)
    wc_last = work_counts()

    # captured step, replayed
    graph = None
    ms_graph = None
    if not args.eager:
        graph = m.capture_step(cams, B.frames, targets, B.expo, B.grads, B.loss, lam=args.lam)
        for _ in range(warmup):
            graph.launch()
        log(f"graph timed regions ({args.repeats} x {steps} steps)")
        runs = []
        for _ in range(max(args.repeats, 1)):
            restore()
            runs.append(timed(torch, graph.launch, steps))
        ms_graph = float(np.median(runs))
    if m.check_overflow():
        raise RuntimeError("instance buffer overflow during the timed steps")
    ms = ms_graph if ms_graph is not None else ms_eager

    # work per step: the mean of the first and last step of the eager region (the stage
    # times are averages over that region; the work grows as the map moves)
    avg = lambda k: (wc_first[k] + wc_last[k]) / 2.0
    n_inst, n_vis, pairs = avg("n_inst"), avg("n_vis"), avg("pairs")
    F = 11 + 3 * (sh + 1) ** 2
    T_total = wc_last["n_tiles"]
    P = sum(c.width * c.height for c in cams)
    tile_passes = (int(np.ceil(np.log2(T_total + 1))) + 7) // 8
    V = len(cams)

    per = {k: (v[0] / max(v[1], 1)) for k, v in stages.items() if v[1] > 0}
    # Algorithmic work per launch of each stage: the HBM bytes the method must move (all
    # stages) and FLOPs (blend kernels, bound by the vector ALU). The blend kernels' list
    # entries are gathers of records that several tiles share and their gradient atomics
    # meet in L2: those are reported as L2 bytes beside the HBM minimum, never inside it.
    l2 = {
        # 36-B record (2D mean, conic with opacity, colour) and two indices per list entry
        "blend": 44.0 * n_inst,
        # the same gathers, plus nine float atomics per instance into the 2D-gradient record
        "blend_backward": 44.0 * n_inst + 36.0 * n_inst,
    }
    work = {
        "project": ("hbm", 4.0 * 14 * n + 4.0 * (F - 14) * n + 64.0 * n_vis + 8.0 * V * n, 0),
        # 20 B per key and pass (4 read up, 8 read + 8 written down); the first pass reads no values
        "depth_sort": ("hbm", (4 * 20.0 - 4.0) * V * n, 0),
        "scan": ("hbm", 12.0 * V * n, 0),
        "duplicate": ("hbm", 24.0 * n_vis + 8.0 * n_inst, 0),
        "sort": ("hbm", (tile_passes * 20.0 - 4.0) * n_inst, 0),
        "ranges": ("hbm", 4.0 * n_inst + 8.0 * T_total, 0),
        # HBM minimum: each visible record once, 8 B of indices per entry, 20 B per pixel out
        "blend": ("alu", 36.0 * n_vis + 8.0 * n_inst + 20.0 * P, FWD_FLOPS_PER_PAIR * float(pairs)),
        "loss": ("hbm", 36.0 * P, 0),   # read out and gt, write dL/dout (3 channels)
        # HBM minimum: records once, indices, 32 B per pixel in, the 2D-gradient record written once
        "blend_backward": ("alu", 36.0 * n_vis + 8.0 * n_inst + 32.0 * P + 48.0 * n_vis,
                           BWD_FLOPS_PER_PAIR * float(pairs)),
        # fused with Adam: read and write parameters, m and v (3 x 4F B each way), read and
        # clear the 48-B 2D-gradient record, read the tile counts
        "project_backward": ("hbm", 24.0 * F * n_vis + 96.0 * n_vis + 4.0 * V * n, 0),
        "adam": ("hbm", 2 * 4.0 * 48 * V, 0),   # exposures of the separate path (a fused step updates them in project_backward)
    }
    names = {"blend_backward": (f"k_blend_bwd<{bpx},false,false>" if args.bwd_mode == 0 else "k_blend_bwd_pg<false>"),
             "blend": f"k_blend_fwd<{fpx},false>",
             "project_backward": f"k_project_bwd<{sh},true,{'true' if len(cams) > 1 else 'false'}>",
             "project": f"k_project_fwd<{sh}>",
             "loss": "k_ssim_tile", "duplicate": "k_dup_lb"}
    tag = f"{workload}_{n // 1000}k_sh{sh}_{args.width}x{args.height}"
    kernel_table = {}
    for k, ms_k in per.items():
        if k not in work:
            continue
        bound_k, bytes_k, flops_k = work[k]
        d = ms_k * 1e-3
        row = {"ms": round(ms_k, 4), "bound": bound_k, "alg_bytes": bytes_k,
               "hbm_frac": round(bytes_k / d / (HBM_PEAK_GBS * 1e9), 4)}
        if k in l2:
            row["l2_bytes"] = l2[k]
        if flops_k:
            row["flops"] = flops_k
            row["valu_frac"] = round(flops_k / d / (FP32_PEAK_TFLOPS * 1e12), 4)
        t_k = recorded_traffic(names[k], tag) if k in names else None
        if t_k is not None:
            row["traffic_bytes"] = t_k
            row["traffic_frac"] = round(t_k / d / (HBM_PEAK_GBS * 1e9), 4)
        v_k = recorded_valu(names[k], tag) if k in names else None
        if v_k is not None:
            row["valu_issue_frac"] = round(v_k / (d * VALU_ISSUE_PER_S), 4)
        kernel_table[k] = row
    dom = max(per, key=lambda k: per[k])
    bound, nbytes, nflops = work[dom]
    dur_s = per[dom] * 1e-3
    if bound == "hbm":
        achieved, peak, unit = nbytes / dur_s / 1e9, HBM_PEAK_GBS, "GB/s"
    else:
        achieved, peak, unit = nflops / dur_s / 1e12, FP32_PEAK_TFLOPS, "TFLOP/s"
    traffic = recorded_traffic(names[dom], tag) if dom in names else None
    roof = dict(bound=bound, kernel=dom, achieved=achieved, peak=peak, unit=unit, frac=achieved / peak,
                traffic=traffic, avg_launch_ms=per[dom])
    valu = recorded_valu(names[dom], tag) if dom in names else None
    if valu is not None:
        # instruction side of an ALU-bound kernel: VALU wave-instructions per launch (SQ
        # counters) over what the device issues in the launch's duration
        roof["valu_issue_frac"] = valu / (dur_s * VALU_ISSUE_PER_S)
    if traffic is not None:
        roof["traffic_unit"] = "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-probe scaled)"
        roof["traffic_GBs"] = traffic / dur_s / 1e9

    result = {
        "metric": METRIC,
        "value": 1000.0 / ms,
        "unit": "iters/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "repeats": args.repeats,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": (("outdoor street (LiDAR-shaped + 20k sky), " if workload == "outdoor" else "")
                                + f"{n} Gaussians, SH{sh}, "
                                + ", ".join(f"{c.width}x{c.height}" for c in cams)
                                + f" per step, loss 0.8 L1 + 0.2 D-SSIM, sparse Adam"),
                   "n_gaussians": n, "sh_degree": sh, "views_per_step": V,
                   "timing": "graph replay" if ms_graph is not None else "eager",
                   "blend_px_per_lane": [fpx, bpx],
                   "tile_split": list(split_config(args)),
                   "autotuned": tuned,
                   "backward_blend": "pixel order" if args.bwd_mode == 0 else "per Gaussian"},
        "roofline": roof,
        "eager_ms_per_step": ms_eager,
        "stages_ms": {k: round(v, 4) for k, v in per.items()},
        "kernels": kernel_table,
        "counts": {"visible_pairs": n_vis, "instances": n_inst, "pairs": pairs, "tiles": T_total,
                   "first_step": wc_first, "last_step": wc_last},
    }

    if with_plain:
        # plain: the same views launched one at a time, gradients summed, one Adam step
        Bp = StepBuffers(torch, gslic, cams, dev)

        def plain():
            for k, c in enumerate(cams):
                m.render([c], [Bp.expo[k]], frames=[Bp.frames[k]])
                m.loss(Bp.frames[k].rgb, targets[k], args.lam, loss_out=Bp.loss[k:k + 1], grad_out=Bp.grads[k])
                m.render_backward([Bp.grads[k]], [Bp.expo[k][12:24]])
            m.adam_step(Bp.expo)

        # the plain path at the batched step's long-list split and with no split (single
        # views of uniform scenes blend faster whole); the faster one is the baseline
        plain_by_split = {}
        for sp in (split_config(args), (0, 256, 1.25)):
            m.set_tile_split(*sp)
            for _ in range(warmup):
                plain()
            restore()
            plain_by_split[",".join(str(x) for x in sp)] = timed(torch, plain, steps)
            if m.check_overflow():
                raise RuntimeError("instance buffer overflow in the plain path")
        m.set_tile_split(*split_config(args))
        ms_plain = min(plain_by_split.values())
        result["plain_ms_per_step"] = ms_plain
        result["plain_ms_per_step_by_split"] = plain_by_split
        result["batched_over_plain"] = ms_plain / ms
        result["batched_eager_over_plain"] = ms_plain / ms_eager
        result["metric"] = "mapping iters/s, 8 uneven keyframes per step (batched vs one view per launch)"
    if workload == "outdoor":
        result["metric"] = "mapping iters/s (fwd+bwd+Adam), outdoor single view, 500k Gaussians 1280x720"
    if graph is not None:
        graph.close()
    m.close()
    if with_cpu and not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        try:
            result["cpu_baseline"] = cpu_baseline(params, target_params, sh, cams[0], args.lam)
        except Exception as e:  # report, never fail the GPU result
            result["cpu_baseline"] = {"error": repr(e)}
    return result


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--repeats", type=int, default=1, help="timed regions of --steps steps; the median is reported")
    ap.add_argument("--workload", choices=["headline", "outdoor", "batch8", "stream", "multi", "schedule"],
                    default="headline")
    ap.add_argument("--duration", type=float, default=None,
                    help="serving workloads: seconds of keyframe arrivals (stream 5, multi 2)")
    ap.add_argument("--budget-gib", type=float, default=32.0, help="multi: HBM admission budget")
    ap.add_argument("--n", type=int, default=1_000_000)
    ap.add_argument("--sh", type=int, default=3)
    ap.add_argument("--width", type=int, default=1280)
    ap.add_argument("--height", type=int, default=720)
    ap.add_argument("--lam", type=float, default=0.2)
    ap.add_argument("--eager", action="store_true", help="time eager steps instead of graph replays")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="headline only: skip the outdoor, batch8, street-drive latency, copy and config-1 CPU legs")
    ap.add_argument("--extra-steps", type=int, default=10, help="timed steps of the batch8 and outdoor legs")
    ap.add_argument("--stream-seconds", type=float, default=3.0, help="arrivals of the street-drive latency leg")
    ap.add_argument("--blend-px", default="1,1",
                    help="pixels per lane of the forward and backward blend kernels (1, 2 or 4)")
    ap.add_argument("--split", default="4096,128,1.25",
                    help="long-list split of the blend: parallel,min_chunk,balance (parallel 0: every tile whole)")
    ap.add_argument("--autotune", action="store_true",
                    help="choose the blend launch shapes by timing runs of mapping steps of every candidate on this map")
    ap.add_argument("--bwd-mode", type=int, default=0,
                    help="backward blend: 0 pixel order, 1 per Gaussian")
    ap.add_argument("--copy-probe", action="store_true",
                    help="first copy 256 MiB device-to-device (a known-size kernel for counter scaling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the mapping step is not "
              f"distributed in this build", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2404_06926_amd import gslic

    if args.workload in ("stream", "multi"):
        print(json.dumps(run_serving(args, torch, gslic)), flush=True)
        return
    if args.workload == "schedule":
        print(json.dumps(run_schedule(args, torch, gslic)), flush=True)
        return

    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream(device=dev)
    torch.cuda.set_stream(stream)
    if args.copy_probe:
        src = torch.ones(64 << 20, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.workload != "headline":
        res = bench_step(torch, gslic, args, dev, args.workload, args.steps, args.warmup,
                         with_plain=args.workload == "batch8")
        print(json.dumps(res), flush=True)
        return

    result = bench_step(torch, gslic, args, dev, "headline", args.steps, args.warmup, with_cpu=True)
    if not args.no_extras:
        # The rest of the metric (the keyframe latency) and the context numbers, each a short
        # leg of its own: the headline map at SH0, the outdoor single view, the 8-view batch
        # against one view per launch, the street-drive keyframe latency, the achievable HBM
        # bandwidth and the oracle's 10k-Gaussian step on one and on all host threads.
        log("headline workload at SH0")
        a0 = argparse.Namespace(**vars(args))
        a0.sh = 0
        h0 = bench_step(torch, gslic, a0, dev, "headline", args.extra_steps, args.warmup)
        result["headline_sh0"] = {"workload": h0["config"]["workload"], "iters_per_s": h0["value"],
                                  "ms_per_step": h0["ms_per_step"], "steps": h0["steps"],
                                  "stages_ms": h0["stages_ms"]}
        log("outdoor workload")
        od = bench_step(torch, gslic, args, dev, "outdoor", args.extra_steps, args.warmup)
        result["outdoor_single_view"] = {"workload": od["config"]["workload"], "iters_per_s": od["value"],
                                         "ms_per_step": od["ms_per_step"], "steps": od["steps"],
                                         "roofline": od["roofline"], "stages_ms": od["stages_ms"],
                                         "counts": {k: od["counts"][k] for k in ("instances", "pairs")}}
        log("batch8 workload")
        b8 = bench_step(torch, gslic, args, dev, "batch8", args.extra_steps, args.warmup, with_plain=True)
        result["batched_over_plain"] = b8["batched_over_plain"]
        result["batch8"] = {"workload": b8["config"]["workload"], "batched_ms_per_step": b8["ms_per_step"],
                            "plain_ms_per_step": b8["plain_ms_per_step"],
                            "plain_ms_per_step_by_split": b8["plain_ms_per_step_by_split"], "steps": b8["steps"],
                            "batched_iters_per_s": b8["value"], "stages_ms": b8["stages_ms"]}
        log("street-drive latency")
        sargs = argparse.Namespace(**vars(args))
        sargs.workload, sargs.duration, sargs.sh = "stream", args.stream_seconds, 3
        st = run_serving(sargs, torch, gslic)
        result["keyframe_latency"] = {"p50_ms": st["latency_ms"]["p50"], "p99_ms": st["latency_ms"]["p99"],
                                      "keyframes": st["config"]["keyframes"], "iters_per_s": st["value"],
                                      "arrivals_s": st["config"]["arrivals_s"],
                                      "final_gaussians": st["final_gaussians"],
                                      "workload": st["config"]["workload"]}
        log("copy bandwidth")
        result["copy_GBs"] = measure_copy(torch, dev)
        if not args.no_cpu_baseline:
            log("cpu config 1")
            try:
                result.setdefault("cpu_baseline", {})["config1"] = cpu_config1()
            except Exception as e:
                result.setdefault("cpu_baseline", {})["config1"] = {"error": repr(e)}
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
