"""Mapping-iteration throughput on one MI355X.

One step = one optimisation iteration of the Gaussian map on one keyframe: project, bin,
sort, blend (with exposure), L1 + D-SSIM loss, backward, sparse Adam (Gaussians and the
keyframe's exposure). Workload: 1M Gaussians volume-uniform at 2-20 m in the frustum of a
1280x720 pinhole camera (f = 1000), SH degree 3, target = render of the same map with
means jittered by N(0, 5 cm). Inputs are synthetic and resident in HBM before timing.

Prints one JSON line. `--gpus N` with N > 1 exits: this build runs on one GPU.
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
# FLOPs per (pixel, list entry) pair, counted from the blend arithmetic
FWD_FLOPS_PER_PAIR = 22
BWD_FLOPS_PER_PAIR = 56


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def build_workload(n, deg, W, H, seed=2024):
    from paper_2404_06926_amd import scenes
    cam = scenes.pinhole(W, H, 1000.0 * W / 1280.0)
    params = scenes.frustum_gaussians(n, deg, cam, seed=seed)
    target_params = scenes.jitter_means(params, 0.05, seed)
    return cam, params, target_params


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
    return dict(value=1.0 / dt, unit="iters/s", cores=threads, kind="oracle",
                sample=f"one full step of the same workload (FP64 oracle, {dt:.1f} s; target render "
                       f"{t_target:.1f} s not counted)")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=1_000_000)
    ap.add_argument("--sh", type=int, default=3)
    ap.add_argument("--width", type=int, default=1280)
    ap.add_argument("--height", type=int, default=720)
    ap.add_argument("--lam", type=float, default=0.2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-stage-timing", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the mapping step is not "
              f"distributed in this build", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2404_06926_amd import gslic

    dev = torch.device("cuda:0")
    log(f"building workload: n={args.n} sh={args.sh} {args.width}x{args.height}")
    cam, params, target_params = build_workload(args.n, args.sh, args.width, args.height)
    H, W = args.height, args.width

    # target image from the jittered map (outside the timed region)
    tmap = gslic.GaussianMap(sh_degree=args.sh, capacity=args.n)
    tmap.add_gaussians(torch.from_numpy(target_params).to(dev))
    target = tmap.render([cam])[0].rgb.clone()
    tmap.close()
    del tmap

    m = gslic.GaussianMap(sh_degree=args.sh, capacity=args.n)
    m.add_gaussians(torch.from_numpy(params).to(dev))
    expo = gslic.identity_exposure_state(dev)
    frame = gslic.Frame(torch.empty(3, H, W, device=dev), torch.empty(H, W, device=dev),
                        torch.empty(H, W, dtype=torch.int32, device=dev))
    loss_buf = torch.empty(1, device=dev)
    grad_buf = torch.empty(3, H, W, device=dev)

    def step():
        m.render([cam], [expo], frames=[frame])
        m.loss(frame.rgb, target, args.lam, loss_out=loss_buf, grad_out=grad_buf)
        m.render_backward([grad_buf], [expo[12:24]])
        m.adam_step([expo])

    # first step plans the instance buffers; then no host wait inside the step
    step()
    torch.cuda.synchronize()
    n_inst0 = m.debug_last_render()["n_inst"]
    m.set_instance_policy(False, int(n_inst0 * 1.5) + 65536)
    log(f"instances {n_inst0}; warmup {args.warmup}")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    if m.check_overflow():
        raise RuntimeError("instance buffer overflow during warmup")
    m.set_stage_timing(not args.no_stage_timing)
    m.stage_times()  # reset

    log(f"timing {args.steps} steps")
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record()
    for _ in range(args.steps):
        step()
    stop.record()
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop) / args.steps
    stages = m.stage_times()
    if m.check_overflow():
        raise RuntimeError("instance buffer overflow during the timed steps")
    m.set_stage_timing(False)

    # work counts of the last step (outside the timed region)
    dbg = m.debug_last_render()
    n_inst = dbg["n_inst"]
    counts = dbg["counts"][0]
    n_vis = int((counts > 0).sum().item())
    pairs = int(frame.n_contrib.to(torch.int64).sum().item())
    F = 11 + 3 * (args.sh + 1) ** 2
    T_total = dbg["n_tiles"]
    P = W * H
    sort_passes = (32 + max(1, int(np.ceil(np.log2(T_total)))) + 7) // 8

    per = {k: (v[0] / max(v[1], 1)) for k, v in stages.items()}
    # algorithmic work per launch of each stage (bytes or FLOPs), see the design doc
    work = {
        "project": ("hbm", 4.0 * 14 * args.n + 4.0 * (F - 14) * n_vis + 64.0 * n_vis + 4.0 * args.n),
        "scan": ("hbm", 8.0 * args.n),
        "duplicate": ("hbm", 40.0 * n_vis + 12.0 * n_inst),
        "sort": ("hbm", sort_passes * 32.0 * n_inst),
        "ranges": ("hbm", 8.0 * n_inst + 8.0 * T_total),
        "blend": ("alu", FWD_FLOPS_PER_PAIR * float(pairs)),
        "loss": ("hbm", 24.0 * P + 36.0 * P + 60.0 * P + 12.0 * P),
        "blend_backward": ("alu", BWD_FLOPS_PER_PAIR * float(pairs)),
        "project_backward": ("hbm", 4.0 * F * n_vis * 2 + 64.0 * n_vis * 2 + 4.0 * args.n),
        "adam": ("hbm", 32.0 * F * n_vis),
    }
    dom = max(per, key=lambda k: per[k]) if not args.no_stage_timing else "blend_backward"
    bound, amount = work[dom]
    dur_s = per[dom] * 1e-3 if per[dom] > 0 else float("nan")
    if bound == "hbm":
        achieved, peak, unit = amount / dur_s / 1e9, HBM_PEAK_GBS, "GB/s"
    else:
        achieved, peak, unit = amount / dur_s / 1e12, FP32_PEAK_TFLOPS, "TFLOP/s"
    roof = dict(bound=bound, kernel=dom, achieved=achieved, peak=peak, unit=unit, frac=achieved / peak,
                traffic=None, avg_launch_ms=per[dom])

    result = {
        "metric": METRIC,
        "value": 1000.0 / ms,
        "unit": "iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{args.n} Gaussians, SH{args.sh}, one {W}x{H} view (f={1000.0 * W / 1280:.0f}), "
                               f"loss 0.8 L1 + 0.2 D-SSIM, sparse Adam", "n_gaussians": args.n,
                   "sh_degree": args.sh, "width": W, "height": H, "views_per_step": 1},
        "roofline": roof,
        "stages_ms": {k: round(v, 4) for k, v in per.items()},
        "counts": {"visible": n_vis, "instances": n_inst, "pairs": pairs, "tiles": T_total},
    }
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        try:
            result["cpu_baseline"] = cpu_baseline(params, target_params, args.sh, cam, args.lam)
        except Exception as e:  # report, never fail the GPU result
            result["cpu_baseline"] = {"error": repr(e)}
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
