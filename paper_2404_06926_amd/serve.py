"""Serving loop: keyframe jobs of many map sessions on one GPU.

A session owns one Gaussian map. Its keyframes arrive over time; each keyframe is one
job (gs_submit_keyframe: append Gaussians from the keyframe's points as in Sec. III-C.1,
keep the keyframe in the session's window, run `iters` optimisation steps over the
window). The scheduler:

* admits sessions in order of their first arrival while the HBM they reserve fits the
  budget, and releases a session's memory when its last job has completed. A session
  reserves the larger of its estimate (sized for its final map and full window) and what
  its map reports holding, so a map that has not grown yet lends no headroom to others;
* gives every admitted session its own stream, keeps at most one job of a session in
  flight (a map is used by one stream at a time) and at most `slots` jobs in flight
  overall, so jobs of different sessions overlap on the device as they arrive and as
  slots free up (continuous batching);
* measures each job's latency as completion minus arrival (the upload of the keyframe's
  image and points happens inside it).

The backend interface (create / submit / poll / close) lets the same scheduler run against
a fake clock-driven backend on the CPU (tests of admission, ordering and accounting) and
against the HIP library on the GPU.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field
from typing import Any, Dict, List, Optional

import numpy as np


@dataclass
class Job:
    """One keyframe of a session."""
    arrival: float                 # seconds after the start of the run
    cam: Any                       # camera with R, t, fx, fy, cx, cy, width, height
    image: Any                     # target image (3, H, W), host memory
    xyz: Optional[Any] = None      # new points (n, 3), host memory
    rgb: Optional[Any] = None      # their colours (n, 3)
    # filled by the scheduler
    dispatched: float = -1.0
    latency: float = -1.0


@dataclass
class SessionSpec:
    sid: int
    jobs: List[Job]
    est_bytes: int                 # HBM the session will hold (used for admission)
    init: Any = None               # backend-specific initial state (e.g. parameter rows)
    sh_degree: int = 3


@dataclass
class _Session:
    spec: SessionSpec
    next_job: int = 0              # first job not yet dispatched
    in_flight: Optional[Any] = None
    handle: Any = None
    admitted_at: float = -1.0
    resident: int = 0              # bytes the backend reports the session holds
    done_jobs: int = 0

    @property
    def reserved(self) -> int:
        return max(self.spec.est_bytes, self.resident)


class FakeBackend:
    """CPU stand-in: a job takes `cost(job)` seconds of a single shared device, jobs of
    concurrent sessions share it equally (processor sharing)."""

    def __init__(self, cost_s=lambda job: 0.01):
        self.cost = cost_s
        self.active: Dict[int, List[float]] = {}   # token -> [remaining work, completion time]
        self.last = None
        self.next_token = 0
        self.created = []
        self.closed = []

    def _advance(self, now):
        if self.last is None:
            self.last = now
        dt = now - self.last
        self.last = now
        live = [t for t, v in self.active.items() if v[1] < 0]
        while dt > 1e-12 and live:
            share = dt / len(live)
            first = min(self.active[t][0] for t in live)
            step = min(share, first)
            for t in live:
                self.active[t][0] -= step
            dt -= step * len(live)
            for t in live:
                if self.active[t][0] <= 1e-12:
                    self.active[t][1] = now - dt
            live = [t for t in live if self.active[t][1] < 0]

    def create(self, spec):
        self.created.append(spec.sid)
        return spec.sid, spec.est_bytes

    def submit(self, handle, job, now):
        self._advance(now)
        tok = self.next_token
        self.next_token += 1
        self.active[tok] = [self.cost(job), -1.0]
        return tok

    def poll(self, token, now):
        self._advance(now)
        t = self.active[token][1]
        return None if t < 0 else t

    def resident(self, handle):
        return None

    def close(self, handle):
        self.closed.append(handle)


class GrowingFakeBackend(FakeBackend):
    """FakeBackend whose sessions report resident bytes that grow with every finished
    job: `start` of the estimate at creation, up to `grow_to` times the estimate."""

    def __init__(self, cost_s=lambda job: 0.01, start=0.3, step=0.25, grow_to=1.0):
        super().__init__(cost_s)
        self.start, self.step, self.grow_to = start, step, grow_to
        self.state = {}                            # handle -> [estimate, jobs done]
        self.owner = {}                            # token -> handle

    def create(self, spec):
        self.created.append(spec.sid)
        self.state[spec.sid] = [spec.est_bytes, 0]
        return spec.sid, int(self.start * spec.est_bytes)

    def submit(self, handle, job, now):
        tok = super().submit(handle, job, now)
        self.owner[tok] = handle
        return tok

    def poll(self, token, now):
        t = super().poll(token, now)
        if t is not None and token in self.owner:
            self.state[self.owner.pop(token)][1] += 1
        return t

    def resident(self, handle):
        est, done = self.state[handle]
        return int(min(self.grow_to, self.start + self.step * done) * est)


class GpuBackend:
    """Sessions on the HIP library: one GaussianMap, one stream and one host worker thread
    per session. A job's library calls run on the session's worker (the library releases
    the GIL and a host wait inside one session's job, such as the instance-count read of a
    render, does not hold up the other sessions); its latency is measured with events on
    the session's stream."""

    def __init__(self, device="cuda", iters=10, window=8, lam=0.2, o_init=0.1, deterministic=False,
                 keep_final=False, threaded=True, capacity=None):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.iters, self.window, self.lam, self.o_init = iters, window, lam, o_init
        self.deterministic = deterministic
        self.keep_final = keep_final
        self.threaded = threaded
        self.capacity = capacity   # initial row capacity of every map (None: the initial rows)
        self.final = {}            # sid -> parameter planes at release (when keep_final)

    def create(self, spec):
        from concurrent.futures import ThreadPoolExecutor
        from . import gslic
        torch = self.torch
        stream = torch.cuda.Stream(device=self.device)
        with torch.cuda.device(self.device), torch.cuda.stream(stream):
            init = spec.init
            n0 = 0 if init is None else init.shape[0]
            m = gslic.GaussianMap(sh_degree=spec.sh_degree, capacity=max(1024, n0, self.capacity or 0),
                                  device=self.device)
            m.set_deterministic(self.deterministic)
            if n0:
                m.add_gaussians(torch.as_tensor(np.ascontiguousarray(init)).to(self.device))
        ex = ThreadPoolExecutor(max_workers=1) if self.threaded else None
        return dict(map=m, stream=stream, keep=None, sid=spec.sid, ex=ex), spec.est_bytes

    def _run(self, h, job, start, done):
        torch = self.torch
        with torch.cuda.device(self.device), torch.cuda.stream(h["stream"]):
            start.record()
            img = torch.as_tensor(job.image).to(self.device, non_blocking=True)
            xyz = rgb = None
            if job.xyz is not None and len(job.xyz):
                xyz = torch.as_tensor(job.xyz).to(self.device, non_blocking=True)
                rgb = torch.as_tensor(job.rgb).to(self.device, non_blocking=True)
            h["map"].submit_keyframe(job.cam, img, xyz, rgb, iters=self.iters, window=self.window,
                                     lam=self.lam, o_init=self.o_init)
            done.record()
            h["keep"] = (img, xyz, rgb)

    def submit(self, h, job, now):
        torch = self.torch
        start = torch.cuda.Event(enable_timing=True)
        done = torch.cuda.Event(enable_timing=True)
        tok = dict(start=start, done=done, t_submit=now, fut=None)
        if h["ex"] is not None:
            tok["fut"] = h["ex"].submit(self._run, h, job, start, done)
        else:
            self._run(h, job, start, done)
        return tok

    def poll(self, tok, now):
        f = tok["fut"]
        if f is not None:
            if not f.done():
                return None
            f.result()   # raises what the job raised
        if not tok["done"].query():
            return None
        return tok["t_submit"] + tok["start"].elapsed_time(tok["done"]) * 1e-3

    def resident(self, h):
        return h["map"].info()[2]

    def close(self, h):
        if h["ex"] is not None:
            h["ex"].shutdown(wait=True)
        h["stream"].synchronize()
        if self.keep_final:
            self.final[h["sid"]] = h["map"].params().clone()
        h["map"].close()


class Scheduler:
    def __init__(self, backend, budget_bytes: int, slots: int = 4, poll_s: float = 5e-5):
        self.backend = backend
        self.budget = budget_bytes
        self.slots = slots
        self.poll_s = poll_s
        self.sessions: List[_Session] = []
        self.log: List[tuple] = []

    def add(self, spec: SessionSpec):
        if spec.est_bytes > self.budget:
            raise ValueError(f"session {spec.sid} needs {spec.est_bytes} B, more than the budget")
        self.sessions.append(_Session(spec))

    def run(self, clock=None, max_wall_s: float = 600.0) -> Dict[str, Any]:
        clock = clock or time.perf_counter
        t0 = clock()
        order = sorted(self.sessions, key=lambda s: s.spec.jobs[0].arrival if s.spec.jobs else 0.0)
        waiting = list(order)          # not yet admitted, first-arrival order
        admitted: List[_Session] = []
        reserved_total = 0             # sum of max(estimate, resident) of admitted sessions
        resident_total = 0             # sum of what admitted sessions report holding
        in_flight = 0
        finished = 0
        total = len(order)
        peak_resident = 0
        admission_wait = {}
        while finished < total:
            now = clock() - t0
            if now > max_wall_s:
                raise TimeoutError("serving run exceeded its wall-clock limit")
            progressed = False
            # reap completed jobs
            for s in admitted:
                if s.in_flight is None:
                    continue
                job, tok = s.in_flight
                t_done = self.backend.poll(tok, now)
                if t_done is None:
                    continue
                job.latency = t_done - job.arrival
                s.in_flight = None
                s.done_jobs += 1
                in_flight -= 1
                progressed = True
                r = self.backend.resident(s.handle)
                if r is not None:
                    reserved_total -= s.reserved
                    resident_total += r - s.resident
                    s.resident = r
                    reserved_total += s.reserved
                    peak_resident = max(peak_resident, resident_total)
                self.log.append(("done", s.spec.sid, now, job.latency))
            # release sessions whose jobs are all done
            for s in list(admitted):
                if s.in_flight is None and s.done_jobs == len(s.spec.jobs):
                    self.backend.close(s.handle)
                    reserved_total -= s.reserved
                    resident_total -= s.resident
                    admitted.remove(s)
                    finished += 1
                    progressed = True
                    self.log.append(("release", s.spec.sid, now))
            # admit in first-arrival order while the budget allows
            while waiting and reserved_total + waiting[0].spec.est_bytes <= self.budget:
                s = waiting.pop(0)
                first = s.spec.jobs[0].arrival if s.spec.jobs else 0.0
                if first > now:
                    waiting.insert(0, s)
                    break
                s.handle, s.resident = self.backend.create(s.spec)
                reserved_total += s.reserved
                resident_total += s.resident
                peak_resident = max(peak_resident, resident_total)
                s.admitted_at = now
                admission_wait[s.spec.sid] = now - first
                admitted.append(s)
                progressed = True
                self.log.append(("admit", s.spec.sid, now))
                if not s.spec.jobs:
                    self.backend.close(s.handle)
                    reserved_total -= s.reserved
                    resident_total -= s.resident
                    admitted.remove(s)
                    finished += 1
            # dispatch: oldest arrived job among idle admitted sessions, while slots are free
            while in_flight < self.slots:
                cand = [s for s in admitted if s.in_flight is None and s.next_job < len(s.spec.jobs)
                        and s.spec.jobs[s.next_job].arrival <= now]
                if not cand:
                    break
                s = min(cand, key=lambda x: x.spec.jobs[x.next_job].arrival)
                job = s.spec.jobs[s.next_job]
                s.next_job += 1
                job.dispatched = now
                s.in_flight = (job, self.backend.submit(s.handle, job, now))
                in_flight += 1
                progressed = True
                self.log.append(("dispatch", s.spec.sid, now))
            if not progressed:
                time.sleep(self.poll_s)
        wall = clock() - t0
        per = {}
        all_lat = []
        for s in order:
            lat = np.array([j.latency for j in s.spec.jobs])
            all_lat.extend(lat.tolist())
            per[s.spec.sid] = dict(jobs=len(lat), p50_ms=float(np.percentile(lat, 50) * 1e3) if len(lat) else None,
                                   p99_ms=float(np.percentile(lat, 99) * 1e3) if len(lat) else None,
                                   admission_wait_s=admission_wait.get(s.spec.sid))
        all_lat = np.array(all_lat)
        return dict(wall_s=wall, sessions=per, jobs=int(all_lat.size),
                    p50_ms=float(np.percentile(all_lat, 50) * 1e3) if all_lat.size else None,
                    p99_ms=float(np.percentile(all_lat, 99) * 1e3) if all_lat.size else None,
                    peak_resident_bytes=int(peak_resident))


def estimate_bytes(n_final: int, sh_degree: int, window: int, width: int, height: int) -> int:
    """HBM a session holds: parameters, gradients and Adam moments (16 F bytes per
    Gaussian), per (view, Gaussian) records of a batch (2 x 64 B + 28 B), instances
    (~8 per visible pair, 20 B each), keyframe buffers (8 floats per pixel) and loss
    scratch."""
    F = 11 + 3 * (sh_degree + 1) ** 2
    P = width * height
    return int(16 * F * n_final * 1.25 + window * n_final * (156 + 160) + window * P * 40 + P * 40)


def poisson_arrivals(rng: np.random.Generator, rate_hz: float, duration_s: float, start: float = 0.0):
    t, out = start, []
    while True:
        t += rng.exponential(1.0 / rate_hz)
        if t >= start + duration_s:
            return out
        out.append(t)
