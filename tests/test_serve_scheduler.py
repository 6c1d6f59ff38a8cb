"""Serving scheduler logic on the CPU with a clock-driven fake device: admission by HBM
budget, one job in flight per session, slot limit, release of finished sessions,
latency accounting. No GPU."""
import numpy as np
import pytest

from paper_2404_06926_amd import serve


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        self.t += 1e-4          # every scheduler look advances time by 0.1 ms
        return self.t


def _jobs(arrivals):
    return [serve.Job(arrival=a, cam=None, image=None) for a in arrivals]


def test_single_session_latency_is_queueing_plus_service():
    clock = FakeClock()
    be = serve.FakeBackend(cost_s=lambda j: 0.010)
    sch = serve.Scheduler(be, budget_bytes=100, slots=4, poll_s=0)
    jobs = _jobs([0.0, 0.001, 0.002])          # arrive faster than they are served
    sch.add(serve.SessionSpec(sid=0, jobs=jobs, est_bytes=10))
    res = sch.run(clock=clock)
    lat = [j.latency for j in jobs]
    # one job in flight per session: they run back to back, 10 ms each
    assert lat[0] == pytest.approx(0.010, abs=1e-3)
    assert lat[1] == pytest.approx(0.020 - 0.001, abs=1e-3)
    assert lat[2] == pytest.approx(0.030 - 0.002, abs=1e-3)
    assert res["jobs"] == 3 and be.closed == [0]


def test_concurrent_sessions_share_the_device_and_slots_cap_concurrency():
    clock = FakeClock()
    be = serve.FakeBackend(cost_s=lambda j: 0.010)
    sch = serve.Scheduler(be, budget_bytes=1000, slots=2, poll_s=0)
    for sid in range(3):
        sch.add(serve.SessionSpec(sid=sid, jobs=_jobs([0.0]), est_bytes=10))
    sch.run(clock=clock)
    lat = sorted(j.latency for s in sch.sessions for j in s.spec.jobs)
    # two in flight share the device (both finish at 20 ms), the third runs alone after
    assert lat[0] == pytest.approx(0.020, abs=1e-3) and lat[1] == pytest.approx(0.020, abs=1e-3)
    assert lat[2] == pytest.approx(0.030, abs=1e-3)
    dispatches = [e for e in sch.log if e[0] == "dispatch"]
    assert len(dispatches) == 3


def test_admission_waits_for_budget_and_releases_memory():
    clock = FakeClock()
    be = serve.FakeBackend(cost_s=lambda j: 0.005)
    sch = serve.Scheduler(be, budget_bytes=100, slots=8, poll_s=0)
    sch.add(serve.SessionSpec(sid=0, jobs=_jobs([0.0, 0.001]), est_bytes=70))
    sch.add(serve.SessionSpec(sid=1, jobs=_jobs([0.0005]), est_bytes=60))   # does not fit beside 0
    res = sch.run(clock=clock)
    ev = [(e[0], e[1]) for e in sch.log if e[0] in ("admit", "release")]
    assert ev.index(("release", 0)) < ev.index(("admit", 1))
    assert res["peak_resident_bytes"] <= 100
    assert res["sessions"][1]["admission_wait_s"] >= 0.009
    with pytest.raises(ValueError):
        sch.add(serve.SessionSpec(sid=2, jobs=_jobs([0.0]), est_bytes=1000))


def test_jobs_of_one_session_keep_arrival_order():
    clock = FakeClock()
    be = serve.FakeBackend(cost_s=lambda j: 0.002)
    sch = serve.Scheduler(be, budget_bytes=1000, slots=3, poll_s=0)
    rng = np.random.default_rng(0)
    for sid in range(4):
        arr = serve.poisson_arrivals(rng, 200.0, 0.05)
        sch.add(serve.SessionSpec(sid=sid, jobs=_jobs(arr), est_bytes=10))
    res = sch.run(clock=clock)
    for s in sch.sessions:
        d = [j.dispatched for j in s.spec.jobs]
        assert d == sorted(d)
        assert all(j.latency > 0 for j in s.spec.jobs)
        assert all(j.dispatched >= j.arrival for j in s.spec.jobs)
    assert res["p99_ms"] >= res["p50_ms"] > 0


def test_estimate_grows_with_map_and_window():
    a = serve.estimate_bytes(100_000, 3, 8, 1280, 720)
    assert serve.estimate_bytes(200_000, 3, 8, 1280, 720) > a
    assert serve.estimate_bytes(100_000, 3, 4, 1280, 720) < a


def test_reservation_covers_the_estimate_while_a_map_is_small():
    # Session 0's map starts at 30% of its estimate and grows with every job. Its
    # reservation stays at the estimate, so session 1 (which fits beside the map's current
    # size but not beside its estimate) waits until session 0 is released, and the bytes
    # the sessions actually hold never exceed the budget.
    clock = FakeClock()
    be = serve.GrowingFakeBackend(cost_s=lambda j: 0.004, start=0.3, step=0.25)
    sch = serve.Scheduler(be, budget_bytes=100, slots=8, poll_s=0)
    sch.add(serve.SessionSpec(sid=0, jobs=_jobs([0.0, 0.001, 0.002, 0.003]), est_bytes=70))
    sch.add(serve.SessionSpec(sid=1, jobs=_jobs([0.0005, 0.001]), est_bytes=60))
    res = sch.run(clock=clock)
    ev = [(e[0], e[1]) for e in sch.log if e[0] in ("admit", "release")]
    assert ev.index(("release", 0)) < ev.index(("admit", 1))
    assert res["peak_resident_bytes"] == 70          # session 0 at full size, alone
    assert res["peak_resident_bytes"] <= 100


def test_growth_past_the_estimate_raises_the_reservation():
    # A map that outgrows its estimate (to 1.5x) reserves what it holds: a session that
    # fits beside the estimate but not beside the grown map is held back until release.
    clock = FakeClock()
    be = serve.GrowingFakeBackend(cost_s=lambda j: 0.004, start=1.0, step=0.25, grow_to=1.5)
    sch = serve.Scheduler(be, budget_bytes=100, slots=8, poll_s=0)
    sch.add(serve.SessionSpec(sid=0, jobs=_jobs([0.0, 0.001, 0.002, 0.02]), est_bytes=40))
    sch.add(serve.SessionSpec(sid=1, jobs=_jobs([0.015]), est_bytes=50))
    res = sch.run(clock=clock)
    ev = [(e[0], e[1]) for e in sch.log if e[0] in ("admit", "release")]
    assert ev.index(("release", 0)) < ev.index(("admit", 1))
    # session 0 peaks at 60 B; session 1 alone grows from 50 to 62 B after its job
    assert res["peak_resident_bytes"] == 62
