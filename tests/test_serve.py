"""Scheduling logic of the served form on the CPU: a simulated device (one
queue of batches at a fixed coefficient rate) and a simulated clock drive
the continuous-batching and plain-batching schedulers."""
import numpy as np
import pytest

from paper_2302_03909_amd.serve import (ContinuousScheduler, Request, StaticBatcher, latency_summary,
                                        run_open_loop)


class SimClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t


class FakeExecutor:
    """A simulated device shared by the batches in flight (processor
    sharing): `rate` coefficients/s in total, split evenly between the
    running batches, plus a fixed launch cost per batch."""

    def __init__(self, clock, rate=1e11, overhead=20e-6, bytes_per_coef=8):
        self.clock, self.rate, self.overhead, self.bpc = clock, rate, overhead, bytes_per_coef
        self.active = []
        self.last = 0.0
        self.max_inflight = 0

    def _update(self):
        now = self.clock()
        dt, k = now - self.last, len(self.active)
        if k and dt > 0:
            for j in self.active:
                j["rem"] -= dt * self.rate / k
        self.last = now

    def prepare(self, r):
        if r.wavelet == "bogus":
            raise ValueError("unsupported wavelet")
        return r.coefficients * self.bpc + 4 * r.n

    def launch(self, batch, slot):
        self._update()
        job = {"rem": self.overhead * self.rate + sum(r.coefficients for r in batch)}
        self.active.append(job)
        self.max_inflight = max(self.max_inflight, len(self.active))
        return job

    def done(self, h):
        self._update()
        if h in self.active and h["rem"] <= 0.5:
            self.active.remove(h)
        return h not in self.active

    def finish(self, r, h):
        pass

    def next_event(self):
        self._update()
        if not self.active:
            return None
        return self.clock() + max(0.0, min(j["rem"] for j in self.active)) * len(self.active) / self.rate


def stream(count, rate_hz, seed=0, lo=10, hi=16, s_lo=16, s_hi=64):
    rng = np.random.default_rng(seed)
    t, out = 0.0, []
    for i in range(count):
        t += rng.exponential(1.0 / rate_hz)
        n = int(2 ** rng.uniform(lo, hi))
        s = int(rng.integers(s_lo, s_hi + 1))
        out.append(Request(i, n, "zero", "morlet", 6.0, np.linspace(2, 50, s), arrival=t))
    return out


def drive(sched, ex, clock, reqs):
    def advance(nxt):
        cands = [x for x in (nxt, ex.next_event()) if x is not None]
        clock.t = max(clock.t, min(cands)) if cands else clock.t + 1e-6
    return run_open_loop(sched, reqs, clock=clock, advance=advance)


def test_continuous_respects_budget_and_completes_all():
    clock = SimClock()
    ex = FakeExecutor(clock)
    reqs = stream(300, 2000.0, seed=1)
    budget = 64 << 20
    sched = ContinuousScheduler(ex, budget_bytes=budget, streams=4, max_batch=32, clock=clock)
    done = drive(sched, ex, clock, reqs)
    assert len(done) == 300 and all(r.error is None for r in done)
    assert sched.peak_used <= budget
    assert max(sched.batches) <= 32
    assert ex.max_inflight <= 4
    assert sched.used == 0 and sched.idle


def test_admission_in_arrival_order():
    clock = SimClock()
    ex = FakeExecutor(clock, rate=2e10)
    reqs = stream(200, 5000.0, seed=2)
    sched = ContinuousScheduler(ex, budget_bytes=64 << 20, streams=2, clock=clock)
    done = drive(sched, ex, clock, reqs)
    assert all(r.error is None for r in done)
    adm = [r.admitted for r in sorted(done, key=lambda r: r.arrival)]
    assert all(a <= b for a, b in zip(adm, adm[1:]))
    assert all(r.done >= r.launched >= r.admitted >= r.arrival for r in done)


def test_oversized_and_unsupported_requests_are_rejected():
    clock = SimClock()
    ex = FakeExecutor(clock)
    reqs = stream(20, 1000.0, seed=3)
    reqs.append(Request(100, 1 << 20, "zero", "morlet", 6.0, np.linspace(2, 50, 64), arrival=0.001))
    reqs.append(Request(101, 1000, "zero", "bogus", None, np.linspace(2, 50, 4), arrival=0.002))
    sched = ContinuousScheduler(ex, budget_bytes=48 << 20, streams=2, clock=clock)
    done = drive(sched, ex, clock, reqs)
    bad = {r.rid: r.error for r in done if r.error is not None}
    assert set(bad) == {100, 101}
    assert "exceeds the budget" in bad[100] and "unsupported" in bad[101]
    assert len(done) == 22


def test_static_batcher_bounds_and_order():
    clock = SimClock()
    ex = FakeExecutor(clock)
    reqs = stream(150, 3000.0, seed=4)
    sched = StaticBatcher(ex, max_batch=16, window=1e-3, clock=clock)
    done = drive(sched, ex, clock, reqs)
    assert len(done) == 150 and max(sched.batches) <= 16
    assert ex.max_inflight == 1


def test_continuous_has_lower_tail_latency_than_plain_batching():
    # same simulated device, 80 % load: the plain batcher waits for whole
    # batches (or its window); continuous batching launches whatever is
    # admitted as soon as the stream is free
    reqs_a = stream(600, 1.0, seed=5)
    mean_coef = np.mean([r.coefficients for r in reqs_a])
    rate_hz = 0.8 * 1e11 / mean_coef
    res = {}
    for name in ("continuous", "static"):
        clock = SimClock()
        ex = FakeExecutor(clock)
        reqs = stream(600, rate_hz, seed=5)
        sched = (ContinuousScheduler(ex, budget_bytes=1 << 30, streams=1, clock=clock) if name == "continuous"
                 else StaticBatcher(ex, max_batch=32, window=2e-3, clock=clock))
        res[name] = latency_summary(drive(sched, ex, clock, reqs), skip=60)
    assert res["continuous"]["p99_ms"] < res["static"]["p99_ms"]
    assert res["continuous"]["p50_ms"] < res["static"]["p50_ms"]


def test_invalid_scheduler_parameters():
    with pytest.raises(ValueError):
        ContinuousScheduler(FakeExecutor(SimClock()), budget_bytes=0)


class SlowPlanExecutor(FakeExecutor):
    """Planning takes real (wall-clock) time, as building device tables does."""

    def prepare(self, r):
        import time
        time.sleep(0.0005)
        return super().prepare(r)


@pytest.mark.parametrize("kind", ["continuous", "static"])
def test_pooled_planning_keeps_order_and_completes(kind):
    # plans built on two background threads: every request completes, bad
    # ones are rejected, admission stays in arrival order, plan_ms recorded
    clock = SimClock()
    ex = SlowPlanExecutor(clock)
    reqs = stream(120, 3000.0, seed=6)
    reqs.append(Request(500, 1000, "zero", "bogus", None, np.linspace(2, 50, 4), arrival=0.003))
    sched = (ContinuousScheduler(ex, budget_bytes=64 << 20, streams=2, clock=clock, planners=2) if kind == "continuous"
             else StaticBatcher(ex, max_batch=16, window=1e-3, clock=clock, planners=2))
    done = drive(sched, ex, clock, reqs)
    sched.close()
    assert len(done) == 121
    assert {r.rid for r in done if r.error is not None} == {500}
    ok = sorted((r for r in done if r.error is None), key=lambda r: r.arrival)
    adm = [r.admitted for r in ok]
    assert all(a <= b for a, b in zip(adm, adm[1:]))
    assert all(r.plan_ms is not None and r.plan_ms >= 0.4 for r in ok)
    assert "plan_ms_p50" in latency_summary(done)
