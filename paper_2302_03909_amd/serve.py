"""Served form of the transform: requests of arbitrary length, scales,
wavelet and boundary arrive over time and are answered from one GPU.

Two schedulers share one executor interface:

* ``ContinuousScheduler`` -- continuous batching.  Requests are admitted in
  arrival order while the device-memory footprint of everything admitted
  (signal, output, workspace and plan tables, ``cwt_footprint_bytes``) stays
  within a budget.  Whenever one of K streams is free, every admitted request
  not yet running is launched on it as one ``cwt_exec_batch``; batches on the
  other streams keep running meanwhile, so new work is appended while
  earlier work is in flight.  A request whose footprint alone exceeds the
  budget is rejected.
* ``StaticBatcher`` -- the plain batched form: collect up to ``max_batch``
  requests or until ``window`` seconds passed since the oldest, run them as
  one batch, wait for it, release, repeat.

Planning (building a request's plan: validation, segment framing, device
tables, on the host and the calling thread's plan stream) happens either
inline in ``poll`` (``planners=0``) or on a pool of ``planners`` host
threads started at ``submit``, so that the polling loop only admits,
launches and collects; a request is admitted once its plan is ready (the
head of the queue waits for its own).  Each request records ``plan_ms``.

``GpuExecutor`` runs batches with the library; tests drive the schedulers
with a simulated executor and clock.  Every result is bit-identical to the
same request transformed alone (``cwt_exec_batch`` guarantees it).

``run_open_loop`` replays a request stream against a scheduler and returns
the completed requests; ``latency_summary`` gives p50/p99 of arrival to
device completion.
"""
from __future__ import annotations

import collections
import concurrent.futures
import dataclasses
import threading
import time
from typing import Any, Callable, Optional

import numpy as np


@dataclasses.dataclass
class Request:
    """One transform request.  ``signal`` is whatever the executor consumes
    (a device tensor for ``GpuExecutor``)."""
    rid: int
    n: int
    boundary: str
    wavelet: str
    param: Optional[float]
    scales: np.ndarray
    precision: str = "fp32"
    signal: Any = None
    arrival: float = 0.0
    # filled in by the scheduler / executor
    footprint: int = 0
    admitted: Optional[float] = None
    launched: Optional[float] = None
    done: Optional[float] = None
    output: Any = None
    error: Optional[str] = None
    plan: Any = None
    plan_ms: Optional[float] = None
    planned: Any = None  # future of a background planning job

    @property
    def coefficients(self) -> int:
        return int(self.n) * int(np.asarray(self.scales).size)


def _plan(ex, r: Request) -> None:
    """Builds the request's plan (sets footprint or error, and plan_ms)."""
    t0 = time.perf_counter()
    try:
        r.footprint = int(ex.prepare(r))
    except Exception as e:  # unsupported request
        r.error = str(e)
    r.plan_ms = (time.perf_counter() - t0) * 1e3


class _Planning:
    """Inline or pooled planning shared by the two schedulers."""

    def __init__(self, executor, planners: int):
        if planners < 0:
            raise ValueError("planners must be >= 0")
        self.ex = executor
        self.pool = concurrent.futures.ThreadPoolExecutor(planners) if planners > 0 else None

    def start(self, r: Request) -> None:
        if self.pool is not None:
            r.planned = self.pool.submit(_plan, self.ex, r)

    def ready(self, r: Request) -> bool:
        """True once the request's plan (or its error) is there; plans it
        inline when there is no pool."""
        if r.planned is not None:
            if not r.planned.done():
                return False
            r.planned.result()
            r.planned = None
            return True
        if r.footprint == 0 and r.error is None:
            _plan(self.ex, r)
        return True

    def close(self) -> None:
        if self.pool is not None:
            self.pool.shutdown(wait=True)


class ContinuousScheduler:
    """Continuous batching over ``streams`` slots within ``budget_bytes``."""

    def __init__(self, executor, budget_bytes: int, streams: int = 2, max_batch: int = 256,
                 clock: Callable[[], float] = time.perf_counter, planners: int = 0):
        if streams < 1 or max_batch < 1 or budget_bytes <= 0:
            raise ValueError("streams, max_batch and budget_bytes must be positive")
        self.planning = _Planning(executor, planners)
        self.ex = executor
        self.budget = int(budget_bytes)
        self.streams = int(streams)
        self.max_batch = int(max_batch)
        self.clock = clock
        self.queue: collections.deque[Request] = collections.deque()
        self.ready: collections.deque[Request] = collections.deque()
        self.inflight: dict[int, tuple[Any, list[Request]]] = {}
        self.used = 0
        self.peak_used = 0
        self.batches: list[int] = []  # sizes of the launched batches

    def submit(self, req: Request) -> None:
        self.planning.start(req)
        self.queue.append(req)

    def close(self) -> None:
        self.planning.close()

    @property
    def idle(self) -> bool:
        return not self.queue and not self.ready and not self.inflight

    def poll(self) -> list[Request]:
        """Advance: collect finished batches, admit, launch.  Returns the
        requests completed (or rejected) by this call."""
        now = self.clock()
        out: list[Request] = []
        for slot in list(self.inflight):
            handle, reqs = self.inflight[slot]
            if self.ex.done(handle):
                for r in reqs:
                    r.done = now
                    self.used -= r.footprint
                    self.ex.finish(r, handle)
                    out.append(r)
                del self.inflight[slot]
        # admission in arrival order (the head waits until it fits)
        while self.queue:
            r = self.queue[0]
            if not self.planning.ready(r):
                break
            if r.error is None and r.footprint > self.budget:
                r.error = f"footprint {r.footprint} bytes exceeds the budget of {self.budget}"
            if r.error is not None:
                self.queue.popleft()
                r.done = now
                out.append(r)
                continue
            if self.used + r.footprint > self.budget:
                break
            self.queue.popleft()
            self.used += r.footprint
            self.peak_used = max(self.peak_used, self.used)
            r.admitted = now
            self.ready.append(r)
        # launch on free streams
        for slot in range(self.streams):
            if not self.ready:
                break
            if slot in self.inflight:
                continue
            batch = [self.ready.popleft() for _ in range(min(self.max_batch, len(self.ready)))]
            for r in batch:
                r.launched = now
            self.inflight[slot] = (self.ex.launch(batch, slot), batch)
            self.batches.append(len(batch))
        return out


class StaticBatcher:
    """Plain batching: up to ``max_batch`` requests, or whatever is pending
    once the oldest has waited ``window`` seconds; one batch at a time, no
    overlap."""

    def __init__(self, executor, max_batch: int = 64, window: float = 2e-3,
                 clock: Callable[[], float] = time.perf_counter, planners: int = 0,
                 budget_bytes: Optional[int] = None):
        self.planning = _Planning(executor, planners)
        self.budget = budget_bytes
        self.ex = executor
        self.max_batch = int(max_batch)
        self.window = float(window)
        self.clock = clock
        self.pending: collections.deque[tuple[float, Request]] = collections.deque()
        self.current: Optional[tuple[Any, list[Request]]] = None
        self.batches: list[int] = []

    def submit(self, req: Request) -> None:
        self.planning.start(req)
        self.pending.append((self.clock(), req))

    def close(self) -> None:
        self.planning.close()

    @property
    def idle(self) -> bool:
        return not self.pending and self.current is None

    def poll(self) -> list[Request]:
        now = self.clock()
        out: list[Request] = []
        if self.current is not None:
            handle, reqs = self.current
            if not self.ex.done(handle):
                return out
            for r in reqs:
                r.done = now
                self.ex.finish(r, handle)
                out.append(r)
            self.current = None
        if self.pending and (len(self.pending) >= self.max_batch or now - self.pending[0][0] >= self.window):
            batch = []
            used = 0
            while self.pending and len(batch) < self.max_batch:
                # the batch takes the planned requests in arrival order,
                # within the footprint budget (if any)
                r = self.pending[0][1]
                if not self.planning.ready(r):
                    break
                if r.error is None and self.budget is not None:
                    if r.footprint > self.budget:
                        r.error = f"footprint {r.footprint} bytes exceeds the budget of {self.budget}"
                    elif used + r.footprint > self.budget:
                        break
                self.pending.popleft()
                if r.error is not None:
                    r.done = now
                    out.append(r)
                    continue
                used += r.footprint
                r.admitted = r.launched = now
                batch.append(r)
            if batch:
                self.current = (self.ex.launch(batch, 0), batch)
                self.batches.append(len(batch))
        return out


class GpuExecutor:
    """Runs batches with ``cwt_exec_batch`` on ``streams`` torch streams
    (default priority).  Plans are cached by request shape (LRU).

    Outputs: with ``keep_outputs`` (the default) each request gets its own
    output tensor, allocated on the launching stream and handed over in
    ``Request.output``.  Otherwise (a consumer that reads each result when
    its batch completes, and benchmarks) every stream owns a device arena of
    ``arena_bytes`` allocated once, and a batch's outputs and workspace are
    carved from its stream's arena: a stream runs one batch at a time, so
    the arena is free again when the next batch is launched on it, and the
    loop allocates no device memory (a batch larger than the arena falls
    back to allocation)."""

    def __init__(self, device="cuda:0", streams: int = 2, plan_cache: int = 256, keep_outputs: bool = True,
                 arena_bytes: int = 0):
        import torch
        import paper_2302_03909_amd as cwt
        self.torch, self.cwt = torch, cwt
        self.device = torch.device(device)
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(streams)]
        self.plans: collections.OrderedDict = collections.OrderedDict()
        self.plan_cache = int(plan_cache)
        self.keep_outputs = keep_outputs
        self._busy_plans: dict[int, int] = collections.Counter()
        self._retired: list = []
        self._lock = threading.Lock()  # plan cache (planning may run on other threads)
        self.launch_s = 0.0  # host time spent in launch()
        self.arena_fallbacks = 0
        self.arenas = ([torch.empty(int(arena_bytes), dtype=torch.uint8, device=self.device) for _ in self.streams]
                       if arena_bytes > 0 and not keep_outputs else None)

    @staticmethod
    def _key(r: Request):
        return (r.n, r.boundary, r.wavelet, r.param, np.asarray(r.scales, dtype=np.float64).tobytes(), r.precision)

    def prepare(self, r: Request) -> int:
        key = self._key(r)
        with self._lock:
            plan = self.plans.get(key)
            if plan is not None:
                self.plans.move_to_end(key)
                self._busy_plans[id(plan)] += 1
        if plan is None:
            built = self.cwt.Plan(r.n, r.boundary, r.wavelet, r.scales, param=r.param, precision=r.precision)
            with self._lock:
                plan = self.plans.get(key)
                if plan is None:
                    plan = built
                    self.plans[key] = plan
                    self._evict()
                else:  # another thread built the same shape meanwhile: keep that one
                    self.plans.move_to_end(key)
                self._busy_plans[id(plan)] += 1
            if plan is not built:
                built.close()
        r.plan = plan
        return plan.footprint_bytes

    def _evict(self):
        # plans still referenced by unfinished requests stay alive
        while len(self.plans) > self.plan_cache:
            key, plan = next(iter(self.plans.items()))
            del self.plans[key]
            if self._busy_plans.get(id(plan), 0) > 0:
                self._retired.append(plan)
            else:
                plan.close()

    def launch(self, batch: list[Request], slot: int):
        t0 = time.perf_counter()
        try:
            return self._launch(batch, slot)
        finally:
            self.launch_s += time.perf_counter() - t0

    def _carve(self, plans, slot):
        """Outputs and workspace of a batch as views of the slot's arena, or
        None when they do not fit."""
        if self.arenas is None:
            return None
        arena = self.arenas[slot]
        off, views = 0, []
        for p in plans:
            _, odt = p._dtypes()
            nb = p.num_scales * p.n * torch_itemsize(odt)
            if off + nb > arena.numel():
                return None
            views.append(arena[off:off + nb].view(odt).view(p.num_scales, p.n))
            off = (off + nb + 255) & ~255
        wb = self.cwt.batch_workspace_bytes(plans)
        if off + max(wb, 1) > arena.numel():
            return None
        return views, arena[off:off + max(wb, 1)]

    def _launch(self, batch: list[Request], slot: int):
        torch = self.torch
        st = self.streams[slot]
        plans = [r.plan for r in batch]
        with torch.cuda.stream(st):
            carved = self._carve(plans, slot)
            if carved is not None:
                outs, ws = carved
            else:
                if self.arenas is not None:
                    self.arena_fallbacks += 1
                outs = [p.empty_output(self.device) for p in plans]
                wb = self.cwt.batch_workspace_bytes(plans)
                ws = torch.empty(max(wb, 1), dtype=torch.uint8, device=self.device)
            self.cwt.exec_batch(plans, [r.signal for r in batch], outs, ws, stream=st)
            ev = torch.cuda.Event()
            ev.record(st)
        return {"event": ev, "outs": outs, "ws": ws, "batch": batch}

    def done(self, handle) -> bool:
        return handle["event"].query()

    def finish(self, r: Request, handle) -> None:
        i = handle["batch"].index(r)
        r.output = handle["outs"][i] if self.keep_outputs else None
        plan = r.plan
        close = False
        with self._lock:
            self._busy_plans[id(plan)] -= 1
            if self._busy_plans[id(plan)] == 0:
                del self._busy_plans[id(plan)]
                if plan in self._retired:
                    self._retired.remove(plan)
                    close = True
        if close:
            plan.close()
        r.plan = None


def torch_itemsize(dt) -> int:
    import torch
    return torch.empty((), dtype=dt).element_size()


def run_open_loop(scheduler, requests: list[Request], clock: Callable[[], float] = time.perf_counter,
                  advance: Optional[Callable[[float], None]] = None, idle_sleep: float = 0.0) -> list[Request]:
    """Submit each request at its arrival time (seconds after the start) and
    poll until all have completed.  ``advance(t)``, if given, moves a
    simulated clock to t when nothing else can happen.  ``idle_sleep``: with
    the real clock, sleep that long after a poll that completed nothing and
    with no arrival due, so that planner threads get the interpreter (a
    spinning loop would hold it for whole switch intervals)."""
    reqs = sorted(requests, key=lambda r: r.arrival)
    t0 = clock()
    for r in reqs:
        r.arrival = t0 + r.arrival
    i, done = 0, []
    while len(done) < len(reqs):
        now = clock()
        while i < len(reqs) and reqs[i].arrival <= now:
            scheduler.submit(reqs[i])
            i += 1
        got = scheduler.poll()
        done.extend(got)
        if advance is not None and not got:
            nxt = reqs[i].arrival if i < len(reqs) else None
            advance(nxt)
        elif idle_sleep > 0 and not got and (i == len(reqs) or reqs[i].arrival > clock()):
            time.sleep(idle_sleep)
    return done


def latency_summary(done: list[Request], skip: int = 0) -> dict:
    """p50 / p99 / mean of arrival -> completion (seconds) over the requests
    that arrived after the first ``skip`` (warm-up), and the throughput."""
    ok = sorted((r for r in done if r.error is None), key=lambda r: r.arrival)[skip:]
    if not ok:
        return {"count": 0}
    lat = np.array([r.done - r.arrival for r in ok])
    span = max(r.done for r in ok) - min(r.arrival for r in ok)
    coeffs = sum(r.coefficients for r in ok)
    out = {"count": len(ok), "p50_ms": float(np.percentile(lat, 50) * 1e3),
           "p99_ms": float(np.percentile(lat, 99) * 1e3), "mean_ms": float(lat.mean() * 1e3),
           "coefficients_per_s": coeffs / span if span > 0 else None,
           "rejected": sum(1 for r in done if r.error is not None)}
    pm = np.array([r.plan_ms for r in ok if r.plan_ms is not None])
    if pm.size:
        out.update({"plan_ms_p50": float(np.percentile(pm, 50)), "plan_ms_p99": float(np.percentile(pm, 99)),
                    "plan_ms_mean": float(pm.mean())})
    return out
