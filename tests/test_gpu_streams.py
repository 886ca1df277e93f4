"""Stream behaviour of the C ABI on the GPU.

* A plan may be destroyed while its work is still queued: its tables are
  released after that work (cwt_destroy orders the release after the plan's
  last call on each stream).  A throw-away plan per call, with no
  synchronisation in between, must give the same outputs as a kept plan.
* Calls on different caller streams run side by side: each caller stream
  gets its own second stream for the local kernels, so nothing orders one
  caller's calls after another's.  Outputs stay bit-identical, and two
  streams finish a set of small calls sooner than one stream."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.mark.parametrize("method", ["fft", "spline"])
def test_plan_destroyed_while_queued(torch_cuda, method):
    import paper_2302_03909_amd as cwt
    torch = torch_cuda
    shapes = [(1 << 16, "zero", "morlet", 6.0, synth.log_scales(2.0, 2.0 ** 12, 24)),
              (50001, "periodic", "mexhat", None, synth.log_scales(1.5, 3000.0, 16)),
              (1 << 15, "zero", "dog", 4.0, synth.log_scales(0.8, 900.0, 12))]
    sigs = [torch.as_tensor(synth.lognormal_field(n, seed=30 + i).astype(np.float32), device="cuda")
            for i, (n, *_rest) in enumerate(shapes)]
    kept = [cwt.Plan(n, bc, w, sc, param=p, precision="fp32", method=method) for n, bc, w, p, sc in shapes]
    refs = [pl(x) for pl, x in zip(kept, sigs)]
    torch.cuda.synchronize()
    outs = []
    for rep in range(4):
        for (n, bc, w, p, sc), x in zip(shapes, sigs):
            # the plan's last reference goes away right after the enqueue
            outs.append(cwt.Plan(n, bc, w, sc, param=p, precision="fp32", method=method)(x))
    torch.cuda.synchronize()
    for i, o in enumerate(outs):
        assert torch.equal(o, refs[i % len(shapes)]), f"call {i} differs from the kept plan's output"


def test_two_caller_streams_overlap(torch_cuda):
    import paper_2302_03909_amd as cwt
    torch = torch_cuda
    n = 1 << 16
    plan = cwt.Plan(n, "zero", "morlet", synth.log_scales(2.0, 1024.0, 32), param=6.0, precision="fp32")
    assert set(plan.scale_path().tolist()) == {cwt.PATH_LOCAL, cwt.PATH_COLUMN}
    x = torch.as_tensor(synth.lognormal_field(n, seed=41).astype(np.float32), device="cuda")
    ref = plan(x)
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    k = 12
    wss = [plan.empty_workspace() for _ in streams]
    outs = [[plan.empty_output() for _ in range(k)] for _ in streams]
    for st, ws in zip(streams, wss):  # first call per caller stream creates its pair
        with torch.cuda.stream(st):
            plan(x, outs[0][0], ws)
    torch.cuda.synchronize()

    def span(nstreams):
        # a spin kernel holds the streams while the calls are enqueued, so the
        # host's enqueue rate does not set the pace; the span runs from the
        # first sequence's start to the last sequence's end
        gate = torch.cuda.Stream()
        with torch.cuda.stream(gate):
            torch.cuda._sleep(20_000_000)
        go = torch.cuda.Event()
        go.record(gate)
        starts, ends = [], []
        for si in range(2):
            st = streams[si] if nstreams == 2 else streams[0]
            ws = wss[si] if nstreams == 2 else wss[0]
            st.wait_event(go)
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(st)
            with torch.cuda.stream(st):
                for o in outs[si]:
                    plan(x, o, ws)
            b.record(st)
            starts.append(a)
            ends.append(b)
        torch.cuda.synchronize()
        return max(starts[0].elapsed_time(b) for b in ends)

    serial = min(span(1) for _ in range(3))
    concurrent = min(span(2) for _ in range(3))
    print(f"{2 * k} calls: one stream {serial:.3f} ms, two streams {concurrent:.3f} ms "
          f"({concurrent / serial:.2f})")
    for row in outs:
        for o in row:
            assert torch.equal(o, ref)
    assert concurrent < 0.95 * serial
