"""Served form on the GPU: requests of mixed shapes go through the
continuous-batching and plain-batching schedulers; every output must equal
the same request transformed alone, bit for bit, and match the FP64 oracle
(Sec. 3, Eq. discreteCWT) within the FP32 bar at sampled positions."""
import numpy as np
import pytest

import oracle
import synth
from tests.helpers import per_scale_rel_l2

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _requests(torch, count=40, seed=11):
    from paper_2302_03909_amd.serve import Request
    out = []
    for i, inst in enumerate(synth.request_stream(count, rate_hz=20000.0, seed=seed, log2_lo=10.0, log2_hi=15.0,
                                                  s_lo=8, s_hi=40)):
        par = {"morlet": 6.0, "mexhat": None, "dog": 4.0}[inst.wavelet]
        sig = torch.as_tensor(inst.signal.astype(np.float32), device="cuda")
        out.append(Request(i, inst.n, inst.boundary, inst.wavelet, par, inst.scales, "fp32", sig,
                           arrival=inst.arrival))
    torch.cuda.synchronize()
    return out


@pytest.mark.parametrize("mode", ["continuous", "static"])
def test_served_outputs_equal_alone(torch_cuda, mode):
    import paper_2302_03909_amd as cwt
    from paper_2302_03909_amd.serve import (ContinuousScheduler, GpuExecutor, StaticBatcher, latency_summary,
                                            run_open_loop)
    reqs = _requests(torch_cuda)
    print(f"serving {len(reqs)} requests ({mode})", flush=True)
    ex = GpuExecutor(streams=2, keep_outputs=True)
    sched = (ContinuousScheduler(ex, budget_bytes=2 << 30, streams=2) if mode == "continuous"
             else StaticBatcher(ex, max_batch=8, window=1e-3))
    done = run_open_loop(sched, reqs)
    torch_cuda.cuda.synchronize()
    assert len(done) == len(reqs) and all(r.error is None for r in done)
    print(latency_summary(done), "batches", sched.batches)
    for r in done:
        alone = cwt.Plan(r.n, r.boundary, r.wavelet, r.scales, param=r.param, precision="fp32")(r.signal)
        torch_cuda.cuda.synchronize()
        assert torch_cuda.equal(r.output, alone), r.rid
    # and every served output matches the FP64 oracle (on the FP32 input) at
    # sampled positions of every scale: the first and last two and 12 more
    worst = 0.0
    for r in done:
        rng = np.random.default_rng(r.rid)
        pos = np.unique(np.concatenate([[0, 1, r.n - 2, r.n - 1], rng.integers(0, r.n, 12)]))
        s = np.asarray(r.scales)
        si = np.repeat(np.arange(s.size), pos.size)
        pi = np.tile(pos, s.size)
        f64 = r.signal.double().cpu().numpy()
        ref = oracle.cwt_points(f64, r.boundary, r.wavelet, s, si, pi, param=r.param).reshape(s.size, pos.size)
        got = r.output[:, torch_cuda.as_tensor(pos, device="cuda")].cpu().numpy().astype(ref.dtype)
        err = per_scale_rel_l2(got, ref)
        worst = max(worst, float(err.max()))
        assert err.max() <= 1e-5, (r.rid, r.n, r.wavelet, float(err.max()))
    print("served outputs vs oracle: max sampled per-scale rel L2", worst)
