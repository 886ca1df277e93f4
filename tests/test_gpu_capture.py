"""cwt_exec under HIP stream capture.  The segmented FFT method forks its
local-group kernels onto a second stream and joins them back; captured into a
graph, that must replay the transform exactly.  The graph is replayed several
times with eager work of another plan and synchronisations in between, and
every replay is compared with the eager result."""
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


@pytest.mark.parametrize("wavelet,param", [("morlet", 6.0), ("dog", 2.0)])
def test_exec_graph_replays_match_eager(torch_cuda, wavelet, param):
    import paper_2302_03909_amd as cwt
    torch = torch_cuda
    n = 1 << 17
    scales = synth.log_scales(2.0, 2.0 ** 12, 24)
    plan = cwt.Plan(n, "zero", wavelet, scales, param=param, precision="fp32")
    paths = set(plan.scale_path().tolist())
    assert paths == {cwt.PATH_LOCAL, cwt.PATH_COLUMN}, "the plan must take both kernel chains"
    f = torch.as_tensor(synth.lognormal_field(n, seed=11).astype(np.float32), device="cuda")
    ws = plan.empty_workspace()
    ref = plan(f, plan.empty_output(), ws)  # eager
    torch.cuda.synchronize()
    # another plan's eager work between replays
    other = cwt.Plan(5000, "periodic", "mexhat", [2.0, 17.0, 90.0], precision="fp32")
    g_in = torch.as_tensor(synth.tones_noise(5000).astype(np.float32), device="cuda")
    g_out = other.empty_output()
    out = plan.empty_output()
    side = torch.cuda.Stream()
    # one eager call on the capture stream creates its paired second stream
    with torch.cuda.stream(side):
        plan(f, out, ws)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=side):
        plan(f, out, ws)
    for rep in range(3):
        out.fill_(float("nan"))
        other(g_in, g_out, other.empty_workspace())
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, ref), f"replay {rep} differs from the eager transform"


@pytest.mark.parametrize("wavelet,param", [("morlet", 6.0), ("dog", 2.0)])
def test_two_stream_execution_equals_serialized(torch_cuda, wavelet, param):
    # with launch timing on, every launch stays on the caller's stream; the
    # two kernel chains write disjoint rows, so the results are bit-identical
    import paper_2302_03909_amd as cwt
    torch = torch_cuda
    n = 200003
    scales = synth.log_scales(2.0, 2.0 ** 13, 40)
    plan = cwt.Plan(n, "zero", wavelet, scales, param=param, precision="fp32")
    f = torch.as_tensor(synth.lognormal_field(n, seed=12).astype(np.float32), device="cuda")
    ws = plan.empty_workspace()
    a = plan(f, plan.empty_output(), ws)
    plan.timing(True)
    b = plan(f, plan.empty_output(), ws)
    plan.timing(False)
    plan.timing_read()
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def test_wps_graph_replays_match_eager(torch_cuda):
    # the statistics epilogue (Sec. 5) under capture: count, forward, reduce,
    # the reducing output kernels and the finalisation replay exactly
    import ctypes
    import paper_2302_03909_amd as cwt
    torch = torch_cuda
    n = 1 << 17
    d = synth.zeldovich_field(n)
    plan = cwt.Plan(n, "periodic", "cwgdw", synth.log_scales(2.0, 2.0 ** 12, 24), precision="fp32")
    f = torch.as_tensor(d.astype(np.float32), device="cuda")
    ws = torch.empty(cwt.wps_workspace_bytes(plan), dtype=torch.uint8, device="cuda")
    ref, ref_c = cwt.exec_wps(plan, f, None, (0.0,), workspace=ws)
    torch.cuda.synchronize()
    wps = torch.empty_like(ref)
    cnt = torch.empty_like(ref_c)
    thr = (ctypes.c_double * 1)(0.0)
    side = torch.cuda.Stream()

    def call():
        rc = cwt.load().cwt_exec_wps(plan.handle, ctypes.c_void_p(f.data_ptr()), None, thr, 1,
                                     ctypes.c_void_p(wps.data_ptr()), ctypes.c_void_p(cnt.data_ptr()),
                                     ctypes.c_void_p(ws.data_ptr()), ctypes.c_void_p(side.cuda_stream))
        assert rc == 0, cwt.load().cwt_last_error()

    with torch.cuda.stream(side):
        call()  # creates the paired second stream of this caller stream
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=side):
        call()
    for rep in range(3):
        wps.fill_(float("nan"))
        cnt.fill_(-1)
        ws.fill_(0xFF)  # stale partial sums must not leak into a replay
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(wps, ref) and torch.equal(cnt, ref_c), f"replay {rep} differs from the eager result"
