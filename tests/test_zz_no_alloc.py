"""cwt_exec_scratch (no allocation: the library's fixed scratch array as
workspace) against cwt_exec with a caller workspace, through the C ABI:
two calls in a row, the second with a smaller input, each output equal to
cwt_exec's bit for bit; a plan whose workspace exceeds the array is
rejected."""
import ctypes

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


def _run_pair(torch, cases):
    import paper_2302_03909_amd as cwt
    lib = cwt.load()
    for k, (n, bc, wav, par, scales, precision, method) in enumerate(cases):
        print(f"no-alloc call {k}: N={n} {bc} {wav} S={len(scales)} {precision} {method}", flush=True)
        plan = cwt.Plan(n, bc, wav, scales, param=par, precision=precision, method=method)
        assert 0 < plan.workspace_bytes <= cwt.scratch_bytes()
        dt = torch.float64 if precision == "fp64" else torch.float32
        x = torch.as_tensor(synth.lognormal_field(n, seed=50 + k), dtype=dt, device="cuda")
        ref = plan(x)
        out = plan.empty_output()
        out.fill_(float("nan"))
        st = torch.cuda.current_stream()
        rc = lib.cwt_exec_scratch(plan.handle, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                  ctypes.c_void_p(st.cuda_stream))
        assert rc == 0, lib.cwt_last_error().decode()
        torch.cuda.synchronize()
        assert torch.equal(out, ref), f"call {k} differs from cwt_exec"


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_scratch_matches_exec_fft(torch_cuda, precision):
    _run_pair(torch_cuda, [
        (1 << 20, "zero", "morlet", 6.0, synth.log_scales(2.0, 2.0 ** 14, 48), precision, "fft"),
        (30001, "periodic", "dog", 2.0, synth.log_scales(1.5, 900.0, 20), precision, "fft"),
    ])


def test_scratch_matches_exec_spline(torch_cuda):
    _run_pair(torch_cuda, [
        (1 << 18, "zero", "mexhat", None, synth.log_scales(1.0, 2.0 ** 12, 24), "fp64", "spline"),
        (5000, "periodic", "morlet", 6.0, [0.8, 3.0, 40.0], "fp64", "spline"),
    ])


def test_scratch_rejects_large_workspace(torch_cuda):
    import paper_2302_03909_amd as cwt
    plan = cwt.Plan(1 << 24, "zero", "mexhat", [2.0, 2.0 ** 16], method="spline", precision="fp32")
    assert plan.workspace_bytes > cwt.scratch_bytes()
    x = torch_cuda.zeros(1 << 24, dtype=torch_cuda.float32, device="cuda")
    out = plan.empty_output()
    with pytest.raises(cwt.CwtError) as e:
        cwt.exec_scratch(plan, x, out)
    assert e.value.code == cwt.CWT_EUNSUPPORTED
