"""Batched execution (cwt_exec_batch): many independent transforms of
different lengths, scales, wavelets, boundaries and precisions in one call.
Every result must be bit-identical to the same plan run alone, and
(spot-checked) agree with the oracle."""
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


def _mixed(torch):
    """Instances of the batch workload's kind, plus an FP64 plan, a
    whole-signal-mode plan and a spline plan (those run one by one inside
    the batch call)."""
    import paper_2302_03909_amd as cwt
    plans, sigs, meta = [], [], []
    for inst in synth.batch_specs(count=40, seed=7, log2_lo=8.0, log2_hi=14.0, s_lo=4, s_hi=24):
        par = 6.0 if inst.wavelet == "morlet" else None
        plans.append(cwt.Plan(inst.n, inst.boundary, inst.wavelet, inst.scales, param=par, precision="fp32"))
        sigs.append(torch.as_tensor(inst.signal.astype(np.float32), device="cuda"))
        meta.append((inst.signal.astype(np.float32).astype(np.float64), inst.boundary, inst.wavelet, par,
                     inst.scales, "fp32"))
    extra = [
        (3001, "zero", "mexhat", None, [1.5, 9.0, 150.0], "fp64", "fft", "segmented"),
        (2048, "periodic", "morlet", 6.0, [2.0, 40.0, 300.0], "fp32", "fft", "whole"),
        (1500, "zero", "morlet", 6.0, [2.0, 30.0], "fp64", "spline", "segmented"),
    ]
    for n, bc, wav, par, scales, prec, method, mode in extra:
        f = np.random.default_rng(n).standard_normal(n)
        dt = torch.float64 if prec == "fp64" else torch.float32
        plans.append(cwt.Plan(n, bc, wav, scales, param=par, precision=prec, method=method, fft_mode=mode))
        sigs.append(torch.as_tensor(f, dtype=dt, device="cuda"))
        meta.append((f if prec == "fp64" else f.astype(np.float32).astype(np.float64), bc, wav, par, scales, prec))
    return plans, sigs, meta


def test_batch_bitwise_equals_single(torch_cuda):
    import paper_2302_03909_amd as cwt
    plans, sigs, _ = _mixed(torch_cuda)
    print(f"batch of {len(plans)} instances", flush=True)
    outs = cwt.exec_batch(plans, sigs)
    torch_cuda.cuda.synchronize()
    for i, (p, s) in enumerate(zip(plans, sigs)):
        alone = p(s)
        torch_cuda.cuda.synchronize()
        assert torch_cuda.equal(outs[i], alone), i


def test_batch_order_independent(torch_cuda):
    import paper_2302_03909_amd as cwt
    plans, sigs, _ = _mixed(torch_cuda)
    a = cwt.exec_batch(plans, sigs)
    perm = np.random.default_rng(3).permutation(len(plans))
    b = cwt.exec_batch([plans[i] for i in perm], [sigs[i] for i in perm])
    torch_cuda.cuda.synchronize()
    for j, i in enumerate(perm):
        assert torch_cuda.equal(a[i], b[j])


def test_batch_matches_oracle(torch_cuda):
    import paper_2302_03909_amd as cwt
    plans, sigs, meta = _mixed(torch_cuda)
    outs = cwt.exec_batch(plans, sigs)
    torch_cuda.cuda.synchronize()
    for i in list(range(0, len(plans) - 3, 7)) + [len(plans) - 3, len(plans) - 2]:
        f, bc, wav, par, scales, prec = meta[i]
        ref = oracle.cwt(f, bc, wav, scales, param=par)
        err = per_scale_rel_l2(outs[i].cpu().numpy(), ref)
        assert err.max() <= (1e-10 if prec == "fp64" else 1e-5), (i, err.max())


def test_batch_of_one_and_empty(torch_cuda):
    import paper_2302_03909_amd as cwt
    plans, sigs, _ = _mixed(torch_cuda)
    out = cwt.exec_batch(plans[:1], sigs[:1])[0]
    torch_cuda.cuda.synchronize()
    assert torch_cuda.equal(out, plans[0](sigs[0]))
    assert cwt.exec_batch([], []) == []
