"""GPU parity of the V97 method (Sec. 3.2) against the oracle's V97
transform: the unit-step sum with the wavelet replaced by
sum_k p(k) beta3(t / 2^i - k), p = q * q12 (Eqs. beta3_wavelet_approx, pj,
qj, q_12), evaluated tap by tap in the time domain.  The library computes it
as the filter chain of Eqs. fir_filter_beta - fir_filter_qi.  The oracle
gets the plan's w~_max (checked separately against its own).  Bars: 1e-10
(FP64 output), 1e-5 (FP32).  Also the error spectrum of the paper's f1 on
the V97 scale grid (Sec. 4.1 prints 0.01 % to 1 %)."""
import numpy as np
import pytest

import oracle
import synth
from tests import closed_forms as cf
from tests.helpers import error_spectrum_percent, per_scale_rel_l2

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-10, "fp32": 1e-5}


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def gpu_v97(torch, f, bc, wav, par, scales, precision):
    import paper_2302_03909_amd as cwt
    plan = cwt.Plan(f.size, bc, wav, scales, param=par, precision=precision, method="v97")
    dt = torch.float64 if precision == "fp64" else torch.float32
    w = plan(torch.as_tensor(f, dtype=dt, device="cuda"))
    torch.cuda.synchronize()
    return plan, w


def ref_rows(f, bc, wav, par, scales, wmax, x):
    return np.stack([oracle.v97_points(f, bc, wav, s, x, param=par, wmax=wmax, nthreads=16) for s in scales])


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("n,bc,wav,par,scales", [
    (4096, "periodic", "morlet", 6.0, [4.6, 7.0, 9.1, 30.0, 300.0]),
    (3001, "zero", "mexhat", None, [1.2, 2.0, 3.3, 40.0, 700.0]),
    (2500, "zero", "cbsw", None, [1.7, 2.0, 4.0, 37.0]),
    (2048, "periodic", "gdw", None, [0.9, 5.0, 61.0]),
    (2000, "zero", "mw", None, [3.1, 4.4, 19.0, 150.0]),
    (1500, "zero", "dog", 4.0, [1.7, 12.0, 1100.0]),
])
def test_v97_parity(torch_cuda, precision, n, bc, wav, par, scales):
    print(f"v97 case N={n} {bc} {wav} S={len(scales)} {precision}", flush=True)
    f = np.random.default_rng(n + 3).standard_normal(n) + 0.1
    plan, w = gpu_v97(torch_cuda, f, bc, wav, par, scales, precision)
    got = w.cpu().numpy()
    wmax = plan.spline_hstar()
    fr = f.astype(np.float32).astype(np.float64) if precision == "fp32" else f
    ref = ref_rows(fr, bc, wav, par, scales, wmax, np.arange(n))
    err = per_scale_rel_l2(got, ref)
    print("max rel L2", err.max())
    assert err.max() <= TOL[precision], (err.max(), int(err.argmax()))


def test_v97_full_size_fp64_mexhat_1m(torch_cuda):
    # N = 2^20 zero-boundary lognormal field, Mexican hat, 64 log scales
    # 2..2^14, FP64: every scale at sampled positions and tile edges
    from tests.test_gpu_spline import tile_edges
    f = synth.lognormal_field(1 << 20, seed=synth.SEED_FIELD_1M)
    scales = synth.log_scales(2.0, 2.0 ** 14, 64)
    plan, w = gpu_v97(torch_cuda, f, "zero", "mexhat", None, scales, "fp64")
    n = f.size
    rng = np.random.default_rng(4)
    pos = np.unique(np.concatenate([[0, 1, n // 2, n - 1], rng.integers(0, n, 8), tile_edges(plan, n)]))
    got = w[:, torch_cuda.as_tensor(pos, device="cuda")].cpu().numpy()
    del w
    ref = ref_rows(f, "zero", "mexhat", None, scales, plan.spline_hstar(), pos)
    err = per_scale_rel_l2(got, ref)
    print("v97 fp64 1M max err", err.max())
    assert err.max() <= 1e-10


def test_v97_paper_error_spectrum(torch_cuda, golden):
    # f1 of Sec. 4 on the V97 grid s = 2^(i + j/8) / w~_max, i < Nint(log2(
    # w~_max N / (c_w pi))) (Sec. 3.2), against its continuous CWT
    n = golden["paper_test_n"]["value"]
    f1 = synth.paper_f1(n)
    lines = []
    for wav in ("cbsw", "gdw", "cwgdw", "mw"):
        wmax = oracle.v97_wmax(wav)
        cw = wmax / 1.34
        nlev = int(round(np.log2(wmax * n / (cw * np.pi))))
        scales = np.array([2.0 ** (i + j / 8) / wmax for i in range(nlev) for j in range(8)])
        a1 = cf.analytic_cwt_f1(wav, None, scales, n)
        if wav != "mw":
            a1 = a1.real
        _, w = gpu_v97(torch_cuda, f1, "periodic", wav, None, scales, "fp64")
        es = error_spectrum_percent(w.cpu().numpy(), a1)
        lines.append(f"{wav} V97 f1 periodic  min {es.min():.1e} %  max {es.max():.1e} %  median {np.median(es):.1e} %")
        assert es.max() < 10 * golden["es_v97_range_percent"]["value"][1]
    print("\n" + "\n".join(lines))
