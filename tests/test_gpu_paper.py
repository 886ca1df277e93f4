"""The paper's own accuracy comparison on the GPU (Sec. 4.1), and parity of
the Table 2 wavelets.

* The CBSW, GDW, CW-GDW and MW of Table 2 in the library's transform (the
  unit-step sum, aliased spectra): FFT method, segmented and whole-signal,
  FP64 and FP32, against the direct-sum oracle; spline method against the
  oracle's exact spline target.  (The CBSW is not band-limited and is
  taken by the analytic form only.)
* psi_mode "analytic" (Eq. discrete_CWT_conv as printed, the bare wavelet
  transform at the DFT bins) against the oracle's numpy form of the same
  equation, on the plan's FFT length.
* Error spectra ES (Eq. error_spectrum) of the paper's test signals f1
  (periodic, Eq. signal_f1) and f2 (zero boundary, Eq. signal_f2), N = 512,
  on the scale grid of Sec. 3.1 with 8 sub-levels, against the continuous
  CWTs (tests/closed_forms), compared with the ranges Sec. 4.1 prints for
  the FFTCWT (periodic below 1e-10 %, zero boundary 1e-8 % to 0.1 %) and the
  M02CWT (0.003 % to 1 % for GDW, CW-GDW and MW), each within a factor 10
  (rounding and the paper's unstated sub-level count differ)."""
import math

import numpy as np
import pytest

import oracle
import synth
from tests import closed_forms as cf
from tests.helpers import error_spectrum_percent, per_scale_rel_l2

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-10, "fp32": 1e-5}
TABLE2 = ["cbsw", "gdw", "cwgdw", "mw"]


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def cw_of(golden, wav):
    return {"cbsw": 0.466094761079290, "gdw": 2 / math.sqrt(5),
            "cwgdw": golden["table2_cwgdw_cw"]["value"], "mw": golden["table2_mw_cw"]["value"]}[wav]


def run(torch, f, bc, wav, scales, precision="fp64", **kw):
    import paper_2302_03909_amd as cwt
    plan = cwt.Plan(f.size, bc, wav, scales, precision=precision, **kw)
    dt = torch.float64 if precision == "fp64" else torch.float32
    w = plan(torch.as_tensor(f, dtype=dt, device="cuda"))
    torch.cuda.synchronize()
    return plan, w.cpu().numpy()


def ref_in(f, precision):
    return f.astype(np.float32).astype(np.float64) if precision == "fp32" else f


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("fft_mode", ["segmented", "whole"])
@pytest.mark.parametrize("wav", ["gdw", "cwgdw", "mw"])
@pytest.mark.parametrize("n,bc", [(3001, "zero"), (4096, "periodic")])
def test_table2_wavelets_fft_parity(torch_cuda, wav, fft_mode, precision, n, bc):
    print(f"table2 fft {wav} {fft_mode} {precision} N={n} {bc}", flush=True)
    f = synth.lognormal_field(n, seed=71)
    scales = synth.log_scales(1.5, 700.0, 12)
    plan, got = run(torch_cuda, f, bc, wav, scales, precision, fft_mode=fft_mode)
    ref = oracle.cwt(ref_in(f, precision), bc, wav, scales)
    assert got.dtype.kind == ("c" if wav == "mw" else "f")
    err = per_scale_rel_l2(got, ref)
    assert err.max() <= TOL[precision], (err.max(), int(err.argmax()))


@pytest.mark.parametrize("wav", ["gdw", "cwgdw", "mw"])
def test_table2_wavelets_spline_parity(torch_cuda, wav, golden):
    f = synth.lognormal_field(3001, seed=72)
    scales = [0.6, 1.5, 3.0, 9.0, 40.0, 300.0]
    plan, got = run(torch_cuda, f, "zero", wav, scales, "fp64", method="spline")
    hs = plan.spline_hstar()
    # Table 3 prints h for these three wavelets (the same AE_M = 5e-4 criterion)
    assert abs(hs - golden["table3_h"][{"gdw": "GDW", "cwgdw": "CW-GDW", "mw": "MW"}[wav]]) < 2e-3
    x = np.arange(f.size)
    ref = np.stack([oracle.spline_target_scale(f, "zero", wav, s, hs, x, nthreads=16) for s in scales])
    err = per_scale_rel_l2(got, ref)
    assert err.max() <= 1e-10, (err.max(), int(err.argmax()))


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("wav", TABLE2 + ["morlet", "mexhat"])
@pytest.mark.parametrize("n,bc", [(512, "periodic"), (512, "zero"), (5000, "zero"), (4608, "periodic")])
def test_analytic_mode_parity(torch_cuda, wav, precision, n, bc):
    import paper_2302_03909_amd as cwt
    print(f"analytic {wav} {precision} N={n} {bc}", flush=True)
    f = synth.tones_noise(n, seed=73) if bc == "periodic" else synth.lognormal_field(n, seed=73)
    scales = synth.log_scales(0.8, 600.0, 16)
    par = 6.0 if wav == "morlet" else None
    plan, got = run(torch_cuda, f, bc, wav, scales, precision, fft_mode="whole", psi_mode="analytic", param=par)
    assert set(plan.scale_path().tolist()) == {cwt.PATH_COLUMN}
    ref = oracle.cwt_analytic(ref_in(f, precision), bc, wav, scales, plan.fft_len, param=par)
    err = per_scale_rel_l2(got, ref)
    assert err.max() <= TOL[precision], (err.max(), int(err.argmax()))


def es_row(tag, es):
    return f"{tag:34s} min {es.min():.1e} %  max {es.max():.1e} %  median {np.median(es):.1e} %"


def test_paper_error_spectra(torch_cuda, golden):
    n = golden["paper_test_n"]["value"]
    f1, f2 = synth.paper_f1(n), synth.paper_f2(n)
    lines = []
    for wav in TABLE2:
        scales = synth.paper_scale_grid(n, cw_of(golden, wav), 8)
        a1 = cf.analytic_cwt_f1(wav, None, scales, n)
        a2 = cf.analytic_cwt_f2(wav, None, scales, n)
        if wav != "mw":
            a1, a2 = a1.real, a2.real
        _, w1 = run(torch_cuda, f1, "periodic", wav, scales, fft_mode="whole", psi_mode="analytic")
        _, w2 = run(torch_cuda, f2, "zero", wav, scales, fft_mode="whole", psi_mode="analytic")
        es1, es2 = error_spectrum_percent(w1, a1), error_spectrum_percent(w2, a2)
        lines += [es_row(f"{wav} FFTCWT f1 periodic", es1), es_row(f"{wav} FFTCWT f2 zero", es2)]
        # FP64 rounding sets this floor; it rises at the smallest scales,
        # whose response to f1's tones is weakest (within 10x of the bound)
        assert es1.max() < 10 * golden["es_fftcwt_periodic_max_percent"]["value"], (wav, es1.max())
        lo, hi = golden["es_fftcwt_zero_range_percent"]["value"]
        assert es2.max() < 10 * hi, (wav, es2.max())
        if wav == "cbsw":
            continue
        # the library's own forms: aliased spectra (the sampled sum) and the
        # spline method (M02)
        _, g1 = run(torch_cuda, f1, "periodic", wav, scales)
        _, g2 = run(torch_cuda, f2, "zero", wav, scales)
        lines += [es_row(f"{wav} aliased f1 periodic", error_spectrum_percent(g1, a1)),
                  es_row(f"{wav} aliased f2 zero", error_spectrum_percent(g2, a2))]
        _, m1 = run(torch_cuda, f1, "periodic", wav, scales, method="spline")
        _, m2 = run(torch_cuda, f2, "zero", wav, scales, method="spline")
        em1, em2 = error_spectrum_percent(m1, a1), error_spectrum_percent(m2, a2)
        lines += [es_row(f"{wav} M02 f1 periodic", em1), es_row(f"{wav} M02 f2 zero", em2)]
        assert em1.max() < 2 * golden["es_m02_range_percent"]["others"][1], (wav, em1.max())
    print("\n" + "\n".join(lines))
