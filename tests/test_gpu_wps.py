"""GPU parity of the statistics epilogue (Sec. 5, Eqs. env_wps, global_wps,
global_wps_env_wps): cwt_exec_wps against the oracle's power spectra of its
FP64 transform, on the 1D Zel'dovich fields of Eq. nonlinear_dens.

Tolerance, derived from the transform's own bar: if the coefficients of a
scale carry a relative L2 error eps (1e-10 FP64, 1e-5 FP32, measured
against max(||W_j||, 1e-3 max_k ||W_k||)), the squares summed over a bin that
holds a fraction q of the scale's power differ by at most
2 eps / sqrt(q) + eps^2 / q relative (Cauchy-Schwarz on
sum (|g| - |r|)(|g| + |r|)); the global spectrum is the case q = 1.

At the full headline size (N = 2^22, 128 scales) the oracle cannot run the
whole transform, so the epilogue is checked there against the power spectra
of cwt_exec's own output (whose parity the FFT tests establish), reduced on
the device in FP64, to the same derived bound with eps doubled."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-10, "fp32": 1e-5}


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def bound(ref, counts, n, eps_w, floor=1e-3):
    """Per-entry relative bound for a [S, nb + 1] spectrum table."""
    nb = ref.shape[1] - 1
    norm = np.sqrt(ref[:, -1] * n)
    eps = eps_w * np.maximum(1.0, floor * norm.max() / norm)
    q = np.empty_like(ref)
    with np.errstate(invalid="ignore", divide="ignore"):
        q[:, :nb] = (counts / n)[None, :] * ref[:, :nb] / ref[:, -1:]
    q[:, nb] = 1.0
    return 2.0 * eps[:, None] / np.sqrt(q) + eps[:, None] ** 2 / q


def check(got, ref, counts_got, counts_ref, n, eps_w, label):
    assert counts_got.tolist() == counts_ref.tolist(), (label, counts_got, counts_ref)
    empty = counts_ref == 0
    if empty.any():
        assert np.all(np.isnan(got[:, :-1][:, empty]))
    keep = np.ones(ref.shape[1], dtype=bool)
    keep[:-1] = ~empty
    b = bound(ref, counts_ref, n, eps_w)[:, keep]
    rel = np.abs(got[:, keep] - ref[:, keep]) / ref[:, keep]
    worst = np.max(rel / (1.05 * b + 1e-13))
    print(f"{label}: max rel err {rel.max():.3e}, worst err/bound {worst:.3f}")
    assert worst <= 1.0, (label, rel.max(), worst)


def run_wps(torch, f, bc, wav, par, scales, precision, env=None, thresholds=(0.0,)):
    import paper_2302_03909_amd as cwt
    plan = cwt.Plan(f.size, bc, wav, scales, param=par, precision=precision)
    dt = torch.float64 if precision == "fp64" else torch.float32
    sig = torch.as_tensor(f, dtype=dt, device="cuda")
    ev = None if env is None else torch.as_tensor(env, dtype=dt, device="cuda")
    w, c = cwt.exec_wps(plan, sig, ev, thresholds)
    torch.cuda.synchronize()
    return plan, w.cpu().numpy(), c.cpu().numpy()


CASES = [
    # n, boundary, wavelet, param, scale range, precision, thresholds, env kind
    (4096, "periodic", "cwgdw", None, (2.0, 1024.0, 24), "fp64", (0.0,), "self"),
    (20000, "periodic", "cwgdw", None, (1.5, 5000.0, 32), "fp64", (0.0,), "self"),
    (12345, "zero", "mexhat", None, (2.0, 3000.0, 28), "fp64", (-0.1, 0.0, 0.3), "self"),
    (12346, "zero", "morlet", 6.0, (2.0, 3000.0, 28), "fp64", (0.0,), "initial"),
    (1 << 16, "periodic", "cwgdw", None, (2.0, 8192.0, 40), "fp32", (-0.2, 0.0, 0.5), "self"),
    (65531, "zero", "dog", 2.0, (2.0, 8192.0, 40), "fp32", (0.0,), "initial"),
    (1 << 16, "periodic", "morlet", 6.0, (2.0, 8192.0, 40), "fp32", (0.0,), "self"),
]


@pytest.mark.parametrize("n,bc,wav,par,sr,precision,thr,envk", CASES)
def test_wps_parity(torch_cuda, n, bc, wav, par, sr, precision, thr, envk):
    d, d0 = synth.zeldovich_field(n, return_initial=True)
    scales = synth.log_scales(*sr)
    env = d0 if envk == "initial" else None
    label = f"N={n} {bc} {wav} {precision} bins={len(thr) + 1} env={envk}"
    print("case", label, flush=True)
    plan, got, cnt = run_wps(torch_cuda, d, bc, wav, par, scales, precision, env, thr)
    # local and band groups both present (scales past one segment's band)
    desc = plan.describe()
    assert "local" in desc and "band" in desc, desc
    ref, rcnt = oracle.cwt_wps(d, bc, wav, scales, env=env, thresholds=thr, param=par, spectral=n > 8192)
    check(got, ref, cnt, rcnt, n, TOL[precision], label)
    # Eq. global_wps_env_wps on the GPU result
    nb = len(thr) + 1
    mix = np.nansum(got[:, :nb] * (cnt / n)[None, :], axis=1)
    assert np.max(np.abs(mix - got[:, nb]) / got[:, nb]) < 1e-12


def test_env_default_is_signal(torch_cuda):
    import paper_2302_03909_amd as cwt
    d = synth.zeldovich_field(8192)
    plan = cwt.Plan(d.size, "periodic", "cwgdw", synth.log_scales(2.0, 2000.0, 16), precision="fp32")
    sig = torch_cuda.as_tensor(d, dtype=torch_cuda.float32, device="cuda")
    a, ca = cwt.exec_wps(plan, sig, None, (0.0,))
    b, cb = cwt.exec_wps(plan, sig, sig.clone(), (0.0,))
    c, _ = cwt.exec_wps(plan, sig, None, (0.0,))
    torch_cuda.cuda.synchronize()
    assert torch_cuda.equal(a, b) and torch_cuda.equal(ca, cb)
    assert torch_cuda.equal(a, c)  # fixed summation order: same bits every run


def test_empty_bin_and_no_threshold(torch_cuda):
    import paper_2302_03909_amd as cwt
    d = synth.zeldovich_field(4096)
    sc = synth.log_scales(2.0, 1000.0, 12)
    plan = cwt.Plan(d.size, "periodic", "cwgdw", sc, precision="fp64")
    sig = torch_cuda.as_tensor(d, device="cuda")
    w, c = cwt.exec_wps(plan, sig, None, (1e6,))  # every position below: bin 1 empty
    w0, c0 = cwt.exec_wps(plan, sig, None, ())  # one bin: env-WPS = global
    torch_cuda.cuda.synchronize()
    w, c, w0, c0 = w.cpu().numpy(), c.cpu().numpy(), w0.cpu().numpy(), c0.cpu().numpy()
    assert c.tolist() == [4096, 0] and np.all(np.isnan(w[:, 1]))
    assert c0.tolist() == [4096] and w0.shape == (12, 2)
    assert np.max(np.abs(w0[:, 0] - w0[:, 1]) / w0[:, 1]) < 1e-14
    assert np.max(np.abs(w[:, 0] - w0[:, 1]) / w0[:, 1]) < 1e-14


def test_bad_arguments(torch_cuda):
    import paper_2302_03909_amd as cwt
    d = synth.zeldovich_field(4096)
    sig = torch_cuda.as_tensor(d, device="cuda")
    plan = cwt.Plan(d.size, "periodic", "cwgdw", [4.0, 40.0], precision="fp64")
    for thr in [(1.0, 0.0), (0.0, 0.0), (float("nan"),), (0.0, 1.0, 2.0, 3.0)]:
        with pytest.raises(cwt.CwtError) as e:
            cwt.exec_wps(plan, sig, None, thr)
        assert e.value.code == cwt.CWT_EINVAL
    sp = cwt.Plan(d.size, "periodic", "mexhat", [4.0, 40.0], precision="fp64", method="spline")
    with pytest.raises(cwt.CwtError) as e:
        cwt.exec_wps(sp, sig, None, (0.0,))
    assert e.value.code == cwt.CWT_EUNSUPPORTED


def device_wps(torch, out, env, thr, n, cplx):
    """Power spectra of a [S, N] coefficient tensor, reduced on the device in
    FP64 (chunks of scales)."""
    k = torch.zeros(n, dtype=torch.int64, device=out.device)
    for t in thr:
        k += (env >= t).to(torch.int64)
    nb = len(thr) + 1
    S = out.shape[0]
    res = np.empty((S, nb + 1))
    for j0 in range(0, S, 8):
        blk = out[j0:j0 + 8]
        p2 = (blk.real.double() ** 2 + blk.imag.double() ** 2) if cplx else blk.double() ** 2
        for b in range(nb):
            m = k == b
            res[j0:j0 + 8, b] = (p2[:, m].sum(dim=1) / m.sum()).cpu().numpy()
        res[j0:j0 + 8, nb] = (p2.sum(dim=1) / n).cpu().numpy()
    counts = np.array([int((k == b).sum()) for b in range(nb)])
    return res, counts


@pytest.mark.parametrize("wav,par,bc", [("cwgdw", None, "periodic"), ("morlet", 6.0, "zero")])
def test_wps_headline_size(torch_cuda, wav, par, bc):
    # N = 2^22, 128 log scales 2..2^16, FP32: the epilogue against the power
    # spectra of the plain transform's output
    import paper_2302_03909_amd as cwt
    torch = torch_cuda
    n = 1 << 22
    d = synth.zeldovich_field(n)
    scales = synth.log_scales(2.0, 65536.0, 128)
    print(f"case headline N=2^22 S=128 {wav} {bc} fp32", flush=True)
    plan = cwt.Plan(n, bc, wav, scales, param=par, precision="fp32")
    sig = torch.as_tensor(d, dtype=torch.float32, device="cuda")
    got, cnt = cwt.exec_wps(plan, sig, None, (0.0,))
    out = plan(sig)
    ref, rcnt = device_wps(torch, out, sig, (0.0,), n, plan.is_complex)
    del out
    torch.cuda.synchronize()
    check(got.cpu().numpy(), ref, cnt.cpu().numpy(), rcnt, n, 2 * TOL["fp32"], f"headline {wav}")


# ---- global spectrum by Parseval (cwt_global_wps) ----------------------------
# For a periodic signal the mean of |W(s, b)|^2 over the period equals
# (1/N^2) sum_m |F[m]|^2 Psi_s(omega_m)^2: no transform is taken.  The same
# derived bound (the q = 1 case, 2 eps + eps^2 with the 1e-3 floor) applies.

@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("wav,par", [("morlet", 6.0), ("dog", 2.0), ("mexhat", None), ("cwgdw", None),
                                     ("gdw", None), ("mw", None)])
def test_parseval_global_spectrum_against_oracle(torch_cuda, precision, wav, par):
    import paper_2302_03909_amd as cwt
    n = 1 << 16
    f = synth.zeldovich_field(n)
    scales = synth.log_scales(2.0, n / 8.0, 24)
    print(f"case parseval N={n} {wav} {precision}", flush=True)
    plan = cwt.Plan(n, "periodic", wav, scales, param=par, precision=precision, fft_mode="whole")
    dt = torch_cuda.float64 if precision == "fp64" else torch_cuda.float32
    got = cwt.global_wps(plan, torch_cuda.as_tensor(f, dtype=dt, device="cuda")).cpu().numpy()
    fr = f.astype(np.float32).astype(np.float64) if precision == "fp32" else f
    ref, counts = oracle.cwt_wps(fr, "periodic", wav, scales, thresholds=(), param=par, spectral=True)
    b = bound(ref, counts, n, TOL[precision])[:, -1]
    rel = np.abs(got - ref[:, -1]) / ref[:, -1]
    print(f"  max rel err {rel.max():.3e}, worst err/bound {np.max(rel / b):.3f}")
    assert np.all(rel <= 1.05 * b + 1e-13)


def test_parseval_matches_the_epilogue_at_the_headline_size(torch_cuda):
    # N = 2^22, 128 scales, CW-GDW, FP32: Parseval on a whole-signal plan
    # against the global column of cwt_exec_wps on the segmented plan
    import paper_2302_03909_amd as cwt
    n = 1 << 22
    f = synth.zeldovich_field(n)
    scales = synth.log_scales(2.0, 2.0 ** 16, 128)
    x = torch_cuda.as_tensor(f, dtype=torch_cuda.float32, device="cuda")
    whole = cwt.Plan(n, "periodic", "cwgdw", scales, precision="fp32", fft_mode="whole")
    seg = cwt.Plan(n, "periodic", "cwgdw", scales, precision="fp32")
    a = cwt.global_wps(whole, x).cpu().numpy()
    w, _ = cwt.exec_wps(seg, x, thresholds=(), with_counts=False)
    b = w.cpu().numpy()[:, -1]
    rel = np.abs(a - b) / b
    print(f"parseval vs epilogue, N=2^22: max rel diff {rel.max():.3e}")
    # each side within the FP32 bar of the FP64 value: 2 (2 eps + eps^2)
    assert rel.max() <= 2 * (2e-5 + 1e-10)
