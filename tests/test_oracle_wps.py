"""Pins of the oracle's wavelet power spectra (Sec. 5, Eqs. env_wps,
global_wps, global_wps_env_wps) and of the 1D Zel'dovich field generator
(Eq. nonlinear_dens): bin bookkeeping by brute force, the partition identity,
a closed form for a pure tone, and the environment dependence the paper
reports for the initial and the evolved field."""
import numpy as np
import pytest

import oracle
import synth
from tests.closed_forms import any_psi_hat


def test_bins_brute_force():
    # bin = number of thresholds <= env; values on a threshold go up; NaN -> 0
    env = np.array([-1.0, 0.0, 1.99, 2.0, 4.5, 5.0, 7.0, np.nan, -np.inf, np.inf])
    thr = (2.0, 5.0)
    want = []
    for e in env:
        k = 0
        for t in thr:
            if e >= t:
                k += 1
        want.append(k)
    assert oracle.wps_bins(env, thr).tolist() == want == [0, 0, 0, 1, 1, 2, 2, 0, 0, 2]


def test_means_brute_force():
    rng = np.random.default_rng(3)
    S, N = 3, 40
    W = rng.standard_normal((S, N)) + 1j * rng.standard_normal((S, N))
    env = rng.integers(0, 6, N).astype(np.float64)
    thr = (1.0, 3.0, 4.0)
    got, counts = oracle.wps(W, env, thr)
    for j in range(S):
        tot = [0.0] * 4
        cnt = [0] * 4
        for x in range(N):
            b = sum(1 for t in thr if env[x] >= t)
            tot[b] += abs(W[j, x]) ** 2
            cnt[b] += 1
        for b in range(4):
            assert abs(got[j, b] - tot[b] / cnt[b]) <= 1e-14 * got[j, b]
        assert abs(got[j, 4] - sum(tot) / N) <= 1e-14 * got[j, 4]
    assert counts.tolist() == cnt


def test_empty_bin_is_nan():
    W = np.ones((2, 8))
    got, counts = oracle.wps(W, np.zeros(8), (1.0,))
    assert counts.tolist() == [8, 0]
    assert np.all(np.isnan(got[:, 1])) and np.allclose(got[:, 0], 1.0) and np.allclose(got[:, 2], 1.0)


def test_partition_identity():
    # Eq. global_wps_env_wps: P(w) = sum_b (N_b / N) P(w, b)
    f = synth.zeldovich_field(2048)
    sc = synth.log_scales(2.0, 200.0, 12)
    w, c = oracle.cwt_wps(f, "periodic", "cwgdw", sc, thresholds=(-0.1, 0.0, 0.2))
    assert c.sum() == f.size and np.all(c > 0)
    mix = (w[:, :4] * (c / f.size)).sum(axis=1)
    assert np.max(np.abs(mix - w[:, 4]) / w[:, 4]) < 1e-13


@pytest.mark.parametrize("wav,par", [("morlet", 6.0), ("mexhat", None), ("cwgdw", None)])
def test_tone_global_closed_form(wav, par):
    # periodic cos(w1 b): W = A e^{i w1 b} + B e^{-i w1 b}, A = conj Psi_s(w1)/2,
    # B = conj Psi_s(-w1)/2; over whole periods the cross term averages out,
    # so the global spectrum is |A|^2 + |B|^2
    n, k = 512, 10
    f = np.cos(2 * np.pi * k * np.arange(n) / n)
    sc = np.array([1.5, 3.0, 7.0, 15.0, 40.0])
    w, _ = oracle.cwt_wps(f, "periodic", wav, sc, param=par)
    w1 = 2 * np.pi * k / n

    def aliased(s, w):  # DTFT of the sampled 1/s-scaled wavelet
        return sum(any_psi_hat(wav, par, np.array([s * (w + 2 * np.pi * q)]))[0] for q in range(-6, 7))

    for j, s in enumerate(sc):
        a = 0.25 * abs(aliased(s, w1)) ** 2
        b = 0.25 * abs(aliased(s, -w1)) ** 2
        assert abs(w[j, -1] - (a + b)) <= 1e-10 * (a + b) + 1e-15, (s, w[j, -1], a + b)


def test_zeldovich_field():
    d, d0 = synth.zeldovich_field(4096, return_initial=True)
    # Eq. nonlinear_dens
    assert np.max(np.abs((d + 1) * (1 - 100.0 * d0) - 1)) < 1e-12
    # the variance of the linear field: sum_m 2 P(k_m) / box with
    # P = 2.5e-6 k^-2, k_m = 2 pi m / 48, over m < n/2; a single draw of a
    # red field scatters around it, so only the order of magnitude is pinned
    m = np.arange(1, 2048)
    var = np.sum(2 * 2.5e-6 / (2 * np.pi * m / 48.0) ** 2 / 48.0)
    assert 0.2 < d0.var() / var < 5.0
    assert abs(d0.mean()) < 1e-15
    with pytest.raises(ValueError):
        synth.zeldovich_field(4096, theta=1000.0)


def test_paper_environment_dependence():
    # Sec. 5: the env-WPSs of the initial (Gaussian) field have the amplitude
    # of the global WPS, while at theta = 100 the overdense one lies above
    # and the underdense one below it (FFTCWT, CW-GDW, split at delta = 0)
    n = 8192
    d, d0 = synth.zeldovich_field(n, return_initial=True)
    sc = synth.log_scales(2.0, n / 8, 16)
    w0, _ = oracle.cwt_wps(d0, "periodic", "cwgdw", sc)
    r0 = w0[:, :2] / w0[:, 2:3]
    assert np.all((r0 > 0.75) & (r0 < 1.33)), r0
    w1, _ = oracle.cwt_wps(d, "periodic", "cwgdw", sc)
    r1 = w1[:, :2] / w1[:, 2:3]
    assert np.all(r1[:, 0] < 0.9) and np.all(r1[:, 1] > 1.1), r1
