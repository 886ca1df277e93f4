"""Pins of the direct-sum oracle: closed forms (tones, Gaussians), Parseval
with an independent DFT, brute force with explicit periodic images, and the
periodic/zero relation."""
import math

import numpy as np
import pytest

import oracle
from tests import closed_forms as cf

SCALES = [2.0, 3.7, 10.0, 50.0, 230.0]   # 230 * chi > 512: several periodic wraps


@pytest.mark.parametrize("wav,par", [("morlet", 6.0), ("mexhat", None), ("dog", 3.0), ("dog", 4.0)])
@pytest.mark.parametrize("kind", ["cos", "sin"])
def test_tone_closed_form_periodic(wav, par, kind):
    n = 512
    for k in (1, 17, 90, 250):
        t = np.arange(n)
        f = np.cos(2 * np.pi * k * t / n) if kind == "cos" else np.sin(2 * np.pi * k * t / n)
        w = oracle.cwt(f, "periodic", wav, SCALES, param=par)
        for j, s in enumerate(SCALES):
            ref = cf.tone_cwt(wav, par, s, n, k, kind)
            if not oracle.is_complex(wav):
                assert np.max(np.abs(ref.imag)) < 1e-12
                ref = ref.real
            scale = max(np.max(np.abs(ref)), 1.0)   # |f| <= 1 and sum_t |psi(t/s)|/s ~ 1
            assert np.max(np.abs(w[j] - ref)) / scale < 1e-13, (k, s)


@pytest.mark.parametrize("wav,par", [("mexhat", None), ("dog", 4.0), ("dog", 1.0), ("morlet", 6.0), ("morlet", 4.0)])
def test_gaussian_closed_form_zero_boundary(wav, par):
    n, x0 = 2048, 1000.3
    for sigma in (8.0, 12.0):
        f = np.exp(-(np.arange(n) - x0) ** 2 / (2 * sigma ** 2))
        scales = [2.0, 7.0, 50.0, 120.0]
        w = oracle.cwt(f, "zero", wav, scales, param=par)
        for j, s in enumerate(scales):
            ref = cf.gaussian_cwt(wav, par, s, np.arange(n), x0, sigma, images=3)
            assert np.max(np.abs(w[j] - ref)) / max(np.max(np.abs(ref)), 1.0) < 1e-13, (sigma, s)


@pytest.mark.parametrize("wav,par", [("morlet", 6.0), ("dog", 3.0), ("mexhat", None)])
def test_parseval_per_scale(wav, par):
    rng = np.random.default_rng(1)
    n = 256
    f = rng.standard_normal(n)
    scales = [0.8, 2.0, 9.3, 40.0]
    w = oracle.cwt(f, "periodic", wav, scales, param=par)
    # DFT by an explicit O(N^2) matrix product
    m = np.arange(n)
    F = np.exp(-2j * np.pi * np.outer(m, m) / n) @ f
    for j, s in enumerate(scales):
        lhs = np.sum(np.abs(w[j]) ** 2)
        rhs = np.sum(np.abs(F) ** 2 * np.abs(cf.psi_aliased(wav, par, s, 2 * np.pi * m / n)) ** 2) / n
        assert abs(lhs - rhs) / rhs < 1e-12


def _neumaier(vals):
    s = 0.0
    c = 0.0
    for v in vals:
        t = s + v
        if abs(s) >= abs(v):
            c += (s - t) + v
        else:
            c += (v - t) + s
        s = t
    return s + c


@pytest.mark.parametrize("bc", ["periodic", "zero"])
@pytest.mark.parametrize("wav,par", [("morlet", 6.0), ("dog", 3.0)])
def test_brute_force_tiny(bc, wav, par):
    # Sum over samples (and explicit periodic images p) instead of over lags.
    rng = np.random.default_rng(7)
    n = 24
    f = rng.standard_normal(n)
    scales = [0.6, 1.5, 4.0, 11.0]
    w = oracle.cwt(f, bc, wav, scales, param=par)
    ch = oracle.chi(wav, par, 1e-17)
    for j, s in enumerate(scales):
        pmax = int(math.ceil(ch * s / n)) + 2 if bc == "periodic" else 0
        for b in range(n):
            terms = []
            for p in range(-pmax, pmax + 1):
                t = np.arange(n) + p * n - b
                terms.append(f * np.conj(oracle.psi(wav, par, t / s)) / s)
            terms = np.concatenate(terms)
            ref = _neumaier(terms.real) + 1j * _neumaier(terms.imag)
            got = w[j, b]
            assert abs(got - ref) <= 1e-14 * max(1.0, abs(ref)), (s, b)


def test_zero_boundary_equals_padded_periodic():
    rng = np.random.default_rng(3)
    n = 300
    f = rng.standard_normal(n)
    scales = [2.0, 6.0, 15.0]
    wz = oracle.cwt(f, "zero", "morlet", scales)
    pad = int(math.ceil(oracle.chi("morlet", 6.0) * 15.0)) + 1
    fp = np.concatenate([f, np.zeros(2 * pad)])
    wp = oracle.cwt(fp, "periodic", "morlet", scales)
    assert np.max(np.abs(wz - wp[:, :n])) < 1e-15


def test_pairwise_sum_accuracy_long_kernel():
    # Long sums (T ~ 2700) against math.fsum on the same products
    rng = np.random.default_rng(11)
    n = 6000
    f = rng.standard_normal(n) + 1.0
    s = 300.0
    pos = np.array([0, 1234, 5999])
    got = oracle.cwt_points(f, "periodic", "mexhat", [s], np.zeros(3, int), pos)
    ch = oracle.chi("mexhat", None, 1e-17)
    tmax = int(math.floor(ch * s))
    t = np.arange(-tmax, tmax + 1)
    k = oracle.psi("mexhat", None, t / s) / s
    for i, b in enumerate(pos):
        ref = math.fsum(f[(b + t) % n] * k)
        assert abs(got[i] - ref) < 1e-15 * np.sum(np.abs(f[(b + t) % n] * k))


def test_points_match_full():
    rng = np.random.default_rng(5)
    n = 512
    f = rng.standard_normal(n)
    scales = [2.0, 20.0, 100.0]
    full = oracle.cwt(f, "zero", "morlet", scales)
    si = rng.integers(0, 3, 50)
    ps = rng.integers(0, n, 50)
    pts = oracle.cwt_points(f, "zero", "morlet", scales, si, ps)
    assert np.array_equal(pts, full[si, ps])


def test_icwt_single_integral_reconstruction():
    # Eq. real_ICWT in the 1/s form: f = mean(f) + (1/K) int_0^inf W(s,.) ds/s
    # for the even Mexican hat, K = sqrt(2 pi)/sqrt(Gamma(5/2)).  A smooth
    # periodic signal (2 and 5 cycles) and dense log scales on [1, 2e4]; the
    # cut of the s-integral at s = 1 (needed so the periodic images of the
    # sampled wavelet stay negligible) bounds the accuracy near 1e-3, which is
    # enough to catch any wrong normalisation power or constant.
    n = 512
    t = np.arange(n)
    f = 1.5 + np.cos(2 * np.pi * 2 * t / n) + 0.4 * np.sin(2 * np.pi * 5 * t / n)
    u = np.linspace(np.log(1.0), np.log(20000.0), 500)
    w = oracle.cwt(f, "periodic", "mexhat", np.exp(u), rel=1e-12)
    k = math.sqrt(2 * math.pi) / math.sqrt(math.gamma(2.5))
    rec = f.mean() + np.trapezoid(w, u, axis=0) / k
    assert np.max(np.abs(rec - f)) < 2e-3


@pytest.mark.parametrize("bc", ["periodic", "zero"])
@pytest.mark.parametrize("wav,par", [("morlet", 6.0), ("mexhat", None), ("dog", 3.0)])
def test_spectral_rows_equal_direct_sum(bc, wav, par):
    # the FFT form of the sum (full-length references) against the direct sum,
    # with scales whose support wraps the period several times
    rng = np.random.default_rng(5)
    n = 300
    f = rng.standard_normal(n) + 0.2
    scales = [0.8, 2.0, 9.3, 40.0, 230.0]
    ref = oracle.cwt(f, bc, wav, scales, param=par)
    for j, row in oracle.cwt_spectral_rows(f, bc, wav, scales, param=par):
        scale = max(np.max(np.abs(ref[j])), 1e-3 * np.max(np.abs(ref)))
        assert np.max(np.abs(row - ref[j])) / scale < 1e-12, (j, np.max(np.abs(row - ref[j])) / scale)


def test_spectral_rows_tone_closed_form():
    n = 1000
    t = np.arange(n)
    f = np.cos(2 * np.pi * 37 * t / n)
    scales = [1.1, 6.0, 75.0, 400.0]
    for j, row in oracle.cwt_spectral_rows(f, "periodic", "morlet", scales, param=6.0):
        ref = cf.tone_cwt("morlet", 6.0, scales[j], n, 37, "cos")
        assert np.max(np.abs(row - ref)) < 1e-13
