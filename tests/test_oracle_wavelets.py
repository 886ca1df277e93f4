"""Pins of the oracle's mother wavelets against the paper's Table 2 and
against closed forms (unit norm, admissibility, Fourier transforms)."""
import math

import numpy as np
import pytest
from scipy import integrate, optimize

import oracle
from tests import closed_forms as cf

WAVELETS = [("morlet", 6.0), ("morlet", 4.0), ("mexhat", None), ("dog", 1.0),
            ("dog", 3.0), ("dog", 4.0)]


@pytest.mark.parametrize("wav,par", WAVELETS)
def test_unit_l2_norm(wav, par):
    x = np.arange(-40, 40, 1.0 / 1024)
    p = oracle.psi(wav, par, x)
    assert abs(np.sum(np.abs(p) ** 2) / 1024 - 1.0) < 1e-12


@pytest.mark.parametrize("wav,par", WAVELETS)
def test_zero_mean(wav, par):
    # psi^(0) = 0 (admissibility; for Morlet this needs the correction term)
    x = np.arange(-40, 40, 1.0 / 1024)
    p = oracle.psi(wav, par, x)
    assert abs(np.sum(p)) / np.sum(np.abs(p)) < 1e-13


def test_morlet4_is_conjugate_of_paper_mw():
    # Table 2 MW: C_N (e^{-4ix} - e^{-8}) e^{-x^2/2}, C_N = e^8/sqrt(1-2e^4+e^16)/pi^{1/4}
    x = np.linspace(-8, 8, 2001)
    assert np.max(np.abs(oracle.psi("morlet", 4.0, x) - np.conj(cf.psi_mw(x)))) < 1e-15


def test_mexhat_textbook_form():
    x = np.linspace(-10, 10, 2001)
    ref = 2.0 / (math.sqrt(3.0) * math.pi ** 0.25) * (1 - x * x) * np.exp(-x * x / 2)
    assert np.max(np.abs(oracle.psi("mexhat", None, x) - ref)) < 1e-15


@pytest.mark.parametrize("wav,par", WAVELETS)
def test_time_domain_matches_fourier_transform(wav, par):
    w = np.linspace(-14, 14, 57)
    num = cf.numeric_ft(lambda x: oracle.psi(wav, par, x), w)
    ana = cf.psi_hat(wav, par, w)
    assert np.max(np.abs(num - ana)) < 1e-13


def test_mw_k_psi_table2(golden):
    # K_psi = int_0^inf psi^(k)/k dk with psi^ from the oracle's time-domain MW
    def integrand(k):
        return (cf.numeric_ft(lambda x: oracle.psi("morlet", 4.0, x), [k])[0] / k).real
    val, _ = integrate.quad(integrand, 1e-12, 16.0, epsabs=1e-14, epsrel=1e-13, limit=200)
    assert abs(val - golden["table2_mw_K"]["value"]) < 1e-10


def test_mw_cw_table2(golden):
    def neg(u):
        ph = cf.numeric_ft(lambda x: oracle.psi("morlet", 4.0, x), [u])[0]
        return -u * abs(ph) ** 2
    r = optimize.minimize_scalar(neg, bracket=(2.0, 4.0, 7.0), tol=1e-12)
    assert abs(1.0 / r.x - golden["table2_mw_cw"]["value"]) < 1e-7


def test_mexhat_k_closed_form():
    # K = int_0^inf psi^(k)/k dk = sqrt(2 pi)/sqrt(Gamma(5/2)) for the Mexican hat
    def integrand(k):
        return (cf.numeric_ft(lambda x: oracle.psi("mexhat", None, x), [k])[0] / k).real
    val, _ = integrate.quad(integrand, 1e-12, 16.0, epsabs=1e-14, epsrel=1e-13, limit=200)
    assert abs(val - math.sqrt(2 * math.pi) / math.sqrt(math.gamma(2.5))) < 1e-10


@pytest.mark.parametrize("wav,par", WAVELETS)
@pytest.mark.parametrize("rel", [1e-17, 1e-9])
def test_chi_radius(wav, par, rel):
    ch = oracle.chi(wav, par, rel)
    xs = np.linspace(0, 40, 400001)
    a = np.abs(oracle.psi(wav, par, xs))
    mx = a.max()
    assert np.all(a[xs > ch] < rel * mx)
    assert np.any(a[(xs > ch - 0.01) & (xs <= ch)] >= rel * mx * 0.5)


def test_paper_wavelet_helpers_table2(golden):
    # The Table 2 helpers used by the AE_M pins are themselves pinned:
    # unit norm, and c_w/K of GDW and CW-GDW against their printed values.
    x = np.arange(-40, 40, 1.0 / 1024)
    for fn in (cf.psi_gdw, cf.psi_cwgdw, cf.psi_mw):
        assert abs(np.sum(np.abs(fn(x)) ** 2) / 1024 - 1) < 1e-12

    def kpsi(fn):
        f = lambda k: (cf.numeric_ft(lambda t: np.conj(fn(t)), [k])[0] / k).real
        return integrate.quad(f, 1e-12, 16.0, epsabs=1e-14, epsrel=1e-13, limit=200)[0]
    assert abs(kpsi(cf.psi_gdw) - 2 * (8 * math.pi / 9) ** 0.25) < 1e-10
    assert abs(kpsi(cf.psi_cwgdw) - 4 * math.pi ** 0.25 / math.sqrt(1 + 5 * math.e)) < 1e-10

    def cw(fn, br):
        neg = lambda u: -u * abs(cf.numeric_ft(fn, [u])[0]) ** 2
        return 1.0 / optimize.minimize_scalar(neg, bracket=br, tol=1e-12).x
    assert abs(cw(cf.psi_gdw, (0.5, 1.1, 2.0)) - 2 / math.sqrt(5)) < 1e-7
    assert abs(cw(cf.psi_cwgdw, (1.5, 2.3, 3.5)) - golden["table2_cwgdw_cw"]["value"]) < 1e-7
