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


TABLE2 = [("cbsw", None), ("gdw", None), ("cwgdw", None), ("mw", None)]


def test_table2_time_domain_forms():
    # the oracle's C implementation against the forms of Table 2 written out
    # here (CBSW from the B-spline of App. B)
    x = np.linspace(-14, 14, 4001)
    cn = math.sqrt(30.0 / 31.0)
    cbsw = cn * (2 * cf.beta_n(3, x) - cf.beta_n(3, x + 1) - cf.beta_n(3, x - 1))
    assert np.max(np.abs(oracle.psi("cbsw", None, x) - cbsw)) < 1e-15
    assert np.max(np.abs(oracle.psi("gdw", None, x) - cf.psi_gdw(x))) < 1e-15
    assert np.max(np.abs(oracle.psi("cwgdw", None, x) - cf.psi_cwgdw(x))) < 1e-15
    assert np.max(np.abs(oracle.psi("mw", None, x) - cf.psi_mw(x))) < 1e-15


@pytest.mark.parametrize("wav,par", TABLE2)
def test_table2_unit_norm_zero_mean(wav, par):
    # C_N of Table 2 makes every wavelet unit-norm; all have zero mean.  The
    # CBSW is piecewise cubic with integer knots: integrate piece by piece.
    if wav == "cbsw":
        f2 = lambda t: oracle.psi(wav, par, [t])[0] ** 2
        f1 = lambda t: oracle.psi(wav, par, [t])[0]
        n2 = sum(integrate.quad(f2, a, a + 1, epsabs=1e-16, epsrel=1e-14)[0] for a in range(-3, 3))
        n1 = sum(integrate.quad(f1, a, a + 1, epsabs=1e-16, epsrel=1e-14)[0] for a in range(-3, 3))
        assert abs(n2 - 1.0) < 1e-13 and abs(n1) < 1e-14
        return
    x = np.arange(-40, 40, 1.0 / 1024)
    p = oracle.psi(wav, par, x)
    assert abs(np.sum(np.abs(p) ** 2) / 1024 - 1.0) < 1e-12
    assert abs(np.sum(p)) / np.sum(np.abs(p)) < 1e-13


@pytest.mark.parametrize("wav,par", TABLE2 + [("morlet", 6.0), ("mexhat", None), ("dog", 3.0)])
def test_psi_hat_is_the_fourier_transform_of_psi(wav, par):
    # oracle.psi_hat (the transforms of Table 2) against the numerical
    # transform of the oracle's time-domain wavelet
    w = np.linspace(-14, 14, 57)
    if wav == "cbsw":
        # compact, piecewise cubic: exact per piece with Gauss-Legendre (degree 3 x smooth)
        num = np.array([sum(integrate.quad(lambda t: (oracle.psi(wav, par, [t])[0] * np.exp(-1j * u * t)).real,
                                           a, a + 1, epsabs=1e-16, epsrel=1e-13)[0] for a in range(-3, 3))
                        for u in w])
        assert np.max(np.abs(num - oracle.psi_hat(wav, par, w).real)) < 1e-12
        assert np.max(np.abs(oracle.psi_hat(wav, par, w).imag)) == 0.0
        return
    num = cf.numeric_ft(lambda x: oracle.psi(wav, par, x), w)
    assert np.max(np.abs(num - oracle.psi_hat(wav, par, w))) < 1e-13
    if wav in ("morlet", "mexhat", "dog"):
        assert np.max(np.abs(oracle.psi_hat(wav, par, w) - cf.psi_hat(wav, par, w))) < 1e-14


def test_table2_cbsw_constants(golden):
    # c_w = 1/argmax u |psi^(u)|^2 (0.466094761079290, Table 2 footnote b) and
    # K_psi = (1/2) sqrt(15/62) (27 ln 3 - 32 ln 2) for the CBSW
    neg = lambda u: -u * abs(oracle.psi_hat("cbsw", None, [u])[0]) ** 2
    r = optimize.minimize_scalar(neg, bracket=(1.0, 2.2, 3.5), tol=1e-12)
    assert abs(1.0 / r.x - 0.466094761079290) < 1e-7
    k = integrate.quad(lambda u: oracle.psi_hat("cbsw", None, [u])[0].real / u, 1e-9, 200.0, limit=2000,
                       epsabs=1e-13, epsrel=1e-12)[0]
    k += integrate.quad(lambda u: oracle.psi_hat("cbsw", None, [u])[0].real / u, 200.0, np.inf, limit=500)[0]
    assert abs(k - 0.5 * math.sqrt(15 / 62) * (27 * math.log(3) - 32 * math.log(2))) < 1e-8


@pytest.mark.parametrize("wav,par", [("mw", None), ("gdw", None), ("cbsw", None), ("morlet", 6.0), ("dog", 3.0)])
def test_analytic_form_tone(wav, par):
    # Eq. discrete_CWT_conv on a periodic tone: the DFT has two bins, so the
    # row is e^{i w b} conj psi^(s w)/2 + e^{-i w b} conj psi^(-s w)/2 exactly
    n = 512
    b = np.arange(n)
    for k in (1, 8, 32, 200):
        w = 2 * np.pi * k / n
        f = np.cos(w * b)
        scales = [1.3, 4.0, 37.0, 300.0]
        got = oracle.cwt_analytic(f, "periodic", wav, scales, n, param=par)
        for j, s in enumerate(scales):
            ref = 0.5 * (np.exp(1j * w * b) * np.conj(oracle.psi_hat(wav, par, [s * w])[0])
                         + np.exp(-1j * w * b) * np.conj(oracle.psi_hat(wav, par, [-s * w])[0]))
            if not oracle.is_complex(wav):
                ref = ref.real
            assert np.max(np.abs(got[j] - ref)) < 2e-13, (k, s)


@pytest.mark.parametrize("bc", ["periodic", "zero"])
@pytest.mark.parametrize("wav,par", [("mw", None), ("gdw", None), ("cwgdw", None), ("morlet", 6.0)])
def test_analytic_form_equals_direct_sum_where_aliasing_vanishes(bc, wav, par):
    # At scales where psi^(s w) is negligible beyond |w| = pi the aliasing
    # images vanish and the printed form equals the sampled sum (direct sum,
    # time domain): an independent check of the frequency-domain code.
    rng = np.random.default_rng(3)
    n = 400
    f = rng.standard_normal(n)
    scales = [6.0, 20.0, 90.0]
    m = n if bc == "periodic" else n + int(np.ceil(oracle.chi(wav, par) * 90.0)) + 7
    a = oracle.cwt_analytic(f, bc, wav, scales, m, param=par)
    d = oracle.cwt(f, bc, wav, scales, param=par)
    for j in range(len(scales)):
        assert np.max(np.abs(a[j] - d[j])) < 1e-12 * max(1.0, np.max(np.abs(d[j]))), (scales[j],)


@pytest.mark.parametrize("wav", ["cbsw", "gdw", "cwgdw", "mw"])
def test_table2_psi_hat_closed_forms(wav):
    # the Table 2 transforms of tests/closed_forms against the oracle's
    # (both pinned by the numerical transform of the time-domain wavelets)
    w = np.linspace(-30, 30, 241)
    assert np.max(np.abs(cf.table2_psi_hat(wav, w) - oracle.psi_hat(wav, None, w))) < 1e-14


def test_analytic_f2_closed_form_matches_direct_integral():
    # the frequency-domain quadrature of the continuous CWT of f2 against the
    # Gaussian closed form of the Mexican hat (GDW is the Mexican hat at
    # scale s sqrt(2), times 2^{1/4})
    n = 512
    scales = [2.0, 17.0, 300.0]
    got = cf.analytic_cwt_f2("gdw", None, scales, n)
    sigma = n / 12.0
    for j, s in enumerate(scales):
        ref = 2 ** 0.25 * cf.gaussian_cwt("mexhat", None, s * math.sqrt(2), np.arange(n), n / 2, sigma)
        assert np.max(np.abs(got[j] - ref)) < 1e-13 * max(1.0, np.max(np.abs(ref)))
