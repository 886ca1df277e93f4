"""Pins of the spline-method oracle: interpolation coefficients against the
paper's recursive filter (App. C), AE_M / h against Table 3, the exact-target
quadrature against B-spline identities (App. B) and brute-force integration,
and convergence of the spline target to the direct sum as h -> 0."""
import math
from fractions import Fraction

import numpy as np
import pytest
from scipy import integrate

import oracle
from tests import closed_forms as cf

Z1 = math.sqrt(3.0) - 2.0   # pole of the cubic B-spline inverse filter (App. C)
D0 = 6.0


def paper_iir(f, boundary):
    """Eqs. iir_filter_real_a/b with n0 = 1, m = 1, and the initial values of
    Eqs. periodic_initial_a/b or zero_initial_a/b; output d0 * f_1."""
    n = f.size
    nl = int(math.ceil(math.log(1e-16) / math.log(abs(Z1))))
    tem = np.empty(n)
    out = np.empty(n)
    if boundary == "periodic":
        tem[0] = sum(Z1 ** l * f[(0 - l) % n] for l in range(nl + 1))
    else:
        tem[0] = f[0]
    for i in range(1, n):
        tem[i] = f[i] + Z1 * tem[i - 1]
    if boundary == "periodic":
        out[n - 1] = -sum(Z1 ** (l + 1) * tem[(n - 1 + l) % n] for l in range(nl))
    else:
        out[n - 1] = -tem[n - 1] * sum(Z1 ** (2 * l - 1) for l in range(1, (nl + 1) // 2 + 1))
    for i in range(n - 2, -1, -1):
        out[i] = Z1 * (out[i + 1] - tem[i])
    return D0 * out


@pytest.mark.parametrize("bc", ["periodic", "zero"])
def test_spline_coeffs_interpolate(bc):
    rng = np.random.default_rng(2)
    f = rng.standard_normal(200)
    c, c0 = oracle.spline_coeffs(f, bc)
    n = f.size
    for i in range(n):
        acc = 0.0
        for k in range(i - 1, i + 2):
            if bc == "periodic":
                acc += c[k % n] * cf.beta_n(3, i - k)
            else:
                acc += c[k - c0] * cf.beta_n(3, i - k)
        assert abs(acc - f[i]) < 1e-14
    if bc == "zero":
        # zero-extended signal: the same identity holds just outside [0, N)
        for i in (-3, -1, n, n + 2):
            acc = sum(c[k - c0] * cf.beta_n(3, i - k) for k in range(i - 1, i + 2))
            assert abs(acc) < 1e-14


@pytest.mark.parametrize("bc", ["periodic", "zero"])
def test_spline_coeffs_match_paper_recursive_filter(bc):
    rng = np.random.default_rng(4)
    f = rng.standard_normal(300)
    c, c0 = oracle.spline_coeffs(f, bc)
    ref = paper_iir(f, bc)
    got = c if bc == "periodic" else c[-c0:-c0 + f.size]
    assert np.max(np.abs(got - ref)) < 1e-13


def test_h_star_table3(golden):
    # Table 3: h where AE_M(h) = 5e-4 for GDW, CW-GDW, MW (with Table 2's chi)
    chis = golden["table2_chi"]
    hs = golden["table3_h"]
    nds = golden["table3_Nd"]
    for name, fn in (("GDW", cf.psi_gdw), ("CW-GDW", cf.psi_cwgdw), ("MW", cf.psi_mw)):
        h = oracle.h_star(fn, chis[name])
        assert abs(h - hs[name]) < 1.5e-3, (name, h)
        assert round(chis[name] / h - 2) == nds[name]


def test_cbsw_exact_target_identity():
    # CBSW = C (2 beta3(x) - beta3(x+1) - beta3(x-1)) (Table 2) is its own spline
    # approximation at h = 1 (Sec. 3.6): at s = 1, delta = 1 the target is
    # sum_n c[n] sum_k d[k] beta7(x + k - n) (App. B, Eq. two_betas).
    rng = np.random.default_rng(9)
    n = 64
    f = rng.standard_normal(n)
    cn = math.sqrt(30.0 / 31.0)
    d = np.array([-cn, 2 * cn, -cn], dtype=np.complex128)
    x = np.arange(n)
    got = oracle.spline_target_d(f, "periodic", d, 1, 1.0, x)
    c, _ = oracle.spline_coeffs(f, "periodic")
    ref = np.zeros(n)
    for xi in range(n):
        for k in (-1, 0, 1):
            for m in range(xi + k - 4, xi + k + 5):
                ref[xi] += c[m % n] * d[k + 1].real * cf.beta_n(7, xi + k - m)
    assert np.max(np.abs(got.real - ref)) < 1e-14
    assert np.max(np.abs(got.imag)) == 0.0


@pytest.mark.parametrize("wav,par,s,delta", [("mexhat", None, 3.0, 1), ("mexhat", None, 6.5, 2),
                                             ("morlet", 6.0, 9.0, 1), ("dog", 4.0, 7.0, 2)])
def test_spline_target_brute_force_quadrature(wav, par, s, delta):
    # (1/s) int f_c(u) conj(psi_h((u-x)/s)) du by adaptive quadrature with the
    # integer knots as break points, on a tiny zero-boundary signal.
    rng = np.random.default_rng(12)
    n = 12
    f = rng.standard_normal(n)
    h = delta / s
    nd = int(math.ceil(oracle.chi(wav, par) / h - 2.0)) + 2
    d = oracle.wavelet_spline_coeffs(wav, par, h, nd)
    c, c0 = oracle.spline_coeffs(f, "zero")

    def fc(u):
        m0 = int(math.floor(u))
        return sum(c[m - c0] * cf.beta_n(3, u - m) for m in range(m0 - 1, m0 + 3)
                   if 0 <= m - c0 < c.size)
    xs = [0, 5, 11]
    got = oracle.spline_target(f, "zero", wav, s, delta, xs, param=par)
    half = (nd + 2) * delta
    for i, x in enumerate(xs):
        lo, hi = x - half, x + half
        brk = list(range(lo + 1, hi))
        def re(u):
            return fc(u) * np.real(np.conj(oracle.spline_approx(d, 1.0, np.array([(u - x) / delta]))[0]))
        def im(u):
            return fc(u) * np.imag(np.conj(oracle.spline_approx(d, 1.0, np.array([(u - x) / delta]))[0]))
        vr = sum(integrate.quad(re, a, a + 1, epsabs=1e-15, epsrel=1e-13)[0] for a in range(lo, hi)) / s
        vi = sum(integrate.quad(im, a, a + 1, epsabs=1e-15, epsrel=1e-13)[0] for a in range(lo, hi)) / s
        ref = vr + 1j * vi if oracle.is_complex(wav) else vr
        assert abs(got[i] - ref) < 1e-13 * max(1.0, abs(ref)), (x, got[i], ref)
        del brk


def test_spline_target_converges_to_direct_sum():
    # As h -> 0 the spline wavelet tends to psi (error ~ h^4) and, for a smooth
    # signal, the CWT of the spline interpolant tends to the unit-step sum.
    n = 256
    f = np.exp(-(np.arange(n) - 128.0) ** 2 / (2 * 10.0 ** 2))
    s = 40.0
    x = np.arange(0, n, 3)
    ref = oracle.cwt_points(f, "zero", "mexhat", [s], np.zeros(x.size, int), x)
    errs = []
    for delta in (16, 8, 4):
        w = oracle.spline_target(f, "zero", "mexhat", s, delta, x)
        errs.append(np.linalg.norm(w - ref) / np.linalg.norm(ref))
    assert errs[0] > 8 * errs[1] > 0
    assert errs[1] > 4 * errs[2]
    assert errs[2] < 1e-5


def test_beta7_at_integers():
    # beta7 sampled on the integers (App. B, Eq. betan, n = 7): the 7-tap
    # smoothing filter used by the spline method.
    vals = {0: Fraction(151, 315), 1: Fraction(397, 1680), 2: Fraction(1, 42), 3: Fraction(1, 5040)}
    for k, v in vals.items():
        assert abs(cf.beta_n(7, k) - float(v)) < 1e-15
        assert abs(cf.beta_n(7, -k) - float(v)) < 1e-15
    assert abs(cf.beta_n(7, 4.0)) < 1e-15


@pytest.mark.parametrize("delta", [1, 2, 3, 4, 7])
def test_integer_dilation_of_beta3(delta):
    # beta3(x/delta) = delta^-3 sum_j box_delta^{*4}[j + 2(delta-1)] beta3(x - j):
    # the generalised two-scale relation (App. B, Eq. two_scale, delta = 2).
    box = np.ones(delta)
    b4 = np.convolve(np.convolve(box, box), np.convolve(box, box))
    off = 2 * (delta - 1)
    x = np.linspace(-2.5 * delta, 2.5 * delta, 1001)
    rhs = np.zeros_like(x)
    for i, b in enumerate(b4):
        rhs += b * cf.beta_n(3, x - (i - off))
    assert np.max(np.abs(cf.beta_n(3, x / delta) - rhs / delta ** 3)) < 1e-13


@pytest.mark.parametrize("delta", [1, 3, 7, 16])
def test_box_identity_exact(delta):
    # Delta_delta^4 applied after Delta^{-4} equals box_delta^4, exactly on integers
    # (App. B, Eqs. rescaled_finite_diff and inverse_finite_diff).
    rng = np.random.default_rng(delta)
    n = 400
    c = [int(v) for v in rng.integers(-1000, 1000, n)]
    g = list(c)
    for _ in range(4):
        acc = 0
        out = []
        for v in g:
            acc += v
            out.append(acc)
        g = out
    for _ in range(4):
        g = [g[i] - (g[i - delta] if i >= delta else 0) for i in range(n)]
    e = list(c)
    for _ in range(4):
        e = [sum(e[i - j] for j in range(delta) if i - j >= 0) for i in range(n)]
    assert g == e


_HSTAR = {}


def _hstar(wav, par):
    key = (wav, par)
    if key not in _HSTAR:
        _HSTAR[key] = oracle.spline_h_star(wav, par)
    return _HSTAR[key]


@pytest.mark.parametrize("wav,par,scales", [
    ("morlet", 6.0, [0.6, 2.0, 5.5, 8.0, 30.0]),
    ("mexhat", None, [0.5, 1.7, 2.6, 9.0]),
    ("dog", 4.0, [0.8, 3.1, 12.0]),
])
def test_spline_target_tone_closed_form(wav, par, scales):
    # Periodic tones against the Fourier-domain form of the spline target
    # (tests/closed_forms.spline_tone_target): pins the quadrature over the
    # merged knots at steps s h between samples (h* s < 1, knot step h*) and
    # on whole samples (h* s >= 1), including the periodic extension of c.
    n = 256
    hs = _hstar(wav, par)
    x = np.arange(n)
    for s in scales:
        h = oracle.spline_step(hs, s)
        nd = int(math.ceil(oracle.chi(wav, par) / h - 2.0)) + 2
        d = oracle.wavelet_spline_coeffs(wav, par, h, nd)
        for k in (3, 40, 101):
            f = np.cos(2 * np.pi * k * x / n)
            got = oracle.spline_target_scale(f, "periodic", wav, s, hs, x, param=par)
            ref = 0.5 * (cf.spline_tone_target(d, h, s, n, k, x) + cf.spline_tone_target(d, h, s, n, -k, x))
            if not oracle.is_complex(wav):
                assert np.max(np.abs(ref.imag)) < 1e-13
                ref = ref.real
            # |f| <= 1 and int |psi_h(y)| dy is of order one: errors are
            # measured against max(|W|, 1), as for the direct sum's tones
            scale = max(np.max(np.abs(ref)), 1.0)
            assert np.max(np.abs(got - ref)) / scale < 1e-12, (s, k, np.max(np.abs(got - ref)) / scale)


@pytest.mark.parametrize("wav,par,s", [("mexhat", None, 1.9), ("morlet", 6.0, 2.3), ("dog", 4.0, 0.7)])
def test_spline_target_fractional_knots_brute_force(wav, par, s):
    # h* s < 1: the knots of psi_h((u - x)/s) sit every s h* samples, between
    # the integers.  Adaptive quadrature over every piece between consecutive
    # knots of the merged set, on a tiny zero-boundary signal.
    rng = np.random.default_rng(14)
    n = 10
    f = rng.standard_normal(n)
    h = _hstar(wav, par)
    assert h * s < 1.0
    step = s * h
    nd = int(math.ceil(oracle.chi(wav, par) / h - 2.0)) + 2
    d = oracle.wavelet_spline_coeffs(wav, par, h, nd)
    c, c0 = oracle.spline_coeffs(f, "zero")

    def fc(u):
        m0 = int(math.floor(u))
        return sum(c[m - c0] * cf.beta_n(3, u - m) for m in range(m0 - 1, m0 + 3) if 0 <= m - c0 < c.size)

    xs = [0, 4, 9]
    got = oracle.spline_target_h(f, "zero", wav, s, h, xs, param=par)
    for i, x in enumerate(xs):
        half = (nd + 2) * step
        knots = sorted(set([x - half, x + half] + list(range(math.floor(x - half) + 1, math.ceil(x + half)))
                           + [x + step * kk for kk in range(-nd - 2, nd + 3)]))
        knots = [v for v in knots if x - half <= v <= x + half]

        def g(u, part):
            v = fc(u) * np.conj(oracle.spline_approx(d, 1.0, np.array([(u - x) / step]))[0])
            return v.real if part == 0 else v.imag
        vr = sum(integrate.quad(g, a, b, args=(0,), epsabs=1e-16, epsrel=1e-13)[0]
                 for a, b in zip(knots[:-1], knots[1:])) / s
        if oracle.is_complex(wav):
            vi = sum(integrate.quad(g, a, b, args=(1,), epsabs=1e-16, epsrel=1e-13)[0]
                     for a, b in zip(knots[:-1], knots[1:])) / s
            ref = vr + 1j * vi
        else:
            ref = vr
        assert abs(got[i] - ref) < 1e-13 * max(1.0, abs(ref)), (x, got[i], ref)


@pytest.mark.parametrize("wav,par", [("morlet", 6.0), ("mexhat", None), ("dog", 4.0)])
def test_spline_step_keeps_ae_m_at_most_5e4(wav, par):
    # Eq. m02cwt_error: the step of every scale is at most h*, so the
    # wavelet's approximation error stays within the 5e-4 that fixes h*
    # (Sec. 3.6, Table 3), also below s = 1/h* where the knots leave the
    # sample grid.
    hs = _hstar(wav, par)
    ch = oracle.chi(wav, par, oracle.SPLINE_CHI_REL)

    def fn(x):
        return oracle.psi(wav, par, x)
    for s in (0.3, 0.99 / hs, 1.0 / hs, 1.01 / hs, 2.5 / hs, 7.2 / hs, 40.0 / hs):
        h = oracle.spline_step(hs, s)
        assert 0.5 * hs < h <= hs
        assert oracle.ae_m(fn, ch, h) <= 5e-4 * (1 + 1e-6), (s, h)


def test_spline_target_step_equals_integer_knots():
    # The merged-knot quadrature with an integer step reduces to the
    # unit-interval quadrature of oracle_spline_target (same integrand, the
    # pieces coincide).
    rng = np.random.default_rng(21)
    f = rng.standard_normal(300)
    for wav, par, s, delta in (("morlet", 6.0, 20.0, 2), ("mexhat", None, 11.0, 4)):
        x = np.arange(0, 300, 7)
        a = oracle.spline_target(f, "zero", wav, s, delta, x, param=par)
        b = oracle.spline_target_h(f, "zero", wav, s, delta / s, x, param=par)
        assert np.max(np.abs(a - b)) <= 1e-14 * max(1.0, np.max(np.abs(a)))


@pytest.mark.parametrize("wav,par,s", [("mexhat", None, 2.0), ("mexhat", None, 40.0), ("morlet", 6.0, 5.0),
                                       ("morlet", 6.0, 300.0)])
def test_spline_target_shift_invariance_at_large_positions(wav, par, s):
    # A periodic signal of 2^20 samples that repeats every 256 samples has a
    # transform that repeats every 256 positions: the target at x and at
    # x + 256 q (positions near 10^6) must agree to rounding.  Evaluating the
    # splines at absolute positions of 10^6 loses about 1e-10 of every
    # argument; the quadrature works relative to the output position.
    n = 1 << 20
    pat = np.random.default_rng(8).standard_normal(256)
    f = np.tile(pat, n // 256)
    hs = _hstar(wav, par)
    x = np.array([3, 100, 255])
    far = x + 256 * 4000
    a = oracle.spline_target_scale(f, "periodic", wav, s, hs, x, param=par)
    b = oracle.spline_target_scale(f, "periodic", wav, s, hs, far, param=par)
    assert np.max(np.abs(a - b)) <= 1e-14 * max(1.0, np.max(np.abs(a))), np.max(np.abs(a - b))
