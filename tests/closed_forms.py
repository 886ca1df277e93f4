"""Closed forms used by the tests to pin the oracle and the HIP path.

Everything here is derived from the wavelet definitions by hand (Fourier
transforms, Gaussian integrals) and written independently of both the oracle
(which works in the time domain) and the HIP library.

FT convention: psi^(w) = int psi(x) e^{-iwx} dx.  For the 1/s correlation
W(s,b) = (1/s) sum_t f[b+t] conj(psi(t/s)), a tone f[n] = e^{i w1 n} gives
W = e^{i w1 b} conj(Psi_s(w1)), Psi_s(w) = sum_q psi^(s (w + 2 pi q)) by the
Poisson summation formula.
"""
from __future__ import annotations

import math

import numpy as np


def psi_hat(wavelet: str, param: float | None, w) -> np.ndarray:
    """Analytic Fourier transform of the unit-norm mother wavelets."""
    w = np.asarray(w, dtype=np.float64)
    wl = wavelet.lower()
    if wl == "morlet":
        w0 = 6.0 if param is None else float(param)
        c = math.pi ** -0.25 / math.sqrt(1 + math.exp(-w0 * w0) - 2 * math.exp(-0.75 * w0 * w0))
        return c * math.sqrt(2 * math.pi) * (np.exp(-0.5 * (w - w0) ** 2)
                                             - math.exp(-0.5 * w0 * w0) * np.exp(-0.5 * w * w))
    m = 2 if wl in ("mexhat", "mexican_hat") else int(param)
    # DOG(m) = (-1)^{m+1} Gamma(m+1/2)^{-1/2} d^m/dx^m e^{-x^2/2}
    return ((-1) ** (m + 1) / math.sqrt(math.gamma(m + 0.5)) * (1j * w) ** m
            * math.sqrt(2 * math.pi) * np.exp(-0.5 * w * w))


def table2_psi_hat(wavelet: str, w) -> np.ndarray:
    """Fourier transforms of the Table 2 wavelets in the e^{-iwx} convention
    used here.  The table prints them for e^{+ikx}; the real ones are even,
    so only the MW changes, to C_N sqrt(2 pi)(e^{-(w+4)^2/2} - e^{-8} e^{-w^2/2})."""
    w = np.asarray(w, dtype=np.float64)
    wl = wavelet.lower()
    if wl == "cbsw":
        cn = math.sqrt(30 / 31)
        with np.errstate(invalid="ignore", divide="ignore"):
            v = 64 * cn * np.sin(w / 2) ** 6 / w ** 4
        return np.where(w == 0, 0.0, v).astype(np.complex128)
    if wl == "gdw":
        cn = 1 / (18 * math.pi) ** 0.25
        return (8 * math.sqrt(math.pi) * cn * w * w * np.exp(-w * w)).astype(np.complex128)
    if wl in ("cwgdw", "cw-gdw"):
        cn = math.sqrt(8 / (1 + 5 * math.e)) / math.pi ** 0.25
        # cosh and sinh times the Gaussian, written so that no factor overflows
        ch = 0.5 * (np.exp(w - w * w / 2) + np.exp(-w - w * w / 2))
        sh = 0.5 * (np.exp(w - w * w / 2) - np.exp(-w - w * w / 2))
        return (math.sqrt(2 * math.pi) * cn * w * (w * ch - sh)).astype(np.complex128)
    if wl == "mw":
        cn = math.exp(8) / math.sqrt(1 - 2 * math.exp(4) + math.exp(16)) / math.pi ** 0.25
        return (math.sqrt(2 * math.pi) * cn * (np.exp(-(w + 4) ** 2 / 2) - math.exp(-8) * np.exp(-w * w / 2))
                ).astype(np.complex128)
    raise ValueError(wavelet)


def any_psi_hat(wavelet: str, param, w) -> np.ndarray:
    wl = wavelet.lower()
    if wl in ("cbsw", "gdw", "cwgdw", "cw-gdw", "mw"):
        return table2_psi_hat(wl, w)
    return psi_hat(wavelet, param, w).astype(np.complex128)


def analytic_cwt_f1(wavelet: str, param, scales, n: int) -> np.ndarray:
    """Continuous CWT (1/s) int f(u) conj(psi((u - b)/s)) du of the paper's
    f1 = 2 cos x + cos(8x)/2 + sin(32x)/4 sampled at x = 2 pi i / n, with
    positions and scales in samples: each tone e^{i w b} gives
    e^{i w b} conj psi^(s w), with no aliasing (the signal is continuous)."""
    b = np.arange(n)
    out = []
    for s in np.asarray(scales, dtype=np.float64):
        acc = np.zeros(n, dtype=np.complex128)
        for amp, k, kind in ((2.0, 1, "cos"), (0.5, 8, "cos"), (0.25, 32, "sin")):
            w = 2 * np.pi * k / n
            ep = np.exp(1j * w * b) * np.conj(any_psi_hat(wavelet, param, [s * w])[0])
            em = np.exp(-1j * w * b) * np.conj(any_psi_hat(wavelet, param, [-s * w])[0])
            acc += amp * (0.5 * (ep + em) if kind == "cos" else (ep - em) / 2j)
        out.append(acc)
    return np.array(out)


def analytic_cwt_f2(wavelet: str, param, scales, n: int) -> np.ndarray:
    """Continuous CWT of the paper's f2 = exp(-x^2/2) sampled at
    x = -6 + 12 i / n: in samples a Gaussian of width sigma = n/12 centred on
    sample n/2, untruncated.  W(s, b) = (1/2 pi) int g^(w) conj(psi^(s w))
    e^{iwb} dw with g^(w) = sqrt(2 pi) sigma e^{-sigma^2 w^2 / 2} e^{-i w n/2},
    by the trapezoid rule on |w| <= 10/sigma, spectrally accurate: its images
    lie 2 pi / dw samples apart, beyond the transform's support."""
    sigma = n / 12.0
    n0 = n / 2.0
    b = np.arange(n)
    smax = float(np.max(scales))
    span = 8.0 * (n + 40.0 * smax)
    dw = 2 * np.pi / span
    wg = np.arange(-10.0 / sigma, 10.0 / sigma + dw / 2, dw)
    g = math.sqrt(2 * math.pi) * sigma * np.exp(-0.5 * (sigma * wg) ** 2) * np.exp(-1j * wg * n0)
    ker = np.exp(1j * np.outer(b, wg))
    out = []
    for s in np.asarray(scales, dtype=np.float64):
        out.append(ker @ (g * np.conj(any_psi_hat(wavelet, param, s * wg))) * dw / (2 * np.pi))
    return np.array(out)


def psi_aliased(wavelet: str, param: float | None, s: float, w, q: int = 6) -> np.ndarray:
    """Psi_s(w) = sum_{|k|<=q} psi^(s (w + 2 pi k)): the DTFT of the sampled,
    1/s-scaled wavelet."""
    w = np.asarray(w, dtype=np.float64)
    acc = np.zeros(w.shape, dtype=np.complex128)
    for k in range(-q, q + 1):
        acc = acc + psi_hat(wavelet, param, s * (w + 2 * np.pi * k))
    return acc


def tone_cwt(wavelet, param, s, n, k, kind="cos"):
    """Periodic CWT of cos(2 pi k t/n) or sin(2 pi k t/n), t = 0..n-1."""
    w1 = 2 * np.pi * k / n
    b = np.arange(n)
    ep = np.exp(1j * w1 * b) * np.conj(psi_aliased(wavelet, param, s, w1))
    em = np.exp(-1j * w1 * b) * np.conj(psi_aliased(wavelet, param, s, -w1))
    if kind == "cos":
        return 0.5 * (ep + em)
    return (ep - em) / 2j


def gaussian_cwt(wavelet, param, s, b, x0, sigma, images=0):
    """Continuous CWT (1/s) int f(x) conj(psi((x-b)/s)) dx of
    f = exp(-(x-x0)^2 / (2 sigma^2)).  With a^2 = sigma^2 + s^2, tau = b - x0:

    DOG(m):  (-1)^{m+1} Gamma(m+1/2)^{-1/2} sqrt(2 pi) sigma s^m a^{-m-1}
             He_m(tau/a) e^{-tau^2/(2a^2)}
    Morlet:  C sqrt(2 pi) sigma/a e^{-tau^2/(2a^2)}
             [exp(i w0 tau s/a^2 - w0^2 sigma^2/(2 a^2)) - e^{-w0^2/2}]

    With images=q > 0 (Morlet only) the Poisson images |k| <= q are added, so
    the result is the unit-step sum over integer x rather than the integral.
    """
    b = np.asarray(b, dtype=np.float64)
    a2 = sigma * sigma + s * s
    a = math.sqrt(a2)
    tau = b - x0
    g = np.exp(-tau * tau / (2 * a2))
    wl = wavelet.lower()
    if wl == "morlet":
        w0 = 6.0 if param is None else float(param)
        c = math.pi ** -0.25 / math.sqrt(1 + math.exp(-w0 * w0) - 2 * math.exp(-0.75 * w0 * w0))

        def gauss(alpha):
            # (1/s) int exp(-(u+tau)^2/(2 sigma^2) - u^2/(2 s^2) - i alpha u) du
            return math.sqrt(2 * math.pi) * sigma / a * np.exp(
                -tau * tau / (2 * a2) + 1j * alpha * tau * s * s / a2
                - alpha * alpha * sigma * sigma * s * s / (2 * a2))
        acc = 0
        for q in range(-images, images + 1):
            # image q of the Poisson sum (positions b are integers)
            acc = acc + gauss(w0 / s + 2 * np.pi * q) - math.exp(-0.5 * w0 * w0) * gauss(2 * np.pi * q)
        return c * acc
    m = 2 if wl in ("mexhat", "mexican_hat") else int(param)
    z = tau / a
    he = {1: z, 2: z * z - 1, 3: z ** 3 - 3 * z, 4: z ** 4 - 6 * z * z + 3}[m]
    return ((-1) ** (m + 1) / math.sqrt(math.gamma(m + 0.5)) * math.sqrt(2 * math.pi) * sigma
            * s ** m * a ** (-m - 1) * he * g)


# Wavelets of the paper's Table 2 (used only to pin the oracle's helpers).

def psi_gdw(x):
    x = np.asarray(x, dtype=np.float64)
    return (18 * math.pi) ** -0.25 * (2 - x * x) * np.exp(-x * x / 4)


def psi_cwgdw(x):
    x = np.asarray(x, dtype=np.float64)
    cn = math.sqrt(8 / (1 + 5 * math.e)) / math.pi ** 0.25
    return cn * ((1 - x * x) * np.cos(x) - x * np.sin(x)) * np.exp((1 - x * x) / 2)


def psi_mw(x):
    x = np.asarray(x, dtype=np.float64)
    cn = math.exp(8) / math.sqrt(1 - 2 * math.exp(4) + math.exp(16)) / math.pi ** 0.25
    return cn * (np.exp(-4j * x) - math.exp(-8)) * np.exp(-x * x / 2)


def beta_n(n: int, x):
    """Centered B-spline of degree n by the explicit truncated-power formula
    beta^n(x) = (1/n!) sum_k (-1)^k C(n+1,k) (x + (n+1)/2 - k)_+^n.
    Evaluated at -|x| (the B-spline is even), where only the first half of
    the terms is active, and set to 0 outside the support; this keeps the
    cancellation in the alternating sum small."""
    x = -np.abs(np.asarray(x, dtype=np.float64))
    out = np.zeros_like(x)
    for k in range(n + 2):
        t = x + (n + 1) / 2 - k
        out += (-1) ** k * math.comb(n + 1, k) * np.where(t > 0, t, 0.0) ** n
    return np.where(x > -(n + 1) / 2, out / math.factorial(n), 0.0)


def numeric_ft(psi_fn, w, half=14.0, step=1.0 / 512):
    """psi^(w) by the trapezoid rule on [-half, half] (spectrally accurate
    for Gaussian-decaying wavelets)."""
    x = np.arange(-half, half + step / 2, step)
    px = psi_fn(x)
    w = np.atleast_1d(np.asarray(w, dtype=np.float64))
    out = np.empty(w.size, dtype=np.complex128)
    for i0 in range(0, w.size, 256):
        ww = w[i0:i0 + 256]
        out[i0:i0 + 256] = (np.exp(-1j * np.outer(ww, x)) @ px) * step
    return out


def bspline3_hat(nu):
    """Fourier transform of the cubic B-spline: (sin(nu/2) / (nu/2))^4."""
    nu = np.asarray(nu, dtype=np.float64)
    return np.sinc(nu / (2 * np.pi)) ** 4


def spline_tone_target(d, h, s, n, k, x):
    """Spline-method target for the periodic tone f[t] = e^{2 pi i k t/n}:
    W(x) = (1/s) int f_c(u) conj(psi_h((u - x)/s)) du in the Fourier domain.

    The periodic spline coefficients are c[t] = f[t] / B(w), B(w) =
    (4 + 2 cos w)/6 the sampled cubic B-spline's symbol, w = 2 pi k/n; by
    Poisson summation f_c(u) = sum_q A_q e^{i nu_q u} with nu_q = w + 2 pi q,
    A_q = bhat(nu_q) / B(w), bhat the B-spline's transform.  The spline
    wavelet psi_h(y) = sum_j d[j] beta3(y/h - j) has the transform
    h D(nu h) bhat(nu h), D(theta) = sum_j d[j] e^{-i j theta}.  Hence
    W(x) = sum_q A_q e^{i nu_q x} conj(h D(s h nu_q) bhat(s h nu_q)).
    The terms fall off like q^-8; |q| <= 600 is kept."""
    d = np.asarray(d, dtype=np.complex128)
    nd = (d.size - 1) // 2
    j = np.arange(-nd, nd + 1)
    w = 2 * np.pi * k / n
    q = np.arange(-600, 601)
    nu = w + 2 * np.pi * q
    amp = bspline3_hat(nu) / ((4.0 + 2.0 * math.cos(w)) / 6.0)
    th = s * h * nu
    dsym = np.exp(-1j * np.outer(th, j)) @ d
    hat = h * dsym * bspline3_hat(th)
    coef = amp * np.conj(hat)
    x = np.asarray(x, dtype=np.float64)
    return np.exp(1j * np.outer(x, nu)) @ coef
