"""FP64 CPU oracle for the multi-scale 1D CWT.

TEST INFRASTRUCTURE ONLY.  Only the tests, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this package.  It shares no
code with the HIP library and never calls it; the only thing both sides use
is the input generator package ``synth``.

Contents
--------
* ``cwt`` / ``cwt_points`` -- the direct O(N * chi * s) sum (Sec. 3,
  Eq. discreteCWT with the 1/s correlation normalisation), in plain C with
  OpenMP (``cwt_oracle.c``).
* ``cwt_spectral_rows`` -- the same sum row by row as an FFT circular
  convolution with the sampled wavelet (scipy.fft as a library primitive),
  for full-length references at sizes the direct sum cannot reach.
* ``psi`` / ``chi`` -- the mother wavelets in the time domain (Morlet, DOG,
  and the CBSW, GDW, CW-GDW and MW of Table 2); ``psi_hat`` their Fourier
  transforms.
* ``cwt_analytic`` -- Eq. discrete_CWT_conv as printed (Sec. 3.1): the bare
  transform of the wavelet at the DFT bins, with numpy FFTs.
* Spline method (Sec. 3.3, App. B, App. C):
  ``spline_coeffs`` (cubic-spline interpolation coefficients c of the
  signal, Eq. interp_coeffs, by a banded solve or an FFT division -- not by
  the recursive filter of App. C), ``wavelet_spline_coeffs`` (d of Eq.
  beta3_wavelet_approx_m02), ``ae_m`` (Eq. m02cwt_error), ``h_star`` (the
  step where AE_M = 5e-4, Sec. 3.6), ``spline_delta`` and
  ``spline_step`` (the reading of the step per scale),
  ``spline_target`` / ``spline_target_h`` / ``spline_target_scale`` (the
  exact CWT of the spline interpolant with the spline wavelet, by
  Gauss-Legendre quadrature over the merged knots of both splines).
* A19 method (Sec. 3.4): ``psi2`` (second derivative), ``a19_pieces`` /
  ``a19_eval`` (the piecewise-cubic wavelet of Eqs. piecewise_polys_psi and
  3rd_derivative_wavelet), ``ae_a`` (Eq. a19cwt_error), ``a19_nchi`` and
  ``a19_target`` (the exact CWT of f_c with that wavelet).
* V97 method (Sec. 3.2): ``wavelet_cw``, ``v97_wmax`` (1.34 c_w), ``q12_filter``
  (Eq. q_12), ``v97_q`` (Eq. qj), ``v97_kernel`` (the approximated wavelet of
  Eqs. beta3_wavelet_approx and pj), ``v97_points`` (the unit-step sum with
  it) and ``ae_v`` (Eq. v97cwt_error).
* Wavelet power spectra (Sec. 5): ``wps_bins``, ``wps`` (Eqs. env_wps and
  global_wps: means of |W|^2 per environment bin and over all positions)
  and ``cwt_wps``.

Readings of the paper that this oracle takes (each is repeated in the
design notes): scales and positions are in samples; the canonical result is
the 1/s correlation with conj(psi) as a unit-step sum; chi is the radius
where |psi| falls below ``rel`` times its maximum; the spline step is
h_s = delta_s / s with delta_s = floor(h* s) whenever h* s >= 1 (every knot
of the wavelet spline on a sample), and h* itself below that (knots between
samples, as the paper keeps h fixed at every scale).

Parity pins: every function above is pinned in ``tests/test_oracle_*.py``
against closed forms, printed constants of Tables 2 and 3, brute force and
invariants.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cwt_oracle.c")
_LIB = os.path.join(_HERE, "libcwt_oracle.so")

MORLET, DOG, CBSW, GDW, CWGDW = 0, 1, 2, 3, 4
PERIODIC, ZERO = 0, 1


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc (-O2, OpenMP, IEEE semantics)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared",
                               "-ffp-contract=off", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        lp = ctypes.POINTER(ctypes.c_long)
        ip = ctypes.POINTER(ctypes.c_int)
        lib.oracle_chi.restype = ctypes.c_double
        lib.oracle_chi.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double]
        lib.oracle_psi.argtypes = [ctypes.c_int, ctypes.c_double, dp, ctypes.c_long, dp, dp]
        lib.oracle_cwt.argtypes = [dp, ctypes.c_long, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                   dp, ctypes.c_int, ctypes.c_double, dp, dp, ctypes.c_int]
        lib.oracle_cwt_points.argtypes = [dp, ctypes.c_long, ctypes.c_int, ctypes.c_int,
                                          ctypes.c_double, dp, ctypes.c_int, ctypes.c_double,
                                          ip, lp, ctypes.c_long, dp, dp, ctypes.c_int]
        lib.oracle_spline_target.argtypes = [dp, ctypes.c_long, ctypes.c_long, dp, dp,
                                             ctypes.c_long, ctypes.c_long, ctypes.c_double,
                                             lp, ctypes.c_long, dp, dp, ctypes.c_int]
        lib.oracle_spline_target_step.argtypes = [dp, ctypes.c_long, ctypes.c_long, dp, dp,
                                                  ctypes.c_long, ctypes.c_double, ctypes.c_double,
                                                  lp, ctypes.c_long, dp, dp, ctypes.c_int]
        lib.oracle_psi2.argtypes = [ctypes.c_int, ctypes.c_double, dp, ctypes.c_long, dp, dp]
        lib.oracle_kernel_sum.argtypes = [dp, ctypes.c_long, ctypes.c_int, dp, dp, ctypes.c_long, lp,
                                          ctypes.c_long, dp, dp, ctypes.c_int]
        lib.oracle_pp_target.argtypes = [dp, ctypes.c_long, ctypes.c_long, dp, dp, ctypes.c_long,
                                         ctypes.c_double, ctypes.c_double, ctypes.c_double, lp,
                                         ctypes.c_long, dp, dp, ctypes.c_int]
        _lib = lib
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _wavelet(wavelet: str, param: float | None):
    w = wavelet.lower()
    if w == "morlet":
        return MORLET, 6.0 if param is None else float(param)
    if w in ("mexhat", "mexican_hat"):
        return DOG, 2.0
    if w == "dog":
        return DOG, 2.0 if param is None else float(param)
    # Table 2: the MW is C_N (e^{-4ix} - e^{-8}) e^{-x^2/2}, the Morlet form
    # with omega0 = -4
    table2 = {"cbsw": (CBSW, 0.0), "gdw": (GDW, 0.0), "cwgdw": (CWGDW, 0.0), "cw-gdw": (CWGDW, 0.0),
              "mw": (MORLET, -4.0)}
    if w in table2:
        return table2[w]
    raise ValueError(wavelet)


def is_complex(wavelet: str) -> bool:
    return wavelet.lower() in ("morlet", "mw")


def psi_hat(wavelet: str, param: float | None, u) -> np.ndarray:
    """Fourier transform psi^(u) = int psi(x) e^{-iux} dx of the unit-norm
    wavelets (the transforms of Table 2, in this sign convention):
    Morlet(w0) C sqrt(2 pi)(e^{-(u-w0)^2/2} - e^{-w0^2/2} e^{-u^2/2});
    DOG(m) (-1)^{m+1} Gamma(m+1/2)^{-1/2} (iu)^m sqrt(2 pi) e^{-u^2/2};
    CBSW 64 C_N sin^6(u/2)/u^4; GDW 8 sqrt(pi) C_N u^2 e^{-u^2};
    CW-GDW sqrt(2 pi) C_N u (u cosh u - sinh u) e^{-u^2/2}."""
    import math
    kind, p = _wavelet(wavelet, param)
    u = np.asarray(u, dtype=np.float64)
    if kind == MORLET:
        c = math.pi ** -0.25 / math.sqrt(1 + math.exp(-p * p) - 2 * math.exp(-0.75 * p * p))
        return (c * math.sqrt(2 * math.pi) * (np.exp(-0.5 * (u - p) ** 2)
                                              - math.exp(-0.5 * p * p) * np.exp(-0.5 * u * u))).astype(np.complex128)
    if kind == DOG:
        m = int(p)
        return ((-1) ** (m + 1) / math.sqrt(math.gamma(m + 0.5)) * (1j * u) ** m
                * math.sqrt(2 * math.pi) * np.exp(-0.5 * u * u))
    if kind == CBSW:
        cn = math.sqrt(30.0 / 31.0)
        with np.errstate(invalid="ignore", divide="ignore"):
            v = 64.0 * cn * np.sin(0.5 * u) ** 6 / u ** 4
        return np.where(u == 0.0, 0.0, v).astype(np.complex128)
    if kind == GDW:
        cn = (18 * math.pi) ** -0.25
        return (8 * math.sqrt(math.pi) * cn * u * u * np.exp(-u * u)).astype(np.complex128)
    cn = math.sqrt(8 / (1 + 5 * math.e)) / math.pi ** 0.25
    # (u cosh u - sinh u) e^{-u^2/2} = ((u - 1) e^{u - u^2/2} + (u + 1) e^{-u - u^2/2}) / 2,
    # which stays finite where cosh u alone would overflow
    v = 0.5 * ((u - 1) * np.exp(u - 0.5 * u * u) + (u + 1) * np.exp(-u - 0.5 * u * u))
    return (math.sqrt(2 * math.pi) * cn * u * v).astype(np.complex128)


def cwt_analytic(f, boundary: str, wavelet: str, scales, m: int, param: float | None = None) -> np.ndarray:
    """The FFT method as written in Sec. 3.1, Eq. discrete_CWT_conv: with
    the signal's DFT on m points (the signal zero-padded to m samples for a
    zero boundary; m = N for a periodic one), each scale's row is the
    inverse DFT of F[k] conj(psi^(s w_k)), w_k = 2 pi k / m the signed
    frequency of bin k in [-m/2, m/2), the bare transform of the wavelet
    (no aliasing images).  The Nyquist bin of an even m takes the mean of
    psi^(s pi) and psi^(-s pi).  [S, N] array, complex for complex
    wavelets."""
    f = np.asarray(f, dtype=np.float64)
    n = f.size
    if boundary == "periodic" and m != n:
        raise ValueError("a periodic signal is transformed on its own length")
    x = np.zeros(m)
    x[:n] = f
    F = np.fft.fft(x)
    k = np.fft.fftfreq(m) * m          # signed bins, Nyquist at -m/2
    w = 2 * np.pi * k / m
    out = []
    for s in np.asarray(scales, dtype=np.float64):
        ph = psi_hat(wavelet, param, s * w)
        if m % 2 == 0:
            ph[m // 2] = 0.5 * (psi_hat(wavelet, param, [-s * np.pi])[0] + psi_hat(wavelet, param, [s * np.pi])[0])
        row = np.fft.ifft(F * np.conj(ph))[:n]
        out.append(row if is_complex(wavelet) else row.real)
    return np.array(out)


def psi(wavelet: str, param: float | None, x) -> np.ndarray:
    kind, p = _wavelet(wavelet, param)
    x = np.ascontiguousarray(np.asarray(x, dtype=np.float64).ravel())
    re = np.empty_like(x)
    im = np.empty_like(x)
    _load().oracle_psi(kind, p, _dp(x), x.size, _dp(re), _dp(im))
    return re + 1j * im if kind == MORLET else re


def chi(wavelet: str, param: float | None = None, rel: float = 1e-17) -> float:
    kind, p = _wavelet(wavelet, param)
    return float(_load().oracle_chi(kind, p, rel))


def cwt(f, boundary: str, wavelet: str, scales, param: float | None = None,
        rel: float = 1e-17, nthreads: int = 0) -> np.ndarray:
    """Full direct-sum transform, [S, N] complex128 (Morlet) or float64."""
    kind, p = _wavelet(wavelet, param)
    f = np.ascontiguousarray(np.asarray(f, dtype=np.float64))
    sc = np.ascontiguousarray(np.asarray(scales, dtype=np.float64))
    n, s = f.size, sc.size
    re = np.empty((s, n))
    im = np.empty((s, n)) if kind == MORLET else None
    bc = PERIODIC if boundary == "periodic" else ZERO
    _load().oracle_cwt(_dp(f), n, bc, kind, p, _dp(sc), s, rel, _dp(re),
                       _dp(im) if im is not None else None, nthreads)
    return re + 1j * im if im is not None else re


def cwt_points(f, boundary: str, wavelet: str, scales, scale_idx, pos,
               param: float | None = None, rel: float = 1e-17, nthreads: int = 0) -> np.ndarray:
    """Direct-sum transform at the outputs (scale_idx[i], pos[i])."""
    kind, p = _wavelet(wavelet, param)
    f = np.ascontiguousarray(np.asarray(f, dtype=np.float64))
    sc = np.ascontiguousarray(np.asarray(scales, dtype=np.float64))
    si = np.ascontiguousarray(np.asarray(scale_idx, dtype=np.int32))
    ps = np.ascontiguousarray(np.asarray(pos, dtype=np.int64))
    re = np.empty(si.size)
    im = np.empty(si.size) if kind == MORLET else None
    bc = PERIODIC if boundary == "periodic" else ZERO
    _load().oracle_cwt_points(_dp(f), f.size, bc, kind, p, _dp(sc), sc.size, rel,
                              si.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                              ps.ctypes.data_as(ctypes.POINTER(ctypes.c_long)), si.size,
                              _dp(re), _dp(im) if im is not None else None, nthreads)
    return re + 1j * im if im is not None else re


def cwt_spectral_rows(f, boundary: str, wavelet: str, scales, param: float | None = None,
                      rel: float = 1e-17, workers: int = -1, rows=None):
    """The same transform as ``cwt`` (the unit-step sum of Sec. 3, Eq.
    discreteCWT), one row at a time, as a circular convolution done with
    FFTs: W_j = f_ext (*) r_j with r_j[-t] = conj(psi(t / s_j)) / s_j for
    |t| <= floor(chi s_j) (time-domain samples, wrapped onto the period N for
    a periodic signal; zero-padded to a length M >= N + T_max + 1 for a zero
    boundary, where the circular convolution equals the linear one on
    [0, N)).  Yields (j, row) for the requested rows (all by default).  For
    full-length checks where the direct sum is too slow; pinned against
    ``cwt`` in the tests."""
    import scipy.fft as sf
    kind, p = _wavelet(wavelet, param)
    f = np.asarray(f, dtype=np.float64)
    n = f.size
    sc = np.asarray(scales, dtype=np.float64)
    ch = chi(wavelet, param, rel)
    rows = range(sc.size) if rows is None else rows
    tmax = max(int(np.floor(ch * sc[j])) for j in rows)
    if boundary == "periodic":
        m = n
    else:
        m = sf.next_fast_len(n + tmax + 1)
    fp = np.zeros(m)
    fp[:n] = f
    cplx = kind == MORLET
    ff = sf.fft(fp, workers=workers) if cplx else sf.rfft(fp, workers=workers)
    for j in rows:
        s = float(sc[j])
        t = np.arange(-int(np.floor(ch * s)), int(np.floor(ch * s)) + 1)
        k = np.conj(psi(wavelet, param, t / s)) / s
        r = np.zeros(m, dtype=np.complex128 if cplx else np.float64)
        np.add.at(r, (-t) % m, k)       # images wrap onto the period
        if cplx:
            w = sf.ifft(ff * sf.fft(r, workers=workers), workers=workers)[:n]
        else:
            w = sf.irfft(ff * sf.rfft(r, workers=workers), n=m, workers=workers)[:n]
        yield j, w


# --------------------------------------------------------------------------
# Spline method (Sec. 3.3, App. B, App. C).

def beta3(x) -> np.ndarray:
    """Cubic B-spline (App. B, Eq. betan with n = 3)."""
    a = np.abs(np.asarray(x, dtype=np.float64))
    out = np.zeros_like(a)
    m1 = a < 1.0
    m2 = (a >= 1.0) & (a < 2.0)
    out[m1] = 2.0 / 3.0 - a[m1] ** 2 + 0.5 * a[m1] ** 3
    out[m2] = (2.0 - a[m2]) ** 3 / 6.0
    return out


def _solve_b3(rhs: np.ndarray) -> np.ndarray:
    """Solve (c[n-1] + 4 c[n] + c[n+1]) / 6 = rhs[n] with c = 0 just outside
    the array (the caller extends the array far enough that this boundary
    value is irrelevant)."""
    from scipy.linalg import solve_banded
    n = rhs.size
    ab = np.zeros((3, n))
    ab[0, 1:] = 1.0 / 6.0
    ab[1, :] = 4.0 / 6.0
    ab[2, :-1] = 1.0 / 6.0
    if np.iscomplexobj(rhs):
        return solve_banded((1, 1), ab, rhs.real) + 1j * solve_banded((1, 1), ab, rhs.imag)
    return solve_banded((1, 1), ab, rhs)


def spline_coeffs(f, boundary: str, pad: int = 48):
    """Cubic-spline interpolation coefficients c of the samples f (Eq.
    interp_coeffs): sum_k c[k] beta3(n - k) = f[n] for every integer n.

    periodic: returns (c, 0), c of length N, by dividing the DFT of f by the
    DFT of the sampled cubic B-spline, (4 + 2 cos w)/6.
    zero: f is zero outside [0, N); returns (c, -pad) with c on
    [-pad, N + pad) from a banded solve on that range (the neglected tail is
    below (2 - sqrt 3)^pad relative)."""
    f = np.asarray(f, dtype=np.float64)
    n = f.size
    if boundary == "periodic":
        w = 2 * np.pi * np.arange(n) / n
        c = np.fft.ifft(np.fft.fft(f) / ((4.0 + 2.0 * np.cos(w)) / 6.0)).real
        return c, 0
    rhs = np.zeros(n + 2 * pad)
    rhs[pad:pad + n] = f
    return _solve_b3(rhs), -pad


def wavelet_spline_coeffs(wavelet: str, param: float | None, h: float, nd: int):
    """d[k], k in [-nd, nd]: cubic-spline interpolation coefficients of the
    samples psi(h k) (Eq. beta3_wavelet_approx_m02, computed as Eq.
    interp_coeffs).  The samples are taken on a range 40 wider than chi/h on
    each side; the solution is then truncated to [-nd, nd]."""
    ch = chi(wavelet, param, 1e-17)
    kmax = max(nd, int(np.ceil(ch / h))) + 40
    k = np.arange(-kmax, kmax + 1)
    smp = psi(wavelet, param, h * k)
    d = _solve_b3(smp)
    mid = kmax
    return d[mid - nd: mid + nd + 1]


def spline_approx(d, h: float, x) -> np.ndarray:
    """psi_h(x) = sum_k d[k] beta3(x/h - k), d indexed from -nd."""
    d = np.asarray(d)
    nd = (d.size - 1) // 2
    x = np.asarray(x, dtype=np.float64)
    y = x / h
    out = np.zeros(x.shape, dtype=d.dtype)
    k0 = np.floor(y).astype(np.int64) - 1
    for j in range(4):
        k = k0 + j
        ok = (k >= -nd) & (k <= nd)
        kk = np.clip(k, -nd, nd)
        out = out + np.where(ok, d[kk + nd] * beta3(y - k), 0.0)
    return out


def ae_m(psi_fn, chi_: float, h: float, npts: int = 20001) -> float:
    """AE_M(h) of Eq. m02cwt_error: sum_n |psi(x_n) - psi_h(x_n)| /
    sum_n |psi(x_n)| on npts uniform points of [-chi, chi]; psi_h uses the
    exact (untruncated) spline interpolation of psi(h k)."""
    kmax = int(np.ceil(chi_ / h)) + 40
    k = np.arange(-kmax, kmax + 1)
    d = _solve_b3(psi_fn(h * k))
    x = np.linspace(-chi_, chi_, npts)
    approx = spline_approx(d, h, x)
    ex = psi_fn(x)
    return float(np.sum(np.abs(ex - approx)) / np.sum(np.abs(ex)))


def h_star(psi_fn, chi_: float, target: float = 5e-4) -> float:
    """Largest-error-below-target step: scan h upward in 0.005 steps until
    AE_M exceeds the target, then bisect the bracketing interval."""
    lo = 0.005
    h = lo
    while ae_m(psi_fn, chi_, h) < target:
        lo = h
        h += 0.005
        if h > 3.0:
            raise RuntimeError("AE_M never reaches the target")
    hi = h
    for _ in range(60):
        mid = 0.5 * (lo + hi)
        if ae_m(psi_fn, chi_, mid) < target:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


SPLINE_CHI_REL = 1e-14   # Table 2 truncates the non-compact wavelets near 1e-14


def spline_h_star(wavelet: str, param: float | None = None) -> float:
    """h* of a supported wavelet: AE_M = 5e-4 on [-chi, chi], chi the
    radius where |psi| < 1e-14 max|psi|."""
    ch = chi(wavelet, param, SPLINE_CHI_REL)
    return h_star(lambda x: psi(wavelet, param, x), ch)


def spline_delta(hstar: float, s: float) -> int:
    """Knot spacing of the spline wavelet at scale s in whole samples:
    delta = floor(h* s) when h* s >= 1 (step h_s = delta / s <= h*), and 0
    below that, where the step is h* itself and the knots s h* k fall
    between samples."""
    return int(np.floor(hstar * s)) if hstar * s >= 1.0 else 0


def spline_step(hstar: float, s: float) -> float:
    """Step h_s of the spline wavelet at scale s: delta / s with delta =
    floor(h* s) >= 1, else h*.  Either way h_s <= h*, so the wavelet's
    approximation error AE_M (Eq. m02cwt_error) stays at or below 5e-4."""
    d = spline_delta(hstar, s)
    return d / s if d >= 1 else float(hstar)


def spline_target(f, boundary: str, wavelet: str, s: float, delta: int, x,
                  param: float | None = None, nthreads: int = 0) -> np.ndarray:
    """Exact CWT of the spline interpolant f_c with the spline wavelet
    psi_h, h = delta/s, at integer positions x (array)."""
    h = delta / s
    ch = chi(wavelet, param, 1e-17)
    nd = int(np.ceil(ch / h - 2.0)) + 2
    d = wavelet_spline_coeffs(wavelet, param, h, nd)
    w = spline_target_d(f, boundary, d, delta, s, x, nthreads)
    return w if is_complex(wavelet) else w.real


def spline_target_h(f, boundary: str, wavelet: str, s: float, h: float, x,
                    param: float | None = None, nthreads: int = 0) -> np.ndarray:
    """Exact CWT of the spline interpolant f_c with the spline wavelet
    psi_h at any step h (knots of psi_h((u - x)/s) every s h samples, not
    necessarily integers), at integer positions x."""
    ch = chi(wavelet, param, 1e-17)
    nd = int(np.ceil(ch / h - 2.0)) + 2
    d = wavelet_spline_coeffs(wavelet, param, h, nd)
    w = spline_target_step_d(f, boundary, d, s * h, s, x, nthreads)
    return w if is_complex(wavelet) else w.real


def spline_target_scale(f, boundary: str, wavelet: str, s: float, hstar: float, x,
                        param: float | None = None, nthreads: int = 0) -> np.ndarray:
    """The spline method's target at scale s for a wavelet of step h*: the
    step h_s of ``spline_step`` (whole-sample knots above s = 1/h*, step h*
    below)."""
    d = spline_delta(hstar, s)
    if d >= 1:
        return spline_target(f, boundary, wavelet, s, d, x, param=param, nthreads=nthreads)
    return spline_target_h(f, boundary, wavelet, s, hstar, x, param=param, nthreads=nthreads)


def _spline_ext(f, boundary: str, half: float):
    """Spline coefficients of f extended over `half` samples beyond each
    end: (c, c0) with c[i] the coefficient of sample c0 + i."""
    n = f.size
    if boundary == "periodic":
        c, _ = spline_coeffs(f, "periodic")
        reps = int(np.ceil(half / n)) + 1
        return np.ascontiguousarray(np.tile(c, 2 * reps + 1)), -reps * n
    cext, c0 = spline_coeffs(f, "zero", pad=max(48, int(np.ceil(half)) + 8))
    return np.ascontiguousarray(cext, dtype=np.float64), c0


def spline_target_step_d(f, boundary: str, d, step: float, s: float, x,
                         nthreads: int = 0) -> np.ndarray:
    """Same as ``spline_target_h`` with explicit wavelet coefficients d[k],
    k in [-nd, nd], and the knot step s h given in samples (complex128)."""
    f = np.asarray(f, dtype=np.float64)
    d = np.asarray(d, dtype=np.complex128)
    nd = (d.size - 1) // 2
    cext, c0 = _spline_ext(f, boundary, (nd + 2) * step + 4)
    dr = np.ascontiguousarray(d.real)
    di = np.ascontiguousarray(d.imag)
    xs = np.ascontiguousarray(np.asarray(x, dtype=np.int64))
    re = np.empty(xs.size)
    im = np.empty(xs.size)
    _load().oracle_spline_target_step(_dp(cext), c0, cext.size, _dp(dr), _dp(di), nd, float(step),
                                      float(s), xs.ctypes.data_as(ctypes.POINTER(ctypes.c_long)),
                                      xs.size, _dp(re), _dp(im), nthreads)
    return re + 1j * im


def spline_target_d(f, boundary: str, d, delta: int, s: float, x,
                    nthreads: int = 0) -> np.ndarray:
    """Same as ``spline_target`` with explicit wavelet coefficients d[k],
    k in [-nd, nd] (complex128 result)."""
    f = np.asarray(f, dtype=np.float64)
    n = f.size
    d = np.asarray(d, dtype=np.complex128)
    nd = (d.size - 1) // 2
    half = (nd + 2) * delta + 4
    if boundary == "periodic":
        c, _ = spline_coeffs(f, "periodic")
        reps = int(np.ceil(half / n)) + 1
        cext = np.tile(c, 2 * reps + 1)
        c0 = -reps * n
    else:
        cext, c0 = spline_coeffs(f, "zero")
    cext = np.ascontiguousarray(cext, dtype=np.float64)
    dr = np.ascontiguousarray(d.real)
    di = np.ascontiguousarray(d.imag)
    xs = np.ascontiguousarray(np.asarray(x, dtype=np.int64))
    re = np.empty(xs.size)
    im = np.empty(xs.size)
    _load().oracle_spline_target(_dp(cext), c0, cext.size, _dp(dr), _dp(di), nd, int(delta),
                                 float(s), xs.ctypes.data_as(ctypes.POINTER(ctypes.c_long)),
                                 xs.size, _dp(re), _dp(im), nthreads)
    return re + 1j * im


# --------------------------------------------------------------------------
# A19CWT (Sec. 3.4).

def psi2(wavelet: str, param: float | None, x) -> np.ndarray:
    """Second derivative of a smooth wavelet, analytic (the A19 method
    needs it, Eq. 3rd_derivative_wavelet)."""
    kind, p = _wavelet(wavelet, param)
    if kind == CBSW:
        raise ValueError("the CBSW is not twice differentiable everywhere")
    x = np.ascontiguousarray(np.asarray(x, dtype=np.float64).ravel())
    re = np.empty_like(x)
    im = np.empty_like(x)
    _load().oracle_psi2(kind, p, _dp(x), x.size, _dp(re), _dp(im))
    return re + 1j * im if kind == MORLET else re


def a19_pieces(wavelet: str, param: float | None, h: float, chi_: float):
    """The wavelet of the A19 method (Sec. 3.4, Eqs. piecewise_polys_psi and
    3rd_derivative_wavelet) on the knots h j: its third derivative is
    constant on each piece, 6 alpha_3 = (e[j+1] - e[j]) / h with e[j] the
    second derivative of psi at h j for |j| <= J = ceil(chi / h) and zero at
    j = -(J+1) and J+1; the function, its first and its second derivative
    vanish at -(J+1) h, and the lower-order coefficients of each piece follow
    from continuity.  Returns (coefficients [pieces, 4] of t^0..t^3, y0, h)
    over the 2J + 2 pieces of [-(J+1) h, (J+1) h)."""
    import math
    J = int(np.ceil(chi_ / h - 1e-9))
    j = np.arange(-J - 1, J + 2)
    e = psi2(wavelet, param, h * j).astype(np.complex128)
    e[0] = 0.0
    e[-1] = 0.0
    npieces = 2 * J + 2
    coef = np.zeros((npieces, 4), dtype=np.complex128)
    # value and slope at the start of each piece: with a3 = (e[k+1] - e[k]) /
    # (6 h), a piece adds (e[k] + e[k+1]) h / 2 to the slope and
    # dv h + (2 e[k] + e[k+1]) h^2 / 6 to the value; each is summed exactly
    # rounded (math.fsum) over all earlier pieces, since psi'' exceeds psi by
    # about w0^2 and plain running sums keep 1e-12 of psi's scale
    dterms_r, dterms_i, vterms_r, vterms_i = [], [], [], []
    for k in range(npieces):
        dv = complex(math.fsum(dterms_r), math.fsum(dterms_i))
        v = complex(math.fsum(vterms_r), math.fsum(vterms_i))
        a3 = (e[k + 1] - e[k]) / (6.0 * h)
        coef[k] = (v, dv, e[k] / 2.0, a3)
        dt = (e[k] + e[k + 1]) * h / 2.0
        vt_a = dv * h
        vt_b = (2.0 * e[k] + e[k + 1]) * h * h / 6.0
        dterms_r.append(dt.real)
        dterms_i.append(dt.imag)
        vterms_r += [vt_a.real, vt_b.real]
        vterms_i += [vt_a.imag, vt_b.imag]
    return coef, -(J + 1) * h, h


def a19_eval(coef, y0: float, h: float, y) -> np.ndarray:
    """The piecewise cubic of ``a19_pieces`` at the points y."""
    y = np.asarray(y, dtype=np.float64)
    k = np.floor((y - y0) / h).astype(np.int64)
    ok = (k >= 0) & (k < coef.shape[0])
    kk = np.clip(k, 0, coef.shape[0] - 1)
    t = y - y0 - h * kk
    c = coef[kk]
    val = ((c[..., 3] * t + c[..., 2]) * t + c[..., 1]) * t + c[..., 0]
    return np.where(ok, val, 0.0)


def ae_a(wavelet: str, param: float | None, chi_: float, nchi: int, npts: int = 20001) -> float:
    """AE_A(N_chi) of Eq. a19cwt_error: the error of the piecewise cubic of
    Eq. piecewise_polys_psi on the 2 N_chi pieces of [-chi, chi], read as
    the cubic spline interpolating psi at the knots -chi + k chi / N_chi
    (the first of the method's two approximations; the second, Eq.
    3rd_derivative_wavelet, is in ``a19_pieces``).  With this reading the
    N_chi that Table 3 prints give AE_A of 6e-4 to 7e-4, "roughly" 5e-4."""
    return ae_m(lambda x: psi(wavelet, param, x), chi_, chi_ / nchi, npts)


def a19_nchi(wavelet: str, param: float | None, chi_: float, target: float = 5e-4) -> int:
    """Smallest N_chi whose AE_A is at most the target (Sec. 3.6)."""
    n = 2
    while ae_a(wavelet, param, chi_, n) > target:
        n += 1
        if n > 4000:
            raise RuntimeError("AE_A never reaches the target")
    return n


def a19_hstar(wavelet: str, param: float | None = None) -> float:
    """Knot step chi / N_chi of the A19 wavelet, chi where |psi| falls below
    1e-14 of its maximum (as for the spline method)."""
    ch = chi(wavelet, param, SPLINE_CHI_REL)
    return ch / a19_nchi(wavelet, param, ch)


def a19_target(f, boundary: str, wavelet: str, s: float, h: float, x,
               param: float | None = None, nthreads: int = 0) -> np.ndarray:
    """The A19 transform at scale s with the wavelet's knots every h: by Eq.
    a19cwt_03 (integration by parts undone) the CWT of the spline
    interpolant f_c with psi_pp, (1/s) int f_c(u) conj(psi_pp((u - x)/s)) du,
    integrated exactly over the merged knots."""
    f = np.asarray(f, dtype=np.float64)
    ch = chi(wavelet, param, SPLINE_CHI_REL)
    coef, y0, hh = a19_pieces(wavelet, param, h, ch)
    half = abs(y0) * s + 4
    cext, c0 = _spline_ext(f, boundary, half)
    ar = np.ascontiguousarray(coef.real.ravel())
    ai = np.ascontiguousarray(coef.imag.ravel())
    xs = np.ascontiguousarray(np.asarray(x, dtype=np.int64))
    re = np.empty(xs.size)
    im = np.empty(xs.size)
    _load().oracle_pp_target(_dp(cext), c0, cext.size, _dp(ar), _dp(ai), coef.shape[0], float(y0), float(hh),
                             float(s), xs.ctypes.data_as(ctypes.POINTER(ctypes.c_long)), xs.size, _dp(re), _dp(im),
                             nthreads)
    w = re + 1j * im
    return w if is_complex(wavelet) else w.real


def a19_target_scale(f, boundary: str, wavelet: str, s: float, hstar: float, x,
                     param: float | None = None, nthreads: int = 0) -> np.ndarray:
    """The A19 target at scale s for the plan step h* = chi / N_chi, with
    the step per scale of ``spline_step``."""
    return a19_target(f, boundary, wavelet, s, spline_step(hstar, s), x, param=param, nthreads=nthreads)


# --------------------------------------------------------------------------
# V97CWT (Sec. 3.2).

def wavelet_cw(wavelet: str, param: float | None = None) -> float:
    """c_w = 1 / argmax |u| |psi^(u)|^2 (Table 2: the ratio of scale to
    pseudo frequency), by a scan and a bounded scalar maximisation."""
    from scipy import optimize
    u = np.linspace(-40.0, 40.0, 160001)
    g = np.abs(u) * np.abs(psi_hat(wavelet, param, u)) ** 2
    u0 = u[int(np.argmax(g))]
    r = optimize.minimize_scalar(lambda v: -abs(v) * abs(psi_hat(wavelet, param, [v])[0]) ** 2,
                                 bounds=(u0 - 1e-3, u0 + 1e-3), method="bounded",
                                 options={"xatol": 1e-14})
    return 1.0 / abs(r.x)


def v97_wmax(wavelet: str, param: float | None = None) -> float:
    """w~_max = 1.34 c_w (Sec. 3.6; Table 3 prints these values)."""
    return 1.34 * wavelet_cw(wavelet, param)


def q12_filter(K: int = 60) -> np.ndarray:
    """Taps |k| <= K of q12, the convolution inverse of the quartic B-spline
    sampled on the integers, (1, 76, 230, 76, 1) / 384 (Eq. q_12), from a
    banded solve with a unit impulse on a range 4K wide."""
    from scipy.linalg import solve_banded
    n = 4 * K + 1
    ab = np.zeros((5, n))
    for d, v in zip(range(5), (1.0, 76.0, 230.0, 76.0, 1.0)):
        ab[d, :] = v / 384.0
    rhs = np.zeros(n)
    rhs[2 * K] = 1.0
    q = solve_banded((2, 2), ab, rhs)
    return q[K:3 * K + 1]


def v97_level(s: float, wmax: float):
    """Octave level i and sub-level factor r in [1, 2) of s = 2^i r / w~_max."""
    t = s * wmax
    if t < 1.0 - 1e-6:
        raise ValueError("V97 scales start at 1 / w~_max")
    i = max(0, int(np.floor(np.log2(max(t, 1.0)))))
    while i > 0 and 2.0 ** i > t:
        i -= 1
    while 2.0 ** (i + 1) <= t:
        i += 1
    return i, t / 2.0 ** i


def v97_q(wavelet: str, param: float | None, r: float, wmax: float, nq: int) -> np.ndarray:
    """q(k) = int_{k-1/2}^{k+1/2} psi(w~_max y / r) dy, |k| <= nq (Eq. qj),
    by adaptive quadrature per cell (cut at the knots of the CBSW)."""
    from scipy import integrate
    cplx = is_complex(wavelet)
    out = np.zeros(2 * nq + 1, dtype=np.complex128)
    knots = [r * m / wmax for m in range(-3, 4)] if wavelet.lower() == "cbsw" else []
    for k in range(-nq, nq + 1):
        cuts = sorted({k - 0.5, k + 0.5} | {y for y in knots if k - 0.5 < y < k + 0.5})
        re = im = 0.0
        for a, b in zip(cuts[:-1], cuts[1:]):
            re += integrate.quad(lambda y: psi(wavelet, param, [wmax * y / r])[0].real, a, b,
                                 epsabs=1e-17, epsrel=1e-14)[0]
            if cplx:
                im += integrate.quad(lambda y: psi(wavelet, param, [wmax * y / r])[0].imag, a, b,
                                     epsabs=1e-17, epsrel=1e-14)[0]
        out[k + nq] = re + 1j * im
    return out


def v97_kernel(wavelet: str, param: float | None, s: float, wmax: float | None = None):
    """Taps t = -T..T of the V97 approximation of the scaled wavelet at scale
    s = 2^i r / w~_max (Eqs. beta3_wavelet_approx and pj):
    psi_v(t) = sum_k p(k) beta3(t / 2^i - k), p = q * q12, returned as
    conj(psi_v(t)) / s (the weights of the unit-step sum), and T."""
    wmax = v97_wmax(wavelet, param) if wmax is None else wmax
    i, r = v97_level(s, wmax)
    ch = chi(wavelet, param, 1e-17)
    nq = int(np.ceil(ch * r / wmax + 0.5))
    q = v97_q(wavelet, param, r, wmax, nq)
    q12 = q12_filter(60)
    p = np.convolve(q, q12)                     # index k + nq + 60
    kp = nq + 60
    step = 2 ** i
    T = step * (kp + 2)
    t = np.arange(-T, T + 1)
    y = t / step
    acc = np.zeros(t.size, dtype=np.complex128)
    k0 = np.floor(y).astype(np.int64) - 1
    for jj in range(4):
        kk = k0 + jj
        ok = (kk >= -kp) & (kk <= kp)
        acc += np.where(ok, p[np.clip(kk + kp, 0, p.size - 1)] * beta3(y - kk), 0.0)
    return np.conj(acc) / s, T


def v97_points(f, boundary: str, wavelet: str, s: float, pos, param: float | None = None,
               wmax: float | None = None, nthreads: int = 0) -> np.ndarray:
    """The V97 transform at scale s and positions pos: the unit-step sum of
    Sec. 3, Eq. discreteCWT, with the wavelet replaced by its V97
    approximation (``v97_kernel``)."""
    k, T = v97_kernel(wavelet, param, s, wmax)
    f = np.ascontiguousarray(np.asarray(f, dtype=np.float64))
    kr = np.ascontiguousarray(k.real)
    ki = np.ascontiguousarray(k.imag)
    ps = np.ascontiguousarray(np.asarray(pos, dtype=np.int64))
    re = np.empty(ps.size)
    im = np.empty(ps.size)
    bc = PERIODIC if boundary == "periodic" else ZERO
    _load().oracle_kernel_sum(_dp(f), f.size, bc, _dp(kr), _dp(ki), T,
                              ps.ctypes.data_as(ctypes.POINTER(ctypes.c_long)), ps.size, _dp(re), _dp(im),
                              nthreads)
    w = re + 1j * im
    return w if is_complex(wavelet) else w.real


def ae_v(wavelet: str, param: float | None, w: float, npts: int = 20001) -> float:
    """AE_V(w) of Eq. v97cwt_error: how well sum_m p(m) beta3(x - m) with
    p = q * q12 (q the cell integrals of psi(w x)) matches psi(w x), on npts
    points of the wavelet's support |x| <= chi / w."""
    ch = chi(wavelet, param, 1e-14)
    nq = int(np.ceil(ch / w + 0.5))
    q = v97_q(wavelet, param, 1.0, w, nq)
    p = np.convolve(q, q12_filter(60))
    kp = nq + 60
    x = np.linspace(-ch / w, ch / w, npts)
    k0 = np.floor(x).astype(np.int64) - 1
    approx = np.zeros(x.size, dtype=np.complex128)
    for jj in range(4):
        kk = k0 + jj
        approx += p[kk + kp] * beta3(x - kk)
    ex = psi(wavelet, param, w * x)
    return float(np.sum(np.abs(ex - approx)) / np.sum(np.abs(ex)))


# ---------------------------------------------------------------------------
# Wavelet power spectra (Sec. 5)

def wps_bins(env, thresholds) -> np.ndarray:
    """Environment bin of every position: the number of thresholds t with
    env >= t (a NaN value compares false everywhere: bin 0)."""
    env = np.asarray(env, dtype=np.float64)
    k = np.zeros(env.shape, dtype=np.int64)
    for t in thresholds:
        k += env >= t
    return k


def wps(W, env, thresholds):
    """Wavelet power spectra of the coefficients W [S, N] (Sec. 5):
    column b < nb of the [S, nb + 1] result is the environment-dependent
    spectrum (Eq. env_wps), the mean of |W|^2 over the positions of bin b
    (NaN when the bin is empty); the last column is the global spectrum
    (Eq. global_wps), the mean over all positions.  Also returns the bin
    sizes N_b."""
    p2 = np.abs(np.asarray(W)) ** 2
    k = wps_bins(env, thresholds)
    nb = len(thresholds) + 1
    out = np.empty((p2.shape[0], nb + 1))
    counts = np.array([np.count_nonzero(k == b) for b in range(nb)], dtype=np.int64)
    for b in range(nb):
        out[:, b] = p2[:, k == b].mean(axis=1) if counts[b] else np.nan
    out[:, nb] = p2.mean(axis=1)
    return out, counts


def cwt_wps(f, boundary: str, wavelet: str, scales, env=None, thresholds=(0.0,),
            param: float | None = None, spectral: bool = False):
    """``wps`` of the canonical transform of f (the direct sum ``cwt``, or
    ``cwt_spectral_rows`` when spectral); env defaults to f itself."""
    if spectral:
        W = np.array([w for _, w in cwt_spectral_rows(f, boundary, wavelet, scales, param)])
    else:
        W = cwt(f, boundary, wavelet, scales, param)
    return wps(W, f if env is None else env, thresholds)
