"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module only draws inputs.  It holds none of the transform's arithmetic:
no wavelet, no spectrum of a wavelet, no scale-dependent step.  Both the HIP
path and the CPU oracle consume what it returns.

Workloads (all seeded with numpy's PCG64):

* ``tones_noise`` -- a periodic three-tone signal plus white noise.  The
  paper's own accuracy tests use a periodic sum of tones (Sec. 4, Eq.
  signal_f1); the tone frequencies here are 40, 300 and 900 cycles per 4096
  samples, scaled with the length.
* ``lognormal_field`` -- a non-periodic 1D density-like field
  delta = exp(g - sigma^2/2) - 1 with g a Gaussian random field of power
  spectrum P(k) ~ k^-1.5 exp(-(k/k_c)^2).  It stands in for the 1D density
  fields of Sec. 5 (Eq. nonlinear_dens), which are also synthetic; the
  paper's own field parameters are not given in the text.
* ``log_scales`` -- scales a * (b/a)^(j/(S-1)), j = 0..S-1, both ends
  included (the paper discretises scales evenly in log, Sec. 3.1).
* ``paper_f1`` / ``paper_f2`` / ``paper_scale_grid`` -- the test signals of
  Sec. 4 (Eqs. signal_f1, signal_f2) and the level/sub-level scale grid of
  Sec. 3.1, for the paper's accuracy comparison.
* ``zeldovich_field`` -- the 1D Zel'dovich density field of Sec. 5 (Eq.
  nonlinear_dens), delta + 1 = 1 / (1 - theta delta_0), delta_0 a periodic
  Gaussian field with P(k) = A k^-2, A = 2.5e-6, on a box of length
  ``box`` (k = 2 pi n / box).  The paper takes the box length and grid from
  another work; here the box is a parameter, 48 by default, which keeps
  theta = 100 before the first orbit crossing (max theta delta_0 < 1).
* ``batch_specs`` / ``request_stream`` -- many uneven instances and a
  Poisson request stream for the batched and served forms.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

SEED_SMALL = 20230209
SEED_FIELD_1M = 20230210
SEED_FIELD_4M = 20230211
SEED_BATCH = 20230212
SEED_SERVE = 20230213
SEED_ZELDOVICH = 20230214


def tones_noise(n: int, seed: int = SEED_SMALL, noise: float = 0.1) -> np.ndarray:
    """sin(2pi*40x) + 0.5 sin(2pi*300x) + 0.3 sin(2pi*900x) + N(0, noise^2),
    x = i/n, with the tone counts scaled by n/4096 (rounded)."""
    rng = np.random.default_rng(seed)
    x = np.arange(n, dtype=np.float64) / n
    k = [max(1, round(c * n / 4096)) for c in (40, 300, 900)]
    f = (np.sin(2 * np.pi * k[0] * x) + 0.5 * np.sin(2 * np.pi * k[1] * x)
         + 0.3 * np.sin(2 * np.pi * k[2] * x))
    return f + noise * rng.standard_normal(n)


def lognormal_field(n: int, seed: int = SEED_FIELD_1M, sigma_g: float = 1.0,
                    slope: float = -1.5, kc_per_n: float | None = None) -> np.ndarray:
    """Lognormal field on n samples.

    g is drawn on a periodic box of 2n samples (so the kept half is not
    periodic), with integer box wavenumbers k, P(k) = k^slope exp(-(k/k_c)^2),
    k_c = 2 * kc_per_n (default kc_per_n = n/8 cycles per n samples), the k=0
    mode set to zero; g is standardised to mean 0 and std sigma_g and
    delta = exp(g - sigma_g^2/2) - 1."""
    rng = np.random.default_rng(seed)
    box = 2 * n
    if kc_per_n is None:
        kc_per_n = n / 8
    kc = 2.0 * kc_per_n
    k = np.arange(box // 2 + 1, dtype=np.float64)
    p = np.zeros_like(k)
    p[1:] = k[1:] ** slope * np.exp(-(k[1:] / kc) ** 2)
    modes = (rng.standard_normal(k.size) + 1j * rng.standard_normal(k.size)) * np.sqrt(p / 2)
    modes[0] = 0.0
    modes[-1] = modes[-1].real
    g = np.fft.irfft(modes, n=box)[:n]
    g = (g - g.mean()) / g.std() * sigma_g
    return np.exp(g - 0.5 * sigma_g ** 2) - 1.0


def zeldovich_field(n: int, theta: float = 100.0, seed: int = SEED_ZELDOVICH, amp: float = 2.5e-6,
                    box: float = 48.0, return_initial: bool = False):
    """Density contrast delta(x, theta) of the 1D Zel'dovich approximation on
    n periodic grid points (Sec. 5, Eq. nonlinear_dens):
    delta + 1 = 1 / (1 - theta delta_0(x)), with delta_0 the linear field at
    theta = 1, a Gaussian random field of power spectrum P(k) = amp k^-2.

    delta_0(x_j) = sum_{m=1}^{n/2-1} 2 Re(a_m e^{i k_m x_j}), x_j = j box / n,
    k_m = 2 pi m / box, a_m complex Gaussian with <|a_m|^2> = P(k_m) / box
    (so <delta_0^2> = sum_m 2 P(k_m) / box).  Raises ValueError when
    theta delta_0 reaches 1 somewhere (past the first orbit crossing).
    return_initial: also return delta_0."""
    rng = np.random.default_rng(seed)
    m = np.arange(n // 2 + 1, dtype=np.float64)
    p = np.zeros_like(m)
    k = 2.0 * np.pi * m[1:] / box
    p[1:] = amp / (k * k)
    a = (rng.standard_normal(m.size) + 1j * rng.standard_normal(m.size)) * np.sqrt(p / box / 2.0)
    a[0] = 0.0
    a[-1] = 0.0  # no Nyquist mode
    # irfft(c) = (1/n) sum_m c_m e^{2 pi i m j / n} + conj. terms
    d0 = np.fft.irfft(a * n, n=n)
    if np.max(theta * d0) >= 1.0:
        raise ValueError(f"theta = {theta} is past the first orbit crossing of this field")
    d = 1.0 / (1.0 - theta * d0) - 1.0
    return (d, d0) if return_initial else d


def paper_f1(n: int = 512) -> np.ndarray:
    """The periodic test signal of Sec. 4 (Eq. signal_f1),
    2 cos x + cos(8x)/2 + sin(32x)/4, sampled at x = 2 pi i / n (period 2 pi)."""
    x = 2 * np.pi * np.arange(n) / n
    return 2 * np.cos(x) + 0.5 * np.cos(8 * x) + 0.25 * np.sin(32 * x)


def paper_f2(n: int = 512) -> np.ndarray:
    """The non-periodic test signal of Sec. 4 (Eq. signal_f2), exp(-x^2/2),
    sampled at x = -6 + 12 i / n on [-6, 6)."""
    x = -6.0 + 12.0 * np.arange(n) / n
    return np.exp(-0.5 * x * x)


def paper_scale_grid(n: int, cw: float, nsubs: int) -> np.ndarray:
    """Scales (in samples) of the log grid of Sec. 3.1: w~ = w~_min
    2^(i + j/nsubs) with w~_min = c_w pi / n (the largest scale), levels
    i = 0 .. Nint(log2 n) - 1 and sub-levels j = 0 .. nsubs - 1; the scale in
    samples is 1/w~ (largest first)."""
    wmin = cw * np.pi / n
    nlev = int(round(np.log2(n)))
    return np.array([1.0 / (wmin * 2.0 ** (i + j / nsubs)) for i in range(nlev) for j in range(nsubs)])


def log_scales(a: float, b: float, s: int) -> np.ndarray:
    if s == 1:
        return np.array([a], dtype=np.float64)
    j = np.arange(s, dtype=np.float64)
    return a * (b / a) ** (j / (s - 1))


@dataclass
class Instance:
    """One transform request: signal, boundary, wavelet and scales."""
    signal: np.ndarray
    boundary: str          # "periodic" | "zero"
    wavelet: str           # "morlet" | "mexhat" | "dog"
    param: float           # omega0 for Morlet, m for DOG (2 for the Mexican hat)
    scales: np.ndarray
    arrival: float = 0.0   # seconds (served form only)

    @property
    def n(self) -> int:
        return int(self.signal.size)

    @property
    def coefficients(self) -> int:
        return int(self.signal.size) * int(self.scales.size)


def _scales_for(n: int, s: int) -> np.ndarray:
    return log_scales(2.0, float(min(n / 8.0, 2.0 ** 16)), s)


def batch_specs(count: int = 4096, seed: int = SEED_BATCH, log2_lo: float = 10.0,
                log2_hi: float = 16.0, s_lo: int = 16, s_hi: int = 96) -> list[Instance]:
    """Uneven instances: lengths log-uniform in [2^log2_lo, 2^log2_hi], scale
    counts uniform in [s_lo, s_hi], half periodic tones+noise and half
    zero-boundary lognormal fields, Morlet(6) / Mexican hat 50/50."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = int(round(2.0 ** rng.uniform(log2_lo, log2_hi)))
        s = int(rng.integers(s_lo, s_hi + 1))
        sub = int(rng.integers(0, 2 ** 31))
        if i % 2 == 0:
            sig, bc = tones_noise(n, seed=sub), "periodic"
        else:
            sig, bc = lognormal_field(n, seed=sub), "zero"
        if rng.uniform() < 0.5:
            wav, par = "morlet", 6.0
        else:
            wav, par = "mexhat", 2.0
        out.append(Instance(sig, bc, wav, par, _scales_for(n, s)))
    return out


def request_specs(count: int, rate_hz: float, seed: int = SEED_SERVE,
                  log2_lo: float = 12.0, log2_hi: float = 22.0, s_lo: int = 32,
                  s_hi: int = 256) -> list[dict]:
    """The draws of ``request_stream`` without the signals: arrival time,
    length, scales, wavelet, boundary and the seed its signal would use."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for _ in range(count):
        t += rng.exponential(1.0 / rate_hz)
        n = int(round(2.0 ** rng.uniform(log2_lo, log2_hi)))
        s = int(rng.integers(s_lo, s_hi + 1))
        sub = int(rng.integers(0, 2 ** 31))
        w = int(rng.integers(0, 3))
        wav, par = [("morlet", 6.0), ("mexhat", 2.0), ("dog", 4.0)][w]
        bc = "periodic" if rng.uniform() < 0.5 else "zero"
        out.append({"arrival": t, "n": n, "scales": _scales_for(n, s), "wavelet": wav, "param": par,
                    "boundary": bc, "seed": sub})
    return out


def request_stream(count: int, rate_hz: float, seed: int = SEED_SERVE,
                   log2_lo: float = 12.0, log2_hi: float = 22.0, s_lo: int = 32,
                   s_hi: int = 256) -> list[Instance]:
    """Poisson arrivals at rate_hz; lengths log-uniform in [2^12, 2^22],
    32-256 scales, wavelet uniform over Morlet(6) / Mexican hat / DOG(4),
    boundary periodic (tones + noise) or zero (lognormal field) 50/50."""
    out = []
    for d in request_specs(count, rate_hz, seed, log2_lo, log2_hi, s_lo, s_hi):
        if d["boundary"] == "periodic":
            sig = tones_noise(d["n"], seed=d["seed"])
        else:
            sig = lognormal_field(d["n"], seed=d["seed"])
        out.append(Instance(sig, d["boundary"], d["wavelet"], d["param"], d["scales"], arrival=d["arrival"]))
    return out


def mean_request_coefficients(log2_lo: float = 12.0, log2_hi: float = 22.0,
                              s_lo: int = 32, s_hi: int = 256) -> float:
    """Expected N*S of ``request_stream`` (N log-uniform, S uniform)."""
    a, b = log2_lo * math.log(2), log2_hi * math.log(2)
    en = (math.exp(b) - math.exp(a)) / (b - a)
    return en * 0.5 * (s_lo + s_hi)
