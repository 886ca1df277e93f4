// cwt_host.h -- host-side helpers shared by the plan sources: error
// reporting, the device-table builder and the wavelet definitions.
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>
#include <complex>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/cwt.h"

namespace cwt {

struct Failure {
    int code;
    std::string msg;
};
[[noreturn]] inline void fail(int code, const std::string &msg) { throw Failure{code, msg}; }

#define HIPCHK(x)                                                                          \
    do {                                                                                   \
        hipError_t e_ = (x);                                                               \
        if (e_ != hipSuccess) ::cwt::fail(CWT_EDEVICE, std::string(#x) + ": " + hipGetErrorString(e_)); \
    } while (0)

// ---------------------------------------------------------------------------
// table upload helper

struct TableBuilder {
    std::vector<char> host;
    int64_t add(const void *data, size_t bytes) {
        size_t off = (host.size() + 255) & ~size_t(255);
        host.resize(off + bytes);
        std::memcpy(host.data() + off, data, bytes);
        return (int64_t)off;
    }
};

// ---------------------------------------------------------------------------
// Wavelets (unit L2 norm; psi^(u) = int psi(x) e^{-iux} dx = i^{-cph}... see
// amp/cph below).  psi^(u) = phase * amp(u) with amp real; conj(phase) = i^cph.

struct Wavelet {
    int kind = 0;   // CWT_MORLET, CWT_MEXHAT, CWT_DOG, CWT_CBSW, CWT_GDW, CWT_CWGDW (CWT_MW is
                    // planned as CWT_MORLET with w0 = -4)
    double w0 = 6.0;
    int m = 2;
    double cmor = 0.0, kappa = 0.0, gnorm = 0.0, cn = 0.0;

    void init() {
        if (kind == CWT_MORLET) {
            kappa = std::exp(-0.5 * w0 * w0);
            cmor = std::pow(M_PI, -0.25) / std::sqrt(1.0 + std::exp(-w0 * w0) - 2.0 * std::exp(-0.75 * w0 * w0));
        } else if (kind == CWT_CBSW) {
            cn = std::sqrt(30.0 / 31.0);  // Table 2
        } else if (kind == CWT_GDW) {
            cn = std::pow(18.0 * M_PI, -0.25);  // Table 2
        } else if (kind == CWT_CWGDW) {
            cn = std::sqrt(8.0 / (1.0 + 5.0 * std::exp(1.0))) * std::pow(M_PI, -0.25);  // Table 2
        } else {
            gnorm = 1.0 / std::sqrt(std::tgamma(m + 0.5));
        }
    }
    bool complex_out() const { return kind == CWT_MORLET; }
    // spectrum limited to a band (Gaussian decay); the cubic B-spline
    // wavelet's transform decays only like u^-4
    bool band_limited() const { return kind != CWT_CBSW; }
    static double bspline3(double x) {
        x = std::fabs(x);
        if (x < 1.0) return 2.0 / 3.0 - x * x + 0.5 * x * x * x;
        if (x < 2.0) return (2.0 - x) * (2.0 - x) * (2.0 - x) / 6.0;
        return 0.0;
    }
    // |psi(x)| in the time domain
    double abs_time(double x) const {
        if (kind == CWT_MORLET) {
            const double g = std::exp(-0.5 * x * x);
            return cmor * g * std::sqrt(std::max(0.0, 1.0 - 2.0 * kappa * std::cos(w0 * x) + kappa * kappa));
        }
        return std::abs(psi_time(x));
    }
    // psi(x) in the time domain:
    //   Morlet(w0)  C (e^{i w0 x} - kappa) e^{-x^2/2}
    //   DOG(m)      -Gamma(m + 1/2)^{-1/2} He_m(x) e^{-x^2/2}
    //   CBSW        C_N (2 beta3(x) - beta3(x + 1) - beta3(x - 1))          (Table 2)
    //   GDW         C_N (2 - x^2) e^{-x^2/4}                                (Table 2)
    //   CW-GDW      C_N ((1 - x^2) cos x - x sin x) e^{(1 - x^2)/2}         (Table 2)
    std::complex<double> psi_time(double x) const {
        if (kind == CWT_MORLET) {
            const double g = std::exp(-0.5 * x * x);
            return cmor * g * std::complex<double>(std::cos(w0 * x) - kappa, std::sin(w0 * x));
        }
        if (kind == CWT_CBSW) return {cn * (2.0 * bspline3(x) - bspline3(x + 1.0) - bspline3(x - 1.0)), 0.0};
        if (kind == CWT_GDW) return {cn * (2.0 - x * x) * std::exp(-0.25 * x * x), 0.0};
        if (kind == CWT_CWGDW)
            return {cn * ((1.0 - x * x) * std::cos(x) - x * std::sin(x)) * std::exp(0.5 * (1.0 - x * x)), 0.0};
        const double g = std::exp(-0.5 * x * x);
        double hm1 = 1.0, h = x;
        for (int n = 1; n < m; ++n) {
            double hn = x * h - n * hm1;
            hm1 = h;
            h = hn;
        }
        return {-h * g * gnorm, 0.0};
    }
    // psi''(x), differentiated by hand from psi_time (the A19 method's
    // third-derivative estimate, Eq. 3rd_derivative_wavelet, needs it):
    //   Morlet  C e^{-x^2/2} [e^{i w0 x} (x^2 - 2 i w0 x - w0^2 - 1) - kappa (x^2 - 1)]
    //   DOG(m)  -Gamma(m + 1/2)^{-1/2} He_{m+2}(x) e^{-x^2/2}
    //   GDW     C_N e^{-x^2/4} (2 x^2 - 2 - (x^2 - 2)^2 / 4)
    //   CW-GDW  C_N e^{(1-x^2)/2} (q'' - 2 x q' + (x^2 - 1) q), q = (1 - x^2) cos x - x sin x
    std::complex<double> psi2_time(double x) const {
        if (kind == CWT_MORLET) {
            const double g = std::exp(-0.5 * x * x);
            const std::complex<double> e(std::cos(w0 * x), std::sin(w0 * x));
            return cmor * g * (e * std::complex<double>(x * x - w0 * w0 - 1.0, -2.0 * w0 * x) - kappa * (x * x - 1.0));
        }
        if (kind == CWT_GDW) {
            const double u = x * x - 2.0;
            return {cn * std::exp(-0.25 * x * x) * (2.0 * x * x - 2.0 - 0.25 * u * u), 0.0};
        }
        if (kind == CWT_CWGDW) {
            const double c = std::cos(x), sn = std::sin(x);
            const double q0 = (1.0 - x * x) * c - x * sn;
            const double q1 = -3.0 * x * c - (2.0 - x * x) * sn;
            const double q2 = (x * x - 5.0) * c + 5.0 * x * sn;
            return {cn * std::exp(0.5 * (1.0 - x * x)) * (q2 - 2.0 * x * q1 + (x * x - 1.0) * q0), 0.0};
        }
        if (kind == CWT_CBSW) return {std::nan(""), 0.0};
        double hm1 = 1.0, h = x;
        for (int n = 1; n < m + 2; ++n) {
            double hn = x * h - n * hm1;
            hm1 = h;
            h = hn;
        }
        return {-h * std::exp(-0.5 * x * x) * gnorm, 0.0};
    }
    // real amplitude of the spectrum psi^(u) = int psi(x) e^{-iux} dx:
    //   Morlet  C sqrt(2 pi) (e^{-(u - w0)^2/2} - kappa e^{-u^2/2})
    //   DOG(m)  Gamma(m + 1/2)^{-1/2} sqrt(2 pi) u^m e^{-u^2/2}   (times the phase i^-cph)
    //   CBSW    64 C_N sin^6(u/2) / u^4                            (Table 2)
    //   GDW     8 sqrt(pi) C_N u^2 e^{-u^2}                        (Table 2)
    //   CW-GDW  sqrt(2 pi) C_N u (u cosh u - sinh u) e^{-u^2/2}    (Table 2)
    double amp(double u) const {
        if (kind == CWT_MORLET)
            return cmor * std::sqrt(2.0 * M_PI) * (std::exp(-0.5 * (u - w0) * (u - w0)) - kappa * std::exp(-0.5 * u * u));
        if (kind == CWT_CBSW) {
            if (std::fabs(u) < 1e-3) {
                // sin^6(u/2)/u^4 = u^2/64 (1 - u^2/4 + ...)
                return cn * u * u * (1.0 - u * u / 4.0);
            }
            const double sh = std::sin(0.5 * u);
            const double s2 = sh * sh;
            return 64.0 * cn * s2 * s2 * s2 / (u * u * u * u);
        }
        if (kind == CWT_GDW) return 8.0 * std::sqrt(M_PI) * cn * u * u * std::exp(-u * u);
        if (kind == CWT_CWGDW) {
            // u cosh(u) e^{-u^2/2} and sinh(u) e^{-u^2/2} as sums of two Gaussians
            const double ep = std::exp(u - 0.5 * u * u), em = std::exp(-u - 0.5 * u * u);
            return std::sqrt(2.0 * M_PI) * cn * u * (0.5 * u * (ep + em) - 0.5 * (ep - em));
        }
        return std::pow(u, m) * std::sqrt(2.0 * M_PI) * std::exp(-0.5 * u * u) * gnorm;
    }
    // DOG(m): psi^ = (-1)^{m+1} i^m amp  ->  conj(phase) = i^{(m+2) mod 4};
    // the others have a real spectrum
    int cph() const { return (kind == CWT_MEXHAT || kind == CWT_DOG) ? (m + 2) % 4 : 0; }
};

}  // namespace cwt
