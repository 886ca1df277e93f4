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
    int kind = 0;   // CWT_MORLET, CWT_MEXHAT, CWT_DOG
    double w0 = 6.0;
    int m = 2;
    double cmor = 0.0, kappa = 0.0, gnorm = 0.0;

    void init() {
        if (kind == CWT_MORLET) {
            kappa = std::exp(-0.5 * w0 * w0);
            cmor = std::pow(M_PI, -0.25) / std::sqrt(1.0 + std::exp(-w0 * w0) - 2.0 * std::exp(-0.75 * w0 * w0));
        } else {
            gnorm = 1.0 / std::sqrt(std::tgamma(m + 0.5));
        }
    }
    bool complex_out() const { return kind == CWT_MORLET; }
    // |psi(x)| in the time domain
    double abs_time(double x) const {
        double g = std::exp(-0.5 * x * x);
        if (kind == CWT_MORLET)
            return cmor * g * std::sqrt(std::max(0.0, 1.0 - 2.0 * kappa * std::cos(w0 * x) + kappa * kappa));
        // probabilists' Hermite polynomial He_m
        double hm1 = 1.0, h = x;
        for (int n = 1; n < m; ++n) {
            double hn = x * h - n * hm1;
            hm1 = h;
            h = hn;
        }
        return std::fabs(h) * g * gnorm;
    }
    // psi(x) in the time domain: Morlet C (e^{i w0 x} - kappa) e^{-x^2/2};
    // DOG(m) -Gamma(m + 1/2)^{-1/2} He_m(x) e^{-x^2/2}
    std::complex<double> psi_time(double x) const {
        double g = std::exp(-0.5 * x * x);
        if (kind == CWT_MORLET) return cmor * g * std::complex<double>(std::cos(w0 * x) - kappa, std::sin(w0 * x));
        double hm1 = 1.0, h = x;
        for (int n = 1; n < m; ++n) {
            double hn = x * h - n * hm1;
            hm1 = h;
            h = hn;
        }
        return {-h * g * gnorm, 0.0};
    }
    // real amplitude of the spectrum
    double amp(double u) const {
        if (kind == CWT_MORLET)
            return cmor * std::sqrt(2.0 * M_PI) * (std::exp(-0.5 * (u - w0) * (u - w0)) - kappa * std::exp(-0.5 * u * u));
        return std::pow(u, m) * std::sqrt(2.0 * M_PI) * std::exp(-0.5 * u * u) * gnorm;
    }
    // DOG(m): psi^ = (-1)^{m+1} i^m amp  ->  conj(phase) = i^{(m+2) mod 4}
    int cph() const { return kind == CWT_MORLET ? 0 : (m + 2) % 4; }
};

}  // namespace cwt
