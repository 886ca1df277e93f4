// cwt_tables.hip -- plan-time device work: the sampled wavelet spectra of the
// segmented FFT method (Sec. 3.1, Eq. discrete_CWT_conv with the aliased
// spectrum), evaluated in FP64 on the device.
//
// Entry e of job k is  Psi_s(2 pi m / L) / L  with  m = m0 + e  (or, for a
// full-spectrum job, the signed bin of e in [0, L)),
//   Psi_s(w) = sum_q A(s (w + 2 pi q)),
// over the images q whose argument lies in the wavelet's band [ulo, uhi];
// A is the real amplitude of the wavelet's Fourier transform:
//   Morlet(w0): C sqrt(2 pi) (e^{-(u - w0)^2/2} - e^{-w0^2/2} e^{-u^2/2})
//               (w0 = -4: the MW of Table 2)
//   DOG(m):     Gamma(m + 1/2)^{-1/2} sqrt(2 pi) u^m e^{-u^2/2}
//   GDW:        8 sqrt(pi) C_N u^2 e^{-u^2}                       (Table 2)
//   CW-GDW:     sqrt(2 pi) C_N u (u cosh u - sinh u) e^{-u^2/2}   (Table 2)
// A shifted job (a band unit whose output columns move by d) stores each
// entry as a complex value, times w_L^{-m d}.
#include <hip/hip_runtime.h>

#include "../../include/cwt.h"
#include "cwt_internal.h"

namespace cwt {

__device__ __forceinline__ double spec_amp(const SpecWavelet &w, double u) {
    const double r2pi = 2.5066282746310005024;
    if (w.kind == CWT_MORLET) {
        const double d = u - w.w0;
        return w.cmor * r2pi * (exp(-0.5 * d * d) - w.kappa * exp(-0.5 * u * u));
    }
    if (w.kind == CWT_GDW) return 8.0 * 1.7724538509055160273 * w.cn * u * u * exp(-u * u);
    if (w.kind == CWT_CWGDW) {
        const double ep = exp(u - 0.5 * u * u), em = exp(-u - 0.5 * u * u);
        return r2pi * w.cn * u * (0.5 * u * (ep + em) - 0.5 * (ep - em));
    }
    double p = 1.0;
    for (int i = 0; i < w.m; ++i) p *= u;
    return p * r2pi * exp(-0.5 * u * u) * w.gnorm;
}

template <typename T>
__global__ __launch_bounds__(256) void spectrum_kernel(SpecWavelet w, const SpecJob *__restrict__ jobs, int njobs,
                                                       T *__restrict__ tab) {
    // job of this block: last job whose first block <= blockIdx.x
    int lo = 0, hi = njobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].block0 <= (int64_t)blockIdx.x) lo = mid;
        else hi = mid - 1;
    }
    const SpecJob jb = jobs[lo];
    const int64_t e = ((int64_t)blockIdx.x - jb.block0) * 256 + threadIdx.x;
    if (e >= jb.count) return;
    int64_t m = jb.m0 + e;
    if (jb.full && m >= jb.L / 2) m -= jb.L;  // signed bin of a full spectrum
    const double tp = 6.283185307179586477;
    const double om = tp * (double)m / (double)jb.L;
    const int64_t q0 = (int64_t)ceil((w.ulo / jb.s - om) / tp), q1 = (int64_t)floor((w.uhi / jb.s - om) / tp);
    double acc = 0.0;
    for (int64_t q = q0; q <= q1; ++q) acc += spec_amp(w, jb.s * (om + tp * (double)q));
    const double v = acc / (double)jb.L;
    if (jb.shift < 0) {
        tab[jb.off + e] = (T)v;
        return;
    }
    // times w_L^{-m shift} = e^{-2 pi i x / L}, x = m shift mod L (exact integer)
    int64_t x = (m % jb.L) * (int64_t)jb.shift % jb.L;
    if (x < 0) x += jb.L;
    double sn, cs;
    sincospi(2.0 * (double)x / (double)jb.L, &sn, &cs);
    tab[jb.off + 2 * e] = (T)(v * cs);
    tab[jb.off + 2 * e + 1] = (T)(-v * sn);
}

hipError_t launch_spectrum_tables(const SpecWavelet &w, const SpecJob *jobs, int njobs, int64_t blocks, void *tab,
                                  bool fp64, hipStream_t st) {
    if (njobs <= 0 || blocks <= 0) return hipSuccess;
    if (fp64)
        hipLaunchKernelGGL(spectrum_kernel<double>, dim3((unsigned)blocks), dim3(256), 0, st, w, jobs, njobs,
                           static_cast<double *>(tab));
    else
        hipLaunchKernelGGL(spectrum_kernel<float>, dim3((unsigned)blocks), dim3(256), 0, st, w, jobs, njobs,
                           static_cast<float *>(tab));
    return hipGetLastError();
}

}  // namespace cwt
