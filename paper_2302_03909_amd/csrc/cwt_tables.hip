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

// Global wavelet power spectrum (Eq. global_wps) of a periodic signal by
// Parseval's identity, without the transform: with F the M-point DFT of the
// period (M = N) and W(s, .) the circular correlation of Eq.
// discrete_CWT_conv with the aliased spectrum,
//   P(s) = (1/N) sum_b |W(s, b)|^2 = (1/M^2) sum_m |F[m]|^2 Psi_s(omega_m)^2.
// Workgroup (c, j) sums chunk c of kParsevalChunk signed bins for scale j,
// over the bins where some image of omega_m falls in the wavelet's band
// [ulo, uhi] / s (every bin when the band spans a period); the chunk sums are
// then added per scale in a fixed order.
template <typename C>
__global__ __launch_bounds__(256) void parseval_part_kernel(SpecWavelet w, const C *__restrict__ F, int64_t M,
                                                           const double *__restrict__ scales,
                                                           double *__restrict__ part) {
    __shared__ double red[256];
    const double tp = 6.283185307179586477;
    const int64_t c = blockIdx.x, j = blockIdx.y;
    const double s = scales[j];
    const int t = threadIdx.x;
    const int64_t half = M / 2;  // signed bins [-half, M - half)
    const int64_t c0 = -half + c * kParsevalChunk;
    const int64_t c1 = (c0 + kParsevalChunk - 1 < M - half - 1) ? c0 + kParsevalChunk - 1 : M - half - 1;
    double acc = 0.0;
    auto visit = [&](int64_t lo, int64_t hi) {  // signed bins lo..hi within this chunk
        lo = lo < c0 ? c0 : lo;
        hi = hi > c1 ? c1 : hi;
        for (int64_t ms = lo + t; ms <= hi; ms += 256) {
            const double om = tp * (double)ms / (double)M;
            const int64_t q0 = (int64_t)ceil((w.ulo / s - om) / tp), q1 = (int64_t)floor((w.uhi / s - om) / tp);
            double psi = 0.0;
            for (int64_t q = q0; q <= q1; ++q) psi += spec_amp(w, s * (om + tp * (double)q));
            const C f = F[ms < 0 ? ms + M : ms];
            acc = fma((double)f.x * (double)f.x + (double)f.y * (double)f.y, psi * psi, acc);
        }
    };
    if ((w.uhi - w.ulo) / s >= tp) {
        visit(c0, c1);
    } else {
        // the images [ulo / s - 2 pi q, uhi / s - 2 pi q] are then disjoint
        const int64_t qa = (int64_t)floor((w.ulo / s - M_PI) / tp), qb = (int64_t)ceil((w.uhi / s + M_PI) / tp);
        for (int64_t q = qa; q <= qb; ++q) {
            const double a = w.ulo / s - tp * (double)q, b = w.uhi / s - tp * (double)q;
            visit((int64_t)ceil(a * (double)M / tp), (int64_t)floor(b * (double)M / tp));
        }
    }
    red[t] = acc;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (t < h) red[t] += red[t + h];
        __syncthreads();
    }
    if (t == 0) part[j * gridDim.x + c] = red[0];
}

__global__ __launch_bounds__(256) void parseval_sum_kernel(const double *__restrict__ part, int nch, int64_t M,
                                                          double *__restrict__ wps) {
    __shared__ double red[256];
    const int j = blockIdx.x, t = threadIdx.x;
    double a = 0.0;
    for (int c = t; c < nch; c += 256) a += part[(int64_t)j * nch + c];
    red[t] = a;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (t < h) red[t] += red[t + h];
        __syncthreads();
    }
    if (t == 0) wps[j] = red[0] / ((double)M * (double)M);
}

hipError_t launch_parseval_wps(const SpecWavelet &w, const void *F, int64_t M, const double *scales, int S,
                               double *part, double *wps, bool fp64, hipStream_t st) {
    if (S <= 0) return hipSuccess;
    const int nch = parseval_chunks(M);
    if (fp64)
        hipLaunchKernelGGL(parseval_part_kernel<double2>, dim3((unsigned)nch, (unsigned)S), dim3(256), 0, st, w,
                           static_cast<const double2 *>(F), M, scales, part);
    else
        hipLaunchKernelGGL(parseval_part_kernel<float2>, dim3((unsigned)nch, (unsigned)S), dim3(256), 0, st, w,
                           static_cast<const float2 *>(F), M, scales, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(parseval_sum_kernel, dim3((unsigned)S), dim3(256), 0, st, part, nch, M, wps);
    return hipGetLastError();
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
