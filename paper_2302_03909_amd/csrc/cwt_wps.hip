// cwt_wps.hip -- statistics epilogue of the segmented FFT method: the
// environment-dependent and global wavelet power spectra of Sec. 5,
//   P(s, bin) = <|W(s, x)|^2> over the positions x whose environment value
//               falls in the bin                              (Eq. env_wps)
//   P(s)      = <|W(s, x)|^2> over all positions              (Eq. global_wps)
// reduced inside the two output kernels (seg_kernels.h, instantiated for 1,
// 2 and up to 4 bins in cwt_wps_b*.hip) instead of writing the S x N
// coefficients.  Every position falls in exactly one bin, so
// P(s) = sum_bin f_bin P(s, bin) with f_bin = N_bin / N (Eq.
// global_wps_env_wps) holds by construction.
//
// Workgroup sums go to fixed slots and are added in a fixed order, so the
// result does not depend on scheduling.
#include "seg_kernels.h"

namespace cwt {

// N_bin partial counts: kWpsCountBlocks workgroups stride over env
template <typename R>
__global__ __launch_bounds__(256) void wps_count_kernel(const R *__restrict__ env, int64_t N, const WpsArgs w,
                                                        uint64_t *__restrict__ cpart) {
    __shared__ uint32_t cnt[kWpsMaxBins];
    if (threadIdx.x < kWpsMaxBins) cnt[threadIdx.x] = 0u;
    __syncthreads();
    uint32_t c[kWpsMaxBins] = {};
    for (int64_t x = (int64_t)blockIdx.x * 256 + threadIdx.x; x < N; x += (int64_t)gridDim.x * 256) {
        const uint32_t b = wps_bin(env, x, true, w);
#pragma unroll
        for (int k = 0; k < kWpsMaxBins; ++k) c[k] += b == (uint32_t)k ? 1u : 0u;
    }
#pragma unroll
    for (int k = 0; k < kWpsMaxBins; ++k)
        if (k < w.nbin && c[k]) atomicAdd(&cnt[k], c[k]);
    __syncthreads();
    if (threadIdx.x < kWpsMaxBins) cpart[(int64_t)blockIdx.x * kWpsMaxBins + threadIdx.x] = cnt[threadIdx.x];
}

// one workgroup per scale: slot sums in a fixed order, then
//   wps[j][bin]  = sum_bin / N_bin   (NaN for an empty bin)
//   wps[j][nbin] = sum over bins / N
// workgroup 0 also writes the counts (if requested)
__global__ __launch_bounds__(256) void wps_finalize_kernel(const double *__restrict__ part,
                                                           const int64_t *__restrict__ base, const WpsArgs w,
                                                           const uint64_t *__restrict__ cpart, int64_t N,
                                                           double *__restrict__ wps, int64_t *__restrict__ counts) {
    __shared__ double sh[256];
    __shared__ double sums[kWpsMaxBins];
    __shared__ uint64_t cn[kWpsMaxBins];
    const int j = blockIdx.x, t = threadIdx.x, nb = w.nbin;
    const int64_t s0 = base[j], s1 = base[j + 1];
    for (int b = 0; b < nb; ++b) {
        double a = 0.0;
        for (int64_t sl = s0 + t; sl < s1; sl += 256) a += part[sl * nb + b];
        sh[t] = a;
        __syncthreads();
        for (int h = 128; h > 0; h >>= 1) {
            if (t < h) sh[t] += sh[t + h];
            __syncthreads();
        }
        if (t == 0) sums[b] = sh[0];
        __syncthreads();
    }
    if (t < nb) {
        uint64_t c = 0;
        for (int k = 0; k < kWpsCountBlocks; ++k) c += cpart[(int64_t)k * kWpsMaxBins + t];
        cn[t] = c;
    }
    __syncthreads();
    double *row = wps + (int64_t)j * (nb + 1);
    if (t < nb) row[t] = cn[t] ? sums[t] / (double)cn[t] : __builtin_nan("");
    if (t == 0) {
        double tot = 0.0;
        for (int b = 0; b < nb; ++b) tot += sums[b];
        row[nb] = tot / (double)N;
    }
    if (j == 0 && counts && t < nb) counts[t] = (int64_t)cn[t];
}

hipError_t launch_wps_count(const void *env, int64_t N, bool fp64, const WpsArgs &w, uint64_t *cpart, hipStream_t st) {
    if (fp64)
        hipLaunchKernelGGL(wps_count_kernel<double>, dim3(kWpsCountBlocks), dim3(256), 0, st,
                           static_cast<const double *>(env), N, w, cpart);
    else
        hipLaunchKernelGGL(wps_count_kernel<float>, dim3(kWpsCountBlocks), dim3(256), 0, st,
                           static_cast<const float *>(env), N, w, cpart);
    return hipGetLastError();
}

hipError_t launch_wps_finalize(const double *part, const int64_t *base, int S, const WpsArgs &w,
                               const uint64_t *cpart, int64_t N, double *wps, int64_t *counts, hipStream_t st) {
    if (S <= 0) return hipSuccess;
    hipLaunchKernelGGL(wps_finalize_kernel, dim3((unsigned)S), dim3(256), 0, st, part, base, w, cpart, N, wps, counts);
    return hipGetLastError();
}

hipError_t launch_out_kernel_wps1(const SegKernelId &id, const BatchArgs &a, int64_t blocks, hipStream_t st);
hipError_t launch_out_kernel_wps2(const SegKernelId &id, const BatchArgs &a, int64_t blocks, hipStream_t st);
hipError_t launch_out_kernel_wps4(const SegKernelId &id, const BatchArgs &a, int64_t blocks, hipStream_t st);

hipError_t launch_seg_kernel_wps(const SegKernelId &id, const BatchArgs &a, int64_t blocks, hipStream_t st) {
    if (blocks <= 0) return hipSuccess;
    if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
    if (id.kind != 0 && id.kind != 3) return launch_seg_kernel(id, a, blocks, st);  // forward, reduce: shared
    // variants specialised on the bin count (1, 2, or up to 4)
    if (a.wps.nbin == 1) return launch_out_kernel_wps1(id, a, blocks, st);
    if (a.wps.nbin == 2) return launch_out_kernel_wps2(id, a, blocks, st);
    if (a.wps.nbin <= kWpsMaxBins) return launch_out_kernel_wps4(id, a, blocks, st);
    return hipErrorInvalidValue;
}

}  // namespace cwt
