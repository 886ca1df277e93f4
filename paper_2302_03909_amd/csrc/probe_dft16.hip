// probe_dft16.hip -- measurement probe, not part of the transform
// (libcwt_probe.so): the throughput of one radix-16 stage of the FFT kernels,
// a 16-point complex DFT of many columns in FP32, done two ways with the
// operands in registers:
//   VALU -- the in-register radix-16 butterfly the FFT kernels use (dftR),
//           one 16-point column per thread;
//   MFMA -- the same DFT as a matrix product Y = F X on the matrix cores:
//           16 columns per wave, four real 16x16x16 products (Fr Xr, -Fi Xi,
//           Fr Xi, Fi Xr), each four v_mfma_f32_16x16x4_f32.
// Both repeat the stage kIters times on their registers (the MFMA form feeds
// its output back as the next input, rows permuted; F is scaled by 1/4, which
// keeps the norm).  A single-stage check against the VALU result confirms the
// operand layout.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <vector>

#include "fft_device.h"

namespace cwt {

typedef float f32x4 __attribute__((ext_vector_type(4)));
constexpr int kIters = 256;

// a DFT and its inverse per iteration, then the 1/16 that undoes their gain
template <int ITERS>
__global__ __launch_bounds__(256) void dft16_valu_kernel(const float2 *__restrict__ in, float2 *__restrict__ out) {
    const int64_t base = ((int64_t)blockIdx.x * 256 + threadIdx.x) * 16;
    float2 v[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) v[r] = in[base + r];
    for (int it = 0; it < ITERS; ++it) {
        dftR<16, -1>(v);
        dftR<16, +1>(v);
#pragma unroll
        for (int r = 0; r < 16; ++r) v[r] = make_float2(v[r].x * 0.0625f, v[r].y * 0.0625f);
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) out[base + r] = v[r];
}

// lane l of a wave holds column l % 16 at rows l / 16 + 4 kb (kb = 0..3):
// the B operand of the kb-th 16x16x4 product; the A operand is
// F[l % 16][4 kb + l / 16] / 4.  The product leaves rows 4 (l / 16) + j of
// column l % 16 in lane l (j = 0..3).
template <int ITERS>
__global__ __launch_bounds__(256) void dft16_mfma_kernel(const float2 *__restrict__ in, float2 *__restrict__ out) {
    const int lane = threadIdx.x & 63;
    const int64_t wave = ((int64_t)blockIdx.x * 256 + threadIdx.x) >> 6;
    const int col = lane & 15, kq = lane >> 4;
    float fr[4], fi[4], fn[4];
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) {
        const int k = 4 * kb + kq;
        float s, c;
        sincospif(-2.0f * (float)((col * k) & 15) / 16.0f, &s, &c);  // row index = col here (A row = lane % 16)
        fr[kb] = 0.25f * c;
        fi[kb] = 0.25f * s;
        fn[kb] = -0.25f * s;
    }
    const int64_t base = wave * 256;  // 16 columns x 16 points, column-major
    float xr[4], xi[4];
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) {
        const float2 x = in[base + col * 16 + 4 * kb + kq];
        xr[kb] = x.x;
        xi[kb] = x.y;
    }
    f32x4 yr = {0.f, 0.f, 0.f, 0.f}, yi = yr;
    for (int it = 0; it < ITERS; ++it) {
        yr = f32x4{0.f, 0.f, 0.f, 0.f};
        yi = yr;
#pragma unroll
        for (int kb = 0; kb < 4; ++kb) {
            yr = __builtin_amdgcn_mfma_f32_16x16x4f32(fr[kb], xr[kb], yr, 0, 0, 0);
            yr = __builtin_amdgcn_mfma_f32_16x16x4f32(fn[kb], xi[kb], yr, 0, 0, 0);
            yi = __builtin_amdgcn_mfma_f32_16x16x4f32(fr[kb], xi[kb], yi, 0, 0, 0);
            yi = __builtin_amdgcn_mfma_f32_16x16x4f32(fi[kb], xr[kb], yi, 0, 0, 0);
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            xr[j] = yr[j];
            xi[j] = yi[j];
        }
    }
    // rows 4 kq + j of column col
#pragma unroll
    for (int j = 0; j < 4; ++j) out[base + col * 16 + 4 * kq + j] = make_float2(yr[j], yi[j]);
}

// one forward DFT per column by the butterfly, for the layout check
__global__ __launch_bounds__(256) void dft16_valu_once(const float2 *__restrict__ in, float2 *__restrict__ out) {
    const int64_t base = ((int64_t)blockIdx.x * 256 + threadIdx.x) * 16;
    float2 v[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) v[r] = in[base + r];
    dftR<16, -1>(v);
#pragma unroll
    for (int r = 0; r < 16; ++r) out[base + r] = make_float2(0.25f * v[r].x, 0.25f * v[r].y);
}

}  // namespace cwt

extern "C" {

// Points per second of each form (16 complex outputs per column and stage)
// and the largest difference between one MFMA stage and one butterfly stage
// (relative to the largest output).  Returns 0, or -4 on a HIP error.
int cwt_probe_dft16(double *valu_points_per_s, double *mfma_points_per_s, double *max_rel_diff) {
    using namespace cwt;
    const int64_t ncols = int64_t(1) << 20, npts = ncols * 16;
    float2 *a = nullptr, *b = nullptr, *c = nullptr;
    auto ok = [](hipError_t e) { return e == hipSuccess; };
    if (!ok(hipMalloc(&a, npts * sizeof(float2))) || !ok(hipMalloc(&b, npts * sizeof(float2))) ||
        !ok(hipMalloc(&c, npts * sizeof(float2))))
        return -4;
    std::vector<float2> h(npts);
    uint32_t st = 12345u;
    for (auto &x : h) {
        st = st * 1664525u + 1013904223u;
        const float re = (float)(st >> 8) / 16777216.0f - 0.5f;
        st = st * 1664525u + 1013904223u;
        const float im = (float)(st >> 8) / 16777216.0f - 0.5f;
        x = make_float2(re, im);
    }
    int rc = 0;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    do {
        if (!ok(hipMemcpy(a, h.data(), npts * sizeof(float2), hipMemcpyHostToDevice))) { rc = -4; break; }
        // layout check: one stage each
        hipLaunchKernelGGL(dft16_valu_once, dim3((unsigned)(ncols / 256)), dim3(256), 0, 0, a, b);
        hipLaunchKernelGGL((dft16_mfma_kernel<1>), dim3((unsigned)(ncols / 16 / 4)), dim3(256), 0, 0, a, c);
        if (!ok(hipDeviceSynchronize())) { rc = -4; break; }
        std::vector<float2> hb(npts), hc(npts);
        if (!ok(hipMemcpy(hb.data(), b, npts * sizeof(float2), hipMemcpyDeviceToHost)) ||
            !ok(hipMemcpy(hc.data(), c, npts * sizeof(float2), hipMemcpyDeviceToHost))) { rc = -4; break; }
        double mx = 0.0, md = 0.0;
        for (int64_t i = 0; i < npts; ++i) {
            mx = std::fmax(mx, std::fabs((double)hb[i].x) + std::fabs((double)hb[i].y));
            md = std::fmax(md, std::fabs((double)hb[i].x - hc[i].x) + std::fabs((double)hb[i].y - hc[i].y));
        }
        *max_rel_diff = md / mx;
        if (!ok(hipEventCreate(&e0)) || !ok(hipEventCreate(&e1))) { rc = -4; break; }
        float ms = 0.f;
        // VALU: 2 stages per iteration
        for (int w = 0; w < 2; ++w)
            hipLaunchKernelGGL((dft16_valu_kernel<kIters>), dim3((unsigned)(ncols / 256)), dim3(256), 0, 0, a, b);
        if (!ok(hipEventRecord(e0, 0))) { rc = -4; break; }
        hipLaunchKernelGGL((dft16_valu_kernel<kIters>), dim3((unsigned)(ncols / 256)), dim3(256), 0, 0, a, b);
        if (!ok(hipEventRecord(e1, 0)) || !ok(hipEventSynchronize(e1)) || !ok(hipEventElapsedTime(&ms, e0, e1))) { rc = -4; break; }
        *valu_points_per_s = (double)npts * 2.0 * kIters / (ms * 1e-3);
        // MFMA: 1 stage per iteration
        for (int w = 0; w < 2; ++w)
            hipLaunchKernelGGL((dft16_mfma_kernel<kIters>), dim3((unsigned)(ncols / 16 / 4)), dim3(256), 0, 0, a, c);
        if (!ok(hipEventRecord(e0, 0))) { rc = -4; break; }
        hipLaunchKernelGGL((dft16_mfma_kernel<kIters>), dim3((unsigned)(ncols / 16 / 4)), dim3(256), 0, 0, a, c);
        if (!ok(hipEventRecord(e1, 0)) || !ok(hipEventSynchronize(e1)) || !ok(hipEventElapsedTime(&ms, e0, e1))) { rc = -4; break; }
        *mfma_points_per_s = (double)npts * kIters / (ms * 1e-3);
    } while (false);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(a);
    (void)hipFree(b);
    (void)hipFree(c);
    return rc;
}

}  // extern "C"
