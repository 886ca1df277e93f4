// cwt_seg.hip -- segmented (overlap-save) FFT method for gfx950.
//
// The product W = IDFT(DFT(f) * conj(Psi_s)) of Sec. 3.1 (Eq.
// discrete_CWT_conv, with the aliased spectrum of the sampled wavelet) is
// evaluated segment by segment: a segment of L = 2^l samples starting Tg
// before its first output yields V = L - 2 Tg valid outputs, because the
// wavelet at every scale of the group is negligible beyond Tg samples.
//
// Small scales (wide spectrum relative to L): local2_kernel takes the full
// L-point FFT of NCOL segments per workgroup, keeps the spectra in registers
// and, for every scale of the group, multiplies and inverts in LDS.
//
// Larger scales (the spectrum at length L occupies B <= P << L bins): the
// segment spectrum is needed only on the band [klo, klo + B).  With L = P Q:
//   forward  X[m] = sum_q w_L^{-q m} DFT_P(x[q + Q p])[m mod P]
//            (seg_forward_kernel: 16 columns q per iteration, FP64 sums,
//             partial sums per column chunk, then seg_reduce_kernel)
//   inverse  W[r + Q p] = DFT_P^{-1}( Y[m] w_L^{m r} )[p],  m = k mod P
//            (seg_inverse_kernel: 16 consecutive columns r per workgroup, so
//             the last FFT pass stores 16-element runs straight to HBM).
#include "cwt_internal.h"
#include "fft_cols.h"

namespace cwt {

template <typename R>
__device__ __forceinline__ R sig_seg(const R *__restrict__ f, int64_t N, int periodic, int64_t idx) {
    if (periodic) {
        int64_t r = idx % N;
        if (r < 0) r += N;
        return f[r];
    }
    return (idx >= 0 && idx < N) ? f[idx] : (R)0;
}

// w_{2^23}^x, x in [0, 2^23), from FP64 tables hi[x >> 11] * lo[x & 2047]
__device__ __forceinline__ double2 w23(const double2 *__restrict__ hi, const double2 *__restrict__ lo, int64_t x) {
    return cmul(hi[x >> 11], lo[x & 2047]);
}

template <typename C> __device__ __forceinline__ C mul_i_pow(C a, int q) {
    switch (q & 3) {
        case 1: return mk<C>(-a.y, a.x);
        case 2: return mk<C>(-a.x, -a.y);
        case 3: return mk<C>(a.y, -a.x);
        default: return a;
    }
}

template <typename C> __device__ __forceinline__ C to_c(double2 v) { return mk<C>((decltype(C::x))v.x, (decltype(C::x))v.y); }
template <typename C> __device__ __forceinline__ double2 to_d(C v) { return make_double2((double)v.x, (double)v.y); }

// ---------------------------------------------------------------------------
// pruned forward transform of the segments, partial sums per column chunk

template <typename R, int P, int NT>
__global__ __launch_bounds__(NT) void seg_forward_kernel(const R *__restrict__ f, int64_t N, int periodic, int lgL,
                                                         int64_t V, int64_t Tg, int iters, int nchunk, int64_t klo,
                                                         int B, const cplx_t<R> *__restrict__ twl_g,
                                                         const double2 *__restrict__ whi,
                                                         const double2 *__restrict__ wlo,
                                                         double2 *__restrict__ Xp) {
    using C = cplx_t<R>;
    constexpr int G = 16;
    constexpr int LD = lds_len(P);
    static_assert(NT >= P, "one band bin per thread");
    __shared__ C buf[G * LD];
    __shared__ C twl[twl_len(P)];
    load_twl<C, P, NT>(twl, twl_g);
    const int64_t L = int64_t(1) << lgL, Q = L >> log2_exact(P);
    const int sh = 23 - lgL;
    const int64_t seg = blockIdx.x / nchunk;
    const int chunk = blockIdx.x % nchunk;
    const int64_t x0 = seg * V - Tg;
    const int tid = threadIdx.x;
    double2 acc = make_double2(0.0, 0.0), base = acc, step = acc, w16 = acc;
    int kap = 0;
    if (tid < B) {
        int64_t mm = (klo + tid) & (L - 1);
        kap = (int)(mm & (P - 1));
        double2 s = w23(whi, wlo, mm << sh);
        step = make_double2(s.x, -s.y);
        double2 s16 = w23(whi, wlo, ((16 * mm) & (L - 1)) << sh);
        w16 = make_double2(s16.x, -s16.y);
        int64_t qf = (int64_t)chunk * iters * G;
        double2 b = w23(whi, wlo, ((qf * mm) & (L - 1)) << sh);
        base = make_double2(b.x, -b.y);
    }
    auto emit = [&](int c, int p, C v) { buf[c * LD + lidx(p)] = v; };
    for (int it = 0; it < iters; ++it) {
        const int64_t q0 = ((int64_t)chunk * iters + it) * G;
        for (int idx = tid; idx < G * P; idx += NT) {
            int g = idx % G, p = idx / G;
            buf[g * LD + lidx(p)] = mk<C>(sig_seg(f, N, periodic, x0 + q0 + g + Q * p), (decltype(C::x))0);
        }
        __syncthreads();
        cols_fft<C, P, G, NT, LD, -1, true>(buf, twl, emit);
        __syncthreads();
        if (tid < B) {
            double2 b = base;
#pragma unroll
            for (int g = 0; g < G; ++g) {
                double2 y = to_d(buf[g * LD + lidx(kap)]);
                acc = cadd(acc, cmul(y, b));
                b = cmul(b, step);
            }
            base = cmul(base, w16);
        }
        __syncthreads();
    }
    if (tid < B) Xp[(seg * nchunk + chunk) * B + tid] = acc;
}

// X[seg][k] = sum over chunks (fixed order) of the partial sums
__global__ void seg_reduce_kernel(const double2 *__restrict__ Xp, int64_t nseg, int nchunk, int B,
                                  double2 *__restrict__ X) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nseg * B) return;
    int64_t seg = t / B;
    int k = (int)(t % B);
    double2 a = make_double2(0.0, 0.0);
    for (int c = 0; c < nchunk; ++c) a = cadd(a, Xp[(seg * nchunk + c) * B + k]);
    X[t] = a;
}

// ---------------------------------------------------------------------------
// band-limited inverse per (segment, scale or scale pair, 16 columns)

template <typename R, int P, int NT, bool PAIR, bool CPLX>
__global__ __launch_bounds__(NT) void seg_inverse_kernel(int64_t N, int lgL, int64_t V, int64_t Tg, int64_t klo, int B,
                                                         const double2 *__restrict__ X,
                                                         const SegItem *__restrict__ items,
                                                         const R *__restrict__ ktab, int cph,
                                                         const cplx_t<R> *__restrict__ gtw,
                                                         const cplx_t<R> *__restrict__ twl_g,
                                                         const double2 *__restrict__ whi,
                                                         const double2 *__restrict__ wlo, R *__restrict__ out) {
    using C = cplx_t<R>;
    constexpr int G = 16;
    constexpr int LD = lds_len(P);
    static_assert(NT >= P, "one slot per thread");
    __shared__ C buf[G * LD];
    __shared__ C ys[P];
    __shared__ C twl[twl_len(P)];
    load_twl<C, P, NT>(twl, twl_g);
    const SegItem d = items[blockIdx.x];
    const int64_t L = int64_t(1) << lgL, Q = L >> log2_exact(P);
    const int sh = 23 - lgL;
    const int tid = threadIdx.x;
    if (tid < B) {
        int64_t mm = (klo + tid) & (L - 1);
        double2 x = X[(int64_t)d.seg * B + tid];
        double ka = (double)ktab[d.ka + tid];
        double kb = (PAIR && d.sb >= 0) ? (double)ktab[d.kb + tid] : 0.0;
        double2 y = cmul(x, make_double2(ka, kb));
        y = mul_i_pow(y, cph);
        y = cmul(y, w23(whi, wlo, ((mm * (int64_t)d.r0) & (L - 1)) << sh));
        ys[tid] = to_c<C>(y);
    }
    __syncthreads();
    {
        const int kap = tid;
        int first = (int)(((int64_t)kap - klo) & (P - 1));
        if (first < B) {
            C y = ys[first];
            const C *gt = gtw + first;
#pragma unroll
            for (int g = 0; g < G; ++g) buf[g * LD + lidx(kap)] = cmul(y, gt[(int64_t)g * B]);
        } else {
#pragma unroll
            for (int g = 0; g < G; ++g) buf[g * LD + lidx(kap)] = mk<C>(0, 0);
        }
    }
    __syncthreads();
    R *rowa = out + (int64_t)d.sa * N * (CPLX ? 2 : 1);
    R *rowb = (PAIR && d.sb >= 0) ? out + (int64_t)d.sb * N : nullptr;
    const int64_t ob = (int64_t)d.seg * V - Tg;
    auto emit = [&](int c, int p, C v) {
        int64_t u = (int64_t)d.r0 + c + Q * p;
        if (u >= Tg && u < Tg + V) {
            int64_t b = ob + u;
            if (b < N) {
                if (CPLX) reinterpret_cast<C *>(rowa)[b] = v;
                else {
                    rowa[b] = v.x;
                    if (rowb) rowb[b] = v.y;
                }
            }
        }
    };
    cols_fft<C, P, G, NT, LD, +1, false>(buf, twl, emit);
}

// ---------------------------------------------------------------------------
// fused full-spectrum segments (small scales)

template <typename R, int L, int NCOL, int NT, bool PAIR, bool CPLX>
__global__ __launch_bounds__(NT) void local2_kernel(const R *__restrict__ f, int64_t N, int periodic, int64_t Tg,
                                                    int64_t V, int64_t nseg, int nscale,
                                                    const int32_t *__restrict__ scale_ids,
                                                    const R *__restrict__ ktab, int cph,
                                                    const cplx_t<R> *__restrict__ twl_g, R *__restrict__ out) {
    using C = cplx_t<R>;
    constexpr int LD = lds_len(L);
    constexpr int E = NCOL * L / NT;
    static_assert((NCOL * L) % NT == 0, "whole elements per thread");
    __shared__ C buf[NCOL * LD];
    __shared__ C twl[twl_len(L)];
    load_twl<C, L, NT>(twl, twl_g);
    const int tid = threadIdx.x;
    constexpr int SEGS = PAIR ? 2 : 1;
    const int64_t seg0 = (int64_t)blockIdx.x * NCOL * SEGS;
    for (int idx = tid; idx < NCOL * L; idx += NT) {
        int c = idx / L, u = idx % L;
        int64_t s = seg0 + (int64_t)c * SEGS;
        R a = sig_seg(f, N, periodic, s * V - Tg + u);
        R b = PAIR ? sig_seg(f, N, periodic, (s + 1) * V - Tg + u) : (R)0;
        buf[c * LD + lidx(u)] = mk<C>(a, b);
    }
    __syncthreads();
    {
        auto emit = [&](int c, int p, C v) { buf[c * LD + lidx(p)] = v; };
        cols_fft<C, L, NCOL, NT, LD, -1, true>(buf, twl, emit);
    }
    __syncthreads();
    C Xr[E];
#pragma unroll
    for (int i = 0; i < E; ++i) {
        int idx = tid + i * NT;
        Xr[i] = buf[(idx / L) * LD + lidx(idx % L)];
    }
    __syncthreads();
    for (int j = 0; j < nscale; ++j) {
        const R *kt = ktab + (int64_t)j * L;
#pragma unroll
        for (int i = 0; i < E; ++i) {
            int idx = tid + i * NT;
            int u = idx % L;
            buf[(idx / L) * LD + lidx(u)] = mul_i_pow(cscale(Xr[i], kt[u]), cph);
        }
        __syncthreads();
        R *row = out + (int64_t)scale_ids[j] * N * (CPLX ? 2 : 1);
        auto emit = [&](int c, int p, C v) {
            if (p < Tg || p >= Tg + V) return;
            int64_t s = seg0 + (int64_t)c * SEGS;
            int64_t b = s * V + (p - Tg);
            if (CPLX) {
                if (b < N) reinterpret_cast<C *>(row)[b] = v;
            } else {
                if (b < N) row[b] = v.x;
                if (PAIR && s + 1 < nseg && b + V < N) row[b + V] = v.y;
            }
        };
        cols_fft<C, L, NCOL, NT, LD, +1, false>(buf, twl, emit);
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// launchers

static constexpr int local2_ncol(int L) { return L >= 1024 ? 1 : 1024 / L; }
static constexpr int local2_nt(int L) { return local2_ncol(L) * L / 16 < 64 ? 64 : local2_ncol(L) * L / 16; }

bool local2_size_ok(int L, int precision) {
    int lmax = precision == 0 ? 4096 : 8192;
    return L >= 64 && L <= lmax && (L & (L - 1)) == 0;
}
int local2_segs_per_block(int L, bool pair) { return local2_ncol(L) * (pair ? 2 : 1); }

template <typename R, int L>
static hipError_t local2_launch_L(const Plan &p, const SegGroup &g, const R *f, R *out, hipStream_t st) {
    constexpr int NCOL = local2_ncol(L);
    constexpr int NT = local2_nt(L);
    using C = cplx_t<R>;
    const R *ktab = static_cast<const R *>(p.d_tab) + g.tab_off;
    const C *twl = tw_at<C>(p, g.twl_off);
    int periodic = p.boundary == 0 ? 1 : 0;
    int64_t per = (int64_t)NCOL * (p.pair_real ? 2 : 1);
    int64_t grid = (g.nseg + per - 1) / per;
    if (grid <= 0) return hipSuccess;
    if (p.cplx_out)
        hipLaunchKernelGGL((local2_kernel<R, L, NCOL, NT, false, true>), dim3((unsigned)grid), dim3(NT), 0, st, f, p.N,
                           periodic, g.Tg, g.V, g.nseg, (int)g.scales.size(), g.d_scales, ktab, p.cph, twl, out);
    else if (p.pair_real)
        hipLaunchKernelGGL((local2_kernel<R, L, NCOL, NT, true, false>), dim3((unsigned)grid), dim3(NT), 0, st, f, p.N,
                           periodic, g.Tg, g.V, g.nseg, (int)g.scales.size(), g.d_scales, ktab, p.cph, twl, out);
    else
        hipLaunchKernelGGL((local2_kernel<R, L, NCOL, NT, false, false>), dim3((unsigned)grid), dim3(NT), 0, st, f, p.N,
                           periodic, g.Tg, g.V, g.nseg, (int)g.scales.size(), g.d_scales, ktab, p.cph, twl, out);
    return hipGetLastError();
}

template <typename R>
static hipError_t local2_typed(const Plan &p, const SegGroup &g, const R *f, R *o, hipStream_t st) {
    switch (g.L) {
        case 64: return local2_launch_L<R, 64>(p, g, f, o, st);
        case 128: return local2_launch_L<R, 128>(p, g, f, o, st);
        case 256: return local2_launch_L<R, 256>(p, g, f, o, st);
        case 512: return local2_launch_L<R, 512>(p, g, f, o, st);
        case 1024: return local2_launch_L<R, 1024>(p, g, f, o, st);
        case 2048: return local2_launch_L<R, 2048>(p, g, f, o, st);
        case 4096: return local2_launch_L<R, 4096>(p, g, f, o, st);
        case 8192:
            if constexpr (sizeof(R) == 4) return local2_launch_L<R, 8192>(p, g, f, o, st);
            return hipErrorInvalidValue;
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_local2(const Plan &p, const SegGroup &g, const void *signal, void *out, hipStream_t st) {
    if (p.precision == 0)
        return local2_typed(p, g, static_cast<const double *>(signal), static_cast<double *>(out), st);
    return local2_typed(p, g, static_cast<const float *>(signal), static_cast<float *>(out), st);
}

bool seg_size_ok(int P, int precision) {
    int pmax = precision == 0 ? 512 : 1024;
    return P >= 64 && P <= pmax && (P & (P - 1)) == 0;
}

template <typename R, int P>
static hipError_t seg_launch_P(const Plan &p, const SegGroup &g, const R *f, void *ws, R *out, hipStream_t st,
                               int phase) {
    constexpr int NT = P;  // 16 columns x P / 16 elements per thread
    using C = cplx_t<R>;
    char *w = static_cast<char *>(ws);
    double2 *Xp = reinterpret_cast<double2 *>(w + g.ws_xp_off);
    double2 *X = reinterpret_cast<double2 *>(w + g.ws_x_off);
    const C *twl = tw_at<C>(p, g.twl_off);
    const double2 *whi = tw_at<double2>(p, p.w23_hi_off), *wlo = tw_at<double2>(p, p.w23_lo_off);
    int periodic = p.boundary == 0 ? 1 : 0;
    if (phase == 0) {
        unsigned fgrid = (unsigned)(g.nseg * g.nchunk);
        hipLaunchKernelGGL((seg_forward_kernel<R, P, NT>), dim3(fgrid), dim3(NT), 0, st, f, p.N, periodic, g.lgL,
                           g.V, g.Tg, g.iters, g.nchunk, g.klo, g.B, twl, whi, wlo, Xp);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        int64_t nred = g.nseg * g.B;
        hipLaunchKernelGGL(seg_reduce_kernel, dim3((unsigned)((nred + 255) / 256)), dim3(256), 0, st, Xp, g.nseg,
                           g.nchunk, g.B, X);
        return hipGetLastError();
    }
    const R *ktab = static_cast<const R *>(p.d_tab);
    const C *gtw = tw_at<C>(p, g.gtw_off);
    unsigned igrid = (unsigned)g.items.size();
    if (igrid == 0) return hipSuccess;
    if (p.cplx_out)
        hipLaunchKernelGGL((seg_inverse_kernel<R, P, NT, false, true>), dim3(igrid), dim3(NT), 0, st, p.N, g.lgL, g.V,
                           g.Tg, g.klo, g.B, X, g.d_items, ktab, p.cph, gtw, twl, whi, wlo, out);
    else
        hipLaunchKernelGGL((seg_inverse_kernel<R, P, NT, true, false>), dim3(igrid), dim3(NT), 0, st, p.N, g.lgL, g.V,
                           g.Tg, g.klo, g.B, X, g.d_items, ktab, p.cph, gtw, twl, whi, wlo, out);
    return hipGetLastError();
}

template <typename R>
static hipError_t seg_typed(const Plan &p, const SegGroup &g, const R *f, void *ws, R *o, hipStream_t st, int phase) {
    switch (g.P) {
        case 64: return seg_launch_P<R, 64>(p, g, f, ws, o, st, phase);
        case 128: return seg_launch_P<R, 128>(p, g, f, ws, o, st, phase);
        case 256: return seg_launch_P<R, 256>(p, g, f, ws, o, st, phase);
        case 512: return seg_launch_P<R, 512>(p, g, f, ws, o, st, phase);
        case 1024:
            if constexpr (sizeof(R) == 4) return seg_launch_P<R, 1024>(p, g, f, ws, o, st, phase);
            return hipErrorInvalidValue;
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_seg(const Plan &p, const SegGroup &g, const void *signal, void *ws, void *out, hipStream_t st,
                      int phase) {
    if (p.precision == 0)
        return seg_typed(p, g, static_cast<const double *>(signal), ws, static_cast<double *>(out), st, phase);
    return seg_typed(p, g, static_cast<const float *>(signal), ws, static_cast<float *>(out), st, phase);
}

std::string seg_kernel_name(const Plan &p, const SegGroup &g, int phase) {
    std::string t = p.precision == 0 ? "f64," : "f32,";
    if (g.kind == SegGroup::LOCAL)
        return "local2_kernel<" + t + std::to_string(g.L) + (p.cplx_out ? ",complex>" : ",real-pair>");
    if (phase == 0) return "seg_forward+reduce<" + t + std::to_string(g.P) + ">";
    return "seg_inverse_kernel<" + t + std::to_string(g.P) + (p.cplx_out ? ",complex>" : ",real-pair>");
}

}  // namespace cwt
