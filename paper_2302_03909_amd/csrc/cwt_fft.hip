// cwt_fft.hip -- FFT method (FFTCWT, Sec. 3.1) for gfx950.
//
// The transform per scale is W = IDFT(F * conj(Psi_s)) / len, where F is the
// DFT of the signal and Psi_s(w) = sum_q psi^(s (w + 2 pi q)) is the DTFT of
// the sampled, 1/s-scaled wavelet (Eq. discrete_CWT_conv with the aliased
// spectrum of the sampled wavelet, so that the result equals the unit-step
// correlation sum exactly).  Three kernels:
//
//   forward_*     FP64 DFT of the whole (zero- or wrap-padded) signal, length
//                 M = M1 * M2, as a four-step transform (two LDS passes).
//   local_kernel  segmented form for scales whose wavelet support is short:
//                 one workgroup per segment of L samples (halo Tg each side)
//                 takes the segment's FFT once and then, for every scale of
//                 its group, multiplies by the L-point spectrum of the wavelet
//                 and runs the inverse FFT, keeping the V = L - 2 Tg valid
//                 outputs (overlap-save).  Output rows are written contiguously.
//   column_kernel band-limited inverse of the whole-signal spectrum for the
//                 large scales: with P | M and Q = M/P, output b = r + Q p
//                 (column r, row p) is the P-point inverse DFT of the band,
//                 folded modulo P and pre-twiddled by w_M^{m r}:
//                   W[r + Q p] = sum_k w_P^{k p} sum_{m = k mod P} X[m] w_M^{m r}.
//                 A workgroup does G consecutive columns so rows are written in
//                 G-element contiguous runs.
#include "cwt_internal.h"
#include "fft_device.h"

namespace cwt {

// ---------------------------------------------------------------------------
// helpers

template <typename R>
__device__ __forceinline__ R sig_at(const R *__restrict__ f, int64_t N, int periodic, int64_t idx) {
    if (periodic) {
        int64_t r = idx % N;
        if (r < 0) r += N;
        return f[r];
    }
    return (idx >= 0 && idx < N) ? f[idx] : (R)0;
}

// x[n] of the whole-signal transform, n in [0, M), promoted to FP64
template <typename R>
__device__ __forceinline__ double fwd_input(const R *__restrict__ f, int64_t N, int mode, int64_t M,
                                            int64_t T, int64_t n) {
    if (mode == LOAD_ZERO) return n < N ? (double)f[n] : 0.0;
    if (mode == LOAD_PERIODIC) return (double)f[n];
    if (n < N + T) return (double)f[n % N];
    if (n >= M - T) {
        int64_t r = (n - M) % N;
        if (r < 0) r += N;
        return (double)f[r];
    }
    return 0.0;
}

// w_M^x = hi[x >> 12] * lo[x & 4095]
template <typename C>
__device__ __forceinline__ C twM(const C *__restrict__ hi, const C *__restrict__ lo, int64_t x) {
    return cmul(hi[x >> 12], lo[x & 4095]);
}

// multiply by i^q
template <typename C> __device__ __forceinline__ C mul_iq(C a, int q) {
    switch (q & 3) {
        case 1: return mk<C>(-a.y, a.x);
        case 2: return mk<C>(-a.x, -a.y);
        case 3: return mk<C>(a.y, -a.x);
        default: return a;
    }
}

// ---------------------------------------------------------------------------
// whole-signal forward transform (FP64)

// single pass: M = P
template <typename RS, int P, int NT>
__global__ __launch_bounds__(NT) void forward_single(const RS *__restrict__ f, int64_t N, int mode,
                                                     int64_t T, const double2 *__restrict__ tw,
                                                     void *__restrict__ Fout, int out_f32) {
    constexpr int LD = lds_len(P);
    __shared__ double2 buf[LD];
    for (int n = threadIdx.x; n < P; n += NT) buf[lidx(n)] = make_double2(fwd_input(f, N, mode, P, T, n), 0.0);
    lds_barrier();
    block_fft<double2, P, 1, NT, LD, -1>(buf, tw);
    for (int k = threadIdx.x; k < P; k += NT) {
        double2 v = buf[lidx(k)];
        if (out_f32) static_cast<float2 *>(Fout)[k] = make_float2((float)v.x, (float)v.y);
        else static_cast<double2 *>(Fout)[k] = v;
    }
}

// four-step pass 1: for n1 in a group of G: Y[k2][n1] = w_M^{-n1 k2} DFT_{M2}(x[n1 + M1 n2])
template <typename RS, int P, int G, int NT>
__global__ __launch_bounds__(NT) void forward_pass1(const RS *__restrict__ f, int64_t N, int mode,
                                                    int64_t M, int64_t T, int64_t M1,
                                                    const double2 *__restrict__ tw,
                                                    const double2 *__restrict__ hi,
                                                    const double2 *__restrict__ lo,
                                                    double2 *__restrict__ Y) {
    constexpr int LD = lds_len(P);
    __shared__ double2 buf[G * LD];
    const int64_t n1_0 = (int64_t)blockIdx.x * G;
    for (int idx = threadIdx.x; idx < G * P; idx += NT) {
        int c = idx % G, n2 = idx / G;
        int64_t n = n1_0 + c + M1 * n2;
        buf[c * LD + lidx(n2)] = make_double2(fwd_input(f, N, mode, M, T, n), 0.0);
    }
    lds_barrier();
    block_fft<double2, P, G, NT, LD, -1>(buf, tw);
    for (int idx = threadIdx.x; idx < G * P; idx += NT) {
        int c = idx % G, k2 = idx / G;
        int64_t n1 = n1_0 + c;
        double2 w = twM(hi, lo, n1 * k2);
        Y[(int64_t)k2 * M1 + n1] = cmulc(buf[c * LD + lidx(k2)], w);
    }
}

// four-step pass 2: for k2 in a group of G: F[k2 + M2 k1] = DFT_{M1}(Y[k2][n1])
template <int P, int G, int NT>
__global__ __launch_bounds__(NT) void forward_pass2(const double2 *__restrict__ Y, int64_t M2,
                                                    const double2 *__restrict__ tw,
                                                    void *__restrict__ Fout, int out_f32) {
    constexpr int LD = lds_len(P);
    __shared__ double2 buf[G * LD];
    const int64_t k2_0 = (int64_t)blockIdx.x * G;
    for (int idx = threadIdx.x; idx < G * P; idx += NT) {
        int c = idx / P, n1 = idx % P;
        buf[c * LD + lidx(n1)] = Y[(k2_0 + c) * P + n1];
    }
    lds_barrier();
    block_fft<double2, P, G, NT, LD, -1>(buf, tw);
    for (int idx = threadIdx.x; idx < G * P; idx += NT) {
        int c = idx % G, k1 = idx / G;
        double2 v = buf[c * LD + lidx(k1)];
        int64_t o = k2_0 + c + M2 * (int64_t)k1;
        if (out_f32) static_cast<float2 *>(Fout)[o] = make_float2((float)v.x, (float)v.y);
        else static_cast<double2 *>(Fout)[o] = v;
    }
}

// ---------------------------------------------------------------------------
// segmented (overlap-save) kernel

template <typename R, int L, int NT, bool PAIR, bool CPLX>
__global__ __launch_bounds__(NT) void local_kernel(const R *__restrict__ f, int64_t N, int periodic,
                                                   int64_t Tg, int64_t V, int64_t nseg, int nscale,
                                                   const int32_t *__restrict__ scale_ids,
                                                   const R *__restrict__ ktab, int cph,
                                                   const cplx_t<R> *__restrict__ tw,
                                                   const double2 *__restrict__ tw64, R *__restrict__ out) {
    using C = cplx_t<R>;
    constexpr int LD = lds_len(L);
    constexpr int E = L / NT;
    static_assert(L % NT == 0, "L must be a multiple of NT");
    // segment forward transform in FP64 (the FP32 inverse buffer aliases it):
    // an FP32 forward would leave rounding noise of order eps |f| in the weak
    // high-frequency bands of red spectra
    __shared__ double2 bufF[LD];
    C *buf = reinterpret_cast<C *>(bufF);
    const int tid = threadIdx.x;
    const int64_t seg = (int64_t)blockIdx.x * (PAIR ? 2 : 1);
    const int64_t x0 = seg * V - Tg;
    for (int u = tid; u < L; u += NT) {
        double a = (double)sig_at(f, N, periodic, x0 + u);
        double b = PAIR ? (double)sig_at(f, N, periodic, x0 + V + u) : 0.0;
        bufF[lidx(u)] = make_double2(a, b);
    }
    lds_barrier();
    block_fft<double2, L, 1, NT, LD, -1>(bufF, tw64);
    C X[E];
#pragma unroll
    for (int i = 0; i < E; ++i) {
        const double2 v = bufF[lidx(tid + i * NT)];
        X[i] = mk<C>((R)v.x, (R)v.y);
    }
    lds_barrier();
    const int64_t b0 = seg * V;
    const bool second = PAIR && (seg + 1 < nseg);
    for (int j = 0; j < nscale; ++j) {
        const R *kt = ktab + (int64_t)j * L;
#pragma unroll
        for (int i = 0; i < E; ++i) {
            int m = tid + i * NT;
            buf[lidx(m)] = mul_iq(cscale(X[i], kt[m]), cph);
        }
        lds_barrier();
        block_fft<C, L, 1, NT, LD, +1>(buf, tw);
        R *row = out + (int64_t)scale_ids[j] * N * (CPLX ? 2 : 1);
        for (int64_t u = tid; u < V; u += NT) {
            int64_t b = b0 + u;
            C v = buf[lidx((int)(Tg + u))];
            if (CPLX) {
                if (b < N) reinterpret_cast<C *>(row)[b] = v;
            } else {
                if (b < N) row[b] = v.x;
                if (second && b + V < N) row[b + V] = v.y;
            }
        }
        lds_barrier();
    }
}

// ---------------------------------------------------------------------------
// band-limited inverse of the whole-signal spectrum (large scales)

template <typename R, int P, int G, int NT, bool PAIR, bool CPLX>
__global__ __launch_bounds__(NT) void column_kernel(const cplx_t<R> *__restrict__ F, int64_t M, int64_t N,
                                                    const ColumnDesc *__restrict__ items,
                                                    const R *__restrict__ tab, int cph,
                                                    const cplx_t<R> *__restrict__ hi,
                                                    const cplx_t<R> *__restrict__ lo,
                                                    const cplx_t<R> *__restrict__ tw, R *__restrict__ out) {
    using C = cplx_t<R>;
    constexpr int LD = lds_len(P);
    __shared__ C buf[G * LD];
    const ColumnDesc d = items[blockIdx.x];
    const int tid = threadIdx.x;
    const int64_t mend = d.mlo + d.B;
    for (int k = tid; k < P; k += NT) {
        C acc[G];
#pragma unroll
        for (int g = 0; g < G; ++g) acc[g] = mk<C>(0, 0);
        int64_t first = (int64_t)k - d.mlo;
        first %= P;
        if (first < 0) first += P;
        for (int64_t m = d.mlo + first; m < mend; m += P) {
            int64_t mm = m % M;
            if (mm < 0) mm += M;
            C fv = F[mm];
            C y;
            if (PAIR) {
                R a = tab[d.taba + (m - d.mlo)];
                R b = d.sb >= 0 ? tab[d.tabb + (m - d.mlo)] : (R)0;
                y = mul_iq(cmul(fv, mk<C>(a, b)), cph);
            } else {
                y = mul_iq(cscale(fv, tab[d.taba + (m - d.mlo)]), cph);
            }
            C base = cmul(y, twM(hi, lo, (mm * d.r0) % M));
            C step = twM(hi, lo, mm);
#pragma unroll
            for (int g = 0; g < G; ++g) {
                acc[g] = cadd(acc[g], base);
                base = cmul(base, step);
            }
        }
#pragma unroll
        for (int g = 0; g < G; ++g) buf[g * LD + lidx(k)] = acc[g];
    }
    lds_barrier();
    block_fft<C, P, G, NT, LD, +1>(buf, tw);
    R *rowa = out + (int64_t)d.sa * N * (CPLX ? 2 : 1);
    R *rowb = (PAIR && d.sb >= 0) ? out + (int64_t)d.sb * N : nullptr;
    for (int idx = tid; idx < G * P; idx += NT) {
        int g = idx % G, p = idx / G;
        int64_t r = d.r0 + g;
        if (r >= d.Q) continue;
        int64_t b = r + d.Q * p;
        if (b >= N) continue;
        C v = buf[g * LD + lidx(p)];
        if (CPLX) reinterpret_cast<C *>(rowa)[b] = v;
        else {
            rowa[b] = v.x;
            if (rowb) rowb[b] = v.y;
        }
    }
}

// ---------------------------------------------------------------------------
// size tables and launchers

bool local_size_ok(int L, int precision) {
    (void)precision;
    int lmax = 4096;
    return L >= 256 && L <= lmax && (L & (L - 1)) == 0;
}
bool column_size_ok(int P, int precision) {
    int pmax = precision == 0 ? 1024 : 2048;
    return P >= 64 && P <= pmax && (P & (P - 1)) == 0;
}
int column_g(int P, int precision) {
    int cap = precision == 0 ? 8192 : 16384;
    int g = cap / P;
    return g > 16 ? 16 : g;
}
int column_nt(int P, int precision) {
    int nt = column_g(P, precision) * P / 16;
    return nt < 64 ? 64 : (nt > 1024 ? 1024 : nt);
}

static const int kFwdSizes[] = {64,  128, 256, 512,  1024, 2048, 4096, 96,   192,  384, 768,  1536,
                                3072, 80, 160, 320, 640, 1280, 2560, 144, 288, 576, 1152, 2304, 4608};
bool fwd_size_ok(int P) {
    for (int s : kFwdSizes)
        if (s == P) return true;
    return false;
}
// columns per workgroup of the forward passes: the largest power of two (<= 16)
// whose FP64 LDS footprint stays within 152 KiB
constexpr int fwd_g(int P) {
    int g = 16;
    while (g > 1 && g * lds_len(P) * 16 > 152 * 1024) g /= 2;
    return g;
}
constexpr int round64(int n) { return ((n + 63) / 64) * 64; }
constexpr int fwd_nt(int P, int G) {
    int nt = round64(G * P / 16);
    return nt < 64 ? 64 : (nt > 1024 ? 1024 : nt);
}

template <typename RS, int P>
static hipError_t fwd_single_launch(const Plan &p, const RS *f, void *F, hipStream_t st) {
    constexpr int NT = fwd_nt(P, 1) > 512 ? 512 : fwd_nt(P, 1);
    const double2 *tw = tw_ptr<double2>(p, P, true);
    hipLaunchKernelGGL((forward_single<RS, P, NT>), dim3(1), dim3(NT), 0, st, f, p.N, p.load_mode, p.Twrap,
                       tw, F, p.precision == 1 ? 1 : 0);
    return hipGetLastError();
}

template <typename RS, int P>
static hipError_t fwd_pass1_launch(const Plan &p, const RS *f, double2 *Y, hipStream_t st) {
    constexpr int G = fwd_g(P);
    constexpr int NT = fwd_nt(P, G);
    if (p.M1 % G) return hipErrorInvalidValue;
    hipLaunchKernelGGL((forward_pass1<RS, P, G, NT>), dim3(p.M1 / G), dim3(NT), 0, st, f, p.N, p.load_mode,
                       p.M, p.Twrap, (int64_t)p.M1, tw_ptr<double2>(p, P, true),
                       tw_at<double2>(p, p.twM64_hi_off), tw_at<double2>(p, p.twM64_lo_off), Y);
    return hipGetLastError();
}

template <int P>
static hipError_t fwd_pass2_launch(const Plan &p, const double2 *Y, void *F, hipStream_t st) {
    constexpr int G = fwd_g(P);
    constexpr int NT = fwd_nt(P, G);
    if (p.M2 % G) return hipErrorInvalidValue;
    hipLaunchKernelGGL((forward_pass2<P, G, NT>), dim3(p.M2 / G), dim3(NT), 0, st, Y, (int64_t)p.M2,
                       tw_ptr<double2>(p, P, true), F, p.precision == 1 ? 1 : 0);
    return hipGetLastError();
}

#define CWT_FWD_SIZES(X) \
    X(64) X(128) X(256) X(512) X(1024) X(2048) X(4096) X(96) X(192) X(384) X(768) X(1536) X(3072) \
    X(80) X(160) X(320) X(640) X(1280) X(2560) X(144) X(288) X(576) X(1152) X(2304) X(4608)

template <typename RS>
static hipError_t forward_typed(const Plan &p, const RS *f, void *ws, hipStream_t st) {
    char *w = static_cast<char *>(ws);
    void *F = w + p.ws_F_off;
    double2 *Y = reinterpret_cast<double2 *>(w + p.ws_Y_off);
    if (p.M2 <= 1) {
        switch (p.M1) {
#define X(S) case S: return fwd_single_launch<RS, S>(p, f, F, st);
            CWT_FWD_SIZES(X)
#undef X
            default: return hipErrorInvalidValue;
        }
    }
    hipError_t e = hipErrorInvalidValue;
    switch (p.M2) {
#define X(S) case S: e = fwd_pass1_launch<RS, S>(p, f, Y, st); break;
        CWT_FWD_SIZES(X)
#undef X
        default: return hipErrorInvalidValue;
    }
    if (e != hipSuccess) return e;
    switch (p.M1) {
#define X(S) case S: return fwd_pass2_launch<S>(p, Y, F, st);
        CWT_FWD_SIZES(X)
#undef X
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_forward(const Plan &p, const void *signal, void *ws, hipStream_t st) {
    if (p.precision == 0) return forward_typed(p, static_cast<const double *>(signal), ws, st);
    return forward_typed(p, static_cast<const float *>(signal), ws, st);
}

template <typename R, int L>
static hipError_t local_launch_L(const Plan &p, const LocalGroup &g, const R *f, R *out, hipStream_t st) {
    constexpr int NT = L / 16 > 1024 ? 1024 : (L / 16 < 64 ? 64 : L / 16);
    using C = cplx_t<R>;
    const R *ktab = static_cast<const R *>(p.d_tab) + g.tab_off;
    const C *tw = tw_ptr<C>(p, L, false);
    const double2 *tw64 = sizeof(R) == 8 ? reinterpret_cast<const double2 *>(tw) : tw_ptr<double2>(p, L, true);
    int periodic = p.boundary == 0 ? 1 : 0;
    int64_t grid = p.pair_real ? (g.nseg + 1) / 2 : g.nseg;
    if (grid <= 0) return hipSuccess;
    if (p.cplx_out)
        hipLaunchKernelGGL((local_kernel<R, L, NT, false, true>), dim3((unsigned)grid), dim3(NT), 0, st, f,
                           p.N, periodic, g.Tg, g.V, g.nseg, (int)g.scales.size(), g.d_scales, ktab, p.cph, tw,
                           tw64, out);
    else if (p.pair_real)
        hipLaunchKernelGGL((local_kernel<R, L, NT, true, false>), dim3((unsigned)grid), dim3(NT), 0, st, f,
                           p.N, periodic, g.Tg, g.V, g.nseg, (int)g.scales.size(), g.d_scales, ktab, p.cph, tw,
                           tw64, out);
    else
        hipLaunchKernelGGL((local_kernel<R, L, NT, false, false>), dim3((unsigned)grid), dim3(NT), 0, st, f,
                           p.N, periodic, g.Tg, g.V, g.nseg, (int)g.scales.size(), g.d_scales, ktab, p.cph, tw,
                           tw64, out);
    return hipGetLastError();
}

std::string local_kernel_name(const Plan &p, const LocalGroup &g) {
    return std::string("local_kernel<") + (p.precision == 0 ? "f64," : "f32,") + std::to_string(g.L) +
           (p.cplx_out ? ",complex>" : (p.pair_real ? ",real-pair>" : ",real>"));
}

std::string column_kernel_name(const Plan &p, const ColumnLaunch &c) {
    return std::string("column_kernel<") + (p.precision == 0 ? "f64," : "f32,") + std::to_string(c.P) + "," +
           std::to_string(c.G) + (p.cplx_out ? ",complex>" : ",real-pair>");
}

hipError_t launch_local(const Plan &p, const LocalGroup &g, const void *signal, void *out, hipStream_t st) {
    if (p.precision == 0) {
        const double *f = static_cast<const double *>(signal);
        double *o = static_cast<double *>(out);
        switch (g.L) {
            case 256: return local_launch_L<double, 256>(p, g, f, o, st);
            case 512: return local_launch_L<double, 512>(p, g, f, o, st);
            case 1024: return local_launch_L<double, 1024>(p, g, f, o, st);
            case 2048: return local_launch_L<double, 2048>(p, g, f, o, st);
            case 4096: return local_launch_L<double, 4096>(p, g, f, o, st);
            default: return hipErrorInvalidValue;
        }
    }
    const float *f = static_cast<const float *>(signal);
    float *o = static_cast<float *>(out);
    switch (g.L) {
        case 256: return local_launch_L<float, 256>(p, g, f, o, st);
        case 512: return local_launch_L<float, 512>(p, g, f, o, st);
        case 1024: return local_launch_L<float, 1024>(p, g, f, o, st);
        case 2048: return local_launch_L<float, 2048>(p, g, f, o, st);
        case 4096: return local_launch_L<float, 4096>(p, g, f, o, st);
        default: return hipErrorInvalidValue;
    }
}

template <typename R, int P, int G>
static hipError_t column_launch_P(const Plan &p, const ColumnLaunch &c, const void *ws, R *out, hipStream_t st) {
    constexpr int NT = fwd_nt(P, G);
    using C = cplx_t<R>;
    const C *F = reinterpret_cast<const C *>(static_cast<const char *>(ws) + p.ws_F_off);
    const R *tab = static_cast<const R *>(p.d_tab);
    const C *hi = tw_at<C>(p, p.twM_hi_off), *lo = tw_at<C>(p, p.twM_lo_off);
    const C *tw = tw_ptr<C>(p, P, false);
    unsigned grid = (unsigned)c.items.size();
    if (grid == 0) return hipSuccess;
    if (p.cplx_out)
        hipLaunchKernelGGL((column_kernel<R, P, G, NT, false, true>), dim3(grid), dim3(NT), 0, st, F, p.M, p.N,
                           c.d_items, tab, p.cph, hi, lo, tw, out);
    else
        hipLaunchKernelGGL((column_kernel<R, P, G, NT, true, false>), dim3(grid), dim3(NT), 0, st, F, p.M, p.N,
                           c.d_items, tab, p.cph, hi, lo, tw, out);
    return hipGetLastError();
}

hipError_t launch_column(const Plan &p, const ColumnLaunch &c, const void *ws, void *out, hipStream_t st) {
    if (p.precision == 0) {
        double *o = static_cast<double *>(out);
        switch (c.P) {
            case 64: return column_launch_P<double, 64, 16>(p, c, ws, o, st);
            case 128: return column_launch_P<double, 128, 16>(p, c, ws, o, st);
            case 256: return column_launch_P<double, 256, 16>(p, c, ws, o, st);
            case 512: return column_launch_P<double, 512, 16>(p, c, ws, o, st);
            case 1024: return column_launch_P<double, 1024, 8>(p, c, ws, o, st);
            default: return hipErrorInvalidValue;
        }
    }
    float *o = static_cast<float *>(out);
    switch (c.P) {
        case 64: return column_launch_P<float, 64, 16>(p, c, ws, o, st);
        case 128: return column_launch_P<float, 128, 16>(p, c, ws, o, st);
        case 256: return column_launch_P<float, 256, 16>(p, c, ws, o, st);
        case 512: return column_launch_P<float, 512, 16>(p, c, ws, o, st);
        case 1024: return column_launch_P<float, 1024, 16>(p, c, ws, o, st);
        case 2048: return column_launch_P<float, 2048, 8>(p, c, ws, o, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace cwt
