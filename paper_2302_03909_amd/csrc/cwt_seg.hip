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

// Raw buffer accesses (vector memory instructions) with the descriptor's
// bounds check: an access whose byte offset lies beyond num_records is
// dropped (store) or returns zero (load), so predicated lanes need no branch
// and every wave issues the same number of memory instructions.
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
constexpr uint32_t kOOB = 0x80000000u;  // beyond every descriptor used here (< 2 GiB)
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void *base, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), 0, (int)bytes, 0x00020000);
}
__device__ __forceinline__ void bstore(float v, __amdgpu_buffer_rsrc_t r, uint32_t off) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, v), r, off, 0, 0);
}
__device__ __forceinline__ void bstore(double v, __amdgpu_buffer_rsrc_t r, uint32_t off) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, off, 0, 0);
}
__device__ __forceinline__ void bstore(float2 v, __amdgpu_buffer_rsrc_t r, uint32_t off) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, off, 0, 0);
}
__device__ __forceinline__ void bstore(double2 v, __amdgpu_buffer_rsrc_t r, uint32_t off) {
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, v), r, off, 0, 0);
}
__device__ __forceinline__ float bload(const float *, __amdgpu_buffer_rsrc_t r, uint32_t off) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}
__device__ __forceinline__ double bload(const double *, __amdgpu_buffer_rsrc_t r, uint32_t off) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}

template <typename C> __device__ __forceinline__ C to_c(double2 v) { return mk<C>((decltype(C::x))v.x, (decltype(C::x))v.y); }
template <typename C> __device__ __forceinline__ double2 to_d(C v) { return make_double2((double)v.x, (double)v.y); }

// ---------------------------------------------------------------------------
// pruned forward transform of the segments, partial sums per column chunk.
// Work item (g, seg, chunk): columns q in [chunk * iters * 16, +iters * 16).

template <typename R, int P, int NT>
__global__ __launch_bounds__(NT) void seg_forward_kernel(const R *__restrict__ f, int64_t N, int periodic,
                                                         const SegGroupDev *__restrict__ groups,
                                                         const SegWork *__restrict__ work,
                                                         const cplx_t<R> *__restrict__ twl_g,
                                                         const double2 *__restrict__ whi,
                                                         const double2 *__restrict__ wlo, char *__restrict__ ws) {
    using C = cplx_t<R>;
    constexpr int G = 16;
    constexpr int LD = lds_len(P);
    constexpr int E = G * P / NT;  // samples per thread per iteration
    static_assert(NT >= P && (G * P) % NT == 0, "launch shape");
    __shared__ C buf[G * LD];
    __shared__ C twl[twl_len(P)];
    load_twl<C, P, NT>(twl, twl_g);
    const SegWork w = work[blockIdx.x];
    const SegGroupDev gd = groups[w.g];
    const int64_t L = int64_t(1) << gd.lgL, Q = L >> log2_exact(P);
    const int sh = 23 - gd.lgL;
    const int64_t x0 = (int64_t)w.seg * gd.V - gd.Tg;
    const int tid = threadIdx.x;
    const int B = gd.B;
    double2 acc = make_double2(0.0, 0.0), base = acc, step = acc, w16 = acc;
    int kap = 0;
    if (tid < B) {
        int64_t mm = (gd.klo + tid) & (L - 1);
        kap = (int)(mm & (P - 1));
        double2 s1 = w23(whi, wlo, mm << sh);
        step = make_double2(s1.x, -s1.y);
        double2 s16 = w23(whi, wlo, ((16 * mm) & (L - 1)) << sh);
        w16 = make_double2(s16.x, -s16.y);
        int64_t qf = (int64_t)w.idx * gd.iters * G;
        double2 b = w23(whi, wlo, ((qf * mm) & (L - 1)) << sh);
        base = make_double2(b.x, -b.y);
    }
    R xn[E];
    {
        const int64_t q0 = (int64_t)w.idx * gd.iters * G;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            int idx = tid + e * NT;
            xn[e] = sig_seg(f, N, periodic, x0 + q0 + (idx % G) + Q * (idx / G));
        }
    }
    auto emit = [&](int c, int p, C v) { buf[c * LD + lidx(p)] = v; };
    for (int it = 0; it < gd.iters; ++it) {
#pragma unroll
        for (int e = 0; e < E; ++e) {
            int idx = tid + e * NT;
            buf[(idx % G) * LD + lidx(idx / G)] = mk<C>(xn[e], (decltype(C::x))0);
        }
        if (it + 1 < gd.iters) {
            const int64_t q1 = ((int64_t)w.idx * gd.iters + it + 1) * G;
#pragma unroll
            for (int e = 0; e < E; ++e) {
                int idx = tid + e * NT;
                xn[e] = sig_seg(f, N, periodic, x0 + q1 + (idx % G) + Q * (idx / G));
            }
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
    if (tid < B) {
        double2 *Xp = reinterpret_cast<double2 *>(ws + gd.xp_off);
        Xp[((int64_t)w.seg * gd.nchunk + w.idx) * B + tid] = acc;
    }
}

// X[seg][k] = sum over the column chunks of the partial sums, 16 bins per
// workgroup, 16 lanes per bin, fixed summation order
__global__ __launch_bounds__(256) void seg_reduce_kernel(const SegGroupDev *__restrict__ groups,
                                                         const SegWork *__restrict__ work, char *__restrict__ ws) {
    __shared__ double2 part[256];
    const SegWork w = work[blockIdx.x];
    const SegGroupDev gd = groups[w.g];
    const int kb = threadIdx.x / 16, lane = threadIdx.x % 16;
    const int k = w.idx * 16 + kb;
    const double2 *Xp = reinterpret_cast<const double2 *>(ws + gd.xp_off);
    double2 a = make_double2(0.0, 0.0);
    if (k < gd.B)
        for (int c = lane; c < gd.nchunk; c += 16) a = cadd(a, Xp[((int64_t)w.seg * gd.nchunk + c) * gd.B + k]);
    part[threadIdx.x] = a;
    __syncthreads();
    for (int st = 8; st > 0; st >>= 1) {
        if (lane < st) part[threadIdx.x] = cadd(part[threadIdx.x], part[threadIdx.x + st]);
        __syncthreads();
    }
    if (lane == 0 && k < gd.B) {
        double2 *X = reinterpret_cast<double2 *>(ws + gd.x_off);
        X[(int64_t)w.seg * gd.B + k] = part[threadIdx.x];
    }
}

// LDS elements for the staged spectrum samples of one BAND group: at most
// 16 KiB, and at least one unit (two tables for a real-wavelet pair) of P bins
constexpr int seg_kls_elems(int rbytes, int P) {
    int n = 16384 / rbytes;
    return n < 2 * P ? 2 * P : n;
}

// ---------------------------------------------------------------------------
// band-limited inverse: work item (g, seg, r0) covers columns r0..r0+15 of one
// segment for every output unit of the group

template <typename R, int P, int NT, bool PAIR, bool CPLX>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(sizeof(R) == 4 && !PAIR ? 3 : 2))) void seg_inverse_kernel(int64_t N, const SegGroupDev *__restrict__ groups,
                                                         const SegUnit *__restrict__ units,
                                                         const SegWork *__restrict__ work,
                                                         const char *__restrict__ ws, const R *__restrict__ ktab,
                                                         int cph, const char *__restrict__ twbase,
                                                         const cplx_t<R> *__restrict__ twl_g,
                                                         const double2 *__restrict__ whi,
                                                         const double2 *__restrict__ wlo, R *__restrict__ out) {
    using C = cplx_t<R>;
    constexpr int G = 16;
    constexpr int LD = lds_len(P);
    constexpr int MAXU = 32;
    constexpr int NB = P / 16;  // pass-0 butterflies per column
    constexpr int KLS = seg_kls_elems(sizeof(R), P);
    static_assert(NT == P, "one pass-0 butterfly per thread");
    __shared__ C buf[G * LD];
    __shared__ C twl[twl_len(P)];
    __shared__ SegUnit us[MAXU];
    __shared__ R kls[KLS];  // spectrum samples of the group's units (and pair partners)
    load_twl<C, P, NT>(twl, twl_g);
    const SegWork w = work[blockIdx.x];
    const SegGroupDev gd = groups[w.g];
    const int nunits = gd.nunits < MAXU ? gd.nunits : MAXU;
    for (int u = threadIdx.x; u < nunits; u += NT) us[u] = units[gd.unit0 + u];
    const int64_t L = int64_t(1) << gd.lgL, Q = L >> log2_exact(P);
    const int sh = 23 - gd.lgL;
    const int tid = threadIdx.x;
    const int B = gd.B;
    const int64_t r0 = w.idx;
    // band spectrum of the segment times w_L^{m r0}, staged in LDS (reuses buf)
    C *xs = buf;
    if (tid < B) {
        int64_t mm = (gd.klo + tid) & (L - 1);
        const double2 *X = reinterpret_cast<const double2 *>(ws + gd.x_off);
        xs[tid] = to_c<C>(cmul(X[(int64_t)w.seg * B + tid], w23(whi, wlo, ((mm * r0) & (L - 1)) << sh)));
    }
    __syncthreads();
    // pass-0 inputs of this thread: column c, positions kap = i + r P/16; the
    // band bin congruent to kap modulo P (if any) and w_L^{m c}
    const int c = tid / NB, i = tid % NB;
    // first(r): band bin congruent to i + r P/16 (valid when < B)
    const int f0 = (int)(((int64_t)i - gd.klo) & (P - 1));
    auto first_of = [&](int r) { return (f0 + r * NB) & (P - 1); };
    C xg[16];
    {
        const C *gtw = reinterpret_cast<const C *>(twbase + gd.gtw_off) + (int64_t)c * B;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            int fr = first_of(r);
            xg[r] = fr < B ? cmul(xs[fr], gtw[fr]) : mk<C>(0, 0);
        }
    }
    // spectrum samples of every unit of the group, staged in LDS once
    for (int t = tid; t < nunits * B; t += NT) {
        const int u = t / B, k = t % B;
        kls[u * B + k] = ktab[us[u].ka + k];
        if constexpr (PAIR) kls[nunits * B + u * B + k] = us[u].sb >= 0 ? ktab[us[u].kb + k] : (R)0;
    }
    // band bin read for position r; bins outside the band read bin 0, which
    // is harmless because xg[r] is zero there.  The phase i^cph of the
    // wavelet's spectrum is common to every unit and folded into xg.
    int fro[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        int fr = first_of(r);
        fro[r] = fr < B ? fr : 0;
        xg[r] = mul_i_pow(xg[r], cph);
    }
    __syncthreads();  // xs (in buf) is no longer read
    const int64_t ob = (int64_t)w.seg * gd.V - gd.Tg;
    const uint32_t eb = (uint32_t)(CPLX ? sizeof(C) : sizeof(R));
    for (int u = 0; u < nunits; ++u) {
        // unit fields are uniform; say so, so that the store descriptors
        // live in scalar registers
        const int sa = __builtin_amdgcn_readfirstlane(us[u].sa);
        const int sb = __builtin_amdgcn_readfirstlane(us[u].sb);
        C v[16];
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const R ka = kls[u * B + fro[r]];
            if constexpr (PAIR) {
                const R kb = kls[nunits * B + u * B + fro[r]];
                v[r] = cmul(xg[r], mk<C>(ka, kb));
            } else {
                v[r] = cscale(xg[r], ka);
            }
        }
        cols_pass0_regs<C, P, G, NT, LD, +1>(buf, v);
        // output b = ob + r0 + cc + Q p, kept when Tg <= r0 + cc + Q p < Tg + V; the
        // descriptor of each row spans exactly its N values, so b >= N is dropped
        const __amdgpu_buffer_rsrc_t ra =
            make_rsrc(out + (int64_t)sa * N * (CPLX ? 2 : 1), (uint32_t)(N * eb));
        const __amdgpu_buffer_rsrc_t rb =
            make_rsrc(out + (int64_t)(PAIR && sb >= 0 ? sb : sa) * N, (uint32_t)(N * eb));
        const bool has_b = PAIR && sb >= 0;
        const int64_t lo_all = gd.Tg - r0, hi_all = gd.Tg + gd.V - r0;
        const int64_t obr = ob + r0;
        auto emit = [&](int cc, int p, C val) {
            const int64_t o = cc + Q * p;
            const uint32_t off = (o >= lo_all && o < hi_all) ? (uint32_t)((obr + o) * (int64_t)eb) : kOOB;
            if (CPLX) bstore(val, ra, off);
            else {
                bstore(val.x, ra, off);
                bstore(val.y, rb, has_b ? off : kOOB);
            }
        };
        cols_fft_after0<C, P, G, NT, LD, +1, false>(buf, twl, emit);
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// fused full-spectrum segments (small scales)

template <typename R, int L, int NCOL, int NT, bool PAIR, bool CPLX>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(sizeof(R) == 4 ? 3 : 2))) void local2_kernel(const R *__restrict__ f, int64_t N, int periodic, int64_t Tg,
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
    // spectra in registers in the pass-0 layout of the inverse transforms:
    // thread t owns column c = t / (L/16), positions i + r L/16
    static_assert(E == 16, "one radix-16 butterfly per thread");
    constexpr int NB = L / 16;
    const int cc = tid / NB, ii = tid % NB;
    C Xr[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) Xr[r] = mul_i_pow(buf[cc * LD + lidx(ii + r * NB)], cph);  // phase i^cph folded in
    R kv[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) kv[r] = ktab[ii + r * NB];
    __syncthreads();
    for (int j = 0; j < nscale; ++j) {
        C v[16];
#pragma unroll
        for (int r = 0; r < 16; ++r) v[r] = cscale(Xr[r], kv[r]);
        if (j + 1 < nscale) {  // prefetch the next scale's spectrum samples
            const R *kt = ktab + (int64_t)(j + 1) * L;
#pragma unroll
            for (int r = 0; r < 16; ++r) kv[r] = kt[ii + r * NB];
        }
        // keep the prefetch loads ahead of this scale's stores (no code emitted)
        asm volatile("" ::: "memory");
        cols_pass0_regs<C, L, NCOL, NT, LD, +1>(buf, v);
        constexpr uint32_t eb = (uint32_t)(CPLX ? sizeof(C) : sizeof(R));
        const __amdgpu_buffer_rsrc_t rr =
            make_rsrc(out + (int64_t)scale_ids[j] * N * (CPLX ? 2 : 1), (uint32_t)(N * eb));
        auto emit = [&](int c, int p, C val) {
            const bool inside = p >= Tg && p < Tg + V;
            const int64_t sgi = seg0 + (int64_t)c * SEGS;
            const int64_t b = sgi * V + (p - Tg);
            const uint32_t off = inside ? (uint32_t)(b * (int64_t)eb) : kOOB;
            if (CPLX) bstore(val, rr, off);
            else {
                bstore(val.x, rr, off);
                if (PAIR) bstore(val.y, rr, (inside && sgi + 1 < nseg) ? (uint32_t)((b + V) * (int64_t)eb) : kOOB);
            }
        };
        cols_fft_after0<C, L, NCOL, NT, LD, +1, false>(buf, twl, emit);
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
    (void)precision;
    int pmax = 512;
    return P >= 64 && P <= pmax && (P & (P - 1)) == 0;
}

template <typename R, int P>
static hipError_t seg_launch_P(const Plan &p, const SegLaunch &l, const R *f, void *ws, R *out, hipStream_t st,
                               int phase) {
    constexpr int NT = P;  // 16 columns x P / 16 elements per thread
    using C = cplx_t<R>;
    char *w = static_cast<char *>(ws);
    const C *twl = tw_at<C>(p, l.twl_off);
    const double2 *whi = tw_at<double2>(p, p.w23_hi_off), *wlo = tw_at<double2>(p, p.w23_lo_off);
    int periodic = p.boundary == 0 ? 1 : 0;
    if (phase == 0) {
        if (l.fwd.empty()) return hipSuccess;
        hipLaunchKernelGGL((seg_forward_kernel<R, P, NT>), dim3((unsigned)l.fwd.size()), dim3(NT), 0, st, f, p.N,
                           periodic, l.d_groups, l.d_fwd, twl, whi, wlo, w);
        return hipGetLastError();
    }
    if (phase == 1) {
        if (l.red.empty()) return hipSuccess;
        hipLaunchKernelGGL(seg_reduce_kernel, dim3((unsigned)l.red.size()), dim3(256), 0, st, l.d_groups, l.d_red, w);
        return hipGetLastError();
    }
    if (l.inv.empty()) return hipSuccess;
    const R *ktab = static_cast<const R *>(p.d_tab);
    const char *twbase = static_cast<const char *>(p.d_tw_all);
    if (p.cplx_out)
        hipLaunchKernelGGL((seg_inverse_kernel<R, P, NT, false, true>), dim3((unsigned)l.inv.size()), dim3(NT), 0, st,
                           p.N, l.d_groups, p.d_units, l.d_inv, w, ktab, p.cph, twbase, twl, whi, wlo, out);
    else
        hipLaunchKernelGGL((seg_inverse_kernel<R, P, NT, true, false>), dim3((unsigned)l.inv.size()), dim3(NT), 0, st,
                           p.N, l.d_groups, p.d_units, l.d_inv, w, ktab, p.cph, twbase, twl, whi, wlo, out);
    return hipGetLastError();
}

template <typename R>
static hipError_t seg_typed(const Plan &p, const SegLaunch &l, const R *f, void *ws, R *o, hipStream_t st, int phase) {
    switch (l.P) {
        case 64: return seg_launch_P<R, 64>(p, l, f, ws, o, st, phase);
        case 128: return seg_launch_P<R, 128>(p, l, f, ws, o, st, phase);
        case 256: return seg_launch_P<R, 256>(p, l, f, ws, o, st, phase);
        case 512: return seg_launch_P<R, 512>(p, l, f, ws, o, st, phase);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_seg(const Plan &p, const SegLaunch &l, const void *signal, void *ws, void *out, hipStream_t st,
                      int phase) {
    if (p.precision == 0)
        return seg_typed(p, l, static_cast<const double *>(signal), ws, static_cast<double *>(out), st, phase);
    return seg_typed(p, l, static_cast<const float *>(signal), ws, static_cast<float *>(out), st, phase);
}

std::string local2_kernel_name(const Plan &p, const SegGroup &g) {
    std::string t = p.precision == 0 ? "f64," : "f32,";
    return "local2_kernel<" + t + std::to_string(g.L) + (p.cplx_out ? ",complex>" : ",real-pair>");
}

std::string seg_kernel_name(const Plan &p, const SegLaunch &l, int phase) {
    std::string t = p.precision == 0 ? "f64," : "f32,";
    if (phase == 0) return "seg_forward_kernel<" + t + std::to_string(l.P) + ">";
    if (phase == 1) return "seg_reduce_kernel<" + t + std::to_string(l.P) + ">";
    return "seg_inverse_kernel<" + t + std::to_string(l.P) + (p.cplx_out ? ",complex>" : ",real-pair>");
}

}  // namespace cwt
