// cwt_seg.hip -- segmented (overlap-save) FFT method for gfx950.
//
// The product W = IDFT(DFT(f) * conj(Psi_s)) of Sec. 3.1 (Eq.
// discrete_CWT_conv, with the aliased spectrum of the sampled wavelet) is
// evaluated segment by segment: a segment of L samples starting Tg before
// its first output yields V = L - 2 Tg valid outputs, because the wavelet at
// every scale of the group is negligible beyond Tg samples (L = 2^l for the
// small scales, L = c 2^l with c odd for the larger ones).
//
// Small scales (wide spectrum relative to L): local2_kernel takes the full
// L-point FFT of NCOL segments per workgroup, keeps the spectra in registers
// and, for every scale of the group, multiplies and inverts in LDS.
//
// Larger scales (the spectrum at length L occupies B <= P << L bins): the
// segment spectrum is needed only on the band [klo, klo + B).  With L = P Q:
//   forward  X[m] = sum_q w_L^{-q m} DFT_P(x[q + Q p])[m mod P]
//            (seg_forward_kernel: 16 real columns q per iteration, packed
//             two per complex P-point FFT, FP64 sums, partial sums per
//             column chunk, then seg_reduce_kernel)
//   inverse  W[r + Q p] = DFT_P^{-1}( Y[m] w_L^{m r} )[p],  m = k mod P
//            (seg_inverse_kernel: 16 consecutive columns r per workgroup, so
//             the last FFT pass stores 16-element runs straight to HBM; 32

#include "seg_kernels.h"

namespace cwt {

// ---------------------------------------------------------------------------
// pruned forward transform of the segments, partial sums per column chunk.
// Work item (g, seg, chunk): columns q in [chunk * iters * 16, +iters * 16).

template <typename R, int P, int NT>
__global__ __launch_bounds__(NT) void seg_forward_kernel(const BatchArgs a) {
    using C = cplx_t<R>;
    constexpr int G = 16;       // real columns per iteration
    constexpr int GC = G / 2;   // complex columns: real columns 2z and 2z+1 share column z
    // column stride = 2 (mod 16) complex elements: the sample scatter below
    // (16 real columns x consecutive rows per wave) then hits distinct banks
    constexpr int LD = lds_len(P) + 1;
    constexpr int E = G * P / NT;  // samples per thread per iteration
    static_assert(NT >= P && (G * P) % NT == 0, "launch shape");
    __shared__ C buf[GC * LD];
    __shared__ C twl[twl_len(P)];
    const Resolved rv = resolve(a);
    const KeyDesc *kd = &rv.kd;
    const R *__restrict__ f = static_cast<const R *>(rv.bi.f);
    char *__restrict__ ws = rv.bi.ws;
    const int64_t N = kd->N;
    const int periodic = kd->periodic;
    const double2 *__restrict__ whi = kd->whi, *__restrict__ wlo = kd->wlo;
    load_twl<C, P, NT>(twl, static_cast<const C *>(kd->twl));
    const SegWork w = cload(kd->work + rv.local);
    const SegGroupDev gd = cload(kd->groups + w.g);
    const int64_t L = gd.L, Q = gd.Q;
    const int cL = __builtin_amdgcn_readfirstlane(gd.cL), kL = __builtin_amdgcn_readfirstlane(gd.lgL);
    const double2 *__restrict__ wsm = reinterpret_cast<const double2 *>(kd->twbase + gd.wsm_off);
    const int tid = threadIdx.x;
    const int B = gd.B;
    // bins of this thread: step = w_L^{-m}, step2 = w_L^{-2m}, w14 =
    // w_L^{-14 m}, w16 = w_L^{-16 m}, and the chunk's first-column factor
    // base0 = w_L^{-q0 m}
    const int64_t q0 = (int64_t)w.idx * gd.iters * G;
    double2 acc = make_double2(0.0, 0.0), base0 = acc, base = acc, step = acc, step2 = acc, w14 = acc, w16 = acc;
    double cc2 = 0.0;  // 2 cos(2 theta), theta = 2 pi m / L
    int kap = 0, kam = 0;
    if (tid < B) {
        const int64_t mm = mod_seg(gd.klo + tid, cL, L);
        kap = (int)(mm & (P - 1));  // P divides L
        kam = (P - kap) & (P - 1);
        double2 s1 = w_seg(whi, wlo, wsm, cL, kL, mm);
        step = make_double2(s1.x, -s1.y);
        step2 = cmul(step, step);
        cc2 = 2.0 * step2.x;
        double2 s14 = w_seg(whi, wlo, wsm, cL, kL, mod_seg(14 * mm, cL, L));
        w14 = make_double2(s14.x, -s14.y);
        double2 s16 = w_seg(whi, wlo, wsm, cL, kL, mod_seg(16 * mm, cL, L));
        w16 = make_double2(s16.x, -s16.y);
        double2 b = w_seg(whi, wlo, wsm, cL, kL, mod_seg(q0 * mm, cL, L));
        base0 = make_double2(b.x, -b.y);
        base = base0;
    }
    // flat loop over (segment, iteration) pairs of this work item: w.pad
    // consecutive segments, gd.iters iterations of 16 columns each; the next
    // step's samples are loaded during this step
    const int total = w.pad * gd.iters;
    // sample e of step t: x[sg V - Tg + q + tid % G + Q (tid / G + e NT / G)]
    // (idx = tid + e NT, NT a multiple of G).  Zero boundary: raw buffer
    // loads over f[0, N) with 32-bit offsets; positions outside, negative
    // ones included (they wrap to large unsigned offsets), read 0.
    const __amdgpu_buffer_rsrc_t fr = make_rsrc(f, (uint32_t)(N * (int64_t)sizeof(R)));
    auto pos0 = [&](int t) {
        const int64_t sg = w.seg + t / gd.iters;
        const int64_t q = q0 + (int64_t)(t % gd.iters) * G;
        return sg * gd.V - gd.Tg + q + (tid % G) + Q * (tid / G);
    };
    const int64_t estep = Q * (NT / G);
    auto load_step = [&](int t, R (&x)[E]) {
        const int64_t x0 = pos0(t);
        if (periodic) {
#pragma unroll
            for (int e = 0; e < E; ++e) x[e] = sig_seg(f, N, 1, x0 + e * estep);
        } else {
            const uint32_t o0 = (uint32_t)(x0 * (int64_t)sizeof(R)), os = (uint32_t)(estep * (int64_t)sizeof(R));
#pragma unroll
            for (int e = 0; e < E; ++e) x[e] = bload((const R *)nullptr, fr, o0 + (uint32_t)e * os);
        }
    };
    R xn[E];
    load_step(0, xn);
    auto emit = [&](int c, int p, C v) { buf[c * LD + lidx(p)] = v; };
    R *bufr = reinterpret_cast<R *>(buf);
    for (int t = 0; t < total; ++t) {
        // real column g of row p -> component g & 1 of complex column g / 2
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int idx = tid + e * NT, g = idx % G;
            bufr[2 * ((g >> 1) * LD + lidx(idx / G)) + (g & 1)] = xn[e];
        }
        if (t + 1 < total) load_step(t + 1, xn);
        lds_barrier();
        cols_fft<C, P, GC, NT, LD, -1, true>(buf, twl, emit);
        lds_barrier();
        if (tid < B) {
            // With Z = DFT(x_{2z} + i x_{2z+1}):  DFT(x_{2z})[k] = (Z[k] + conj Z[-k]) / 2
            // and DFT(x_{2z+1})[k] = (Z[k] - conj Z[-k]) / 2i (the 1/2 is applied
            // once per step).  The sum over the 16 columns,
            //   sum_z ye_z e^{-2 i theta z} + e^{-i theta} sum_z yo_z e^{-2 i theta z},
            // is taken by two Goertzel recurrences at angle 2 theta (even and
            // odd columns): s_z = y_z + 2 cos(2 theta) s_{z-1} - s_{z-2}, and
            //   sum_{z<8} y_z e^{-2 i theta z} = e^{-14 i theta} (s_7 - e^{-2 i theta} s_6).
            // Eight terms per recurrence keep its rounding at a few tens of ulps.
            double2 e1 = make_double2(0.0, 0.0), e2 = e1, o1 = e1, o2 = e1;
#pragma unroll
            for (int z = 0; z < GC; ++z) {
                const double2 zk = to_d(buf[z * LD + lidx(kap)]), zm = to_d(buf[z * LD + lidx(kam)]);
                const double2 ye = make_double2(zk.x + zm.x, zk.y - zm.y);
                const double2 yo = make_double2(zk.y + zm.y, zm.x - zk.x);
                const double2 en = make_double2(fma(cc2, e1.x, ye.x - e2.x), fma(cc2, e1.y, ye.y - e2.y));
                const double2 on = make_double2(fma(cc2, o1.x, yo.x - o2.x), fma(cc2, o1.y, yo.y - o2.y));
                e2 = e1;
                e1 = en;
                o2 = o1;
                o1 = on;
            }
            const double2 te = csub(e1, cmul(step2, e2)), tq = csub(o1, cmul(step2, o2));
            const double2 sum = cmul(cmul(base, w14), cadd(te, cmul(step, tq)));
            acc = cadd(acc, make_double2(0.5 * sum.x, 0.5 * sum.y));
            base = cmul(base, w16);
            if (t % gd.iters == gd.iters - 1) {  // segment complete
                const int64_t sg = w.seg + t / gd.iters;
                double2 *Xp = reinterpret_cast<double2 *>(ws + gd.xp_off);
                Xp[(sg * gd.nchunk + w.idx) * B + tid] = acc;
                acc = make_double2(0.0, 0.0);
                base = base0;
            }
        }
        lds_barrier();
    }
}

// X[seg][k] = sum over the column chunks of the partial sums, 16 bins per
// workgroup, 16 lanes per bin, fixed summation order; w.pad consecutive
// segments per workgroup
__global__ __launch_bounds__(256) void seg_reduce_kernel(const BatchArgs args) {
    const Resolved rv = resolve(args);
    char *__restrict__ ws = rv.bi.ws;
    const SegWork w = cload(rv.kd.work + rv.local);
    const SegGroupDev gd = cload(rv.kd.groups + w.g);
    const int kb = threadIdx.x / 16, lane = threadIdx.x % 16;
    const int k = w.idx * 16 + kb;
    const double2 *Xp = reinterpret_cast<const double2 *>(ws + gd.xp_off);
    double2 *X = reinterpret_cast<double2 *>(ws + gd.x_off);
    for (int64_t sg = w.seg; sg < (int64_t)w.seg + w.pad; ++sg) {
        double2 a = make_double2(0.0, 0.0);
        if (k < gd.B)
            for (int c = lane; c < gd.nchunk; c += 16) a = cadd(a, Xp[(sg * gd.nchunk + c) * gd.B + k]);
        // the 16 lanes of a bin are consecutive lanes of one wave: fixed-order
        // butterfly reduction across them, no LDS
#pragma unroll
        for (int st = 8; st > 0; st >>= 1) {
            a.x += __shfl_xor(a.x, st, 16);
            a.y += __shfl_xor(a.y, st, 16);
        }
        if (lane == 0 && k < gd.B) X[sg * gd.B + k] = a;
    }
}


// ---------------------------------------------------------------------------
// launchers

bool local2_size_ok(int L, int precision) {
    (void)precision;
    int lmax = 4096;
    return L >= 64 && L <= lmax && (L & (L - 1)) == 0;
}
int local2_segs_per_block(int L, bool pair, bool fp64) {
    (void)pair;  // real pairs share an inverse between two scales, not segments
    return local2_ncol(L, fp64);
}

bool seg_size_ok(int P, int precision) {
    (void)precision;
    int pmax = 512;
    return P >= 64 && P <= pmax && (P & (P - 1)) == 0;
}

template <typename R, int P>
static hipError_t seg_launch_P(int kind, const BatchArgs &a, int64_t blocks, hipStream_t st) {
    constexpr int NT = P;  // 16 columns x P / 16 elements per thread
    if (kind == 1)
        hipLaunchKernelGGL((seg_forward_kernel<R, P, NT>), dim3((unsigned)blocks), dim3(NT), 0, st, a);
    else
        hipLaunchKernelGGL(seg_reduce_kernel, dim3((unsigned)blocks), dim3(256), 0, st, a);
    return hipGetLastError();
}

template <typename R>
static hipError_t seg_typed(int kind, int P, const BatchArgs &a, int64_t blocks, hipStream_t st) {
    switch (P) {
        case 64: return seg_launch_P<R, 64>(kind, a, blocks, st);
        case 128: return seg_launch_P<R, 128>(kind, a, blocks, st);
        case 256: return seg_launch_P<R, 256>(kind, a, blocks, st);
        case 512: return seg_launch_P<R, 512>(kind, a, blocks, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_seg_kernel(const SegKernelId &id, const BatchArgs &a, int64_t blocks, hipStream_t st) {
    if (blocks <= 0) return hipSuccess;
    if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
    const bool fp64 = id.precision == 0;
    if (id.kind == 0 || id.kind == 3) return launch_out_kernel<false>(id, a, blocks, st);
    if (id.kind == 2) return seg_launch_P<float, 64>(2, a, blocks, st);  // precision-free
    return fp64 ? seg_typed<double>(id.kind, id.size, a, blocks, st) : seg_typed<float>(id.kind, id.size, a, blocks, st);
}

std::string seg_kernel_id_name(const SegKernelId &id, bool wps) {
    const std::string t = id.precision == 0 ? "f64," : "f32,";
    const std::string c = std::string(id.cplx ? ",complex" : ",real-pair") + (wps ? ",wps>" : ">");
    switch (id.kind) {
        case 0: return "local2_kernel<" + t + std::to_string(id.size) + c;
        case 1: return "seg_forward_kernel<" + t + std::to_string(id.size) + ">";
        case 2: return "seg_reduce_kernel<" + t + std::to_string(id.size) + ">";
        default: return "seg_inverse_kernel<" + t + std::to_string(id.size) + c;
    }
}

}  // namespace cwt
