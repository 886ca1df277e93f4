// cwt_spline.hip -- spline method (Sec. 3.3).
//
// Scales with h* s >= 1 use an integer knot spacing delta (below); scales
// with h* s < 1 keep the step h* and sum exact taps over the spline
// coefficients c themselves, W[x] = sum_t Omega_s(t) c[x + t] (the taps are
// built with the plan), in the same tap kernel with delta = 1 and c read in
// place of the box sums.
//
// With psi_h(y) = sum_n d[n] beta3(y/h - n) (Eq. beta3_wavelet_approx_m02) and
// f_c = sum_k c[k] beta3(u - k) (Eq. beta3_signal), the transform
// W(s, x) = (1/s) int f_c(u) conj psi_h((u - x)/s) du is, for h = delta / s
// with integer delta,
//
//   W[x] = 1 / (s delta^3) sum_{n=-nd}^{nd} conj(d[n]) S[x + n delta],
//   S[y] = (box_delta^4 (beta7 * c))[y + 2 delta - 2],
//
// using beta3(v/delta) = delta^{-3} sum_j B[j] beta3(v - j) (B = box_delta^4
// impulse response, centred), int beta3(u - k) beta3(u - m) du = beta7(k - m)
// (App. B, Eqs. two_betas, rescaled_beta) and beta7 sampled on the integers
// (151/315, 397/1680, 1/42, 1/5040).  box_delta^4 = Delta_delta^4 Delta^{-4}
// (App. B, Eqs. rescaled_finite_diff, inverse_finite_diff) is the paper's
// four running sums g of Eq. cumsum4_coeffs followed by delta-spaced
// differences.  Here the running sums are taken in 128-bit integers, modulo
// 2^128, of the fixed-point coefficients q = rint(c 2^F) convolved with the
// integer taps 5040 beta7 = (1, 120, 1191, 2416, 1191, 120, 1): the delta-spaced
// fourth difference of the wrapped sums is the exact integer box sum whenever
// that sum fits (|.| < 2^127, guaranteed by the choice of F), so the
// precision loss of long running sums (Sec. 3.3, App. D) does not arise and no
// segmentation of the sums is needed.  The sums are shared by every scale.
//
// Kernels (one exec):
//   spl_maxabs   partial max |f| per block of 1024 samples
//   spl_exponent F = qbits - e, 3 max|f| = m 2^e, 0.5 <= m < 1  (|c| <= 3 max|f|)
//   spl_sums<0>  per block: c (61-tap FIR, Eq. interp_coeffs), q, q7, local
//                running-sum state; c 2^F stored when a scale sums exact taps
//   spl_carry    exclusive scan of the block states
//   spl_sums<1>  per block: the fourth running sum H of q7, stored (16 B each)
//   spl_tap      per (scale, tile): S from H (5 loads, exact), FP64 taps
#include <hip/hip_runtime.h>

#include <string>
#include <type_traits>

#include "../../include/cwt.h"
#include "cwt_internal.h"
#include "fft_device.h"

namespace cwt {

typedef unsigned __int128 u128;
typedef __int128 i128;

constexpr int kSB = 2048;       // positions per block: 8 per thread halves the block scans of 4 per thread
constexpr int kSNT = 256;       // threads per block
constexpr int kSPT = kSB / kSNT;  // positions per thread
constexpr int kFIR = 30;        // prefilter half length: (2 - sqrt 3)^31 < 2e-18

// running-sum state of a run of positions: the four sums at its end, each
// started from zero at its beginning
struct Sums {
    u128 y1, y2, y3, y4;
};

// C(t + 1, 2) and C(t + 2, 3) for t < 2^32, dividing the factors by 2 and 3
// before the 128-bit products (no 128-bit division)
__device__ __forceinline__ void binoms(uint64_t t, u128 &c2, u128 &c3) {
    uint64_t a = t, b = t + 1, c = t + 2;
    if ((t & 1) == 0) a >>= 1;  // exactly one of t, t + 1 is even
    else b >>= 1;
    c2 = (u128)a * (u128)b;
    if (a % 3 == 0) a /= 3;  // one of t, t + 1, t + 2 is a multiple of 3 (halving keeps that)
    else if (b % 3 == 0) b /= 3;
    else c /= 3;
    c3 = (u128)a * (u128)b * (u128)c;
}

// state after run A followed by run B of length t < 2^32 (B's sums started at zero)
__device__ __forceinline__ Sums sums_then(const Sums &a, const Sums &b, uint64_t tt) {
    u128 c2, c3;
    binoms(tt, c2, c3);
    const u128 t = tt;
    Sums r;
    r.y1 = a.y1 + b.y1;
    r.y2 = a.y2 + t * a.y1 + b.y2;
    r.y3 = a.y3 + t * a.y2 + c2 * a.y1 + b.y3;
    r.y4 = a.y4 + t * a.y3 + c2 * a.y2 + c3 * a.y1 + b.y4;
    return r;
}

__device__ __forceinline__ double i128_to_double(u128 v) {
    const i128 s = (i128)v;
    const long long hi = (long long)(s >> 64);
    const unsigned long long lo = (unsigned long long)s;
    return (double)hi * 0x1p64 + (double)lo;
}

// NaN-propagating maximum
__device__ __forceinline__ double nmax(double a, double b) { return (b > a || b != b) ? b : a; }

template <typename R>
__device__ __forceinline__ double sig_ext(const R *__restrict__ f, int64_t N, int periodic, int64_t x) {
    if (periodic) {
        int64_t m = x % N;
        if (m < 0) m += N;
        return (double)f[m];
    }
    return (x >= 0 && x < N) ? (double)f[x] : 0.0;
}

template <typename R>
__global__ __launch_bounds__(kSNT) void spl_maxabs_kernel(const R *__restrict__ f, int64_t N, double *__restrict__ part) {
    __shared__ double red[kSNT];
    const int64_t base = (int64_t)blockIdx.x * kSB;
    double m = 0.0;
    for (int k = threadIdx.x; k < kSB; k += kSNT) {
        const int64_t i = base + k;
        if (i < N) m = nmax(m, fabs((double)f[i]));
    }
    red[threadIdx.x] = m;
    lds_barrier();
    for (int s = kSNT / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] = nmax(red[threadIdx.x], red[threadIdx.x + s]);
        lds_barrier();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// fx[0] = F, fx[1] = 1 if max|f| is not finite
__global__ __launch_bounds__(kSNT) void spl_exponent_kernel(const double *__restrict__ part, int nb, int qbits,
                                                            int *__restrict__ fx) {
    __shared__ double red[kSNT];
    double m = 0.0;
    for (int k = threadIdx.x; k < nb; k += kSNT) m = nmax(m, part[k]);
    red[threadIdx.x] = m;
    lds_barrier();
    for (int s = kSNT / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] = nmax(red[threadIdx.x], red[threadIdx.x + s]);
        lds_barrier();
    }
    if (threadIdx.x == 0) {
        const double b = 3.0 * red[0];
        int F = 0, bad = 0;
        if (!(b <= 1.7e308)) bad = 1;  // inf or NaN
        else if (b > 0.0) {
            int e;
            (void)frexp(b, &e);
            F = qbits - e;
        }
        fx[0] = F;
        fx[1] = bad;
    }
}

// powers z1^t, t = 0..kFIR, z1 = sqrt(3) - 2
struct ZPow {
    double v[kFIR + 1];
    constexpr ZPow() : v() {
        const double z = -0.26794919243112270647;
        double a = 1.0;
        for (int t = 0; t <= kFIR; ++t) {
            v[t] = a;
            a *= z;
        }
    }
};
__constant__ ZPow kZ = ZPow();

// lane i gets v of lane i - d of its wave (its own v when i < d)
__device__ __forceinline__ u128 shfl_up_u128(u128 v, int d) {
    const uint64_t lo = __shfl_up((unsigned long long)(uint64_t)v, d, 64);
    const uint64_t hi = __shfl_up((unsigned long long)(uint64_t)(v >> 64), d, 64);
    return ((u128)hi << 64) | lo;
}
__device__ __forceinline__ Sums shfl_up_sums(const Sums &a, int d) {
    return {shfl_up_u128(a.y1, d), shfl_up_u128(a.y2, d), shfl_up_u128(a.y3, d), shfl_up_u128(a.y4, d)};
}

// Block b covers array indices [b kSB, (b + 1) kSB), position x = index - E.
// FINAL = 0: writes the block's running-sum state (from zero) to state[b].
// FINAL = 1: adds the carry-in carry[b] and writes H[index] (fourth sum).
// C (FINAL = 0, may be null): c 2^F at every index of the block.
template <typename R, int FINAL>
__global__ __launch_bounds__(kSNT) void spl_sums_kernel(const R *__restrict__ f, int64_t N, int periodic, int64_t E,
                                                        int64_t len, const int *__restrict__ fx,
                                                        Sums *__restrict__ state, const Sums *__restrict__ carry,
                                                        u128 *__restrict__ H, double *__restrict__ C) {
    constexpr int FS = kSB + 6 + 2 * kFIR;  // samples on [x0 - 3 - kFIR, x0 + kSB + 3 + kFIR)
    constexpr int QS = kSB + 6;             // q on [x0 - 3, x0 + kSB + 3)
    __shared__ double fs[FS];
    __shared__ long long qs[QS];
    __shared__ Sums wtot[kSNT / 64];
    const int tid = threadIdx.x;
    const int F = fx[0], bad = fx[1];
    const int64_t l0 = (int64_t)blockIdx.x * kSB;
    const int64_t x0 = l0 - E;
    for (int k = tid; k < FS; k += kSNT) fs[k] = sig_ext(f, N, periodic, x0 - 3 - kFIR + k);
    lds_barrier();
    // spline coefficients c = (beta3)^{-1} f (Eq. interp_coeffs) as the
    // symmetric FIR sqrt(3) sum_t z1^|t| f[x - t], then fixed point
    for (int k = tid; k < QS; k += kSNT) {
        const double *fc = fs + k + kFIR;
        double c = fc[0];
#pragma unroll
        for (int t = 1; t <= kFIR; ++t) c = fma(kZ.v[t], fc[-t] + fc[t], c);
        c *= 1.7320508075688772935;
        const double cf = bad ? 0.0 : ldexp(c, F);
        qs[k] = (long long)rint(cf);
        if (!FINAL && C != nullptr && k >= 3 && k < kSB + 3 && l0 + k - 3 < len) C[l0 + k - 3] = cf;
    }
    lds_barrier();
    // 5040 beta7 * q at this thread's positions, local running sums
    Sums loc = {0, 0, 0, 0};
    i128 q7v[kSPT];
#pragma unroll
    for (int e = 0; e < kSPT; ++e) {
        const long long *qq = qs + tid * kSPT + e + 3;
        const i128 q7 = (i128)qq[0] * 2416 + ((i128)qq[-1] + qq[1]) * 1191 + ((i128)qq[-2] + qq[2]) * 120 +
                        ((i128)qq[-3] + qq[3]);
        q7v[e] = q7;
        loc.y1 += (u128)q7;
        loc.y2 += loc.y1;
        loc.y3 += loc.y2;
        loc.y4 += loc.y3;
    }
    // inclusive scan of the thread states (each covers kSPT positions): within
    // each wave with shuffles, then the totals of the earlier waves in front
    const int lane = tid & 63, wv = tid >> 6;
    Sums inc = loc;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const Sums left = shfl_up_sums(inc, d);
        if (lane >= d) inc = sums_then(left, inc, (uint64_t)(d * kSPT));
    }
    if (lane == 63) wtot[wv] = inc;
    lds_barrier();
    Sums pre = {0, 0, 0, 0};  // waves before this one
    for (int v = 0; v < wv; ++v) pre = sums_then(pre, wtot[v], (uint64_t)(64 * kSPT));
    if (!FINAL) {
        if (tid == kSNT - 1) state[blockIdx.x] = sums_then(pre, inc, (uint64_t)(64 * kSPT));
        return;
    }
    // absolute state before this thread's first position: carry-in, earlier
    // waves, earlier lanes of this wave
    const Sums excl = shfl_up_sums(inc, 1);
    Sums st = sums_then(carry[blockIdx.x], pre, (uint64_t)(wv * 64 * kSPT));
    if (lane > 0) st = sums_then(st, excl, (uint64_t)(lane * kSPT));
#pragma unroll
    for (int e = 0; e < kSPT; ++e) {
        st.y1 += (u128)q7v[e];
        st.y2 += st.y1;
        st.y3 += st.y2;
        st.y4 += st.y3;
        const int64_t l = l0 + tid * kSPT + e;
        if (l < len) H[l] = st.y4;
    }
}

// exclusive scan of the block states: carry[b] = running sums just before
// block b.  One wave: each lane combines a contiguous run of states, the
// lanes' totals are scanned across the wave with shuffles (no barriers), and
// each lane then writes the carries of its run.
constexpr int kCNT = 64;
__global__ __launch_bounds__(kCNT) void spl_carry_kernel(const Sums *__restrict__ state, int nblk,
                                                         Sums *__restrict__ carry) {
    const int lane = threadIdx.x;
    const int per = (nblk + kCNT - 1) / kCNT;
    const int b0 = min(nblk, lane * per), b1 = min(nblk, b0 + per);
    Sums acc = {0, 0, 0, 0};
    for (int b = b0; b < b1; ++b) acc = sums_then(acc, state[b], (uint64_t)kSB);
    int64_t len = (int64_t)(b1 - b0) * kSB;  // positions acc covers
    for (int d = 1; d < kCNT; d <<= 1) {
        const Sums left = shfl_up_sums(acc, d);
        const int64_t llen = __shfl_up((long long)len, d, kCNT);
        if (lane >= d) {
            acc = sums_then(left, acc, (uint64_t)len);
            len += llen;
        }
    }
    Sums st = shfl_up_sums(acc, 1);
    if (lane == 0) st = {0, 0, 0, 0};
    for (int b = b0; b < b1; ++b) {
        carry[b] = st;
        st = sums_then(st, state[b], (uint64_t)kSB);
    }
}

// Tap sums.  Positions x = i delta + r0 + r (row i, column r < R); the tile
// holds rows [i0, i0 + I).  S rows m <-> i = i0 - nd + m, m < I + ntap, kept
// in LDS at R (m + m/16) + r: one spare row per 16 makes the strides between
// the 16-row groups of neighbouring threads odd (no bank conflicts).
constexpr int kSTile = 8192;  // S values per tile (rows with spares included), 64 KiB
__device__ __forceinline__ int stile_idx(int m, int R, int r) { return R * (m + (m >> 4)) + r; }

// LDS: the S tile (stile doubles), then the tile's taps d' (ntap double2).
// The launch passes the largest such size over the plan's scales.
// Registers are budgeted for three waves per SIMD (three workgroups per CU
// where the S tile allows): stated explicitly, the real form keeps its tap
// window in fewer registers and both forms schedule their row loads better
// (about 2 % faster); four would need spills in the tap loop and run slower.
template <typename OUT, bool CPLX>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void spl_tap_kernel(int64_t N, int64_t E, const SplineScaleDev *__restrict__ scl,
                                                      const SplineWork *__restrict__ work,
                                                      const u128 *__restrict__ H, const double *__restrict__ C,
                                                      const double2 *__restrict__ dtab,
                                                      const int *__restrict__ fx, OUT *__restrict__ out) {
    extern __shared__ double lds[];
    const SplineWork w = work[blockIdx.x];
    const SplineScaleDev p = scl[w.j];
    const int tid = threadIdx.x;
    const int R = w.R;
    const int ngrp = 256 / p.R;  // row groups of 16 (I = 16 ngrp)
    const int r = tid % p.R, g = tid / p.R;
    const bool active = r < R && g < ngrp;
    const int64_t delta = p.delta;
    const int I = p.I, nd = p.nd, ntap = p.ntap;
    const int rowsS = I + ntap;
    double *S = lds;
    double2 *dl = reinterpret_cast<double2 *>(lds + R * (rowsS + rowsS / 16 + 1));
    // first 256 taps: loaded now, written to LDS after the S rows (their
    // latency overlaps the H row loads)
    const double2 d0 = tid < ntap ? dtab[p.d_off + tid] : make_double2(0.0, 0.0);
    const int64_t nrows = (N + delta - 1) / delta;
    // S rows that some output of the tile uses with a nonzero tap; the H
    // rows of later S rows are clamped (their finite values meet zero taps or
    // outputs beyond N only)
    const int mvalid = (int)min((int64_t)rowsS, min((int64_t)I, nrows - w.i0) + 2 * nd);
    const int64_t rho_max = w.i0 - nd + mvalid + 1;
    const int F = fx[0];
    const int bad = fx[1];
    if (p.mode == 1) {
        // S read directly from C (c 2^F for the spline method's exact taps,
        // F_i for the V97 method): S row m, column r is C at position
        // (i0 - nd + m) delta + r0 + r; rows past the last one some output
        // uses are clamped.  All threads load, consecutive threads take
        // consecutive columns of a row.
        const double *cp = C + (E + (w.i0 - nd) * delta + w.r0);
        for (int idx = tid; idx < rowsS * R; idx += 256) {
            const int m = idx / R, rr = idx - m * R;
            S[stile_idx(m, R, rr)] = cp[(int64_t)min(m, mvalid - 1) * delta + rr];
        }
    } else if (active) {
        // rows in batches of BR: S rows m0..m0+BR-1 need H rows i - 2 .. i + 2,
        // i.e. the BR + 4 rows starting at i0 - nd + m0 - 2, loaded together
        // (one memory latency per batch; batches as large as the register
        // budget of each form allows measured best: 20 rows complex, 24 real)
        constexpr int BR = CPLX ? 20 : 24;
        const int ch = BR * ((rowsS + BR * ngrp - 1) / (BR * ngrp));
        const int mb = g * ch, me = min(rowsS, mb + ch);
        // H row rho of this column: H[E + r0 + r - 2 + rho delta], read with
        // raw buffer loads and 32-bit byte offsets (H holds N + 2E < 2^27 values)
        const __amdgpu_buffer_rsrc_t hr = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<u128 *>(H), 0, (int)__builtin_amdgcn_readfirstlane((uint32_t)((N + 2 * E) * 16)), 0x00020000);
        const uint32_t hb = (uint32_t)((E + w.r0 + r - 2) * 16), hs = (uint32_t)(delta * 16);
        const int32_t rho0 = (int32_t)(w.i0 - nd - 2), rmax = (int32_t)rho_max;
        for (int m0 = mb; m0 < me; m0 += BR) {
            u128 h[BR + 4];
#pragma unroll
            for (int q = 0; q < BR + 4; ++q) {
                const int32_t rho = min(rho0 + m0 + q, rmax);
                h[q] = __builtin_bit_cast(u128, __builtin_amdgcn_raw_buffer_load_b128(hr, hb + (uint32_t)rho * hs, 0, 0));
            }
            // S = fourth difference at spacing delta, taken as four rounds of
            // first differences over the BR + 4 rows (subtractions modulo
            // 2^128 instead of the weighted sum's multiplies and adds)
#pragma unroll
            for (int d = 0; d < 4; ++d) {
#pragma unroll
                for (int q = 0; q < BR + 3 - d; ++q) h[q] = h[q + 1] - h[q];
            }
#pragma unroll
            for (int k = 0; k < BR; ++k)
                if (m0 + k < me) S[stile_idx(m0 + k, R, r)] = i128_to_double(h[k]);
        }
    }
    if (tid < ntap) dl[tid] = d0;
    for (int k = tid + 256; k < ntap; k += 256) dl[k] = dtab[p.d_off + k];
    lds_barrier();
    if (!active) return;
    const int u0 = g * 16;
    // rows u0 + m for m in [16 q, 16 q + 16) start at stile_idx(u0 + 16 q) and
    // are R apart: a block of 8 rows starting at a multiple of 8 has constant
    // offsets
    const double *Sc = S + stile_idx(u0, R, r);
    auto rowp = [&](int m) { return Sc + R * (m + (m >> 4)); };  // m relative to u0, u0 % 16 == 0
    double ar[16], ai[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
        ar[u] = 0.0;
        ai[u] = 0.0;
    }
    if constexpr (CPLX) {
        // window of S rows u0 + nb .. u0 + nb + 23, shifted by 8 rows per
        // block of 8 taps; the next block's rows are loaded before this
        // block's multiply-adds, the taps per tap (the complex form's
        // register budget has no room for more)
        double win[24], nxt[8];
        {
            const double *p0 = rowp(0), *p1 = rowp(16);
#pragma unroll
            for (int k = 0; k < 16; ++k) win[k] = p0[k * R];
#pragma unroll
            for (int k = 0; k < 8; ++k) win[16 + k] = p1[k * R];
        }
        for (int nb = 0; nb < ntap; nb += 8) {
            if (nb + 8 < ntap) {
                const double *pn = rowp(nb + 24);
#pragma unroll
                for (int k = 0; k < 8; ++k) nxt[k] = pn[k * R];
            }
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                const double2 dv = dl[nb + t];
#pragma unroll
                for (int u = 0; u < 16; ++u) {
                    ar[u] = fma(dv.x, win[u + t], ar[u]);
                    ai[u] = fma(dv.y, win[u + t], ai[u]);
                }
            }
#pragma unroll
            for (int k = 0; k < 16; ++k) win[k] = win[8 + k];
#pragma unroll
            for (int k = 0; k < 8; ++k) win[16 + k] = nxt[k];
        }
    } else {
        // S rows u0 + nb .. in four rotating blocks of 8 registers: the
        // 8-tap step k (taps nb + 8k ..) reads rows nb + 8k .. nb + 8k + 22
        // from blocks k, k + 1, k + 2 (mod 4) and loads the next step's last
        // block into block k + 3, and the next step's taps, before its
        // multiply-adds; nb is a multiple of 32, so every row's block is known
        // at compile time and no register moves between steps
        double blk[4][8], tr[2][8];
        {
            const double *p0 = rowp(0), *p1 = rowp(16);
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                blk[0][k] = p0[k * R];
                blk[1][k] = p0[(8 + k) * R];
                blk[2][k] = p1[k * R];
            }
#pragma unroll
            for (int t = 0; t < 8; ++t) tr[0][t] = dl[t].x;
        }
        auto step = [&](int nb, auto kc) {
            constexpr int K = decltype(kc)::value;
            const int nbk = nb + 8 * K;
            if (nbk >= ntap) return;
            if (nbk + 8 < ntap) {
                const double *pn = rowp(nbk + 24);
#pragma unroll
                for (int k = 0; k < 8; ++k) blk[(K + 3) & 3][k] = pn[k * R];
#pragma unroll
                for (int t = 0; t < 8; ++t) tr[(K + 1) & 1][t] = dl[nbk + 8 + t].x;
            }
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                const double dv = tr[K & 1][t];
#pragma unroll
                for (int u = 0; u < 16; ++u) ar[u] = fma(dv, blk[(K + ((u + t) >> 3)) & 3][(u + t) & 7], ar[u]);
            }
        };
        for (int nb = 0; nb < ntap; nb += 32) {
            step(nb, std::integral_constant<int, 0>{});
            step(nb, std::integral_constant<int, 1>{});
            step(nb, std::integral_constant<int, 2>{});
            step(nb, std::integral_constant<int, 3>{});
        }
    }
    const double nan = __builtin_nan("");
    OUT *row = out + (int64_t)w.j * N * (CPLX ? 2 : 1);
#pragma unroll
    for (int u = 0; u < 16; ++u) {
        const int64_t x = (w.i0 + u0 + u) * delta + w.r0 + r;
        if (x < N) {
            const double vr = bad ? nan : ldexp(ar[u], -F);
            if (CPLX) {
                const double vi = bad ? nan : ldexp(ai[u], -F);
                row[2 * x] = (OUT)vr;
                row[2 * x + 1] = (OUT)vi;
            } else {
                row[x] = (OUT)vr;
            }
        }
    }
}

template <typename R>
static hipError_t spline_sums(const Plan &p, const R *f, char *ws, hipStream_t st) {
    double *part = reinterpret_cast<double *>(ws + p.ws_maxp_off);
    int *fx = reinterpret_cast<int *>(ws + p.ws_fx_off);
    Sums *state = reinterpret_cast<Sums *>(ws + p.ws_state_off);
    Sums *carry = reinterpret_cast<Sums *>(ws + p.ws_carry_off);
    u128 *H = reinterpret_cast<u128 *>(ws + p.ws_H_off);
    double *C = p.spl_direct ? reinterpret_cast<double *>(ws + p.ws_C_off) : nullptr;
    const int periodic = p.boundary == CWT_PERIODIC;
    hipLaunchKernelGGL(spl_maxabs_kernel<R>, dim3(p.spl_nb0), dim3(kSNT), 0, st, f, p.N, part);
    hipLaunchKernelGGL(spl_exponent_kernel, dim3(1), dim3(kSNT), 0, st, part, p.spl_nb0, p.spl_qbits, fx);
    hipLaunchKernelGGL((spl_sums_kernel<R, 0>), dim3(p.spl_nblk), dim3(kSNT), 0, st, f, p.N, periodic, p.spl_E,
                       p.spl_len, fx, state, carry, H, C);
    hipLaunchKernelGGL(spl_carry_kernel, dim3(1), dim3(kCNT), 0, st, state, p.spl_nblk, carry);
    hipLaunchKernelGGL((spl_sums_kernel<R, 1>), dim3(p.spl_nblk), dim3(kSNT), 0, st, f, p.N, periodic, p.spl_E,
                       p.spl_len, fx, state, carry, H, nullptr);
    return hipGetLastError();
}

template <typename OUT>
static hipError_t spline_taps(const Plan &p, char *ws, void *out, hipStream_t st) {
    const int *fx = reinterpret_cast<const int *>(ws + p.ws_fx_off);
    const u128 *H = reinterpret_cast<const u128 *>(ws + p.ws_H_off);
    const double *C = p.spl_direct ? reinterpret_cast<const double *>(ws + p.ws_C_off) : nullptr;
    const double2 *dt = reinterpret_cast<const double2 *>(p.d_dtab);
    const dim3 grid((unsigned)p.spl_work.size());
    const size_t lds = (size_t)p.spl_lds_bytes;
    if (p.cplx_out)
        hipLaunchKernelGGL((spl_tap_kernel<OUT, true>), grid, dim3(256), lds, st, p.N, p.spl_E, p.d_spl, p.d_spl_work,
                           H, C, dt, fx, reinterpret_cast<OUT *>(out));
    else
        hipLaunchKernelGGL((spl_tap_kernel<OUT, false>), grid, dim3(256), lds, st, p.N, p.spl_E, p.d_spl, p.d_spl_work,
                           H, C, dt, fx, reinterpret_cast<OUT *>(out));
    return hipGetLastError();
}

hipError_t launch_spline(const Plan &p, const void *signal, void *out, void *ws, hipStream_t st, int phase) {
    char *w = reinterpret_cast<char *>(ws);
    const bool fp64 = p.precision == CWT_FP64;
    if (phase == 0)
        return fp64 ? spline_sums(p, reinterpret_cast<const double *>(signal), w, st)
                    : spline_sums(p, reinterpret_cast<const float *>(signal), w, st);
    return fp64 ? spline_taps<double>(p, w, out, st) : spline_taps<float>(p, w, out, st);
}

std::string spline_kernel_name(const Plan &p, int phase) {
    const std::string t = p.precision == CWT_FP64 ? "f64" : "f32";
    if (phase == 0) return "spline_sums<" + t + ">";
    return "spl_tap_kernel<" + t + (p.cplx_out ? ",complex>" : ",real>");
}


// ---------------------------------------------------------------------------
// V97 method (Sec. 3.2): the filter chain of Eqs. fir_filter_beta,
// iir_filter_0, fir_filter_hi and iir_filter_i, in FP64.  An f buffer holds
// positions [-E, N + E) (zero boundary; the chain's support ends 2^(i+1) + 1
// samples beyond the signal, inside E, so reads past the buffer are zeros) or
// [0, N) read with wrapped indices (periodic).  The F array always holds
// [-E, N + E), filled on the part the tap sums read.

// value of an f buffer at position x
__device__ __forceinline__ double fbuf(const double *__restrict__ b, int64_t N, int periodic, int64_t E, int64_t x) {
    if (periodic) {
        int64_t m = x % N;
        if (m < 0) m += N;
        return b[m];
    }
    const int64_t i = x + E;
    return (i >= 0 && i < N + 2 * E) ? b[i] : 0.0;
}

// f_0 = f * beta3 sampled: (f[x-1] + 4 f[x] + f[x+1]) / 6 (Eq. fir_filter_beta);
// thread 0 also clears the scaling exponent and flag the tap kernel reads
template <typename R>
__global__ __launch_bounds__(256) void v97_f0_kernel(const R *__restrict__ f, int64_t N, int periodic, int64_t E,
                                                     int64_t flen, double *__restrict__ out, int *__restrict__ fx) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i == 0) {
        fx[0] = 0;
        fx[1] = 0;
    }
    if (i >= flen) return;
    const int64_t x = periodic ? i : i - E;
    const double a = sig_ext(f, N, periodic, x - 1), b = sig_ext(f, N, periodic, x),
                 c = sig_ext(f, N, periodic, x + 1);
    out[i] = (a + c + 4.0 * b) * (1.0 / 6.0);
}

// f_{a+1} = f_a * [h] upsampled by 2^a, h = (1, 4, 6, 4, 1) / 8 (Eq. h_filter
// with n = 3; Eq. fir_filter_hi)
__global__ __launch_bounds__(256) void v97_h_kernel(const double *__restrict__ in, int64_t N, int periodic, int64_t E,
                                                    int64_t flen, int64_t step, double *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= flen) return;
    const int64_t x = periodic ? i : i - E;
    const double v = 6.0 * fbuf(in, N, periodic, E, x) +
                     4.0 * (fbuf(in, N, periodic, E, x - step) + fbuf(in, N, periodic, E, x + step)) +
                     (fbuf(in, N, periodic, E, x - 2 * step) + fbuf(in, N, periodic, E, x + 2 * step));
    out[i] = v * 0.125;
}

// F_a = f_a * [q12] upsampled by 2^a (Eq. iir_filter_i), taps |k| <= K, on
// positions [-EF, N + EF) of the F array
__global__ __launch_bounds__(256) void v97_q12_kernel(const double *__restrict__ in, int64_t N, int periodic, int64_t E,
                                                      int64_t EF, int64_t step, const double *__restrict__ q12, int K,
                                                      double *__restrict__ F) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= N + 2 * EF) return;
    const int64_t x = i - EF;
    double acc = q12[K] * fbuf(in, N, periodic, E, x);
    for (int k = 1; k <= K; ++k)
        acc = fma(q12[K + k], fbuf(in, N, periodic, E, x - k * step) + fbuf(in, N, periodic, E, x + k * step), acc);
    F[x + E] = acc;
}

template <typename OUT>
static hipError_t v97_taps(const Plan &p, const Plan::V97Step &sp, char *ws, void *out, hipStream_t st) {
    const int *fx = reinterpret_cast<const int *>(ws + p.ws_fx_off);
    const double *C = reinterpret_cast<const double *>(ws + p.ws_C_off);
    const double2 *dt = reinterpret_cast<const double2 *>(p.d_dtab);
    const dim3 grid((unsigned)(sp.w1 - sp.w0));
    const size_t lds = (size_t)p.spl_lds_bytes;
    const SplineWork *work = p.d_spl_work + sp.w0;
    if (p.cplx_out)
        hipLaunchKernelGGL((spl_tap_kernel<OUT, true>), grid, dim3(256), lds, st, p.N, p.spl_E, p.d_spl, work, nullptr,
                           C, dt, fx, reinterpret_cast<OUT *>(out));
    else
        hipLaunchKernelGGL((spl_tap_kernel<OUT, false>), grid, dim3(256), lds, st, p.N, p.spl_E, p.d_spl, work,
                           nullptr, C, dt, fx, reinterpret_cast<OUT *>(out));
    return hipGetLastError();
}

hipError_t launch_v97(const Plan &p, size_t k, const void *signal, void *out, void *ws, hipStream_t st) {
    char *w = reinterpret_cast<char *>(ws);
    const Plan::V97Step &sp = p.v97_steps[k];
    const int periodic = p.boundary == CWT_PERIODIC;
    double *fb[2] = {reinterpret_cast<double *>(w + p.ws_fa_off), reinterpret_cast<double *>(w + p.ws_fb_off)};
    const int64_t E = p.spl_E;
    const bool fp64 = p.precision == CWT_FP64;
    if (sp.kind == 0) {
        const dim3 grid((unsigned)((p.v97_flen + 255) / 256));
        int *fx = reinterpret_cast<int *>(w + p.ws_fx_off);
        if (fp64)
            hipLaunchKernelGGL(v97_f0_kernel<double>, grid, dim3(256), 0, st, reinterpret_cast<const double *>(signal),
                               p.N, periodic, E, p.v97_flen, fb[sp.dst], fx);
        else
            hipLaunchKernelGGL(v97_f0_kernel<float>, grid, dim3(256), 0, st, reinterpret_cast<const float *>(signal),
                               p.N, periodic, E, p.v97_flen, fb[sp.dst], fx);
        return hipGetLastError();
    }
    if (sp.kind == 1) {
        const dim3 grid((unsigned)((p.v97_flen + 255) / 256));
        hipLaunchKernelGGL(v97_h_kernel, grid, dim3(256), 0, st, fb[sp.src], p.N, periodic, E, p.v97_flen,
                           int64_t(1) << sp.a, fb[sp.dst]);
        return hipGetLastError();
    }
    if (sp.kind == 2) {
        // the part of F the tap sums of this level read
        int64_t EF = 16;
        for (const Plan::V97Step &t : p.v97_steps)
            if (t.kind == 3 && t.a == sp.a)
                for (int32_t q = t.w0; q < t.w1; ++q) {
                    const SplineScaleDev &sc = p.spl[p.spl_work[q].j];
                    EF = std::max<int64_t>(EF, (int64_t)(sc.nd + 2) * sc.delta + 16);
                }
        EF = std::min(EF, E);
        const dim3 grid((unsigned)((p.N + 2 * EF + 255) / 256));
        hipLaunchKernelGGL(v97_q12_kernel, grid, dim3(256), 0, st, fb[sp.src], p.N, periodic, E, EF,
                           int64_t(1) << sp.a, p.d_v97_q12, p.v97_nq12, reinterpret_cast<double *>(w + p.ws_C_off));
        return hipGetLastError();
    }
    return fp64 ? v97_taps<double>(p, sp, w, out, st) : v97_taps<float>(p, sp, w, out, st);
}

std::string v97_kernel_name(const Plan &p, size_t k) {
    static const char *nm[4] = {"v97_f0_kernel", "v97_h_kernel", "v97_q12_kernel", "spl_tap_kernel"};
    const Plan::V97Step &sp = p.v97_steps[k];
    if (sp.kind == 3)
        return std::string("spl_tap_kernel<") + (p.precision == CWT_FP64 ? "f64" : "f32") +
               (p.cplx_out ? ",complex>" : ",real>");
    return nm[sp.kind];
}

}  // namespace cwt
