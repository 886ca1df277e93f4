// fft_cols.h -- workgroup FFT of NCOL columns of length P held in LDS, with
// per-pass twiddle tables in LDS and a last pass that hands every output to
// a caller functor straight from registers (no final LDS round trip).
//
// Pass j has radix R_j (radix_of), sub-transform size Ns_j (ns_before); its
// twiddles e^{+2 pi i r k / (R_j Ns_j)}, r in [1, R_j), k in [0, Ns_j), sit
// at twl[twl_off(P, j) + (r - 1) Ns_j + k], so the threads of a wave read
// consecutive entries.  The table is generated in FP64 on the host and stored
// in the kernel's precision.
#pragma once
#include "fft_device.h"

namespace cwt {

constexpr int twl_off(int P, int pass) {
    int off = 0;
    for (int j = 0; j < pass; ++j) {
        int ns = ns_before(P, j);
        if (ns > 1) off += (radix_of(P, j) - 1) * ns;
    }
    return off;
}
constexpr int twl_len(int P) { return twl_off(P, num_passes(P)) > 0 ? twl_off(P, num_passes(P)) : 1; }

// middle pass: LDS -> LDS, column-major thread mapping (consecutive threads
// take consecutive butterflies of one column)
// Twiddles of butterfly k: e^{+2 pi i r k/(R Ns)}, r = 1..R-1, read from the
// table (TWCALC = false) or, TWCALC = true (FP64 only), w^1 evaluated with
// sincospi and the other powers formed by products.  The FP64 segment
// transforms of FP32 plans use the latter: a table read from global memory
// in the middle of a pass would expose its full latency.
template <typename C, int R, int NS, int SIGN, bool TWCALC>
__device__ __forceinline__ void apply_twiddles(const C *tab, int k, C (&v)[R]) {
    if constexpr (TWCALC) {
        static_assert(sizeof(decltype(C::x)) == 8, "computed twiddles are FP64");
        double sn, cs;
        sincospi((double)(2 * k) / (double)(R * NS), &sn, &cs);
        const C w1 = mk<C>(cs, sn);
        C w = w1;  // w^r along the chain: two twiddles live, not R - 1
#pragma unroll
        for (int r = 1; r < R; ++r) {
            if (r > 1) w = cmul(w, w1);
            v[r] = SIGN > 0 ? cmul(v[r], w) : cmulc(v[r], w);
        }
    } else {
#pragma unroll
        for (int r = 1; r < R; ++r) {
            const C w = tab[k + (r - 1) * NS];
            v[r] = SIGN > 0 ? cmul(v[r], w) : cmulc(v[r], w);
        }
    }
}

template <typename C, int P, int NCOL, int NT, int LD, int SIGN, int PASS, bool TWCALC = false>
__device__ __forceinline__ void cols_pass_mid(C *buf, const C *twl) {
    constexpr int R = radix_of(P, PASS);
    constexpr int NS = ns_before(P, PASS);
    constexpr int NB = NCOL * (P / R);
    constexpr int PER = (NB + NT - 1) / NT;
    const int tid = threadIdx.x;
    C v[PER][R];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        int gb = tid + q * NT;
        if (NB % NT == 0 || gb < NB) {
            int c = gb / (P / R), i = gb % (P / R);
#pragma unroll
            for (int r = 0; r < R; ++r) v[q][r] = buf[c * LD + lidx(i + r * (P / R)) + col_skew<LD>(c)];
        }
    }
    lds_barrier();
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        int gb = tid + q * NT;
        if (NB % NT == 0 || gb < NB) {
            int c = gb / (P / R), i = gb % (P / R);
            int k = i % NS;
            if constexpr (NS > 1) apply_twiddles<C, R, NS, SIGN, TWCALC>(twl + twl_off(P, PASS), k, v[q]);
            dftR<R, SIGN>(v[q]);
            int base = (i - k) * R + k;
#pragma unroll
            for (int r = 0; r < R; ++r) buf[c * LD + lidx(base + r * NS) + col_skew<LD>(c)] = v[q][r];
        }
    }
    lds_barrier();
}

// last pass: column-fastest thread mapping (consecutive threads take the same
// butterfly of consecutive columns) or, POSFAST, position-fastest (consecutive
// threads take consecutive butterflies of one column, so that for each r they
// emit consecutive positions); outputs go to emit(col, p, value).
// SYNC: barrier between the LDS reads and the emits (needed when emit writes
// back into buf).
template <typename C, int P, int NCOL, int NT, int LD, int SIGN, bool SYNC, class F, bool TWCALC = false,
          bool POSFAST = false>
__device__ __forceinline__ void cols_pass_last(C *buf, const C *twl, F &emit) {
    constexpr int PASS = num_passes(P) - 1;
    constexpr int R = radix_of(P, PASS);
    constexpr int NS = ns_before(P, PASS);  // = P / R
    constexpr int NB = NCOL * (P / R);
    constexpr int PER = (NB + NT - 1) / NT;
    const int tid = threadIdx.x;
    C v[PER][R];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        int gb = tid + q * NT;
        if (NB % NT == 0 || gb < NB) {
            int c = POSFAST ? gb / (P / R) : gb % NCOL, i = POSFAST ? gb % (P / R) : gb / NCOL;
#pragma unroll
            for (int r = 0; r < R; ++r) v[q][r] = buf[c * LD + lidx(i + r * (P / R)) + col_skew<LD>(c)];
        }
    }
    if constexpr (SYNC) lds_barrier();
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        int gb = tid + q * NT;
        if (NB % NT == 0 || gb < NB) {
            int c = POSFAST ? gb / (P / R) : gb % NCOL, i = POSFAST ? gb % (P / R) : gb / NCOL;
            if constexpr (NS > 1) apply_twiddles<C, R, NS, SIGN, TWCALC>(twl + twl_off(P, PASS), i, v[q]);
            dftR<R, SIGN>(v[q]);
#pragma unroll
            for (int r = 0; r < R; ++r) emit(c, i + r * NS, v[q][r]);
        }
    }
}

// The (column, position) pairs cols_pass_last hands this thread, in the order
// of its emit calls: fn(k, col, p) for emit k = 0, 1, ...
template <int P, int NCOL, int NT, bool POSFAST, class F>
__device__ __forceinline__ void cols_last_positions(F &&fn) {
    constexpr int PASS = num_passes(P) - 1;
    constexpr int R = radix_of(P, PASS);
    constexpr int NS = ns_before(P, PASS);
    constexpr int NB = NCOL * (P / R);
    constexpr int PER = (NB + NT - 1) / NT;
    const int tid = threadIdx.x;
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        int gb = tid + q * NT;
        if (NB % NT == 0 || gb < NB) {
            int c = POSFAST ? gb / (P / R) : gb % NCOL, i = POSFAST ? gb % (P / R) : gb / NCOL;
#pragma unroll
            for (int r = 0; r < R; ++r) fn(q * R + r, c, i + r * NS);
        }
    }
}

template <typename C, int P, int NCOL, int NT, int LD, int SIGN, int PASS, bool TWCALC = false>
__device__ __forceinline__ void cols_mid_from(C *buf, const C *twl) {
    if constexpr (PASS + 1 < num_passes(P)) {
        cols_pass_mid<C, P, NCOL, NT, LD, SIGN, PASS, TWCALC>(buf, twl);
        cols_mid_from<C, P, NCOL, NT, LD, SIGN, PASS + 1, TWCALC>(buf, twl);
    }
}

// Full transform of NCOL columns in buf (filled and synchronised by the
// caller).  Outputs are emitted in natural order positions p.
template <typename C, int P, int NCOL, int NT, int LD, int SIGN, bool SYNC_LAST, class F, bool TWCALC = false>
__device__ __forceinline__ void cols_fft(C *buf, const C *twl, F &emit) {
    cols_mid_from<C, P, NCOL, NT, LD, SIGN, 0, TWCALC>(buf, twl);
    cols_pass_last<C, P, NCOL, NT, LD, SIGN, SYNC_LAST, F, TWCALC>(buf, twl, emit);
}

// Pass 0 (radix 16, Ns = 1) from registers: thread t owns butterfly
// (c, i) = (t / (P/16), t % (P/16)) with inputs v[r] = x_c[i + r P/16]; the
// outputs go to LDS and the function ends with a barrier.
template <typename C, int P, int NCOL, int NT, int LD, int SIGN>
__device__ __forceinline__ void cols_pass0_regs(C *buf, C *v) {
    static_assert(radix_of(P, 0) == 16 && NCOL * (P / 16) == NT, "one radix-16 butterfly per thread");
    const int c = threadIdx.x / (P / 16), i = threadIdx.x % (P / 16);
    dftR<16, SIGN>(v);
#pragma unroll
    for (int r = 0; r < 16; ++r) buf[c * LD + lidx(i * 16 + r) + col_skew<LD>(c)] = v[r];
    lds_barrier();
}

// remaining passes after cols_pass0_regs
template <typename C, int P, int NCOL, int NT, int LD, int SIGN, bool SYNC_LAST, class F, bool POSFAST = false>
__device__ __forceinline__ void cols_fft_after0(C *buf, const C *twl, F &emit) {
    static_assert(num_passes(P) >= 2, "at least two passes");
    cols_mid_from<C, P, NCOL, NT, LD, SIGN, 1>(buf, twl);
    cols_pass_last<C, P, NCOL, NT, LD, SIGN, SYNC_LAST, F, false, POSFAST>(buf, twl, emit);
}

// copy a per-pass twiddle table from global memory into LDS: every load is
// issued before the first LDS write, through the global address space (a
// flat load would also count as an LDS operation, so later LDS waits would
// wait for it too)
template <typename C, int P, int NT>
__device__ __forceinline__ void load_twl(C *twl_s, const C *__restrict__ twl_g) {
    constexpr int N = twl_len(P), K = (N + NT - 1) / NT;
#if defined(__HIP_DEVICE_COMPILE__)
    const __attribute__((address_space(1))) C *g = (const __attribute__((address_space(1))) C *)twl_g;
#else
    const C *g = twl_g;  // host pass of the kernel templates; never executed
#endif
    C v[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int j = threadIdx.x + k * NT;
        if (N % NT == 0 || j < N) v[k] = g[j];
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int j = threadIdx.x + k * NT;
        if (N % NT == 0 || j < N) twl_s[j] = v[k];
    }
}

}  // namespace cwt
