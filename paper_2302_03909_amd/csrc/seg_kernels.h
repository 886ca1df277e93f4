// seg_kernels.h -- device helpers and the two output kernels of the
// segmented FFT method (band inverse and fused small-scale segments),
// shared by the transform (cwt_seg.hip) and the statistics epilogue
// (cwt_wps.hip), which instantiate them with and without the reduction.
#pragma once
#include <type_traits>

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

// w_L^x, x in [0, L), for a segment length L = c 2^k: w_{2^k}^y w_L^z with
// x = c y + z (wsm[z] = w_L^z, read only when c > 1)
__device__ __forceinline__ double2 w_seg(const double2 *__restrict__ hi, const double2 *__restrict__ lo,
                                         const double2 *__restrict__ wsm, int c, int k, int64_t x) {
    if (c == 1) return w23(hi, lo, x << (23 - k));
    const uint32_t y = (uint32_t)x / (uint32_t)c, z = (uint32_t)x - y * (uint32_t)c;
    return cmul(w23(hi, lo, (int64_t)y << (23 - k)), wsm[z]);
}
// v modulo the segment length L = c 2^k (either sign of v)
__device__ __forceinline__ int64_t mod_seg(int64_t v, int c, int64_t L) {
    if (c == 1) return v & (L - 1);
    const int64_t r = v % L;
    return r < 0 ? r + L : r;
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
// and every wave issues the same number of memory instructions.  The stores
// (the transform's output, written once and far larger than the caches)
// carry the non-temporal hint, so they stream to HBM instead of displacing
// the signal, spectra and tables the other kernels read.
constexpr int kStoreNT = 2;  // cache-policy operand: nt
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
constexpr uint32_t kOOB = 0x80000000u;  // beyond every descriptor used here (< 2 GiB)
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void *base, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), 0, (int)bytes, 0x00020000);
}
__device__ __forceinline__ void bstore(float v, __amdgpu_buffer_rsrc_t r, uint32_t off) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, v), r, off, 0, kStoreNT);
}
__device__ __forceinline__ void bstore(double v, __amdgpu_buffer_rsrc_t r, uint32_t off) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, off, 0, kStoreNT);
}
__device__ __forceinline__ void bstore(float2 v, __amdgpu_buffer_rsrc_t r, uint32_t off) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, off, 0, kStoreNT);
}
__device__ __forceinline__ void bstore(double2 v, __amdgpu_buffer_rsrc_t r, uint32_t off) {
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, v), r, off, 0, kStoreNT);
}
__device__ __forceinline__ float bload(const float *, __amdgpu_buffer_rsrc_t r, uint32_t off) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}
__device__ __forceinline__ double bload(const double *, __amdgpu_buffer_rsrc_t r, uint32_t off) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}

__device__ __forceinline__ float2 bload(const float2 *, __amdgpu_buffer_rsrc_t r, uint32_t off) {
    return __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
__device__ __forceinline__ double2 bload(const double2 *, __amdgpu_buffer_rsrc_t r, uint32_t off) {
    return __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
}

template <typename C> __device__ __forceinline__ C to_c(double2 v) { return mk<C>((decltype(C::x))v.x, (decltype(C::x))v.y); }
template <typename C> __device__ __forceinline__ double2 to_d(C v) { return make_double2((double)v.x, (double)v.y); }

// Read-only data that every lane of a workgroup reads at the same address:
// loaded through the constant address space, i.e. with scalar loads into
// scalar registers (the tables are never written while a launch runs).
template <typename T> __device__ __forceinline__ T cload(const T *p) {
#if defined(__HIP_DEVICE_COMPILE__)
    return *(const __attribute__((address_space(4))) T *)p;
#else
    return *p;  // host pass of the kernel templates; never executed
#endif
}

// Values that are the same in every lane, marked as such so that they stay in
// scalar registers (buffer descriptors built from them must be scalar).
__device__ __forceinline__ int64_t uni(int64_t v) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}
template <typename T> __device__ __forceinline__ T *uni(T *p) { return (T *)uni((int64_t)p); }
template <typename T> __device__ __forceinline__ const T *uni(const T *p) { return (const T *)uni((int64_t)p); }

// The launch key, caller buffers and local block index of this workgroup.
struct Resolved {
    KeyDesc kd;
    BatchInst bi;
    int64_t local;
};
__device__ __forceinline__ Resolved resolve(const BatchArgs &a) {
    Resolved rv;
    if (a.nranges == 0) {
        rv = {a.k0, a.i0, (int64_t)blockIdx.x};
    } else {
        const int64_t b = blockIdx.x;
        int lo = cload(a.coarse + (b >> 8)), hi = cload(a.coarse + (b >> 8) + 1);
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (cload(a.ranges + mid).block0 <= b) lo = mid;
            else hi = mid - 1;
        }
        const BatchRange r = cload(a.ranges + lo);
        rv = {cload(r.key), cload(a.insts + r.inst), (int64_t)blockIdx.x - r.block0};
    }
    rv.bi.f = uni(rv.bi.f);
    rv.bi.out = uni(rv.bi.out);
    rv.bi.ws = uni(rv.bi.ws);
    rv.local = uni(rv.local);
    KeyDesc &k = rv.kd;
    k.N = uni(k.N);
    k.Tg = uni(k.Tg);
    k.V = uni(k.V);
    k.nseg = uni(k.nseg);
    k.groups = uni(k.groups);
    k.units = uni(k.units);
    k.work = uni(k.work);
    k.ktab = uni(k.ktab);
    k.twbase = uni(k.twbase);
    k.twl = uni(k.twl);
    k.whi = uni(k.whi);
    k.wlo = uni(k.wlo);
    k.scale_ids = uni(k.scale_ids);
    k.wps_base = uni(k.wps_base);
    rv.bi.env = uni(rv.bi.env);
    rv.bi.part = uni(rv.bi.part);
    k.periodic = __builtin_amdgcn_readfirstlane(k.periodic);
    k.cph = __builtin_amdgcn_readfirstlane(k.cph);
    k.nscale = __builtin_amdgcn_readfirstlane(k.nscale);
    return rv;
}



// ---------------------------------------------------------------------------
// statistics epilogue (Sec. 5, Eqs. env_wps and global_wps): each thread
// keeps, for the 16 outputs its last FFT pass emits, a 4-bit code (its
// environment bin, or kNoBin for a position that is not an output), and adds
// |w|^2 per bin instead of storing w.

constexpr uint32_t kNoBin = 15;

// bin of env[b] (b an output position): the number of thresholds <= env[b]
template <typename R>
__device__ __forceinline__ uint32_t wps_bin(const R *__restrict__ env, int64_t b, bool kept, const WpsArgs &w) {
    if (!kept) return kNoBin;
    const double e = (double)env[b];
    uint32_t k = 0;
#pragma unroll
    for (int j = 0; j < kWpsMaxBins - 1; ++j) k += (j < w.nbin - 1 && e >= w.thr[j]) ? 1u : 0u;
    return k;
}
__device__ __forceinline__ void put_code(uint32_t (&codes)[4], int k, uint32_t code) {
    codes[k >> 3] |= code << ((k & 7) * 4);
}
__device__ __forceinline__ uint32_t get_code(const uint32_t (&codes)[4], int k) {
    return (codes[k >> 3] >> ((k & 7) * 4)) & 15u;
}
// acc[bin(code)] += x^2 (codes of other bins, and kNoBin, add nothing): one
// compare, select and fused multiply-add per bin
template <int NB, typename A>
__device__ __forceinline__ void wps_acc(A (&acc)[kWpsMaxBins], uint32_t code, A x) {
#pragma unroll
    for (int b = 0; b < NB; ++b) acc[b] = fma(x, code == (uint32_t)b ? x : (A)0, acc[b]);
}
// the same for |x + i y|^2
template <int NB, typename A>
__device__ __forceinline__ void wps_acc(A (&acc)[kWpsMaxBins], uint32_t code, A x, A y) {
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const bool in = code == (uint32_t)b;
        acc[b] = fma(y, in ? y : (A)0, fma(x, in ? x : (A)0, acc[b]));
    }
}
// Sum over the 64 lanes of a wave with DPP moves (VALU only, no LDS round
// trip): lane pairs and quads by quad permutations, rows of 16 by row shifts
// of 4 and 8, then the row totals broadcast upward (lane 15 of each row into
// the next row, lane 31 into rows 2 and 3).  Lane 63 ends with the total;
// the summation order is fixed.  Lanes a move does not write, and sources
// outside the row, contribute 0.
template <int CTRL, int ROWMASK>
__device__ __forceinline__ float dpp_move(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, ROWMASK, 0xf, true));
}
template <int CTRL, int ROWMASK>
__device__ __forceinline__ double dpp_move(double v) {
    const u32x2 h = __builtin_bit_cast(u32x2, v);
    u32x2 r;
    r.x = (unsigned)__builtin_amdgcn_update_dpp(0, (int)h.x, CTRL, ROWMASK, 0xf, true);
    r.y = (unsigned)__builtin_amdgcn_update_dpp(0, (int)h.y, CTRL, ROWMASK, 0xf, true);
    return __builtin_bit_cast(double, r);
}
template <typename A>
__device__ __forceinline__ A wave_total(A v) {
    v += dpp_move<0xb1, 0xf>(v);   // quad_perm(1, 0, 3, 2)
    v += dpp_move<0x4e, 0xf>(v);   // quad_perm(2, 3, 0, 1)
    v += dpp_move<0x114, 0xf>(v);  // row_shr:4
    v += dpp_move<0x118, 0xf>(v);  // row_shr:8: lanes 12..15 of a row hold its total
    v += dpp_move<0x142, 0xa>(v);  // row_bcast:15 into rows 1 and 3
    v += dpp_move<0x143, 0xc>(v);  // row_bcast:31 into rows 2 and 3
    return v;
}
// per-wave sums parked in LDS: red[(wave * 2 + half) * kWpsMaxBins + bin]
template <int NB, typename A>
__device__ __forceinline__ void wps_park(const A (&acc)[kWpsMaxBins], double *red, int half) {
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const A t = wave_total(acc[b]);
        if ((threadIdx.x & 63) == 63) red[((threadIdx.x >> 6) * 2 + half) * kWpsMaxBins + b] = (double)t;
    }
}
// after a barrier: the workgroup's sums (waves added in order) to its slot
template <int NT>
__device__ __forceinline__ void wps_store(const double *red, int half, double *__restrict__ part, int64_t slot,
                                          int nbin) {
    const int t = threadIdx.x;
    if (t < nbin) {
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < NT / 64; ++w) s += red[(w * 2 + half) * kWpsMaxBins + t];
        part[slot * nbin + t] = s;
    }
}

// LDS elements for the staged spectrum samples of one BAND group: at most
// kSegKlsBytes, and at least one unit (two tables for a real-wavelet pair) of
// P bins
constexpr int seg_kls_elems(int rbytes, int P) {
    int n = kSegKlsBytes / rbytes;
    return n < 2 * P ? 2 * P : n;
}

// ---------------------------------------------------------------------------
// band-limited inverse: work item (g, seg, r0) covers columns r0..r0+15 of one
// segment for every output unit of the group.  Real output takes two real
// transforms per complex one: either two scales (unit sa, sb: real and
// imaginary part), or, in a column-pair group, the adjacent columns
// r0 + 2c, r0 + 2c + 1 of one scale as complex column c (work item r0..r0+31).
// Every column of a real output has a Hermitian P-point spectrum, so
// Z_{2c} + i Z_{2c+1} inverts to W_{2c} + i W_{2c+1}; each lane then holds two
// neighbouring outputs and stores them with one 8-byte store, 16 lanes
// filling a whole 128-byte line (a line written as two 64-byte halves, by two
// stores of one wave or of two workgroups, streams at about two thirds of the
// rate).
// A row that starts inside a line (N not a multiple of the line length) is
// shifted: for that unit the work item computes columns r0 - dsh .. instead
// (dsh = the row's offset in its line), so its runs again start on lines.
// Since W[t] = sum_k Y[k] w_L^{k t} for any t modulo L, the shift only
// multiplies the unit's spectrum samples by w_L^{-k dsh} (folded into complex
// samples at plan time, staged a chunk of units at a time), and column r < 0
// of row p is the output t = r + Q p (+ L when negative).

template <typename R, int P, int NT, bool PAIR, bool CPLX, int RED = 0>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(sizeof(R) == 4 && !PAIR ? 3 : 2))) void seg_inverse_kernel(
    const BatchArgs a) {
    using C = cplx_t<R>;
    constexpr int G = 16;
    // skewed columns for 8-byte elements (a 16-byte access is served 16
    // lanes at a time, where the plain stride is already conflict-free)
    constexpr int LD = P == 256 && sizeof(C) == 8 ? kLdSkew256 : lds_len(P);
    constexpr int MAXU = 32;
    constexpr int NB = P / 16;  // pass-0 butterflies per column
    constexpr int KLS = seg_kls_elems(sizeof(R), P);
    static_assert(NT == P, "one pass-0 butterfly per thread");
    __shared__ C buf[cols_len(G, LD)];
    __shared__ C twl[twl_len(P)];
    // spectrum samples of the group's units (and pair partners); complex
    // samples of shifted units in chunks of kls_chunk units
    __shared__ __align__(16) R kls[KLS];
    __shared__ double red[RED ? (NT / 64) * 2 * kWpsMaxBins : 1];  // statistics: per-wave sums
    const Resolved rv = resolve(a);
    const KeyDesc *kd = &rv.kd;
    const char *__restrict__ ws = rv.bi.ws;
    R *__restrict__ out = static_cast<R *>(rv.bi.out);
    const int64_t N = kd->N;
    const int cph = kd->cph;
    const R *__restrict__ ktab = static_cast<const R *>(kd->ktab);
    const char *__restrict__ twbase = kd->twbase;
    const SegUnit *__restrict__ units = kd->units;
    const double2 *__restrict__ whi = kd->whi, *__restrict__ wlo = kd->wlo;
    const SegWork w = cload(kd->work + rv.local);
    const SegGroupDev gd = cload(kd->groups + w.g);
    const int nunits = gd.nunits < MAXU ? gd.nunits : MAXU;
    const bool cp = PAIR && gd.colpair;              // column pairs of one scale (uniform)
    const bool shf = gd.cshift && (CPLX || cp);      // shifted single-row units (uniform)
    const bool codd = cp && gd.colodd;               // column pairs of an odd-length signal (uniform)
    const int64_t L = gd.L, Q = gd.Q;
    const int cL = __builtin_amdgcn_readfirstlane(gd.cL), kL = __builtin_amdgcn_readfirstlane(gd.lgL);
    const double2 *__restrict__ wsm = reinterpret_cast<const double2 *>(twbase + gd.wsm_off);
    const int tid = threadIdx.x;
    const int B = gd.B;
    const int64_t r0 = w.idx;
    // Every global read of the set-up is a buffer load issued before the
    // first wait (flat loads would also count as LDS operations), so the
    // set-up costs one memory latency instead of one per load.
    // pass-0 inputs of this thread: column c, positions kap = i + r P/16; the
    // band bin congruent to kap modulo P (if any) and w_L^{m c}
    const int c = tid / NB, i = tid % NB;
    // first(r): band bin congruent to i + r P/16 (valid when < B)
    const int f0 = (int)(((int64_t)i - gd.klo) & (P - 1));
    auto first_of = [&](int r) { return (f0 + r * NB) & (P - 1); };
    // w_L^{m c} of the band bins this thread reads; 0 for positions outside
    // the band (out-of-range offsets read 0)
    C gv[16];
    {
        const __amdgpu_buffer_rsrc_t gr =
            make_rsrc(uni(twbase + gd.gtw_off), __builtin_amdgcn_readfirstlane((uint32_t)(16 * B * (int)sizeof(C))));
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int fr = first_of(r);
            gv[r] = bload((const C *)nullptr, gr, fr < B ? (uint32_t)((c * B + fr) * (int)sizeof(C)) : kOOB);
        }
    }
    // band spectrum of the segment times w_L^{m r0}, staged in LDS (reuses buf)
    C *xs = buf;
    if (tid < B) {
        const int64_t mm = mod_seg(gd.klo + tid, cL, L);
        const double2 *X = reinterpret_cast<const double2 *>(ws + gd.x_off);
        xs[tid] = to_c<C>(cmul(X[(int64_t)w.seg * B + tid], w_seg(whi, wlo, wsm, cL, kL, mod_seg(mm * r0, cL, L))));
    }
    load_twl<C, P, NT>(twl, static_cast<const C *>(kd->twl));
    const __amdgpu_buffer_rsrc_t kr = make_rsrc(ktab, 0x7ffffff0u);
    // shifted units (uniform): their complex samples, with the shift phase
    // folded in, are staged kls_chunk units at a time (two reals per bin)
    const bool sh_path = !RED && (shf || codd);
    const int kls_chunk = sh_path ? KLS / (2 * B) : nunits;
    auto stage_complex = [&](int ub, int ue) {
        C *klc = reinterpret_cast<C *>(kls);
        if (tid < B) {
            for (int u0 = ub; u0 < ue; u0 += 8) {
                C kc[8];
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const int u = u0 + j < ue ? u0 + j : ue - 1;
                    const SegUnit su = cload(units + gd.unit0 + u);
                    kc[j] = bload((const C *)nullptr, kr, (uint32_t)((uni(su.kb) + 2 * tid) * (int64_t)sizeof(R)));
                }
#pragma unroll
                for (int j = 0; j < 8; ++j)
                    if (u0 + j < ue) klc[(u0 + j - ub) * B + tid] = kc[j];
            }
        }
    };
    // spectrum samples of every unit of the group (and pair partners),
    // staged in LDS once, eight units per batch of loads
    if (sh_path) {
        stage_complex(0, kls_chunk < nunits ? kls_chunk : nunits);
    } else if (tid < B) {
        for (int u0 = 0; u0 < nunits; u0 += 8) {
            R ka[8], kb[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int u = u0 + j < nunits ? u0 + j : nunits - 1;
                const SegUnit su = cload(units + gd.unit0 + u);
                ka[j] = bload(ktab, kr, (uint32_t)((uni(su.ka) + tid) * (int64_t)sizeof(R)));
                if constexpr (PAIR)
                    kb[j] = __builtin_amdgcn_readfirstlane(su.sb) >= 0
                                ? bload(ktab, kr, (uint32_t)((uni(su.kb) + tid) * (int64_t)sizeof(R)))
                                : (R)0;
            }
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                if (u0 + j < nunits) {
                    kls[(u0 + j) * B + tid] = ka[j];
                    if constexpr (PAIR)
                        if (!cp) kls[nunits * B + (u0 + j) * B + tid] = kb[j];
                }
            }
        }
    }
    lds_barrier();
    C xg[16];
    // band bin read for position r; bins outside the band read bin 0, which
    // is harmless because xg[r] is zero there.  The phase i^cph of the
    // wavelet's spectrum is common to every unit and folded into xg.
    int fro[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int fr = first_of(r);
        fro[r] = fr < B ? fr : 0;
        xg[r] = mul_i_pow(cmul(xs[fro[r]], gv[r]), cph);
    }
    lds_barrier();  // xs (in buf) is no longer read
    // 32-bit position arithmetic: t < L <= 2^23, and byte offsets are taken
    // modulo 2^32 (every kept one is below the 2 GiB of a row descriptor)
    const int64_t ob = (int64_t)w.seg * gd.V - gd.Tg;
    const uint32_t eb = (uint32_t)(CPLX ? sizeof(C) : sizeof(R));
    const uint32_t obe = (uint32_t)ob * eb;
    const int32_t tlo = (int32_t)gd.Tg, thi = (int32_t)(gd.Tg + gd.V);
    const int32_t Li = (int32_t)L, Qi = (int32_t)Q;
    // statistics: bin codes of the outputs this thread emits (unshifted
    // columns; with column pairs two outputs, t and t + 1, per emit)
    uint32_t codes[4] = {0u, 0u, 0u, 0u};
    const int nbin = RED ? a.wps.nbin : 0;
    if constexpr (RED) {
        const R *__restrict__ env = static_cast<const R *>(rv.bi.env);
        cols_last_positions<P, G, NT, false>([&](int k, int cc, int p) {
            const int32_t t = (int32_t)r0 + (cp ? 2 * cc : cc) + Qi * p;
            auto code = [&](int32_t tt) {
                return wps_bin(env, ob + tt, tt >= tlo && tt < thi && ob + tt < N, a.wps);
            };
            if (cp) {
                put_code(codes, 2 * k, code(t));
                put_code(codes, 2 * k + 1, code(t + 1));
            } else {
                put_code(codes, k, code(t));
            }
        });
    }
    auto units_loop = [&](auto cp_const, auto sh_const, auto odd_const) {
        constexpr bool CP = decltype(cp_const)::value;
        constexpr bool SH = decltype(sh_const)::value;
        constexpr bool ODD = decltype(odd_const)::value;
        for (int u = 0; u < nunits; ++u) {
            // unit fields are uniform; say so, so that the store descriptors
            // live in scalar registers (no waterfall loop around the stores)
            const SegUnit su = cload(units + gd.unit0 + u);
            const int sa = __builtin_amdgcn_readfirstlane(su.sa);
            const int sb = __builtin_amdgcn_readfirstlane(su.sb);
            const int dl = SH ? __builtin_amdgcn_readfirstlane(su.dsh) : 0;
            C v[16];
            if constexpr (SH) {
                // the next chunk of complex samples (every read of the
                // previous chunk ended before the last unit's final barrier)
                const int uk = u % kls_chunk;
                if (u > 0 && uk == 0) {
                    stage_complex(u, u + kls_chunk < nunits ? u + kls_chunk : nunits);
                    lds_barrier();
                }
                // samples times w_L^{-m dsh}, m = klo + fro[r]: the shift of
                // the unit's columns by dsh
                const C *klc = reinterpret_cast<const C *>(kls) + uk * B;
#pragma unroll
                for (int r = 0; r < 16; ++r) v[r] = cmul(xg[r], klc[fro[r]]);
            }
            if constexpr (!SH) {
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    if constexpr (PAIR && !CP) {
                        const R ka = kls[u * B + fro[r]];
                        const R kb = kls[nunits * B + u * B + fro[r]];
                        v[r] = cmul(xg[r], mk<C>(ka, kb));
                    } else {
                        v[r] = cscale(xg[r], kls[u * B + fro[r]]);
                    }
                }
            }
            cols_pass0_regs<C, P, G, NT, LD, +1>(buf, v);
            // output b = ob + t, t = r0 - dsh + col + Q p modulo L (col = cc,
            // or 2 cc and the next one for column pairs); only t < 0 wraps.
            // Kept when Tg <= t < Tg + V; the descriptor of each row spans
            // exactly its N values, so b >= N is dropped.  Column pairs of an
            // even N: t, Tg, V and N are even, so both outputs are kept or
            // dropped.  Odd N (ODD): a pair can straddle the row end or a
            // window edge, or wrap (t = -1, 0); such a pair is stored as two
            // single outputs, each kept or dropped on its own.
            if constexpr (RED) {
                // |w|^2 per bin: sa takes the real parts (or both outputs of a
                // column pair, or the complex values), sb the imaginary parts
                R acc_a[kWpsMaxBins] = {}, acc_b[kWpsMaxBins] = {};
                int k = 0;
                auto remit = [&](int, int, C val) {
                    if constexpr (CPLX) {
                        wps_acc<RED>(acc_a, get_code(codes, k), val.x, val.y);
                    } else if constexpr (CP) {
                        wps_acc<RED>(acc_a, get_code(codes, 2 * k), val.x);
                        wps_acc<RED>(acc_a, get_code(codes, 2 * k + 1), val.y);
                    } else {
                        wps_acc<RED>(acc_a, get_code(codes, k), val.x);
                        wps_acc<RED>(acc_b, get_code(codes, k), val.y);
                    }
                    ++k;
                };
                cols_fft_after0<C, P, G, NT, LD, +1, false>(buf, twl, remit);
                const bool has_b = PAIR && !CP && sb >= 0;
                wps_park<RED>(acc_a, red, 0);
                if (has_b) wps_park<RED>(acc_b, red, 1);
                lds_barrier();
                const int64_t slot = rv.local - gd.inv0;
                wps_store<NT>(red, 0, rv.bi.part, cload(kd->wps_base + sa) + slot, nbin);
                if (has_b) wps_store<NT>(red, 1, rv.bi.part, cload(kd->wps_base + sb) + slot, nbin);
                continue;
            }
            const __amdgpu_buffer_rsrc_t ra =
                make_rsrc(out + (int64_t)sa * N * (CPLX ? 2 : 1), (uint32_t)(N * eb));
            const __amdgpu_buffer_rsrc_t rb =
                make_rsrc(out + (int64_t)(PAIR && sb >= 0 ? sb : sa) * N, (uint32_t)(N * eb));
            const bool has_b = PAIR && sb >= 0;
            const int32_t t0 = (int32_t)r0 - dl;
            auto emit = [&](int cc, int p, C val) {
                int32_t t = t0 + (CP ? 2 * cc : cc) + Qi * p;
                if constexpr (ODD) {
                    int32_t ty = t + 1;
                    if constexpr (SH) {
                        t += t < 0 ? Li : 0;
                        ty += ty < 0 ? Li : 0;
                    }
                    const bool kx = t >= tlo && t < thi, ky = ty >= tlo && ty < thi;
                    // b + 1 < N: the pair lies inside the row
                    if (kx && ky && ty == t + 1 && (int64_t)ob + ty < N) {
                        bstore(val, ra, obe + (uint32_t)t * eb);
                    } else {
                        bstore(val.x, ra, kx ? obe + (uint32_t)t * eb : kOOB);
                        bstore(val.y, ra, ky ? obe + (uint32_t)ty * eb : kOOB);
                    }
                    return;
                }
                if constexpr (SH) t += t < 0 ? Li : 0;
                const uint32_t off = (t >= tlo && t < thi) ? obe + (uint32_t)t * eb : kOOB;
                if (CPLX || CP) bstore(val, ra, off);
                else {
                    bstore(val.x, ra, off);
                    bstore(val.y, rb, has_b ? off : kOOB);
                }
            };
            cols_fft_after0<C, P, G, NT, LD, +1, false>(buf, twl, emit);
            lds_barrier();
        }
    };
    using T_ = std::true_type;
    using F_ = std::false_type;
    if constexpr (RED) {
        // no column shift: the shift only aligns stores
        if (PAIR && cp) units_loop(T_{}, F_{}, F_{});
        else units_loop(F_{}, F_{}, F_{});
    } else if constexpr (PAIR) {
        if (!cp) units_loop(F_{}, F_{}, F_{});
        else if (codd) units_loop(T_{}, T_{}, T_{});  // odd N: pairs may straddle edges; always shifted
        else if (shf) units_loop(T_{}, T_{}, F_{});
        else units_loop(T_{}, F_{}, F_{});
    } else {
        if (shf) units_loop(F_{}, T_{}, F_{});
        else units_loop(F_{}, F_{}, F_{});
    }
}

// ---------------------------------------------------------------------------
// fused full-spectrum segments (small scales)

// G columns of L points per workgroup (G L = 16 NT): one radix-16 butterfly
// per thread in every pass of the inverse.  The segment transform is taken in
// FP64 whatever the plan precision: an FP32 forward spreads rounding noise of
// order eps |f| over every bin, which for red spectra swamps the weak
// high-frequency bands the small scales read.  To keep the FP64 forward
// within the LDS of the inverse buffer, it runs on G/2 complex columns: real
// segments 2z and 2z+1 share column z as real and imaginary part; with
// Z = DFT(a + i b),  A[k] = (Z[k] + conj Z[-k]) / 2 and
// B[k] = (Z[k] - conj Z[-k]) / (2 i).  With G = 1 the single column takes the
// whole FP64 buffer.
// Real wavelets (PAIR): the spectrum of a scale, phase folded into X, is
// Hermitian (real and even, or imaginary and odd), so X K_a + i X K_b inverts
// to w_a + i w_b: one inverse yields two scales, real part and imaginary part.
template <typename R, int L, int G, int NT, bool PAIR, bool CPLX, int RED = 0>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(sizeof(R) == 4 ? 3 : 2))) void local2_kernel(
    const BatchArgs a) {
    using C = cplx_t<R>;
    constexpr int LD = lds_len(L);
    static_assert(G * L == 16 * NT, "one radix-16 butterfly per thread");
    constexpr int FCOL = G >= 2 ? G / 2 : 1;           // FP64 columns per round
    constexpr int NROUND = 1;                           // forward rounds
    constexpr bool TWO = G >= 2;                        // two real segments per FP64 column
    constexpr int BUF_BYTES = (FCOL * LD * 16 > G * LD * (int)sizeof(C)) ? FCOL * LD * 16 : G * LD * (int)sizeof(C);
    __shared__ double2 bufF[BUF_BYTES / 16];
    C *buf = reinterpret_cast<C *>(bufF);
    __shared__ C twl[twl_len(L)];
    __shared__ double red[RED ? (NT / 64) * 2 * kWpsMaxBins : 1];  // statistics: per-wave sums
    const Resolved rv = resolve(a);
    const KeyDesc *kd = &rv.kd;
    const R *__restrict__ f = static_cast<const R *>(rv.bi.f);
    R *__restrict__ out = static_cast<R *>(rv.bi.out);
    const int64_t N = kd->N, Tg = kd->Tg, V = kd->V;
    const int periodic = __builtin_amdgcn_readfirstlane(kd->periodic);
    const int nscale = kd->nscale, cph = kd->cph;
    const int32_t *__restrict__ scale_ids = kd->scale_ids;
    const R *__restrict__ ktab = static_cast<const R *>(kd->ktab);
    // pass twiddles in LDS: needed by the FP64 forward of FP64 plans (FP32
    // plans evaluate those, and load the table after the forward)
    if constexpr (sizeof(R) == 8) load_twl<C, L, NT>(twl, static_cast<const C *>(kd->twl));
    const double2 *twF = reinterpret_cast<const double2 *>(twl);
    const int tid = threadIdx.x;
    constexpr int SEGS = 1;  // segments per inverse column
    const int64_t seg0 = rv.local * G * SEGS;
    // inverse pass-0 layout: thread t owns column cc = t / (L/16), positions
    // ii + r L/16
    constexpr int NB = L / 16;
    const int cc = tid / NB, ii = tid % NB;
    C Xr[16];
    // Zero boundary: raw buffer loads over f[0, N) with 32-bit offsets;
    // positions outside, negative ones included (they wrap to large unsigned
    // offsets), read 0.  All loads of a round are issued before the first
    // LDS write.
    const __amdgpu_buffer_rsrc_t fr = make_rsrc(f, (uint32_t)(N * (int64_t)sizeof(R)));
    constexpr int EL = FCOL * L / NT;  // FP64 column elements per thread and round
    static_assert((FCOL * L) % NT == 0, "whole column elements per thread");
    constexpr bool TWOSEG = TWO;
#pragma unroll
    for (int h = 0; h < NROUND; ++h) {
        // FP64 column z of this round: segments s0(z) and s0(z) + 1
        R xa[EL], xb[EL];
        auto pos = [&](int e) {
            const int idx = tid + e * NT, z = idx / L, u = idx % L;
            const int64_t s = seg0 + (TWO ? 2 * (int64_t)z : (int64_t)(h * FCOL + z) * SEGS);
            return s * V - Tg + u;
        };
        if (periodic) {
#pragma unroll
            for (int e = 0; e < EL; ++e) {
                xa[e] = sig_seg(f, N, 1, pos(e));
                xb[e] = TWOSEG ? sig_seg(f, N, 1, pos(e) + V) : (R)0;
            }
        } else {
#pragma unroll
            for (int e = 0; e < EL; ++e) {
                const int64_t pa = pos(e);
                xa[e] = bload((const R *)nullptr, fr, (uint32_t)(pa * (int64_t)sizeof(R)));
                xb[e] = TWOSEG ? bload((const R *)nullptr, fr, (uint32_t)((pa + V) * (int64_t)sizeof(R))) : (R)0;
            }
        }
#pragma unroll
        for (int e = 0; e < EL; ++e) {
            const int idx = tid + e * NT;
            bufF[(idx / L) * LD + lidx(idx % L)] = make_double2((double)xa[e], (double)xb[e]);
        }
        lds_barrier();
        {
            auto emit = [&](int c, int p, double2 v) { bufF[c * LD + lidx(p)] = v; };
            cols_fft<double2, L, FCOL, NT, LD, -1, true, decltype(emit), sizeof(R) == 4>(bufF, twF, emit);
        }
        lds_barrier();
        // spectra of this thread's column, phase i^cph folded in
        if constexpr (TWO) {
            const int z = cc >> 1;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int k = ii + r * NB;
                const double2 zk = bufF[z * LD + lidx(k)], zm = bufF[z * LD + lidx((L - k) & (L - 1))];
                // even column: (Z[k] + conj Z[-k]) / 2; odd: (Z[k] - conj Z[-k]) / (2 i)
                const double2 x = (cc & 1) ? make_double2(0.5 * (zk.y + zm.y), -0.5 * (zk.x - zm.x))
                                           : make_double2(0.5 * (zk.x + zm.x), 0.5 * (zk.y - zm.y));
                Xr[r] = to_c<C>(mul_i_pow(x, cph));
            }
        } else {
            const int z = cc - h * FCOL;
            if (z >= 0 && z < FCOL) {
#pragma unroll
                for (int r = 0; r < 16; ++r) Xr[r] = to_c<C>(mul_i_pow(bufF[z * LD + lidx(ii + r * NB)], cph));
            }
        }
        lds_barrier();
    }
    if constexpr (sizeof(R) == 4) {
        load_twl<C, L, NT>(twl, static_cast<const C *>(kd->twl));
        lds_barrier();
    }
    // spectrum samples through buffer loads: flat loads would also count as
    // LDS operations and make every LDS wait wait for them
    const __amdgpu_buffer_rsrc_t kr = make_rsrc(ktab, (uint32_t)((int64_t)nscale * L * (int64_t)sizeof(R)));
    // scales per inverse: one (complex output) or two (real pair)
    constexpr int SPI = PAIR ? 2 : 1;
    R kv[SPI][16];
    auto load_kv = [&](int j) {
#pragma unroll
        for (int h = 0; h < SPI; ++h) {
            // a missing second scale reads beyond the table: zeros
            const uint32_t o = j + h < nscale ? (uint32_t)((j + h) * L * (int)sizeof(R)) : kOOB;
#pragma unroll
            for (int r = 0; r < 16; ++r) kv[h][r] = bload(ktab, kr, o + (uint32_t)((ii + r * NB) * sizeof(R)));
        }
    };
    load_kv(0);
    constexpr uint32_t eb = (uint32_t)(CPLX ? sizeof(C) : sizeof(R));
    // statistics: bin codes of the 16 outputs this thread emits
    uint32_t codes[4] = {0u, 0u, 0u, 0u};
    const int nbin = RED ? a.wps.nbin : 0;
    if constexpr (RED) {
        const R *__restrict__ env = static_cast<const R *>(rv.bi.env);
        cols_last_positions<L, G, NT, true>([&](int k, int c, int p) {
            const int64_t b = (seg0 + (int64_t)c * SEGS) * V + (p - Tg);
            put_code(codes, k, wps_bin(env, b, p >= Tg && p < Tg + V && b < N, a.wps));
        });
    }
    for (int j = 0; j < nscale; j += SPI) {
        C v[16];
#pragma unroll
        for (int r = 0; r < 16; ++r) v[r] = PAIR ? cmul(Xr[r], mk<C>(kv[0][r], kv[1][r])) : cscale(Xr[r], kv[0][r]);
        if (j + SPI < nscale) load_kv(j + SPI);  // prefetch the next scales' spectrum samples
        // keep the prefetch loads ahead of this scale's stores (no code emitted)
        asm volatile("" ::: "memory");
        cols_pass0_regs<C, L, G, NT, LD, +1>(buf, v);
        if constexpr (RED) {
            // |w|^2 per bin: scale j takes the real parts (or the complex
            // values), scale j + 1 the imaginary parts
            R acc_a[kWpsMaxBins] = {}, acc_b[kWpsMaxBins] = {};
            int k = 0;
            auto remit = [&](int, int, C val) {
                const uint32_t code = get_code(codes, k);
                if constexpr (CPLX) {
                    wps_acc<RED>(acc_a, code, val.x, val.y);
                } else {
                    wps_acc<RED>(acc_a, code, val.x);
                    wps_acc<RED>(acc_b, code, val.y);
                }
                ++k;
            };
            cols_fft_after0<C, L, G, NT, LD, +1, false, decltype(remit), true>(buf, twl, remit);
            const bool has_b = PAIR && j + 1 < nscale;
            wps_park<RED>(acc_a, red, 0);
            if (has_b) wps_park<RED>(acc_b, red, 1);
            lds_barrier();
            wps_store<NT>(red, 0, rv.bi.part, cload(kd->wps_base + cload(scale_ids + j)) + rv.local, nbin);
            if (has_b) wps_store<NT>(red, 1, rv.bi.part, cload(kd->wps_base + cload(scale_ids + j + 1)) + rv.local, nbin);
            continue;
        }
        const __amdgpu_buffer_rsrc_t rr =
            make_rsrc(out + (int64_t)cload(scale_ids + j) * N * (CPLX ? 2 : 1), (uint32_t)(N * eb));
        const bool has_b = PAIR && j + 1 < nscale;
        const __amdgpu_buffer_rsrc_t rb =
            make_rsrc(out + (int64_t)cload(scale_ids + (has_b ? j + 1 : j)) * N, (uint32_t)(N * eb));
        // position-fastest last pass: consecutive lanes store consecutive
        // outputs of one segment
        auto emit = [&](int c, int p, C val) {
            const bool inside = p >= Tg && p < Tg + V;
            const int64_t sgi = seg0 + (int64_t)c * SEGS;
            const int64_t b = sgi * V + (p - Tg);
            const uint32_t off = inside ? (uint32_t)(b * (int64_t)eb) : kOOB;
            if (CPLX) bstore(val, rr, off);
            else {
                bstore(val.x, rr, off);
                bstore(val.y, rb, has_b ? off : kOOB);
            }
        };
        cols_fft_after0<C, L, G, NT, LD, +1, false, decltype(emit), true>(buf, twl, emit);
        lds_barrier();
    }
}

// ---------------------------------------------------------------------------
// launchers of the two output kernels (RED > 0: the statistics variants
// for up to RED environment bins)

// local2 columns per workgroup: 4096 points (FP32) or 2048 points (FP64), at
// least one
constexpr int local2_ncol(int L, bool fp64) { return (fp64 ? 2048 : 4096) / L > 1 ? (fp64 ? 2048 : 4096) / L : 1; }
constexpr int local2_nt(int L, bool fp64) { return local2_ncol(L, fp64) * L / 16; }

template <typename R, int L, int RED>
hipError_t local2_launch_L(const BatchArgs &a, int64_t blocks, bool cplx, hipStream_t st) {
    constexpr int NCOL = local2_ncol(L, sizeof(R) == 8);
    constexpr int NT = local2_nt(L, sizeof(R) == 8);
    if (cplx)
        hipLaunchKernelGGL((local2_kernel<R, L, NCOL, NT, false, true, RED>), dim3((unsigned)blocks), dim3(NT), 0, st, a);
    else
        hipLaunchKernelGGL((local2_kernel<R, L, NCOL, NT, true, false, RED>), dim3((unsigned)blocks), dim3(NT), 0, st, a);
    return hipGetLastError();
}

template <typename R, int RED>
hipError_t local2_typed(int L, const BatchArgs &a, int64_t blocks, bool cplx, hipStream_t st) {
    switch (L) {
        case 64: return local2_launch_L<R, 64, RED>(a, blocks, cplx, st);
        case 128: return local2_launch_L<R, 128, RED>(a, blocks, cplx, st);
        case 256: return local2_launch_L<R, 256, RED>(a, blocks, cplx, st);
        case 512: return local2_launch_L<R, 512, RED>(a, blocks, cplx, st);
        case 1024: return local2_launch_L<R, 1024, RED>(a, blocks, cplx, st);
        case 2048: return local2_launch_L<R, 2048, RED>(a, blocks, cplx, st);
        case 4096: return local2_launch_L<R, 4096, RED>(a, blocks, cplx, st);
        default: return hipErrorInvalidValue;
    }
}

template <typename R, int P, int RED>
hipError_t inverse_launch_P(const BatchArgs &a, int64_t blocks, bool cplx, hipStream_t st) {
    constexpr int NT = P;  // 16 columns x P / 16 elements per thread
    if (cplx)
        hipLaunchKernelGGL((seg_inverse_kernel<R, P, NT, false, true, RED>), dim3((unsigned)blocks), dim3(NT), 0, st, a);
    else
        hipLaunchKernelGGL((seg_inverse_kernel<R, P, NT, true, false, RED>), dim3((unsigned)blocks), dim3(NT), 0, st, a);
    return hipGetLastError();
}

template <typename R, int RED>
hipError_t inverse_typed(int P, const BatchArgs &a, int64_t blocks, bool cplx, hipStream_t st) {
    switch (P) {
        case 64: return inverse_launch_P<R, 64, RED>(a, blocks, cplx, st);
        case 128: return inverse_launch_P<R, 128, RED>(a, blocks, cplx, st);
        case 256: return inverse_launch_P<R, 256, RED>(a, blocks, cplx, st);
        case 512: return inverse_launch_P<R, 512, RED>(a, blocks, cplx, st);
        default: return hipErrorInvalidValue;
    }
}

// kind 0 (local2) or 3 (band inverse)
template <int RED>
hipError_t launch_out_kernel(const SegKernelId &id, const BatchArgs &a, int64_t blocks, hipStream_t st) {
    const bool fp64 = id.precision == 0, cplx = id.cplx != 0;
    if (id.kind == 0)
        return fp64 ? local2_typed<double, RED>(id.size, a, blocks, cplx, st)
                    : local2_typed<float, RED>(id.size, a, blocks, cplx, st);
    if (id.kind == 3)
        return fp64 ? inverse_typed<double, RED>(id.size, a, blocks, cplx, st)
                    : inverse_typed<float, RED>(id.size, a, blocks, cplx, st);
    return hipErrorInvalidValue;
}

}  // namespace cwt
