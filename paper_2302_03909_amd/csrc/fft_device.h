// fft_device.h -- workgroup-level mixed-radix Stockham FFT for gfx950.
//
// A workgroup of NT threads transforms NCOL independent P-point sequences
// that sit in LDS.  Every pass of radix R reads R values per butterfly into
// registers, applies the twiddles, runs an in-register radix-R DFT and
// writes the results back in Stockham (self-sorting) order, so the result
// is in natural order without a bit-reversal pass:
//
//   pass with sub-transform size Ns, butterfly i in [0, P/R):
//     v[r] = x[i + r P/R],  k = i mod Ns,
//     v[r] *= w_{R Ns}^{sign r k},  v = DFT_R(v),
//     y[(i - k) R + k + r Ns] = v[r].
//
// sign = +1 computes sum_n x[n] e^{+2 pi i n k / P} (inverse, unnormalised),
// sign = -1 the forward transform.  Twiddles come from a table
// tw[j] = e^{+2 pi i j / P} generated in FP64 on the host and stored in the
// kernel's precision.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cwt {

// Workgroup barrier that orders LDS accesses only.  __syncthreads() also
// waits until every global store the wave issued has completed, which
// serialises a kernel's output stores with its next FFT; the kernels here
// never read back, within a launch, global memory that another wave wrote,
// so their barriers need only the LDS fence.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

template <typename R> struct cplx_of;
template <> struct cplx_of<float> { using type = float2; };
template <> struct cplx_of<double> { using type = double2; };
template <typename R> using cplx_t = typename cplx_of<R>::type;

template <typename C> __device__ __forceinline__ C mk(decltype(C::x) a, decltype(C::x) b) {
    C c;
    c.x = a;
    c.y = b;
    return c;
}
template <typename C> __device__ __forceinline__ C cadd(C a, C b) { return mk<C>(a.x + b.x, a.y + b.y); }
template <typename C> __device__ __forceinline__ C csub(C a, C b) { return mk<C>(a.x - b.x, a.y - b.y); }
template <typename C> __device__ __forceinline__ C cmul(C a, C b) {
    return mk<C>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
template <typename C> __device__ __forceinline__ C cmulc(C a, C b) {
    return mk<C>(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
template <typename C> __device__ __forceinline__ C cscale(C a, decltype(C::x) s) { return mk<C>(a.x * s, a.y * s); }
// multiply by sign * i
template <int SIGN, typename C> __device__ __forceinline__ C mul_si(C a) {
    return SIGN > 0 ? mk<C>(-a.y, a.x) : mk<C>(a.y, -a.x);
}
// multiply by w = (c, SIGN * s)
template <int SIGN, typename C>
__device__ __forceinline__ C mul_cs(C a, decltype(C::x) c, decltype(C::x) s) {
    return SIGN > 0 ? mk<C>(a.x * c - a.y * s, a.x * s + a.y * c)
                    : mk<C>(a.x * c + a.y * s, a.y * c - a.x * s);
}

// ---- small DFTs, in place, natural output order -------------------------
template <int SIGN, typename C> __device__ __forceinline__ void dft2(C &a, C &b) {
    C t = a;
    a = cadd(t, b);
    b = csub(t, b);
}

template <int SIGN, typename C> __device__ __forceinline__ void dft4(C &x0, C &x1, C &x2, C &x3) {
    C a = cadd(x0, x2), b = csub(x0, x2), c = cadd(x1, x3), d = mul_si<SIGN>(csub(x1, x3));
    x0 = cadd(a, c);
    x2 = csub(a, c);
    x1 = cadd(b, d);
    x3 = csub(b, d);
}

template <int SIGN, typename C> __device__ __forceinline__ void dft3(C &x0, C &x1, C &x2) {
    using R = decltype(C::x);
    const R h = (R)0.86602540378443864676;  // sin(2 pi / 3)
    C t1 = cadd(x1, x2), t2 = csub(x1, x2);
    C m = mk<C>(x0.x - (R)0.5 * t1.x, x0.y - (R)0.5 * t1.y);
    C r = mul_si<SIGN>(cscale(t2, h));
    x0 = cadd(x0, t1);
    x1 = cadd(m, r);
    x2 = csub(m, r);
}

template <int SIGN, typename C> __device__ __forceinline__ void dft5(C &x0, C &x1, C &x2, C &x3, C &x4) {
    using R = decltype(C::x);
    const R c1 = (R)0.30901699437494742410, c2 = (R)-0.80901699437494742410;
    const R s1 = (R)0.95105651629515357212, s2 = (R)0.58778525229247312917;
    C a1 = cadd(x1, x4), b1 = csub(x1, x4), a2 = cadd(x2, x3), b2 = csub(x2, x3);
    C y0 = cadd(x0, cadd(a1, a2));
    C p1 = mk<C>(x0.x + c1 * a1.x + c2 * a2.x, x0.y + c1 * a1.y + c2 * a2.y);
    C p2 = mk<C>(x0.x + c2 * a1.x + c1 * a2.x, x0.y + c2 * a1.y + c1 * a2.y);
    C q1 = mul_si<SIGN>(mk<C>(s1 * b1.x + s2 * b2.x, s1 * b1.y + s2 * b2.y));
    C q2 = mul_si<SIGN>(mk<C>(s2 * b1.x - s1 * b2.x, s2 * b1.y - s1 * b2.y));
    x0 = y0;
    x1 = cadd(p1, q1);
    x4 = csub(p1, q1);
    x2 = cadd(p2, q2);
    x3 = csub(p2, q2);
}

// 8 = 2 x 4: A[n1][k1] = DFT4_{n2} x[n1 + 2 n2]; A *= w8^{n1 k1}; X[k1 + 4 k2] = DFT2_{n1}
template <int SIGN, typename C> __device__ __forceinline__ void dft8(C *v) {
    using R = decltype(C::x);
    const R r2 = (R)0.70710678118654752440;
    C a0 = v[0], a1 = v[2], a2 = v[4], a3 = v[6];
    C b0 = v[1], b1 = v[3], b2 = v[5], b3 = v[7];
    dft4<SIGN>(a0, a1, a2, a3);
    dft4<SIGN>(b0, b1, b2, b3);
    b1 = mul_cs<SIGN>(b1, r2, r2);
    b2 = mul_si<SIGN>(b2);
    b3 = mul_cs<SIGN>(b3, -r2, r2);
    dft2<SIGN>(a0, b0);
    dft2<SIGN>(a1, b1);
    dft2<SIGN>(a2, b2);
    dft2<SIGN>(a3, b3);
    v[0] = a0; v[1] = a1; v[2] = a2; v[3] = a3;
    v[4] = b0; v[5] = b1; v[6] = b2; v[7] = b3;
}

// 9 = 3 x 3
template <int SIGN, typename C> __device__ __forceinline__ void dft9(C *v) {
    using R = decltype(C::x);
    // w9^1, w9^2, w9^4 as (cos, sin)
    const R c1 = (R)0.76604444311897803520, s1 = (R)0.64278760968653932632;
    const R c2 = (R)0.17364817766693034885, s2 = (R)0.98480775301220805936;
    const R c4 = (R)-0.93969262078590838405, s4 = (R)0.34202014332566873304;
    C a[3][3];
#pragma unroll
    for (int n1 = 0; n1 < 3; ++n1) {
        a[n1][0] = v[n1];
        a[n1][1] = v[n1 + 3];
        a[n1][2] = v[n1 + 6];
        dft3<SIGN>(a[n1][0], a[n1][1], a[n1][2]);
    }
    a[1][1] = mul_cs<SIGN>(a[1][1], c1, s1);
    a[1][2] = mul_cs<SIGN>(a[1][2], c2, s2);
    a[2][1] = mul_cs<SIGN>(a[2][1], c2, s2);
    a[2][2] = mul_cs<SIGN>(a[2][2], c4, s4);
#pragma unroll
    for (int k1 = 0; k1 < 3; ++k1) {
        C y0 = a[0][k1], y1 = a[1][k1], y2 = a[2][k1];
        dft3<SIGN>(y0, y1, y2);
        v[k1] = y0;
        v[k1 + 3] = y1;
        v[k1 + 6] = y2;
    }
}

// 16 = 4 x 4: A[n1][k1] = DFT4_{n2} x[n1 + 4 n2]; A *= w16^{n1 k1}; X[k1 + 4 k2] = DFT4_{n1}
template <int SIGN, typename C> __device__ __forceinline__ void dft16(C *v) {
    using R = decltype(C::x);
    const R c1 = (R)0.92387953251128675613, s1 = (R)0.38268343236508977173;  // w16^1
    const R r2 = (R)0.70710678118654752440;                                  // w16^2
    C a[4][4];
#pragma unroll
    for (int n1 = 0; n1 < 4; ++n1) {
        a[n1][0] = v[n1];
        a[n1][1] = v[n1 + 4];
        a[n1][2] = v[n1 + 8];
        a[n1][3] = v[n1 + 12];
        dft4<SIGN>(a[n1][0], a[n1][1], a[n1][2], a[n1][3]);
    }
    a[1][1] = mul_cs<SIGN>(a[1][1], c1, s1);   // w^1
    a[1][2] = mul_cs<SIGN>(a[1][2], r2, r2);   // w^2
    a[1][3] = mul_cs<SIGN>(a[1][3], s1, c1);   // w^3
    a[2][1] = mul_cs<SIGN>(a[2][1], r2, r2);   // w^2
    a[2][2] = mul_si<SIGN>(a[2][2]);           // w^4
    a[2][3] = mul_cs<SIGN>(a[2][3], -r2, r2);  // w^6
    a[3][1] = mul_cs<SIGN>(a[3][1], s1, c1);   // w^3
    a[3][2] = mul_cs<SIGN>(a[3][2], -r2, r2);  // w^6
    a[3][3] = mul_cs<SIGN>(a[3][3], -c1, -s1); // w^9
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
        C y0 = a[0][k1], y1 = a[1][k1], y2 = a[2][k1], y3 = a[3][k1];
        dft4<SIGN>(y0, y1, y2, y3);
        v[k1] = y0;
        v[k1 + 4] = y1;
        v[k1 + 8] = y2;
        v[k1 + 12] = y3;
    }
}

template <int R, int SIGN, typename C> __device__ __forceinline__ void dftR(C *v) {
    if constexpr (R == 2) dft2<SIGN>(v[0], v[1]);
    else if constexpr (R == 3) dft3<SIGN>(v[0], v[1], v[2]);
    else if constexpr (R == 4) dft4<SIGN>(v[0], v[1], v[2], v[3]);
    else if constexpr (R == 5) dft5<SIGN>(v[0], v[1], v[2], v[3], v[4]);
    else if constexpr (R == 8) dft8<SIGN>(v);
    else if constexpr (R == 9) dft9<SIGN>(v);
    else if constexpr (R == 16) dft16<SIGN>(v);
    else static_assert(R == 16, "unsupported radix");
}

// ---- radix schedules -------------------------------------------------------
// P = r * 2^k with r in {1, 3, 5, 9}: the odd radix first, then radix-16
// passes, then one pass of radix 2, 4 or 8 for the remaining power of two.
constexpr int odd_part(int p) { return (p % 9 == 0) ? 9 : (p % 5 == 0) ? 5 : (p % 3 == 0) ? 3 : 1; }
constexpr int log2_exact(int p) { int k = 0; while ((1 << k) < p) ++k; return k; }
constexpr int num_passes(int p) {
    int r = odd_part(p);
    int k = log2_exact(p / r);
    return (r > 1 ? 1 : 0) + k / 4 + (k % 4 ? 1 : 0);
}
constexpr int radix_of(int p, int pass) {
    int r = odd_part(p);
    int k = log2_exact(p / r);
    if (r > 1) {
        if (pass == 0) return r;
        --pass;
    }
    if (pass < k / 4) return 16;
    return 1 << (k % 4);
}
constexpr int ns_before(int p, int pass) {
    int ns = 1;
    for (int i = 0; i < pass; ++i) ns *= radix_of(p, i);
    return ns;
}

// LDS layout: one padding element every 16.  The LDS has 64 banks of 4
// bytes and serves an 8-byte access 32 lanes at a time.  The radix-16 first
// pass has each lane write 16 consecutive elements (lane stride 16); with the
// padding that stride becomes 17 elements, odd, so 32 lanes of one column hit
// distinct banks.  Unit-stride accesses stay contiguous within each run of 16
// (32 lanes of them span 33 slots, so one slot is hit twice).
__device__ __forceinline__ int lidx(int j) { return j + (j >> 4); }
constexpr int lds_len(int p) { return p + p / 16 + 1; }

// Columns start at c LD, except in the skewed layout of 16 columns of 256
// 8-byte points (stride kLdSkew256 = 272, 16 mod 32 elements): column c starts at
// c 272 + 2 floor(c / 2), i.e. at element 2 sigma(c) modulo 32 with
// sigma(c) = floor(c / 2) + 8 (c mod 2) a permutation of 0..15.  Then the
// radix-16 first pass (columns 2h and 2h + 1 in one 32-lane half, 16 elements
// apart) and the column-fastest last pass (columns 0..15 at one position in
// 16 lanes, the next position in the other 16) both touch 32 distinct 8-byte
// slots per half-wave; with the plain stride 273 the first pass conflicts
// two-way.  The columns need 16 LD + 14 elements.
constexpr int kLdSkew256 = 272;
constexpr int cols_len(int ncol, int ld) { return ld == kLdSkew256 ? ncol * ld + 2 * ((ncol - 1) / 2) : ncol * ld; }

// the shift of column c beyond c LD (element c LD + lidx(j) + col_skew(c));
// added last, so that the code of every unskewed layout stays as it was
// (written as one function of the column start, the same addresses led the
// compiler to a different register allocation, with spills, in the local
// kernels)
template <int LD> __device__ __forceinline__ int col_skew(int c) {
    if constexpr (LD == kLdSkew256) return c & ~1;
    else return 0;
}

// One Stockham pass over NCOL columns held in LDS (column c starts at c*LD).
template <typename C, int P, int NCOL, int NT, int LD, int SIGN, int R, int NS>
__device__ __forceinline__ void stockham_pass(C *buf, const C *__restrict__ tw) {
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
            for (int r = 0; r < R; ++r) v[q][r] = buf[c * LD + lidx(i + r * (P / R))];
        }
    }
    lds_barrier();
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        int gb = tid + q * NT;
        if (NB % NT == 0 || gb < NB) {
            int c = gb / (P / R), i = gb % (P / R);
            int k = i % NS;
            if constexpr (NS > 1) {
#pragma unroll
                for (int r = 1; r < R; ++r) {
                    C w = tw[(r * k) * (P / (R * NS))];
                    v[q][r] = SIGN > 0 ? cmul(v[q][r], w) : cmulc(v[q][r], w);
                }
            }
            dftR<R, SIGN>(v[q]);
            int base = (i - k) * R + k;
#pragma unroll
            for (int r = 0; r < R; ++r) buf[c * LD + lidx(base + r * NS)] = v[q][r];
        }
    }
    lds_barrier();
}

template <typename C, int P, int NCOL, int NT, int LD, int SIGN, int PASS>
__device__ __forceinline__ void block_fft_from(C *buf, const C *__restrict__ tw) {
    if constexpr (PASS < num_passes(P)) {
        stockham_pass<C, P, NCOL, NT, LD, SIGN, radix_of(P, PASS), ns_before(P, PASS)>(buf, tw);
        block_fft_from<C, P, NCOL, NT, LD, SIGN, PASS + 1>(buf, tw);
    }
}

// In-place FFT of NCOL columns of length P in LDS.  Callers must
// lds_barrier() after filling buf; the function ends with a barrier.
template <typename C, int P, int NCOL, int NT, int LD, int SIGN>
__device__ __forceinline__ void block_fft(C *buf, const C *__restrict__ tw) {
    block_fft_from<C, P, NCOL, NT, LD, SIGN, 0>(buf, tw);
}

}  // namespace cwt
