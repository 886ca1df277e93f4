// cwt_spline_plan.cpp -- host side of the spline method (Sec. 3.3, App. B,
// App. C, Sec. 3.6 Eq. m02cwt_error).
//
// Per plan: h*, the largest knot step whose spline wavelet reaches the
// accuracy AE_M = 5e-4 (Eq. m02cwt_error, Table 3).  Per scale s, the step
// h_s of the wavelet spline psi_h (Eq. beta3_wavelet_approx_m02, its
// coefficients d_s computed as Eq. interp_coeffs on the samples psi(h_s k),
// N_d = ceil(chi / h_s - 2) + 2 on each side):
//   h* s >= 1: h_s = delta / s with the integer knot spacing
//              delta = floor(h* s) in samples (h_s in (h*/2, h*]); the tap
//              sum runs on the exact box sums of the running sums;
//   h* s <  1: h_s = h*, the paper's fixed step, whose knots s h* k fall
//              between samples.  W[x] = sum_t c[x + t] Omega_s(t) with the
//              exact taps Omega_s(t) = (1/s) int beta3(v - t)
//              conj(psi_h(v / s)) dv on the spline coefficients c (Eq.
//              beta3_signal), evaluated here by Gauss-Legendre quadrature
//              over the merged knots; |t| <= (N_d + 2) s h* + 2.
// Either way h_s <= h*, so AE_M <= 5e-4 at every scale.  Also the tiling of
// the tap-sum launch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "cwt_host.h"
#include "cwt_internal.h"

namespace cwt {

using cd = std::complex<double>;

// cubic B-spline (App. B, Eq. betan with n = 3)
static double bspline3(double x) {
    x = std::fabs(x);
    if (x < 1.0) return 2.0 / 3.0 - x * x + 0.5 * x * x * x;
    if (x < 2.0) return (2.0 - x) * (2.0 - x) * (2.0 - x) / 6.0;
    return 0.0;
}

// Support radius used by the spline method: one grid step past the last point
// of the grid i / 4096 (0 <= i <= 64 * 4096) where |psi| >= rel * max|psi|.
static double spline_chi(const Wavelet &w, double rel) {
    const double step = 1.0 / 4096.0;
    const int n = 64 * 4096;
    double mx = 0.0;
    for (int i = 0; i <= n; ++i) mx = std::max(mx, std::abs(w.psi_time(i * step)));
    double last = 0.0;
    for (int i = 0; i <= n; ++i)
        if (std::abs(w.psi_time(i * step)) >= rel * mx) last = i * step;
    return last + step;
}

// Cubic-spline interpolation coefficients of v (zero outside the array), in
// place: the causal and anticausal first-order recursions of App. C with the
// pole z1 = sqrt(3) - 2 and gain d0 = 6.  The anticausal start value is the
// exact sum of the zero-extended causal output.
static void interp_coeffs(std::vector<cd> &v) {
    const double z = std::sqrt(3.0) - 2.0;
    const size_t n = v.size();
    for (size_t k = 1; k < n; ++k) v[k] += z * v[k - 1];
    v[n - 1] = (-z / (1.0 - z * z)) * v[n - 1];
    for (size_t k = n - 1; k-- > 0;) v[k] = z * (v[k + 1] - v[k]);
    for (auto &x : v) x *= 6.0;
}

// coefficients of psi(h k), k in [-K, K], stored at k + K
static std::vector<cd> wavelet_coeffs(const Wavelet &w, double h, int K) {
    std::vector<cd> v(2 * (size_t)K + 1);
    for (int k = -K; k <= K; ++k) v[(size_t)(k + K)] = w.psi_time(h * k);
    interp_coeffs(v);
    return v;
}

// psi_h(x) = sum_k d[k] beta3(x/h - k)
static cd spline_eval(const std::vector<cd> &d, int K, double h, double x) {
    const double y = x / h;
    const long k0 = (long)std::floor(y) - 1;
    cd acc = 0.0;
    for (long k = k0; k <= k0 + 3; ++k)
        if (k >= -K && k <= K) acc += d[(size_t)(k + K)] * bspline3(y - (double)k);
    return acc;
}

// AE_M(h) of Eq. m02cwt_error on 20001 uniform points of [-chi, chi]; the
// spline uses the untruncated coefficients (40 beyond chi / h on each side)
static double ae_m(const Wavelet &w, double chi, double h) {
    const int K = (int)std::ceil(chi / h) + 40;
    const std::vector<cd> d = wavelet_coeffs(w, h, K);
    const int npts = 20001;
    const double dx = 2.0 * chi / (npts - 1);
    double num = 0.0, den = 0.0;
    for (int i = 0; i < npts; ++i) {
        const double x = i == npts - 1 ? chi : -chi + i * dx;
        const cd ex = w.psi_time(x);
        num += std::abs(ex - spline_eval(d, K, h, x));
        den += std::abs(ex);
    }
    return num / den;
}

// h*: scan h upward in steps of 0.005 until AE_M reaches 5e-4, then bisect the
// bracketing interval (60 halvings)
static double h_star(const Wavelet &w, double chi) {
    const double target = 5e-4;
    double lo = 0.005, h = lo;
    while (ae_m(w, chi, h) < target) {
        lo = h;
        h += 0.005;
        if (h > 3.0) fail(CWT_EUNSUPPORTED, "spline method: AE_M never reaches 5e-4 for this wavelet");
    }
    double hi = h;
    for (int it = 0; it < 60; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (ae_m(w, chi, mid) < target) lo = mid;
        else hi = mid;
    }
    return 0.5 * (lo + hi);
}

static double cached_h_star(const Wavelet &w, double chi) {
    static std::mutex mu;
    static std::map<std::tuple<int, double, int>, double> cache;
    const auto key = std::make_tuple(w.kind, w.kind == CWT_MORLET ? w.w0 : 0.0, w.kind == CWT_MORLET ? 0 : w.m);
    {
        std::lock_guard<std::mutex> g(mu);
        auto it = cache.find(key);
        if (it != cache.end()) return it->second;
    }
    const double h = h_star(w, chi);
    std::lock_guard<std::mutex> g(mu);
    cache[key] = h;
    return h;
}

// Omega_s(t) = (1/s) int beta3(v - t) conj(psi_h(v / s)) dv for |t| <= Tt:
// both factors are cubic between consecutive points of the merged knot set
// (the integers and s h k), so 4-point Gauss-Legendre on each piece is exact.
static std::vector<cd> exact_taps(const std::vector<cd> &d, int K, int nd, double h, double s, int Tt) {
    static const double gx[4] = {-0.86113631159405257522, -0.33998104358485626480, 0.33998104358485626480,
                                 0.86113631159405257522};
    static const double gw[4] = {0.34785484513745385737, 0.65214515486254614263, 0.65214515486254614263,
                                 0.34785484513745385737};
    // the spline with its coefficients truncated to |k| <= nd
    std::vector<cd> dt(d.size(), cd(0.0));
    for (int k = -nd; k <= nd; ++k) dt[(size_t)(k + K)] = d[(size_t)(k + K)];
    const double step = s * h;
    std::vector<cd> om(2 * (size_t)Tt + 1);
    for (int t = -Tt; t <= Tt; ++t) {
        const double lo = t - 2.0, hi = t + 2.0;
        std::vector<double> cut;
        for (int i = t - 2; i <= t + 2; ++i) cut.push_back((double)i);
        for (long k = (long)std::ceil(lo / step); (double)k * step < hi; ++k)
            if ((double)k * step > lo) cut.push_back((double)k * step);
        std::sort(cut.begin(), cut.end());
        cd acc = 0.0;
        for (size_t i = 0; i + 1 < cut.size(); ++i) {
            const double a = cut[i], b = cut[i + 1];
            if (!(b > a)) continue;
            const double mid = 0.5 * (a + b), hw = 0.5 * (b - a);
            for (int q = 0; q < 4; ++q) {
                const double v = mid + hw * gx[q];
                acc += hw * gw[q] * bspline3(v - (double)t) * std::conj(spline_eval(dt, K, h, v / s));
            }
        }
        om[(size_t)(t + Tt)] = acc / s;
    }
    return om;
}

// B-spline coefficients a[k], k in [-K, K] (at k + K), of the A19 wavelet at
// step h (Sec. 3.4): the C^2 piecewise cubic on the knots h k whose second
// derivative interpolates e[k] = psi''(h k), |k| <= J = ceil(chi / h) (zero
// beyond), linearly between the knots (its third derivative on a piece is
// then the difference quotient of Eq. 3rd_derivative_wavelet), and that
// vanishes to the left of -(J + 1) h.  With psi(y) = sum_k a[k] beta3(y/h - k),
// psi''(h m) = (a[m+1] - 2 a[m] + a[m-1]) / h^2, so a is h^2 times the
// double running sum of e: a[k] = h^2 sum_{m < k} (k - m) e[m].
// The two running sums are compensated (Neumaier): psi'' is larger than psi
// by about w0^2 and the sums run over hundreds of knots, so plain sums would
// leave about 1e-12 of psi's scale in a.
struct CompSum {
    double s = 0.0, c = 0.0;
    void add(double x) {
        const double t = s + x;
        c += std::fabs(s) >= std::fabs(x) ? (s - t) + x : (x - t) + s;
        s = t;
    }
    double value() const { return s + c; }
};
static std::vector<cd> a19_coeffs(const Wavelet &w, double h, int K, double chi) {
    const int J = (int)std::ceil(chi / h - 1e-9);
    std::vector<cd> a(2 * (size_t)K + 1, cd(0.0));
    CompSum s1r, s1i, s2r, s2i;  // running sums of e and of the first sum
    for (int k = -K; k <= K; ++k) {
        a[(size_t)(k + K)] = h * h * cd(s2r.value(), s2i.value());
        const cd e = (k >= -J && k <= J) ? w.psi2_time(h * k) : cd(0.0);
        s1r.add(e.real());
        s1i.add(e.imag());
        s2r.add(s1r.s);
        s2r.add(s1r.c);
        s2i.add(s1i.s);
        s2i.add(s1i.c);
    }
    return a;
}

// Work items of the tap-sum launch for scale j (knot spacing delta, ntap
// taps): tiles of R <= 32 columns (consecutive positions) x I = 16 floor(256 /
// R) rows (positions delta apart); the S tile holds R (I + ntap) values plus
// one spare row per 16, and the taps follow it in LDS.  Wide tiles measured
// best although they repeat more halo rows per output: R = 32 against 16
// took the tap kernel 0.36 against 0.39 ms (Mexican hat, 53 taps, N = 2^20,
// 64 scales); R = 8 and 4 were slower (0.45, 0.64 ms).  Each row's R outputs
// are one store run, and each thread's H loads are R-lane runs.  (Morlet's
// 155-tap tiles do not fit 32 columns and stay at 16.)
static void add_tiles(Plan &p, int j, SplineScaleDev &sc, int64_t delta, int ntap) {
    auto tile_fits = [&](int r) {
        const int rows_s = 16 * (256 / r) + ntap;
        return r * (rows_s + rows_s / 16 + 1) + 2 * ntap <= 8192;  // 64 KiB of LDS
    };
    int rmax = 32;
    while (rmax > 1 && !tile_fits(rmax)) rmax /= 2;
    if (!tile_fits(rmax)) fail(CWT_EUNSUPPORTED, "spline method: wavelet support too long for the tap tile");
    const int64_t nck = (delta + rmax - 1) / rmax;
    const int R = (int)((delta + nck - 1) / nck);
    sc.R = R;
    sc.I = 16 * (256 / R);
    {
        const int64_t rows_s = sc.I + ntap;
        const int64_t lds = 8 * (int64_t)R * (rows_s + rows_s / 16 + 1) + 16 * (int64_t)ntap;
        p.spl_lds_bytes = std::max(p.spl_lds_bytes, lds);
    }
    const int64_t rows = (p.N + delta - 1) / delta;
    for (int64_t i0 = 0; i0 < rows; i0 += sc.I)
        for (int64_t k = 0; k < nck; ++k) {
            const int64_t r0 = k * R;
            if (r0 >= delta) break;
            SplineWork wk;
            wk.j = j;
            wk.r0 = (int32_t)r0;
            wk.R = (int32_t)std::min<int64_t>(R, delta - r0);
            wk.pad = 0;
            wk.i0 = i0;
            p.spl_work.push_back(wk);
        }
}

static const int kSplineBlock = 2048;  // elements per block of the running sums and the max|f| reduction (= kSB of the kernels)

void build_spline_plan(Plan &p, const Wavelet &w, TableBuilder &) {
    const double chi14 = spline_chi(w, 1e-14);  // truncation used for h* (Table 2 keeps |psi| near 1e-14)
    const double chi17 = spline_chi(w, 1e-17);  // truncation of d_s
    const bool a19 = p.method == CWT_METHOD_A19;
    p.hstar = cached_h_star(w, chi14);
    if (a19) {
        // N_chi: the fewest pieces on [-chi, chi] whose interpolating cubic
        // spline meets AE_A = 5e-4, i.e. knot step chi / N_chi <= h*
        const double nchi = std::ceil(chi14 / p.hstar - 1e-12);
        p.hstar = chi14 / nchi;
    }
    p.path.assign(p.S, PATH_SPLINE);
    p.spl.resize(p.S);
    p.spl_delta.resize(p.S);
    p.spl_work.clear();
    p.spl_lds_bytes = 0;

    std::vector<cd> dtab;
    int64_t delta_max = 1, E = 16;
    p.spl_ntaps.assign(p.S, 0);
    p.spl_direct = false;
    for (int j = 0; j < p.S; ++j) {
        const double s = p.scales[j];
        const double fl = std::floor(p.hstar * s);
        if (fl > 1e9) fail(CWT_EUNSUPPORTED, "spline method: scale too large");
        const bool direct = fl < 1.0;  // knots between samples: exact taps on c
        const int64_t delta = direct ? 1 : (int64_t)fl;
        const double h = direct ? p.hstar : (double)delta / s;
        const int nd = (int)std::ceil(chi17 / h - 2.0) + 2;
        if (nd > 1800) fail(CWT_EUNSUPPORTED, "spline method: more than 3601 wavelet coefficients at this scale");
        const int K = std::max(nd, (int)std::ceil(chi17 / h)) + 40;
        const std::vector<cd> dk = a19 ? a19_coeffs(w, h, K, chi14) : wavelet_coeffs(w, h, K);
        SplineScaleDev &sc = p.spl[j];
        sc.d_off = (int64_t)dtab.size();
        int ntap;
        if (direct) {
            // W[x] = sum_{|t| <= Tt} Omega_s(t) c[x + t], run as a tap sum of
            // spacing 1 over c itself (tap n <-> t = n - Tt)
            const int Tt = (int)std::ceil((double)(nd + 2) * h * s) + 2;
            const std::vector<cd> om = exact_taps(dk, K, nd, h, s, Tt);
            ntap = (2 * Tt + 1 + 7) / 8 * 8;
            sc.delta = 1;
            sc.nd = Tt;
            sc.mode = 1;
            for (int n = 0; n < ntap; ++n) dtab.push_back(n <= 2 * Tt ? om[(size_t)n] : cd(0.0));
            p.spl_ntaps[j] = 2 * Tt + 1;
            p.spl_direct = true;
            E = std::max<int64_t>(E, (int64_t)Tt + 16);
        } else {
            ntap = (2 * nd + 1 + 7) / 8 * 8;
            sc.delta = (int32_t)delta;
            sc.nd = nd;
            sc.mode = 0;
            const double kscale = 1.0 / (5040.0 * s * (double)delta * (double)delta * (double)delta);
            for (int n = 0; n < ntap; ++n)
                dtab.push_back(n <= 2 * nd ? std::conj(dk[(size_t)(K - nd + n)]) * kscale : cd(0.0));
            p.spl_ntaps[j] = 2 * nd + 1;
        }
        sc.ntap = ntap;
        add_tiles(p, j, sc, delta, ntap);
        if (direct) {
            p.spl_delta[j] = 0;
            p.path[j] = PATH_SPLINE_DIRECT;
            continue;
        }
        p.spl_delta[j] = (int32_t)delta;
        delta_max = std::max(delta_max, delta);
        E = std::max<int64_t>(E, (int64_t)(nd + 3) * delta + 16);
    }
    // most expensive tiles first
    std::stable_sort(p.spl_work.begin(), p.spl_work.end(), [&](const SplineWork &a, const SplineWork &b) {
        return p.spl[a.j].ntap > p.spl[b.j].ntap;
    });
    if (p.N + 2 * E > (int64_t(1) << 31)) fail(CWT_EUNSUPPORTED, "spline method: signal plus wavelet support above 2^31");
    p.spl_E = E;
    p.spl_len = p.N + 2 * E;
    // the tap kernel addresses the running sums with 32-bit byte offsets
    if (p.spl_len * 16 >= (int64_t(1) << 31))
        fail(CWT_EUNSUPPORTED, "spline method: signal plus wavelet support above 2^27 samples");
    // fixed-point bits: |5040 beta7 * box^4 q| <= 5040 delta^4 max|q| must stay below 2^127
    const int qb = (int)std::floor(127.0 - std::log2(5040.0) - 4.0 * std::log2((double)delta_max)) - 1;
    p.spl_qbits = std::min(62, qb);
    if (p.spl_qbits < 40) fail(CWT_EUNSUPPORTED, "spline method: knot spacing too large for 128-bit running sums");
    p.spl_nb0 = (int32_t)((p.N + kSplineBlock - 1) / kSplineBlock);
    p.spl_nblk = (int32_t)((p.spl_len + kSplineBlock - 1) / kSplineBlock);

    size_t ws = 0;
    auto take = [&](size_t bytes) {
        size_t off = (ws + 255) & ~size_t(255);
        ws = off + bytes;
        return off;
    };
    p.ws_maxp_off = take((size_t)p.spl_nb0 * sizeof(double));
    p.ws_fx_off = take(16);
    p.ws_state_off = take((size_t)p.spl_nblk * 64);
    p.ws_carry_off = take((size_t)p.spl_nblk * 64);
    p.ws_H_off = take((size_t)p.spl_len * 16);
    p.ws_C_off = p.spl_direct ? take((size_t)p.spl_len * 8) : 0;
    p.ws_bytes = ws;
    if (p.host_only) return;

    auto upload = [&](const void *src, size_t bytes, void **dst) {
        HIPCHK(hipMalloc(dst, bytes));
        p.table_bytes += bytes;
        HIPCHK(hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice));
    };
    upload(dtab.data(), dtab.size() * sizeof(cd), &p.d_dtab);
    upload(p.spl.data(), p.spl.size() * sizeof(SplineScaleDev), reinterpret_cast<void **>(&p.d_spl));
    p.d_extra.push_back(p.d_spl);
    upload(p.spl_work.data(), p.spl_work.size() * sizeof(SplineWork), reinterpret_cast<void **>(&p.d_spl_work));
    p.d_extra.push_back(p.d_spl_work);
}

}  // namespace cwt

namespace cwt {

// Gauss-Legendre nodes and weights on [-1, 1] (Newton on the Legendre
// recurrence from the Chebyshev guesses).
static void gauss_legendre(int n, std::vector<double> &x, std::vector<double> &w) {
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    for (int i = 0; i < n; ++i) {
        double z = std::cos(M_PI * (i + 0.75) / (n + 0.5)), dp = 0.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
            const double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        x[i] = z;
        w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

// c_w = 1 / argmax_u |u| |psi^(u)|^2 (Table 2): a 1/256 scan of [-64, 64],
// then golden-section refinement of the best bracket
static double wavelet_cw(const Wavelet &w) {
    auto g = [&](double u) { return std::fabs(u) * w.amp(u) * w.amp(u); };
    const double step = 1.0 / 256.0;
    double best = 0.0, ub = 1.0;
    for (double u = -64.0; u <= 64.0; u += step)
        if (g(u) > best) {
            best = g(u);
            ub = u;
        }
    double a = ub - step, b = ub + step;
    const double gr = 0.5 * (std::sqrt(5.0) - 1.0);
    double c = b - gr * (b - a), d = a + gr * (b - a);
    for (int it = 0; it < 200 && b - a > 1e-15 * std::fabs(ub); ++it) {
        if (g(c) > g(d)) b = d;
        else a = c;
        c = b - gr * (b - a);
        d = a + gr * (b - a);
    }
    return 1.0 / std::fabs(0.5 * (a + b));
}

// q12: the inverse filter of the sampled quartic B-spline (1, 76, 230, 76, 1)
// / 384 (Eq. q_12), taps |k| <= K, by the trapezoid rule on the unit circle
// (its images lie 4096 taps apart, where the taps are below 1e-1800)
static std::vector<double> q12_taps(int K) {
    const int M = 4096;
    std::vector<double> q(2 * (size_t)K + 1, 0.0);
    for (int k = -K; k <= K; ++k) {
        double acc = 0.0;
        for (int m = 0; m < M; ++m) {
            const double om = 2.0 * M_PI * m / M;
            const double b4 = (230.0 + 152.0 * std::cos(om) + 2.0 * std::cos(2.0 * om)) / 384.0;
            acc += std::cos(om * k) / b4;
        }
        q[(size_t)(k + K)] = acc / M;
    }
    return q;
}

// V97 method (Sec. 3.2).  Scale s = 2^i r / w~_max, 1 <= r < 2: taps
// conj(q_r(k)) / s at spacing 2^i on F_i = f * beta3 * h * [h]2 * ... *
// [h]2^(i-1) * [q12]2^i, q_r(k) = int_{k-1/2}^{k+1/2} psi(w~_max y / r) dy.
void build_v97_plan(Plan &p, const Wavelet &w) {
    const double chi17 = spline_chi(w, 1e-17);
    p.v97_wmax = 1.34 * wavelet_cw(w);  // Table 3: w~_max = 1.34 c_w
    p.hstar = p.v97_wmax;
    p.path.assign(p.S, PATH_SPLINE_DIRECT);
    p.spl.resize(p.S);
    p.spl_delta.resize(p.S);
    p.spl_ntaps.assign(p.S, 0);
    p.spl_work.clear();
    p.spl_lds_bytes = 0;
    p.spl_direct = true;
    p.v97_nq12 = 40;  // (2 - sqrt 3)-like decay: |q12[k]| < 0.362^k, below 1e-17 past 40
    std::vector<double> gx, gw;
    gauss_legendre(16, gx, gw);
    std::vector<double> g4x, g4w;
    gauss_legendre(4, g4x, g4w);
    std::vector<cd> dtab;
    std::map<int, std::vector<int>> level_scales;
    std::map<int, int64_t> level_ef;
    for (int j = 0; j < p.S; ++j) {
        const double s = p.scales[j];
        const double t = s * p.v97_wmax;
        if (!(t >= 1.0 - 1e-6))
            fail(CWT_EUNSUPPORTED, "V97 method: scales below 1 / w~_max = " + std::to_string(1.0 / p.v97_wmax) +
                                       " samples are not supported");
        int i = std::max(0, (int)std::floor(std::log2(std::max(t, 1.0))));
        while (i > 0 && std::ldexp(1.0, i) > t) --i;
        while (std::ldexp(1.0, i + 1) <= t) ++i;
        if (i > 30) fail(CWT_EUNSUPPORTED, "V97 method: scale too large");
        const double r = t / std::ldexp(1.0, i);
        const int64_t delta = int64_t(1) << i;
        const int nq = (int)std::ceil(chi17 * r / p.v97_wmax + 0.5);
        // cell integrals of psi(w~_max y / r); the cubic B-spline wavelet is
        // cut at its knots y = r m / w~_max so that each piece is a cubic
        std::vector<cd> q(2 * (size_t)nq + 1);
        for (int k = -nq; k <= nq; ++k) {
            std::vector<double> cut = {k - 0.5, k + 0.5};
            if (w.kind == CWT_CBSW)
                for (int m = -3; m <= 3; ++m) {
                    const double y = r * m / p.v97_wmax;
                    if (y > k - 0.5 && y < k + 0.5) cut.push_back(y);
                }
            std::sort(cut.begin(), cut.end());
            const std::vector<double> &nx = w.kind == CWT_CBSW ? g4x : gx;
            const std::vector<double> &nw = w.kind == CWT_CBSW ? g4w : gw;
            cd acc = 0.0;
            for (size_t c = 0; c + 1 < cut.size(); ++c) {
                const double mid = 0.5 * (cut[c] + cut[c + 1]), hw = 0.5 * (cut[c + 1] - cut[c]);
                for (size_t g = 0; g < nx.size(); ++g)
                    acc += hw * nw[g] * w.psi_time(p.v97_wmax * (mid + hw * nx[g]) / r);
            }
            q[(size_t)(k + nq)] = acc;
        }
        SplineScaleDev &sc = p.spl[j];
        const int ntap = (2 * nq + 1 + 7) / 8 * 8;
        sc.delta = (int32_t)delta;
        sc.nd = nq;
        sc.ntap = ntap;
        sc.mode = 1;
        sc.d_off = (int64_t)dtab.size();
        for (int n = 0; n < ntap; ++n) dtab.push_back(n <= 2 * nq ? std::conj(q[(size_t)n]) / s : cd(0.0));
        p.spl_ntaps[j] = 2 * nq + 1;
        p.spl_delta[j] = (int32_t)delta;
        level_scales[i].push_back(j);
        level_ef[i] = std::max<int64_t>(level_ef[i], (int64_t)(nq + 2) * delta + 16);
    }
    // arrays: F on [-EF, N + EF) inside [-E, N + E); f buffers on [-E, N + E)
    // (zero boundary: f_i vanishes beyond 2^(i+1) + 1 samples of the signal)
    // or [0, N) with wrapped reads (periodic)
    int64_t E = 16;
    for (auto &kv : level_ef)
        E = std::max<int64_t>(E, kv.second + (int64_t)(p.v97_nq12 + 2) * (int64_t(1) << kv.first) + 16);
    if (p.N + 2 * E > (int64_t(1) << 31)) fail(CWT_EUNSUPPORTED, "V97 method: signal plus filter support above 2^31");
    p.spl_E = E;
    p.spl_len = p.N + 2 * E;
    p.v97_flen = p.boundary == CWT_PERIODIC ? p.N : p.spl_len;
    // launch sequence: f_0, then per level: advance f, F_i, tap sums
    p.v97_steps.clear();
    p.v97_steps.push_back({0, 0, -1, 0, 0, 0});
    int cur = 0, buf = 0;
    for (auto &kv : level_scales) {
        const int i = kv.first;
        while (cur < i) {
            p.v97_steps.push_back({1, cur, buf, 1 - buf, 0, 0});
            buf = 1 - buf;
            ++cur;
        }
        p.v97_steps.push_back({2, i, buf, -1, 0, 0});
        const int32_t w0 = (int32_t)p.spl_work.size();
        for (int j : kv.second) add_tiles(p, j, p.spl[j], p.spl[j].delta, p.spl[j].ntap);
        p.v97_steps.push_back({3, i, -1, -1, w0, (int32_t)p.spl_work.size()});
    }
    size_t ws = 0;
    auto take = [&](size_t bytes) {
        size_t off = (ws + 255) & ~size_t(255);
        ws = off + bytes;
        return off;
    };
    p.ws_fx_off = take(16);
    p.ws_fa_off = take((size_t)p.v97_flen * 8);
    p.ws_fb_off = take((size_t)p.v97_flen * 8);
    p.ws_C_off = take((size_t)p.spl_len * 8);
    p.ws_bytes = ws;
    if (p.host_only) return;
    auto upload = [&](const void *src, size_t bytes, void **dst) {
        HIPCHK(hipMalloc(dst, bytes));
        p.table_bytes += bytes;
        HIPCHK(hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice));
    };
    const std::vector<double> q12 = q12_taps(p.v97_nq12);
    upload(q12.data(), q12.size() * sizeof(double), reinterpret_cast<void **>(&p.d_v97_q12));
    p.d_extra.push_back(p.d_v97_q12);
    upload(dtab.data(), dtab.size() * sizeof(cd), &p.d_dtab);
    upload(p.spl.data(), p.spl.size() * sizeof(SplineScaleDev), reinterpret_cast<void **>(&p.d_spl));
    p.d_extra.push_back(p.d_spl);
    upload(p.spl_work.data(), p.spl_work.size() * sizeof(SplineWork), reinterpret_cast<void **>(&p.d_spl_work));
    p.d_extra.push_back(p.d_spl_work);
}

}  // namespace cwt
