// cwt_plan.cpp -- plan construction and the C ABI (include/cwt.h).
//
// Host math is FP64 throughout: wavelet spectra, truncation radii, band
// edges, twiddle tables and the spline parameters are computed here once per
// plan and uploaded as small device tables.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <limits>
#include <map>
#include <tuple>
#include <mutex>
#include <cstring>
#include <new>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/cwt.h"
#include "cwt_internal.h"
#include "cwt_host.h"

namespace cwt {

static thread_local std::string g_err;

// radius beyond which |psi| < rel * max|psi|
static double time_radius_scan(const Wavelet &w, double rel);
static double time_radius(const Wavelet &w, double rel) {
    static std::mutex mu;
    static std::map<std::tuple<int, double, int, double>, double> cache;
    const auto key = std::make_tuple(w.kind, w.w0, w.m, rel);
    std::lock_guard<std::mutex> g(mu);
    auto it = cache.find(key);
    if (it != cache.end()) return it->second;
    return cache[key] = time_radius_scan(w, rel);
}
static double time_radius_scan(const Wavelet &w, double rel) {
    const double step = 1.0 / 1024.0;
    double mx = 0.0;
    for (int i = 0; i <= 64 * 1024; ++i) mx = std::max(mx, w.abs_time(i * step));
    double last = 0.0;
    for (int i = 0; i <= 64 * 1024; ++i)
        if (w.abs_time(i * step) >= rel * mx) last = i * step;
    return last + step;
}

// [ulo, uhi] outside of which |psi^(u)| < rel * max|psi^|
static void spectral_band_scan(const Wavelet &w, double rel, double &ulo, double &uhi);
static void spectral_band(const Wavelet &w, double rel, double &ulo, double &uhi) {
    static std::mutex mu;
    static std::map<std::tuple<int, double, int, double>, std::pair<double, double>> cache;
    const auto key = std::make_tuple(w.kind, w.w0, w.m, rel);
    std::lock_guard<std::mutex> g(mu);
    auto it = cache.find(key);
    if (it == cache.end()) {
        double a, b;
        spectral_band_scan(w, rel, a, b);
        it = cache.emplace(key, std::make_pair(a, b)).first;
    }
    ulo = it->second.first;
    uhi = it->second.second;
}
static void spectral_band_scan(const Wavelet &w, double rel, double &ulo, double &uhi) {
    const double step = 1.0 / 512.0, lim = 64.0;
    double mx = 0.0;
    for (double u = -lim; u <= lim; u += step) mx = std::max(mx, std::fabs(w.amp(u)));
    ulo = lim;
    uhi = -lim;
    for (double u = -lim; u <= lim; u += step)
        if (std::fabs(w.amp(u)) >= rel * mx) {
            ulo = std::min(ulo, u);
            uhi = std::max(uhi, u);
        }
    ulo -= 2 * step;
    uhi += 2 * step;
}

// Psi_s(omega) = sum_q amp(s (omega + 2 pi q)), q over the images that can reach the band
// Psi_s(omega) = sum_q psi^(s (omega + 2 pi q)) (amplitude part), summed over
// the images whose argument lies in the wavelet's band [ulo, uhi] (outside
// it |psi^| < rel max|psi^|, the plan's truncation level)
static double psi_aliased(const Wavelet &w, double s, double omega, double ulo, double uhi) {
    const double tp = 2.0 * M_PI;
    const long q0 = (long)std::ceil((ulo / s - omega) / tp), q1 = (long)std::floor((uhi / s - omega) / tp);
    double acc = 0.0;
    for (long q = q0; q <= q1; ++q) acc += w.amp(s * (omega + tp * (double)q));
    return acc;
}

// ---------------------------------------------------------------------------
// FFT length helpers

static int64_t pow2_part(int64_t m) { return m & (-m); }

static bool smooth_form(int64_t m, int &r, int64_t &p2) {
    p2 = pow2_part(m);
    int64_t o = m / p2;
    if (o == 1 || o == 3 || o == 5 || o == 9) {
        r = (int)o;
        return true;
    }
    return false;
}

// M = M1 * M2 with M2 a power of two in [64, 4096] and M1 a supported size,
// or M itself a supported size (single pass).
static bool factor_fft(int64_t M, int32_t &M1, int32_t &M2) {
    if (M <= 4608 && fwd_size_ok((int)M)) {
        M1 = (int32_t)M;
        M2 = 1;
        return true;
    }
    int best = -1;
    for (int64_t m2 = 4096; m2 >= 64; m2 /= 2) {
        if (M % m2) continue;
        int64_t m1 = M / m2;
        if (m1 > 4608 || !fwd_size_ok((int)m1)) continue;
        // prefer balanced factors
        int64_t score = std::llabs((int64_t)std::log2((double)m1) - (int64_t)std::log2((double)m2));
        if (best < 0 || score < best) {
            best = (int)score;
            M1 = (int32_t)m1;
            M2 = (int32_t)m2;
        }
    }
    return best >= 0;
}

static int64_t smallest_fft_len(int64_t need) {
    int64_t best = -1;
    for (int r : {1, 3, 5, 9}) {
        int64_t p2 = 64;
        while (r * p2 < need) p2 *= 2;
        int64_t m = r * p2;
        int32_t a, b;
        if (!factor_fft(m, a, b)) continue;
        if (best < 0 || m < best) best = m;
    }
    return best;
}

static int64_t next_pow2(int64_t x) {
    int64_t p = 1;
    while (p < x) p *= 2;
    return p;
}

template <typename R>
static void push_twiddles(TableBuilder &tb, int64_t P, std::vector<std::pair<int32_t, int64_t>> &offs) {
    for (auto &e : offs)
        if (e.first == P) return;
    std::vector<R> v(2 * P);
    for (int64_t j = 0; j < P; ++j) {
        // e^{+2 pi i j / P}, argument reduced in long double
        long double a = 2.0L * M_PIl * (long double)j / (long double)P;
        v[2 * j] = (R)std::cos(a);
        v[2 * j + 1] = (R)std::sin(a);
    }
    offs.push_back({(int32_t)P, tb.add(v.data(), v.size() * sizeof(R))});
}

template <typename R>
static void push_twM(TableBuilder &tb, int64_t M, int64_t &hi_off, int64_t &lo_off) {
    int64_t nh = (M + 4095) / 4096;
    std::vector<R> hi(2 * nh), lo(2 * 4096);
    for (int64_t j = 0; j < nh; ++j) {
        long double a = 2.0L * M_PIl * (long double)(j * 4096) / (long double)M;
        hi[2 * j] = (R)std::cos(a);
        hi[2 * j + 1] = (R)std::sin(a);
    }
    for (int64_t j = 0; j < 4096; ++j) {
        long double a = 2.0L * M_PIl * (long double)j / (long double)M;
        lo[2 * j] = (R)std::cos(a);
        lo[2 * j + 1] = (R)std::sin(a);
    }
    hi_off = tb.add(hi.data(), hi.size() * sizeof(R));
    lo_off = tb.add(lo.data(), lo.size() * sizeof(R));
}

// ---------------------------------------------------------------------------
// plan construction


// per-pass twiddle table of a P-point transform (layout of fft_cols.h):
// pass j with radix R_j and sub-size Ns_j > 1 stores e^{+2 pi i r k/(R_j Ns_j)}
// at (r - 1) Ns_j + k
static int host_odd_part(int p) { return (p % 9 == 0) ? 9 : (p % 5 == 0) ? 5 : (p % 3 == 0) ? 3 : 1; }
static std::vector<int> host_radices(int p) {
    std::vector<int> r;
    int o = host_odd_part(p);
    int k = 0;
    while ((o << k) < p) ++k;
    if (o > 1) r.push_back(o);
    for (int i = 0; i < k / 4; ++i) r.push_back(16);
    if (k % 4) r.push_back(1 << (k % 4));
    return r;
}
// Twiddle tables depend only on their size; each is computed once (long
// double arguments) and copied into every plan that needs it.
template <typename R>
static const std::vector<R> &pass_twiddles(int P) {
    static std::mutex mu;
    static std::map<int, std::vector<R>> cache;
    std::lock_guard<std::mutex> g(mu);
    auto it = cache.find(P);
    if (it != cache.end()) return it->second;
    std::vector<R> v;
    int ns = 1;
    for (int rad : host_radices(P)) {
        if (ns > 1)
            for (int r = 1; r < rad; ++r)
                for (int k = 0; k < ns; ++k) {
                    long double a = 2.0L * M_PIl * (long double)(r * k) / (long double)(rad * ns);
                    v.push_back((R)std::cos(a));
                    v.push_back((R)std::sin(a));
                }
        ns *= rad;
    }
    if (v.empty()) v.assign(2, (R)0);
    return cache.emplace(P, std::move(v)).first->second;
}
template <typename R>
static int64_t push_pass_twiddles(TableBuilder &tb, int P) {
    const std::vector<R> &v = pass_twiddles<R>(P);
    return tb.add(v.data(), v.size() * sizeof(R));
}
// w_{2^23}^x = hi[x >> 11] * lo[x & 2047] (FP64)
static const std::pair<std::vector<double>, std::vector<double>> &w23_tables() {
    static const std::pair<std::vector<double>, std::vector<double>> t = [] {
        const int64_t L = int64_t(1) << 23;
        std::vector<double> hi(2 * 4096), lo(2 * 2048);
        for (int64_t j = 0; j < 4096; ++j) {
            long double a = 2.0L * M_PIl * (long double)(j * 2048) / (long double)L;
            hi[2 * j] = (double)std::cos(a);
            hi[2 * j + 1] = (double)std::sin(a);
        }
        for (int64_t j = 0; j < 2048; ++j) {
            long double a = 2.0L * M_PIl * (long double)j / (long double)L;
            lo[2 * j] = (double)std::cos(a);
            lo[2 * j + 1] = (double)std::sin(a);
        }
        return std::make_pair(std::move(hi), std::move(lo));
    }();
    return t;
}
// e^{+2 pi i x / L}, L = 2^lg <= 2^23, from the split tables (FP64, ~1 ulp)
static std::complex<double> w23_at(int64_t x, int lg) {
    const auto &t = w23_tables();
    const int64_t y = (x & ((int64_t(1) << lg) - 1)) << (23 - lg);
    const std::complex<double> a(t.first[2 * (y >> 11)], t.first[2 * (y >> 11) + 1]);
    const std::complex<double> b(t.second[2 * (y & 2047)], t.second[2 * (y & 2047) + 1]);
    return a * b;
}
// e^{+2 pi i x / L} for a segment length L = c 2^lg (FP64; the split tables
// when c = 1, else from long double)
static std::complex<double> wL_at(int64_t x, int64_t L, int c, int lg) {
    if (c == 1) return w23_at(x, lg);
    int64_t r = x % L;
    if (r < 0) r += L;
    const long double a = 2.0L * M_PIl * (long double)r / (long double)L;
    return {(double)std::cos(a), (double)std::sin(a)};
}
static void push_w23(TableBuilder &tb, int64_t &hi_off, int64_t &lo_off) {
    const auto &t = w23_tables();
    hi_off = tb.add(t.first.data(), t.first.size() * sizeof(double));
    lo_off = tb.add(t.second.data(), t.second.size() * sizeof(double));
}

static const int64_t kMaxN = int64_t(1) << 26;

void build_spline_plan(Plan &p, const Wavelet &w, TableBuilder &tb);  // cwt_spline_plan.cpp
void build_v97_plan(Plan &p, const Wavelet &w);                       // cwt_spline_plan.cpp

static void build_fft_plan(Plan &p, const Wavelet &w, int64_t fft_len_opt) {
    const bool fp64 = p.precision == CWT_FP64;
    // largest segment transform that keeps its spectrum in registers without spills
    const int lmax = 4096;  // FP64 segment forward in LDS
    const int pmax = fp64 ? 1024 : 2048;
    p.path.assign(p.S, PATH_LOCAL);
    // local if the halo fits a quarter of the largest segment transform (the
    // literal form of Eq. discrete_CWT_conv, psi_mode ANALYTIC, takes every
    // scale through the whole-signal spectrum)
    const bool analytic = p.psi_mode == CWT_PSI_ANALYTIC;
    int64_t tcol = 0;
    std::vector<int> col;
    for (int j = 0; j < p.S; ++j) {
        if (p.T[j] * 4 <= lmax && !analytic) {
            p.path[j] = PATH_LOCAL;
        } else {
            p.path[j] = PATH_COLUMN;
            col.push_back(j);
            tcol = std::max(tcol, p.T[j]);
        }
    }
    p.pair_real = !p.cplx_out;

    // spectrum tables are built as doubles, converted at upload
    std::vector<double> tab;

    // ---- local groups: L = smallest power of two >= 8 T (at least 256), or
    // lmax when the halo needs it
    {
        std::vector<std::pair<int, int>> lj;  // (L, scale)
        for (int j = 0; j < p.S; ++j) {
            if (p.path[j] != PATH_LOCAL) continue;
            int64_t L = std::max<int64_t>(256, next_pow2(8 * p.T[j] + 1));
            if (L > lmax) L = lmax;
            lj.push_back({(int)L, j});
        }
        std::sort(lj.begin(), lj.end());
        double ulo, uhi;
        spectral_band(w, p.rel, ulo, uhi);
        size_t i = 0;
        while (i < lj.size()) {
            LocalGroup g;
            g.L = lj[i].first;
            while (i < lj.size() && lj[i].first == g.L) {
                g.scales.push_back(lj[i].second);
                g.Tg = std::max(g.Tg, p.T[lj[i].second]);
                ++i;
            }
            g.V = g.L - 2 * g.Tg;
            if (g.V <= 0) fail(CWT_EUNSUPPORTED, "internal: segment too short for the halo");
            g.nseg = (p.N + g.V - 1) / g.V;
            g.tab_off = (int64_t)tab.size();
            for (int j : g.scales) {
                double s = p.scales[j];
                for (int m = 0; m < g.L; ++m) {
                    int ms = m < g.L / 2 ? m : m - g.L;
                    tab.push_back(psi_aliased(w, s, 2.0 * M_PI * ms / g.L, ulo, uhi) / g.L);
                }
            }
            p.groups.push_back(std::move(g));
        }
    }

    // ---- whole-signal FFT and band-limited columns
    if (!col.empty()) {
        int64_t need;
        if (p.boundary == CWT_PERIODIC) {
            int r;
            int64_t p2;
            int32_t a, b;
            if (smooth_form(p.N, r, p2) && p2 >= 64 && factor_fft(p.N, a, b)) {
                p.M = p.N;
                p.load_mode = LOAD_PERIODIC;
            } else if (analytic) {
                // the printed form takes the DFT of the period itself
                fail(CWT_EUNSUPPORTED, "psi_mode ANALYTIC with a periodic signal needs N of the form "
                                       "2^a * {1,3,5,9}, 2^a >= 64");
            } else {
                p.load_mode = LOAD_WRAP;
                p.Twrap = tcol;
            }
            need = p.N + 2 * tcol;
        } else {
            p.load_mode = LOAD_ZERO;
            need = p.N + tcol + 1;
        }
        if (p.M == 0) {
            if (fft_len_opt > 0) {
                int r;
                int64_t p2;
                int32_t a, b;
                if (fft_len_opt < need || !smooth_form(fft_len_opt, r, p2) || p2 < 64 || !factor_fft(fft_len_opt, a, b))
                    fail(CWT_EUNSUPPORTED, "fft_len too short or not of the form 2^a*{1,3,5,9} (2^a >= 64)");
                p.M = fft_len_opt;
            } else {
                p.M = smallest_fft_len(need);
            }
        }
        if (p.M <= 0 || !factor_fft(p.M, p.M1, p.M2))
            fail(CWT_EUNSUPPORTED, "signal plus wavelet support exceeds the largest supported FFT length");
        int r;
        int64_t p2;
        smooth_form(p.M, r, p2);

        double ulo = -1e300, uhi = 1e300;  // a spectrum without a band spans every bin
        if (w.band_limited()) spectral_band(w, p.rel, ulo, uhi);
        // spectrum sample at signed bin m: aliased (the sampled wavelet), or
        // analytic (psi^(s w) at |w| <= pi only, Eq. discrete_CWT_conv; the
        // Nyquist bin of an even length, where the paper leaves the sign of
        // w open, takes the mean of psi^(s pi) and psi^(-s pi))
        auto spec = [&](double s, int64_t m) {
            int64_t ms = m % p.M;
            if (ms < 0) ms += p.M;
            if (ms >= (p.M + 1) / 2) ms -= p.M;  // signed bin in [-M/2, M/2)
            const double om = 2.0 * M_PI * (double)ms / (double)p.M;
            if (!analytic) return psi_aliased(w, s, om, ulo, uhi) / (double)p.M;
            if (2 * ms == -p.M) return 0.5 * (w.amp(-s * M_PI) + w.amp(s * M_PI)) / (double)p.M;
            return w.amp(s * om) / (double)p.M;
        };
        struct Band {
            int j;
            int64_t mlo, B;
        };
        std::vector<Band> bands;
        for (int j : col) {
            double s = p.scales[j];
            int64_t mlo = -p.M / 2, B = p.M;
            if (w.band_limited()) {
                mlo = (int64_t)std::floor(p.M * ulo / (2.0 * M_PI * s)) - 1;
                const int64_t mhi = (int64_t)std::ceil(p.M * uhi / (2.0 * M_PI * s)) + 1;
                B = mhi - mlo + 1;
            }
            if (B >= p.M) {
                mlo = -p.M / 2;
                B = p.M;
            }
            bands.push_back({j, mlo, B});
        }
        // pair real-wavelet scales (neighbours in band width share one complex transform)
        std::vector<std::pair<int, int>> units;  // indices into bands
        if (p.pair_real) {
            std::vector<int> order(bands.size());
            for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
            std::sort(order.begin(), order.end(), [&](int a, int b) { return bands[a].B < bands[b].B; });
            for (size_t i = 0; i < order.size(); i += 2)
                units.push_back({order[i], i + 1 < order.size() ? order[i + 1] : -1});
        } else {
            for (size_t i = 0; i < bands.size(); ++i) units.push_back({(int)i, -1});
        }
        for (auto &u : units) {
            const Band &A = bands[u.first];
            int64_t mlo = A.mlo, mend = A.mlo + A.B;
            if (u.second >= 0) {
                const Band &Bb = bands[u.second];
                mlo = std::min(mlo, Bb.mlo);
                mend = std::max(mend, Bb.mlo + Bb.B);
            }
            int64_t B = mend - mlo;
            if (B >= p.M) {
                mlo = -p.M / 2;
                B = p.M;
            }
            int64_t P = std::max<int64_t>(64, next_pow2(B));
            P = std::min<int64_t>(P, pmax);
            P = std::min<int64_t>(P, p2);
            if (!column_size_ok((int)P, p.precision))
                fail(CWT_EUNSUPPORTED, "FFT length has too small a power-of-two factor for the band-limited path");
            int G = column_g((int)P, p.precision);
            int64_t Q = p.M / P;
            ColumnDesc d{};
            d.sa = bands[u.first].j;
            d.sb = u.second >= 0 ? bands[u.second].j : -1;
            d.mlo = mlo;
            d.B = B;
            d.Q = Q;
            d.taba = (int64_t)tab.size();
            for (int64_t m = mlo; m < mlo + B; ++m) tab.push_back(spec(p.scales[d.sa], m));
            d.tabb = d.taba;
            if (d.sb >= 0) {
                d.tabb = (int64_t)tab.size();
                for (int64_t m = mlo; m < mlo + B; ++m) tab.push_back(spec(p.scales[d.sb], m));
            }
            ColumnLaunch *cl = nullptr;
            for (auto &c : p.columns)
                if (c.P == P) cl = &c;
            if (!cl) {
                p.columns.push_back(ColumnLaunch{});
                cl = &p.columns.back();
                cl->P = (int32_t)P;
                cl->G = G;
            }
            for (int64_t r0 = 0; r0 < Q; r0 += G) {
                d.r0 = r0;
                cl->items.push_back(d);
            }
        }
    }

    // workspace: F (plan precision complex) then the four-step intermediate (FP64 complex)
    if (p.M > 0) {
        size_t fbytes = (size_t)p.M * (fp64 ? 16 : 8);
        p.ws_F_off = 0;
        p.ws_Y_off = (fbytes + 255) & ~size_t(255);
        p.ws_bytes = p.M2 > 1 ? p.ws_Y_off + (size_t)p.M * 16 : fbytes;
    }
    p.tab_elems = (int64_t)tab.size();
    if (p.host_only) return;

    // ---- upload: spectrum table (plan precision) and twiddles
    if (!tab.empty()) {
        size_t bytes = tab.size() * (fp64 ? 8 : 4);
        HIPCHK(hipMalloc(&p.d_tab, bytes));
        p.table_bytes += bytes;
        if (fp64) {
            HIPCHK(hipMemcpy(p.d_tab, tab.data(), bytes, hipMemcpyHostToDevice));
        } else {
            std::vector<float> t32(tab.begin(), tab.end());
            HIPCHK(hipMemcpy(p.d_tab, t32.data(), bytes, hipMemcpyHostToDevice));
        }
    }
    TableBuilder tb;
    for (auto &g : p.groups) {
        if (fp64) push_twiddles<double>(tb, g.L, p.tw_off);
        else {
            push_twiddles<float>(tb, g.L, p.tw_off);
            push_twiddles<double>(tb, g.L, p.tw64_off);  // FP64 segment forward transforms
        }
    }
    for (auto &c : p.columns) {
        if (fp64) push_twiddles<double>(tb, c.P, p.tw_off);
        else push_twiddles<float>(tb, c.P, p.tw_off);
    }
    if (p.M > 0) {
        push_twiddles<double>(tb, p.M1, p.tw64_off);
        if (p.M2 > 1) {
            push_twiddles<double>(tb, p.M2, p.tw64_off);
            push_twM<double>(tb, p.M, p.twM64_hi_off, p.twM64_lo_off);
        }
        if (fp64) {
            if (p.twM64_hi_off < 0) push_twM<double>(tb, p.M, p.twM64_hi_off, p.twM64_lo_off);
            p.twM_hi_off = p.twM64_hi_off;
            p.twM_lo_off = p.twM64_lo_off;
        } else {
            push_twM<float>(tb, p.M, p.twM_hi_off, p.twM_lo_off);
        }
    }
    if (!tb.host.empty()) {
        HIPCHK(hipMalloc(&p.d_tw_all, tb.host.size()));
        p.table_bytes += tb.host.size();
        HIPCHK(hipMemcpy(p.d_tw_all, tb.host.data(), tb.host.size(), hipMemcpyHostToDevice));
    }
    for (auto &g : p.groups) {
        HIPCHK(hipMalloc(&g.d_scales, g.scales.size() * sizeof(int32_t)));
        p.table_bytes += g.scales.size() * sizeof(int32_t);
        HIPCHK(hipMemcpy(g.d_scales, g.scales.data(), g.scales.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    }
    for (auto &c : p.columns) {
        size_t bytes = c.items.size() * sizeof(ColumnDesc);
        HIPCHK(hipMalloc(&c.d_items, bytes));
        p.table_bytes += bytes;
        HIPCHK(hipMemcpy(c.d_items, c.items.data(), bytes, hipMemcpyHostToDevice));
    }
}


// Segmented FFT plan.  Every scale gets a segment length L = 2^l >= 8 T
// (T its half-support, at least 64 samples).  If the spectrum of its wavelet
// at that length spans a sixteenth of L or more, the scale joins a LOCAL
// group (full-spectrum fused kernel); otherwise a BAND group keyed by (L, P)
// with P >= the band width, whose length may then shrink to c 2^k (c odd).
// Halo of a segment group, rounded up to 16 samples: the kept outputs of
// every segment then start on a 16-sample boundary (V = L - 2 Tg is a
// multiple of 16 too), so the 16-column output runs of the kernels fill whole
// cache lines instead of straddling two.  Any halo >= the largest T of the
// group gives the same outputs.
static int64_t align_halo(int64_t t, int64_t a = 16) { return (t + a - 1) & ~(a - 1); }

// Stream of the calling thread for plan construction and release
// (non-blocking, default priority): plan tables are allocated, filled and
// freed in its order, so building or destroying a plan never waits for the
// work other streams are running (release waits for the plan's own calls
// only, through the events of note_use).
static hipStream_t plan_stream() {
    static thread_local hipStream_t st = nullptr;
    if (!st) HIPCHK(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    return st;
}

// Shortest single segment that holds the whole signal for a wavelet of
// radius T.  Zero boundary: the signal at offset 0 followed by zeros; the
// circular correlation over L >= N + T + 1 samples then reads, for every
// output b in [0, N), the true neighbours f[b + t], |t| <= T, or zeros (the
// left neighbours of the first outputs wrap into the zero tail).  Periodic
// boundary: halos of T wrapped samples on both sides.
static int64_t single_segment_len(const Plan &p, int64_t T) {
    return p.boundary == CWT_ZERO ? p.N + T + 1 : p.N + 2 * align_halo(T);
}

// Frames a segment group: halo Tg, kept outputs V per segment, segment count,
// with Tg and V multiples of a (16, or 32 for column pairs).  A zero-boundary
// group whose segment holds the whole signal uses the single-segment framing
// above (no left halo, V = N).
static bool single_segment(const Plan &p, const SegGroup &g) {
    return p.boundary == CWT_ZERO && g.L >= p.N + g.Tg + 1;
}
static void frame_group(const Plan &p, SegGroup &g, int64_t a = 16) {
    if (single_segment(p, g)) {
        g.Tg = 0;
        g.V = p.N;
        g.nseg = 1;
        return;
    }
    g.Tg = align_halo(g.Tg, a);
    g.V = g.L - 2 * g.Tg;
    if (g.V <= 0) fail(CWT_EUNSUPPORTED, "internal: segment too short for the halo");
    g.nseg = (p.N + g.V - 1) / g.V;
}

static void build_seg_plan(Plan &p, const Wavelet &w) {
    const bool fp64 = p.precision == CWT_FP64;
    const int lmax_local = 4096;
    const int pmax = 512;
    const int lg_max = 23;
    double ulo, uhi;
    spectral_band(w, p.rel, ulo, uhi);
    p.pair_real = !p.cplx_out;
    p.path.assign(p.S, PATH_LOCAL);

    struct Cand {
        int j, lg;
        int64_t klo, khi;
    };
    std::vector<Cand> loc, band;
    for (int j = 0; j < p.S; ++j) {
        double s = p.scales[j];
        // 8 T per segment for long signals, at least 256 samples (a group of
        // shorter segments holds only the few smallest scales, too few to
        // amortise its segment transforms); a short signal is a single
        // segment just long enough for it and the halos (see single_segment)
        int64_t L = std::min(std::max<int64_t>(256, next_pow2(8 * p.T[j] + 1)),
                             std::max<int64_t>(64, next_pow2(single_segment_len(p, p.T[j]))));
        int lg = 0;
        while ((int64_t(1) << lg) < L) ++lg;
        if (lg > lg_max) fail(CWT_EUNSUPPORTED, "scale too large for the segmented transform (wavelet support above 2^20 samples)");
        int64_t klo = (int64_t)std::floor(L * ulo / (2.0 * M_PI * s)) - 1;
        int64_t khi = (int64_t)std::ceil(L * uhi / (2.0 * M_PI * s)) + 1;
        int64_t B = khi - klo + 1;
        int64_t P = std::max<int64_t>(64, next_pow2(B));
        if (P * 16 > L || P > pmax) {
            if (L > lmax_local) fail(CWT_EUNSUPPORTED, "wavelet band too wide for the segment length");
            loc.push_back({j, lg, 0, 0});
        } else {
            band.push_back({j, lg, klo, khi});
            p.path[j] = PATH_COLUMN;
        }
    }
    // spectrum samples: evaluated on the device at the end (jobs); tab_n
    // counts the table's elements
    std::vector<SpecJob> jobs;
    int64_t tab_n = 0;
    // shift >= 0: complex entries, the samples times w_L^{-m shift}
    auto add_job = [&](double s, int64_t L, int64_t m0, int64_t count, bool full, int32_t shift = -1) {
        SpecJob jb{};
        if (shift >= 0) tab_n += tab_n & 1;  // complex entries start on an even element
        jb.off = tab_n;
        jb.m0 = m0;
        jb.count = count;
        jb.L = L;
        jb.s = s;
        jb.full = full ? 1 : 0;
        jb.shift = shift;
        jobs.push_back(jb);
        tab_n += shift >= 0 ? 2 * count : count;
        return jb.off;
    };
    TableBuilder tb;
    push_w23(tb, p.w23_hi_off, p.w23_lo_off);
    size_t ws = 0;
    auto ws_take = [&](size_t bytes) {
        size_t off = (ws + 255) & ~size_t(255);
        ws = off + bytes;
        return off;
    };

    // Local scales of an FP32 plan of a long signal whose segments would be
    // at most 2048 samples long are taken together at the longest of those
    // lengths: the cost per scale of a local group hardly depends on L up to
    // 2048 (the output stores dominate), while every group pays one FP64
    // transform of all its segments.  (At the longer length a short signal
    // would compute more halo, and FP64 groups of 2048 run at half the
    // occupancy, so neither is merged.)
    if (!fp64) {
        int lgm = 0;
        for (auto &c : loc)
            if (c.lg <= 11) lgm = std::max(lgm, c.lg);
        if (lgm > 0 && p.N >= (int64_t(8) << lgm))
            for (auto &c : loc)
                if (c.lg <= 11) c.lg = lgm;
    }
    // LOCAL groups by L
    std::sort(loc.begin(), loc.end(), [](const Cand &a, const Cand &b) { return a.lg < b.lg || (a.lg == b.lg && a.j < b.j); });
    for (size_t i = 0; i < loc.size();) {
        SegGroup g;
        g.kind = SegGroup::LOCAL;
        g.lgL = loc[i].lg;
        g.L = 1 << g.lgL;
        while (i < loc.size() && loc[i].lg == g.lgL) {
            g.scales.push_back(loc[i].j);
            g.Tg = std::max(g.Tg, p.T[loc[i].j]);
            ++i;
        }
        frame_group(p, g);
        g.tab_off = tab_n;
        for (int j : g.scales) add_job(p.scales[j], g.L, 0, g.L, true);
        g.twl_off = fp64 ? push_pass_twiddles<double>(tb, g.L) : push_pass_twiddles<float>(tb, g.L);
        p.segs.push_back(std::move(g));
    }

    // BAND groups by (L, P), at most kMaxUnits output units each
    const int kMaxUnits = 32;
    std::sort(band.begin(), band.end(), [](const Cand &a, const Cand &b) { return a.lg < b.lg || (a.lg == b.lg && a.j < b.j); });
    const int per_unit = p.pair_real ? 2 : 1;
    // Output elements per 128-byte line: complex rows, and real FP32 rows
    // written as column pairs.  When N is not a multiple of it, rows start
    // inside a line, and the inverse shifts each unit's columns so that its
    // store runs start on line boundaries (a phase applied in registers).
    const int64_t line_e = 128 / ((p.cplx_out ? 2 : 1) * (fp64 ? 8 : 4));
    for (size_t i = 0; i < band.size();) {
        SegGroup g;
        g.kind = SegGroup::BAND;
        g.lgL = band[i].lg;
        g.L = 1 << g.lgL;
        int64_t klo = band[i].klo, khi = band[i].khi;
        std::vector<int> js;
        // add scales of the same L while the union band still fits P (capped at pmax and L/16)
        while (i < band.size() && band[i].lg == g.lgL && (int)js.size() < kMaxUnits * per_unit) {
            int64_t nlo = std::min(klo, band[i].klo), nhi = std::max(khi, band[i].khi);
            int64_t P = std::max<int64_t>(64, next_pow2(nhi - nlo + 1));
            if (!js.empty() && (P > pmax || P * 16 > g.L)) break;
            // the inverse stages all spectrum samples of a group in LDS
            int64_t kls_cap = std::max<int64_t>(2 * P, kSegKlsBytes / (fp64 ? 8 : 4));
            // (a real-wavelet pair takes two tables even when its second scale is absent)
            int64_t ntab = ((int64_t)js.size() + 1 + per_unit - 1) / per_unit * per_unit;
            if (!js.empty() && ntab * (nhi - nlo + 1) > kls_cap) break;
            klo = nlo;
            khi = nhi;
            js.push_back(band[i].j);
            ++i;
        }
        g.scales.assign(js.begin(), js.end());
        g.klo = klo;
        g.B = (int32_t)(khi - klo + 1);
        g.P = (int32_t)std::max<int64_t>(64, next_pow2(g.B));
        for (int j : js) g.Tg = std::max(g.Tg, p.T[j]);
        // Segment length: of L = 2^lg and the shorter L = c 2^k (c odd, at most
        // 15, 2^k >= 32 P so that Q = L / P is a multiple of 32) whose band
        // still fits P, the one that computes the fewest positions, nseg L.
        // The power of two set by the halo (about 8 T) can leave the last
        // segment, or a single segment holding the whole signal, mostly beyond
        // the signal's end.
        {
            auto band_at = [&](int64_t Lc, int64_t &lo, int64_t &hi) {
                lo = std::numeric_limits<int64_t>::max();
                hi = std::numeric_limits<int64_t>::min();
                for (int j : js) {
                    const double s = p.scales[j];
                    lo = std::min(lo, (int64_t)std::floor(Lc * ulo / (2.0 * M_PI * s)) - 1);
                    hi = std::max(hi, (int64_t)std::ceil(Lc * uhi / (2.0 * M_PI * s)) + 1);
                }
            };
            auto cost_of = [&](int64_t Lc) {
                if (p.boundary == CWT_ZERO && Lc >= p.N + g.Tg + 1) return Lc;  // single segment
                const int64_t V = Lc - 2 * align_halo(g.Tg, p.pair_real && !fp64 ? 32 : 16);
                return V > 0 ? (p.N + V - 1) / V * Lc : std::numeric_limits<int64_t>::max();
            };
            int64_t best = cost_of(g.L), bestL = g.L;
            int bestc = 1, bestk = g.lgL;
            for (int c = 3; c <= 15; c += 2)
                for (int k = 0; (int64_t(c) << k) < g.L; ++k) {
                    const int64_t Lc = int64_t(c) << k;
                    if ((int64_t(1) << k) < 32 * (int64_t)g.P) continue;
                    int64_t lo, hi;
                    band_at(Lc, lo, hi);
                    if (hi - lo + 1 > g.P) continue;
                    const int64_t cst = cost_of(Lc);
                    if (cst < best) {
                        best = cst;
                        bestL = Lc;
                        bestc = c;
                        bestk = k;
                    }
                }
            if (bestc != 1) {
                int64_t lo, hi;
                band_at(bestL, lo, hi);
                g.L = (int32_t)bestL;
                g.cL = bestc;
                g.lgL = bestk;
                klo = lo;
                khi = hi;
                g.klo = lo;
                g.B = (int32_t)(hi - lo + 1);
            }
        }
        const int64_t Q = g.L / g.P;
        const int64_t iters_total = Q / 16;
        // Real FP32 output with rows of at least 32 columns: the inverse packs
        // adjacent columns 2g, 2g + 1 of one scale into one complex column
        // (each column's output is real), so that every lane stores two
        // neighbouring outputs and a 16-lane run fills a 128-byte line.  With
        // the column shift below every pair starts on an even element; for an
        // odd N a pair can straddle the row end or a window edge, and the
        // inverse then stores its two outputs separately.  Needs one unit per
        // scale and V, Tg multiples of 32 (or V = N).  (FP64 runs of 16 columns
        // fill whole lines already.)
        g.colpair = p.pair_real && !fp64 && Q >= 32 && (int)js.size() <= kMaxUnits &&
                            (single_segment(p, g) || g.L > 2 * align_halo(g.Tg, 32))
                        ? 1
                        : 0;
        g.colodd = g.colpair && p.N % 2 != 0 ? 1 : 0;
        frame_group(p, g, g.colpair ? 32 : 16);
        // column chunks of the forward: enough workgroups to fill the device,
        // at most 256 partial sums per bin.  A chunk keeps at least two
        // 16-column iterations: a wave reads 16 consecutive FP32 columns (half
        // a 128-byte line) per row, and the other half is then read by the
        // same workgroup one iteration later instead of by another workgroup,
        // often on another XCD with its own L2.
        int64_t nchunk = 1;
        while (nchunk * 4 <= iters_total && nchunk * 2 <= 256 && g.nseg * nchunk < 2048) nchunk *= 2;
        while (iters_total % nchunk != 0) --nchunk;  // whole chunks (Q / 16 need not be a power of two)
        g.nchunk = (int32_t)nchunk;
        g.iters = (int32_t)(iters_total / nchunk);
        // column shift of a single-row unit: its row starts dsh elements past
        // a line boundary (for an output aligned to 128 bytes; the result
        // does not depend on it).  Segment starts and first columns are
        // multiples of the line length already.
        const bool scale_pairs = p.pair_real && !g.colpair;
        std::vector<int32_t> dsh(js.size(), 0);
        if (!scale_pairs)
            for (size_t u = 0; u < js.size(); ++u) {
                dsh[u] = (int32_t)(((int64_t)js[u] * p.N) % line_e);
                if (dsh[u] != 0) g.cshift = 1;
            }
        if (g.colodd) g.cshift = 1;  // the odd-length path is a shifted one
        // spectrum samples of each scale on the group band; a shifted group
        // also gets them as complex values with the unit's shift phase
        // w_L^{-m dsh} folded in (the statistics variants, which never shift,
        // read the real ones)
        std::vector<int64_t> koff(js.size()), kcoff(js.size(), 0);
        for (size_t u = 0; u < js.size(); ++u) {
            koff[u] = add_job(p.scales[js[u]], g.L, g.klo, g.B, false);
            if (g.cshift) kcoff[u] = add_job(p.scales[js[u]], g.L, g.klo, g.B, false, dsh[u]);
        }
        // column factors, g < 16: w_L^{m g}, or w_L^{2 m g} (1 + i w_L^m) for
        // the column pair (2g, 2g + 1)
        {
            std::vector<double> gt(2 * 16 * (size_t)g.B);
            for (int gg = 0; gg < 16; ++gg)
                for (int k = 0; k < g.B; ++k) {
                    const std::complex<double> v =
                        g.colpair ? wL_at((g.klo + k) * 2 * gg, g.L, g.cL, g.lgL) *
                                        (1.0 + std::complex<double>(0.0, 1.0) * wL_at(g.klo + k, g.L, g.cL, g.lgL))
                                  : wL_at((g.klo + k) * gg, g.L, g.cL, g.lgL);
                    gt[2 * ((size_t)gg * g.B + k)] = v.real();
                    gt[2 * ((size_t)gg * g.B + k) + 1] = v.imag();
                }
            if (fp64) g.gtw_off = tb.add(gt.data(), gt.size() * sizeof(double));
            else {
                std::vector<float> g32(gt.begin(), gt.end());
                g.gtw_off = tb.add(g32.data(), g32.size() * sizeof(float));
            }
        }
        // output units: single scales (complex output, column pairs) or
        // scale pairs (other real output)
        g.unit0 = (int32_t)p.units.size();
        for (size_t u = 0; u < js.size(); u += scale_pairs ? 2 : 1) {
            SegUnit un{};
            un.sa = js[u];
            un.ka = koff[u];
            if (scale_pairs && u + 1 < js.size()) {
                un.sb = js[u + 1];
                un.kb = koff[u + 1];
            } else {
                un.sb = -1;
                un.kb = g.cshift ? kcoff[u] : koff[u];
            }
            un.dsh = dsh[u];
            p.units.push_back(un);
        }
        g.nunits = (int32_t)p.units.size() - g.unit0;
        {
            const int64_t need = (scale_pairs ? 2 : 1) * (int64_t)g.nunits;
            if (need * g.B > std::max<int64_t>(2 * g.P, kSegKlsBytes / (fp64 ? 8 : 4)))
                fail(CWT_EUNSUPPORTED, "internal: band group tables exceed the staging area");
        }
        g.ws_xp_off = ws_take((size_t)g.nseg * g.nchunk * g.B * 16);
        // one column chunk: the partial sums are the band spectra (no reduce)
        g.ws_x_off = g.nchunk == 1 ? g.ws_xp_off : ws_take((size_t)g.nseg * g.B * 16);
        // attach to the launch of its P
        SegLaunch *sl = nullptr;
        for (auto &l : p.seg_launches)
            if (l.P == g.P) sl = &l;
        if (!sl) {
            p.seg_launches.push_back(SegLaunch{});
            sl = &p.seg_launches.back();
            sl->P = g.P;
            sl->twl_off = fp64 ? push_pass_twiddles<double>(tb, g.P) : push_pass_twiddles<float>(tb, g.P);
        }
        const int32_t gi = (int32_t)sl->gdev.size();
        SegGroupDev gd{};
        gd.lgL = g.lgL;
        gd.B = g.B;
        gd.nchunk = g.nchunk;
        gd.iters = g.iters;
        gd.unit0 = g.unit0;
        gd.nunits = g.nunits;
        gd.colpair = g.colpair;
        gd.cshift = g.cshift;
        gd.colodd = g.colodd;
        gd.inv0 = (int32_t)sl->inv.size();
        gd.V = g.V;
        gd.Tg = g.Tg;
        gd.klo = g.klo;
        gd.nseg = g.nseg;
        gd.xp_off = (int64_t)g.ws_xp_off;
        gd.x_off = (int64_t)g.ws_x_off;
        gd.gtw_off = g.gtw_off;
        gd.L = g.L;
        gd.Q = g.L / g.P;
        gd.cL = g.cL;
        if (g.cL > 1) {
            // w_L^z, z < c: with w_L^{c y + z} = w_{2^k}^y w_L^z the kernels
            // take the rest from the 2^23 split tables
            std::vector<double> sm(2 * (size_t)g.cL);
            for (int z = 0; z < g.cL; ++z) {
                const std::complex<double> v = wL_at(z, g.L, g.cL, g.lgL);
                sm[2 * (size_t)z] = v.real();
                sm[2 * (size_t)z + 1] = v.imag();
            }
            gd.wsm_off = tb.add(sm.data(), sm.size() * sizeof(double));
        }
        sl->gdev.push_back(gd);
        sl->groups.push_back((int32_t)p.segs.size());
        sl->out_rows += (double)js.size();
        // forward items cover `pad` consecutive segments, about 256 items
        // per group: each workgroup then has enough work to repay its set-up
        // (twiddle tables, band factors); reduce items one segment each
        const int64_t nkb = (g.B + 15) / 16;
        const int64_t fsw = std::max<int64_t>(1, g.nseg * g.nchunk / 256);
        const int64_t rsw = 1;
        for (int64_t sg = 0; sg < g.nseg; sg += fsw)
            for (int32_t c = 0; c < g.nchunk; ++c)
                sl->fwd.push_back({gi, (int32_t)sg, c, (int32_t)std::min(fsw, g.nseg - sg)});
        if (g.nchunk > 1)
            for (int64_t sg = 0; sg < g.nseg; sg += rsw)
                for (int32_t kb = 0; kb < nkb; ++kb)
                    sl->red.push_back({gi, (int32_t)sg, kb, (int32_t)std::min(rsw, g.nseg - sg)});
        for (int64_t sg = 0; sg < g.nseg; ++sg)
            for (int64_t r0 = 0; r0 < Q; r0 += g.colpair ? 32 : 16) sl->inv.push_back({gi, (int32_t)sg, (int32_t)r0, 0});
        p.segs.push_back(std::move(g));
    }
    p.ws_bytes = ws;
    p.tab_elems = tab_n;
    // statistics epilogue slots: one per workgroup that writes outputs of
    // the scale (local blocks; inverse work items of a band group)
    {
        std::vector<int64_t> nslot(p.S, -1);
        auto own = [&](int32_t j, int64_t n) {
            if (j < 0 || j >= p.S || nslot[j] >= 0) fail(CWT_EINVAL, "internal: scale in two segment groups");
            nslot[j] = n;
        };
        for (auto &g : p.segs) {
            if (g.kind == SegGroup::LOCAL) {
                const int64_t per = local2_segs_per_block(g.L, p.pair_real, fp64);
                for (int32_t j : g.scales) own(j, (g.nseg + per - 1) / per);
            } else {
                const int64_t Q = (int64_t)g.L / g.P, cols = g.colpair ? 32 : 16;
                const int64_t n = g.nseg * ((Q + cols - 1) / cols);
                for (int32_t u = g.unit0; u < g.unit0 + g.nunits; ++u) {
                    own(p.units[u].sa, n);
                    if (p.units[u].sb >= 0) own(p.units[u].sb, n);
                }
            }
        }
        p.wps_base.assign(p.S + 1, 0);
        for (int32_t j = 0; j < p.S; ++j) {
            if (nslot[j] < 0) fail(CWT_EINVAL, "internal: scale in no segment group");
            p.wps_base[j + 1] = p.wps_base[j] + nslot[j];
        }
    }
    if (p.host_only) return;

    // One device allocation holds every table of the plan:
    //   twiddles | spectrum samples | spectrum jobs | scale ids | units |
    //   per band size: groups, forward / reduce / inverse work | launch keys
    const size_t eb = fp64 ? 8 : 4;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = (off + 255) & ~size_t(255);
        off = o + bytes;
        return o;
    };
    const size_t o_tw = take(tb.host.size());
    const size_t o_tab = take((size_t)tab_n * eb);
    int64_t spec_blocks = 0;
    for (auto &jb : jobs) {
        jb.block0 = spec_blocks;
        spec_blocks += (jb.count + 255) / 256;
    }
    const size_t o_jobs = take(jobs.size() * sizeof(SpecJob));
    std::vector<size_t> o_sc(p.segs.size(), 0);
    for (size_t gi = 0; gi < p.segs.size(); ++gi)
        if (p.segs[gi].kind == SegGroup::LOCAL) o_sc[gi] = take(p.segs[gi].scales.size() * sizeof(int32_t));
    const size_t o_units = take(p.units.size() * sizeof(SegUnit));
    struct LaunchOffs {
        size_t groups, fwd, red, inv;
    };
    std::vector<LaunchOffs> o_l;
    for (auto &l : p.seg_launches)
        o_l.push_back({take(l.gdev.size() * sizeof(SegGroupDev)), take(l.fwd.size() * sizeof(SegWork)),
                       take(l.red.size() * sizeof(SegWork)), take(l.inv.size() * sizeof(SegWork))});
    size_t nkeys = 0;
    for (auto &g : p.segs) nkeys += g.kind == SegGroup::LOCAL ? 1 : 0;
    nkeys += 3 * p.seg_launches.size();
    const size_t o_keys = take(nkeys * sizeof(KeyDesc));
    const size_t o_wps = take(p.wps_base.size() * sizeof(int64_t));
    const size_t total = off;

    hipStream_t pst = plan_stream();
    HIPCHK(hipMallocAsync(&p.d_arena, total, pst));
    p.table_bytes += total;
    char *base = static_cast<char *>(p.d_arena);
    p.d_tw_all = base + o_tw;
    p.d_tab = base + o_tab;
    std::vector<char> img(total, 0);
    auto put = [&](size_t o, const void *src, size_t bytes) {
        if (bytes) std::memcpy(img.data() + o, src, bytes);
    };
    put(o_tw, tb.host.data(), tb.host.size());
    put(o_jobs, jobs.data(), jobs.size() * sizeof(SpecJob));
    for (size_t gi = 0; gi < p.segs.size(); ++gi) {
        SegGroup &g = p.segs[gi];
        if (g.kind != SegGroup::LOCAL) continue;
        put(o_sc[gi], g.scales.data(), g.scales.size() * sizeof(int32_t));
        g.d_scales = reinterpret_cast<int32_t *>(base + o_sc[gi]);
    }
    put(o_units, p.units.data(), p.units.size() * sizeof(SegUnit));
    p.d_units = reinterpret_cast<SegUnit *>(base + o_units);
    put(o_wps, p.wps_base.data(), p.wps_base.size() * sizeof(int64_t));
    p.d_wps_base = reinterpret_cast<int64_t *>(base + o_wps);
    for (size_t li = 0; li < p.seg_launches.size(); ++li) {
        SegLaunch &l = p.seg_launches[li];
        put(o_l[li].groups, l.gdev.data(), l.gdev.size() * sizeof(SegGroupDev));
        put(o_l[li].fwd, l.fwd.data(), l.fwd.size() * sizeof(SegWork));
        put(o_l[li].red, l.red.data(), l.red.size() * sizeof(SegWork));
        put(o_l[li].inv, l.inv.data(), l.inv.size() * sizeof(SegWork));
        l.d_groups = reinterpret_cast<SegGroupDev *>(base + o_l[li].groups);
        l.d_fwd = reinterpret_cast<SegWork *>(base + o_l[li].fwd);
        l.d_red = reinterpret_cast<SegWork *>(base + o_l[li].red);
        l.d_inv = reinterpret_cast<SegWork *>(base + o_l[li].inv);
    }

    // launch keys
    const char *tw = static_cast<const char *>(p.d_tw_all);
    const char *dtab = static_cast<const char *>(p.d_tab);
    KeyDesc kb{};
    kb.N = p.N;
    kb.periodic = p.boundary == CWT_PERIODIC ? 1 : 0;
    kb.cph = p.cph;
    kb.units = p.d_units;
    kb.ktab = dtab;
    kb.twbase = tw;
    kb.whi = reinterpret_cast<const double2 *>(tw + p.w23_hi_off);
    kb.wlo = reinterpret_cast<const double2 *>(tw + p.w23_lo_off);
    kb.wps_base = p.d_wps_base;
    p.keys.clear();
    for (auto &g : p.segs) {
        if (g.kind != SegGroup::LOCAL) continue;
        KeyDesc k = kb;
        k.ktab = dtab + (size_t)g.tab_off * eb;
        k.twl = tw + g.twl_off;
        k.Tg = g.Tg;
        k.V = g.V;
        k.nseg = g.nseg;
        k.nscale = (int32_t)g.scales.size();
        k.scale_ids = g.d_scales;
        const int64_t per = local2_segs_per_block(g.L, p.pair_real, fp64);
        g.blocks = (g.nseg + per - 1) / per;
        g.key = (int32_t)p.keys.size();
        p.keys.push_back(k);
    }
    for (auto &l : p.seg_launches) {
        KeyDesc k = kb;
        k.groups = l.d_groups;
        k.twl = tw + l.twl_off;
        const SegWork *lists[3] = {l.d_fwd, l.d_red, l.d_inv};
        for (int ph = 0; ph < 3; ++ph) {
            k.work = lists[ph];
            l.key[ph] = (int32_t)p.keys.size();
            p.keys.push_back(k);
        }
    }
    put(o_keys, p.keys.data(), p.keys.size() * sizeof(KeyDesc));
    p.d_keys = reinterpret_cast<KeyDesc *>(base + o_keys);

    // upload and evaluate the spectra on the stream of this thread, then wait
    // for it only (work of other streams keeps running)
    HIPCHK(hipMemcpyAsync(base, img.data(), total, hipMemcpyHostToDevice, pst));
    SpecWavelet sw{};
    sw.kind = w.kind;
    sw.m = w.m;
    sw.w0 = w.w0;
    sw.cmor = w.cmor;
    sw.kappa = w.kappa;
    sw.gnorm = w.gnorm;
    sw.cn = w.cn;
    sw.ulo = ulo;
    sw.uhi = uhi;
    HIPCHK(launch_spectrum_tables(sw, reinterpret_cast<const SpecJob *>(base + o_jobs), (int)jobs.size(),
                                  spec_blocks, p.d_tab, fp64, pst));
    HIPCHK(hipStreamSynchronize(pst));
}

static hipStream_t plan_stream();

// Records, on `st`, that the plan's work enqueued so far on that stream must
// finish before its tables are released.  Skipped while `st` is capturing a
// graph: a graph keeps no claim on the plan, so the caller keeps the plan
// alive while the graph may still be launched.
static bool capturing(hipStream_t st) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    return hipStreamIsCapturing(st, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone;
}
static std::shared_ptr<UseEvent> record_use(hipStream_t st) {
    auto e = std::make_shared<UseEvent>();
    if (!e->ev) fail(CWT_EDEVICE, "hipEventCreateWithFlags failed");
    HIPCHK(hipEventRecord(e->ev, st));
    return e;
}
static void note_use(Plan &p, hipStream_t st, const std::shared_ptr<UseEvent> &e) {
    std::lock_guard<std::mutex> g(p.use_mu);
    for (auto &u : p.last_use)
        if (u.first == st) {
            u.second = e;
            return;
        }
    if (p.last_use.size() >= 16) {
        // bound the list: the oldest stream's last call is waited for here
        HIPCHK(hipEventSynchronize(p.last_use.front().second->ev));
        p.last_use.erase(p.last_use.begin());
    }
    p.last_use.push_back({st, e});
}
static void note_use(Plan &p, hipStream_t st) {
    if (!capturing(st)) note_use(p, st, record_use(st));
}

static void free_plan(Plan *p) {
    if (!p) return;
    if (p->d_arena) {
        // every table of a segmented plan sits in the arena; its stream-ordered
        // release waits for the plan's last call on every stream that used it
        try {
            hipStream_t pst = plan_stream();
            for (auto &e : p->last_use) (void)hipStreamWaitEvent(pst, e.second->ev, 0);
            (void)hipFreeAsync(p->d_arena, pst);
        } catch (...) {
            for (auto &e : p->last_use) (void)hipEventSynchronize(e.second->ev);
            (void)hipFree(p->d_arena);
        }
        p->last_use.clear();
        for (void *x : p->d_extra)
            if (x) (void)hipFree(x);
        for (auto &r : p->timing_recs) {
            (void)hipEventDestroy(r.a);
            (void)hipEventDestroy(r.b);
        }
        for (auto e : p->event_pool) (void)hipEventDestroy(e);
        delete p;
        return;
    }
    // separately allocated tables: wait for the plan's last calls first
    for (auto &e : p->last_use) (void)hipEventSynchronize(e.second->ev);
    p->last_use.clear();
    if (p->d_tab) (void)hipFree(p->d_tab);
    if (p->d_tw_all) (void)hipFree(p->d_tw_all);
    if (p->d_dtab) (void)hipFree(p->d_dtab);
    for (auto &g : p->groups)
        if (g.d_scales) (void)hipFree(g.d_scales);
    for (auto &c : p->columns)
        if (c.d_items) (void)hipFree(c.d_items);
    for (auto &g : p->segs)
        if (g.d_scales) (void)hipFree(g.d_scales);
    if (p->d_units) (void)hipFree(p->d_units);
    if (p->d_keys) (void)hipFree(p->d_keys);
    for (auto &l : p->seg_launches) {
        if (l.d_groups) (void)hipFree(l.d_groups);
        if (l.d_fwd) (void)hipFree(l.d_fwd);
        if (l.d_red) (void)hipFree(l.d_red);
        if (l.d_inv) (void)hipFree(l.d_inv);
    }
    for (void *x : p->d_extra)
        if (x) (void)hipFree(x);
    for (auto &r : p->timing_recs) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    for (auto e : p->event_pool) (void)hipEventDestroy(e);
    delete p;
}

static Plan *make_plan(int64_t N, int32_t boundary, cwt_wavelet wv, const double *scales, int32_t S,
                       const cwt_opts *opts) {
    if (N < 2) fail(CWT_EINVAL, "N must be >= 2");
    if (N > kMaxN) fail(CWT_EUNSUPPORTED, "N above 2^26");
    if (S < 1) fail(CWT_EINVAL, "S must be >= 1");
    if (S > 65536) fail(CWT_EUNSUPPORTED, "S above 65536");
    if (!scales) fail(CWT_EINVAL, "scales is NULL");
    if (boundary != CWT_PERIODIC && boundary != CWT_ZERO) fail(CWT_EINVAL, "unknown boundary");
    int precision = opts ? opts->precision : CWT_FP64;
    int method = opts ? opts->method : CWT_METHOD_FFT;
    int64_t fft_len = opts ? opts->fft_len : 0;
    if (precision != CWT_FP64 && precision != CWT_FP32) fail(CWT_EINVAL, "unknown precision");
    if (method != CWT_METHOD_FFT && method != CWT_METHOD_SPLINE && method != CWT_METHOD_A19 &&
        method != CWT_METHOD_V97)
        fail(CWT_EINVAL, "unknown method");
    if (fft_len < 0) fail(CWT_EINVAL, "fft_len must be >= 0");
    if (opts && opts->fft_mode != CWT_FFT_SEGMENTED && opts->fft_mode != CWT_FFT_WHOLE)
        fail(CWT_EINVAL, "unknown fft_mode");
    const int psi_mode = opts ? opts->psi_mode : CWT_PSI_ALIASED;
    if (psi_mode != CWT_PSI_ALIASED && psi_mode != CWT_PSI_ANALYTIC) fail(CWT_EINVAL, "unknown psi_mode");
    const int fft_mode = opts ? opts->fft_mode : CWT_FFT_SEGMENTED;
    if (psi_mode == CWT_PSI_ANALYTIC && (method != CWT_METHOD_FFT || fft_mode != CWT_FFT_WHOLE))
        fail(CWT_EINVAL, "psi_mode ANALYTIC needs the FFT method with fft_mode WHOLE");
    Wavelet w;
    w.kind = wv.kind;
    if (wv.kind == CWT_MORLET) {
        if (!(std::isfinite(wv.param) && wv.param > 0.0)) fail(CWT_EINVAL, "Morlet omega0 must be finite and > 0");
        w.w0 = wv.param;
    } else if (wv.kind == CWT_MEXHAT) {
        w.m = 2;
    } else if (wv.kind == CWT_DOG) {
        if (!(std::isfinite(wv.param) && wv.param >= 1.0 && wv.param <= 16.0 && wv.param == std::floor(wv.param)))
            fail(CWT_EINVAL, "DOG order must be an integer in [1, 16]");
        w.m = (int)wv.param;
    } else if (wv.kind == CWT_MW) {
        // Table 2's MW: C_N (e^{-4ix} - e^{-8}) e^{-x^2/2} = Morlet(-4)
        w.kind = CWT_MORLET;
        w.w0 = -4.0;
    } else if (wv.kind == CWT_CBSW || wv.kind == CWT_GDW || wv.kind == CWT_CWGDW) {
        if (wv.kind == CWT_CBSW && psi_mode != CWT_PSI_ANALYTIC && method != CWT_METHOD_V97)
            fail(CWT_EUNSUPPORTED, "the cubic B-spline wavelet's spectrum is not band-limited: it is supported "
                                   "by the FFT method with fft_mode WHOLE and psi_mode ANALYTIC, and by the V97 "
                                   "method");
    } else {
        fail(CWT_EINVAL, "unknown wavelet kind");
    }
    w.init();
    for (int j = 0; j < S; ++j)
        if (!(std::isfinite(scales[j]) && scales[j] > 0.0)) fail(CWT_EINVAL, "scales must be finite and > 0");

    Plan *p = new Plan();
    try {
        p->N = N;
        p->boundary = boundary;
        p->kind = wv.kind;
        p->param = w.kind == CWT_MORLET ? w.w0 : (double)w.m;
        p->psi_mode = psi_mode;
        p->precision = precision;
        p->method = method;
        p->host_only = opts && opts->host_only != 0;
        p->single_stream = opts && opts->single_stream != 0;
        p->S = S;
        p->scales.assign(scales, scales + S);
        p->cplx_out = w.complex_out();
        p->cph = w.cph();
        p->rel = precision == CWT_FP64 ? 1e-16 : 1e-9;
        p->chi = time_radius(w, p->rel);
        p->T.resize(S);
        for (int j = 0; j < S; ++j) p->T[j] = (int64_t)std::ceil(p->chi * scales[j]);
        if (method == CWT_METHOD_FFT) {
            p->fft_mode = fft_mode;
            if (p->fft_mode == CWT_FFT_WHOLE) build_fft_plan(*p, w, fft_len);
            else build_seg_plan(*p, w);
            // cwt_global_wps: a periodic whole-signal plan whose FFT is the
            // DFT of the period, the aliased spectrum of a band-limited wavelet
            if (p->fft_mode == CWT_FFT_WHOLE && boundary == CWT_PERIODIC && p->M == N &&
                psi_mode == CWT_PSI_ALIASED && w.band_limited()) {
                double ulo, uhi;
                spectral_band(w, p->rel, ulo, uhi);
                p->spec_w = SpecWavelet{w.kind, w.m, w.w0, w.cmor, w.kappa, w.gnorm, w.cn, ulo, uhi};
                p->spec_ok = true;
                // the chunk sums follow the transform's workspace
                p->ws_pars_off = (p->ws_bytes + 255) & ~size_t(255);
                p->ws_bytes = p->ws_pars_off + (size_t)S * parseval_chunks(p->M) * sizeof(double);
                if (!p->host_only) {
                    void *d = nullptr;
                    HIPCHK(hipMalloc(&d, (size_t)S * sizeof(double)));
                    p->d_extra.push_back(d);
                    HIPCHK(hipMemcpy(d, scales, (size_t)S * sizeof(double), hipMemcpyHostToDevice));
                    p->d_scales64 = static_cast<const double *>(d);
                }
            }
        } else if (method == CWT_METHOD_V97) {
            build_v97_plan(*p, w);
        } else {
            TableBuilder tb;
            build_spline_plan(*p, w, tb);
        }
    } catch (...) {
        free_plan(p);
        throw;
    }
    return p;
}

static hipEvent_t pool_event(Plan &p) {
    if (!p.event_pool.empty()) {
        hipEvent_t e = p.event_pool.back();
        p.event_pool.pop_back();
        return e;
    }
    hipEvent_t e;
    HIPCHK(hipEventCreate(&e));
    return e;
}

// The segmented launches of a plan in execution order (local groups, then per
// band size: forward, reduce, inverse), with their kernel instantiation,
// launch key, workgroup count and algorithmic bytes.
template <typename F>
static void for_each_seg_launch(const Plan &p, F &&fn) {
    const double nn = (double)p.N;
    const double sb = p.precision == CWT_FP64 ? 8.0 : 4.0;
    const double eb = (p.precision == CWT_FP64 ? 8.0 : 4.0) * (p.cplx_out ? 2.0 : 1.0);
    const int32_t cplx = p.cplx_out ? 1 : 0;
    for (auto &g : p.segs)
        if (g.kind == SegGroup::LOCAL)
            fn(SegKernelId{0, g.L, p.precision, cplx}, g.key, g.blocks, nn * sb + nn * (double)g.scales.size() * eb);
    for (auto &l : p.seg_launches) {
        double xbytes = 0.0;
        for (auto &gd : l.gdev) xbytes += (double)gd.nseg * gd.B * 16.0;
        // (the forward and reduce kernels do not depend on the output type)
        fn(SegKernelId{1, l.P, p.precision, 0}, l.key[0], (int64_t)l.fwd.size(),
           nn * sb * (double)l.gdev.size() + xbytes);
        fn(SegKernelId{2, l.P, p.precision, 0}, l.key[1], (int64_t)l.red.size(), 2.0 * xbytes);
        fn(SegKernelId{3, l.P, p.precision, cplx}, l.key[2], (int64_t)l.inv.size(), nn * l.out_rows * eb + xbytes);
    }
}

// Second stream paired with the caller's stream (one per calling thread,
// device and caller stream; non-blocking, default priority) with a
// fork/join event pair.  The local-group kernels of a call run on it while
// the band kernels (forward, reduce, inverse, which depend on each other) run
// on the caller's stream: the two chains write disjoint output rows and only
// read the signal, and running them side by side lets one chain's
// latency-bound phases (segment loads and transforms, launch tails) overlap
// the other's output stores.  Calls on different caller streams get
// different side streams, so nothing orders them against each other.
struct SideStream {
    hipStream_t st = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
};
static SideStream &side_stream(hipStream_t caller) {
    static thread_local std::map<std::pair<int, hipStream_t>, SideStream> m;
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    SideStream &s = m[std::make_pair(dev, caller)];
    if (!s.st) {
        HIPCHK(hipStreamCreateWithFlags(&s.st, hipStreamNonBlocking));
        HIPCHK(hipEventCreateWithFlags(&s.fork, hipEventDisableTiming));
        HIPCHK(hipEventCreateWithFlags(&s.join, hipEventDisableTiming));
    }
    return s;
}

// Stream assignment of one call's segmented launches: local kernels (kind 0)
// on the side stream when the call also has band launches (and launch timing
// is off, so that timed durations are each kernel's own), everything else on
// the caller's stream.  begin() forks after the work already queued on the
// caller's stream, end() joins.
struct SegStreams {
    hipStream_t main, side;
    SideStream *ss = nullptr;
    SegStreams(hipStream_t st, bool split) : main(st), side(st) {
        if (!split) return;
        ss = &side_stream(st);
        side = ss->st;
        HIPCHK(hipEventRecord(ss->fork, main));
        HIPCHK(hipStreamWaitEvent(side, ss->fork, 0));
    }
    hipStream_t of(int kind) const { return kind == 0 ? side : main; }
    void end() {
        if (!ss) return;
        HIPCHK(hipEventRecord(ss->join, side));
        HIPCHK(hipStreamWaitEvent(main, ss->join, 0));
        ss = nullptr;
    }
};

// Runs `launch` and, when timing is on, brackets it with events on `st`.
template <typename F>
static void timed(Plan &p, hipStream_t st, const std::string &name, double bytes, const char *what, F &&launch) {
    hipEvent_t a = nullptr, b = nullptr;
    if (p.timing) {
        a = pool_event(p);
        b = pool_event(p);
        HIPCHK(hipEventRecord(a, st));
    }
    hipError_t e = launch();
    if (e != hipSuccess) fail(CWT_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
    if (p.timing) {
        HIPCHK(hipEventRecord(b, st));
        p.timing_recs.push_back({name, a, b, bytes});
    }
}

}  // namespace cwt

// ---------------------------------------------------------------------------
// C ABI

using cwt::Failure;
using cwt::Plan;

struct cwt_plan_s {
    Plan *p;
};

template <typename F> static int guarded(F &&f) {
    try {
        cwt::g_err.clear();
        return f();
    } catch (const Failure &e) {
        cwt::g_err = e.msg;
        return e.code;
    } catch (const std::bad_alloc &) {
        cwt::g_err = "host allocation failed";
        return CWT_ENOMEM;
    } catch (const std::exception &e) {
        cwt::g_err = e.what();
        return CWT_EINVAL;
    } catch (...) {
        cwt::g_err = "unknown failure";
        return CWT_EINVAL;
    }
}

extern "C" {

int cwt_plan(cwt_plan_t *out, int64_t N, int32_t boundary, cwt_wavelet wavelet, const double *scales, int32_t S,
             const cwt_opts *opts) {
    if (out) *out = nullptr;
    return guarded([&]() -> int {
        if (!out) cwt::fail(CWT_EINVAL, "out is NULL");
        Plan *p = cwt::make_plan(N, boundary, wavelet, scales, S, opts);
        cwt_plan_s *h = new (std::nothrow) cwt_plan_s{p};
        if (!h) {
            cwt::free_plan(p);
            cwt::fail(CWT_ENOMEM, "host allocation failed");
        }
        *out = h;
        return CWT_OK;
    });
}

int cwt_destroy(cwt_plan_t plan) {
    return guarded([&]() -> int {
        if (!plan) return CWT_OK;
        cwt::free_plan(plan->p);
        delete plan;
        return CWT_OK;
    });
}

int cwt_out_is_complex(cwt_plan_t plan) {
    if (!plan) return CWT_EINVAL;
    return plan->p->cplx_out ? 1 : 0;
}

int64_t cwt_out_elems(cwt_plan_t plan) {
    if (!plan) return -1;
    return plan->p->N * (int64_t)plan->p->S;
}

int32_t cwt_out_elem_bytes(cwt_plan_t plan) {
    if (!plan) return CWT_EINVAL;
    int b = plan->p->precision == CWT_FP64 ? 8 : 4;
    return plan->p->cplx_out ? 2 * b : b;
}

size_t cwt_workspace_bytes(cwt_plan_t plan) { return plan ? plan->p->ws_bytes : 0; }

size_t cwt_footprint_bytes(cwt_plan_t plan) {
    if (!plan) return 0;
    const Plan &p = *plan->p;
    size_t eb = (size_t)cwt_out_elem_bytes(plan);
    size_t sig = (size_t)p.N * (p.precision == CWT_FP64 ? 8 : 4);
    return sig + eb * (size_t)p.N * (size_t)p.S + p.ws_bytes + p.table_bytes;
}

}  // extern "C"

namespace cwt {

// One transform on `stream`.  bare: every launch on `stream`, no launch
// timing and no release event (nothing is created, not even an event).
static int exec_impl(cwt_plan_t plan, const void *signal, void *out, void *workspace, void *stream, bool bare) {
    if (!plan) fail(CWT_EINVAL, "plan is NULL");
    if (!signal || !out) fail(CWT_EINVAL, "signal/out is NULL");
    Plan &p = *plan->p;
    if (p.host_only) fail(CWT_EINVAL, "plan was built host-only");
    if (p.ws_bytes > 0 && !workspace) fail(CWT_EINVAL, "workspace is NULL");
    size_t ealign = p.precision == CWT_FP64 ? 8 : 4;
    if ((uintptr_t)signal % ealign || (uintptr_t)out % ealign)
        fail(CWT_EINVAL, "signal/out not aligned to the element size");
    if (workspace && (uintptr_t)workspace % 256) fail(CWT_EINVAL, "workspace not 256-byte aligned");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const double sb = p.precision == CWT_FP64 ? 8.0 : 4.0;
    const double eb = (double)cwt_out_elem_bytes(plan);
    const double nn = (double)p.N;
    const bool timing = p.timing && !bare;
    auto run = [&](hipStream_t ks, const std::string &name, double bytes, const char *what, auto &&launch) {
        if (timing) {
            timed(p, ks, name, bytes, what, launch);
            return;
        }
        const hipError_t e = launch();
        if (e != hipSuccess) fail(CWT_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
    };
    if (p.method == CWT_METHOD_V97) {
        for (size_t k = 0; k < p.v97_steps.size(); ++k) {
            const auto &sp = p.v97_steps[k];
            const double bytes = sp.kind == 3 ? nn * eb * (double)p.S : 8.0 * (double)p.spl_len;
            run(st, v97_kernel_name(p, k), bytes, "V97 launch",
                [&] { return launch_v97(p, k, signal, out, workspace, st); });
        }
        if (!bare) note_use(p, st);
        return CWT_OK;
    }
    if (p.method != CWT_METHOD_FFT) {
        run(st, spline_kernel_name(p, 0), nn * sb + 16.0 * (double)p.spl_len, "spline sums launch",
            [&] { return launch_spline(p, signal, out, workspace, st, 0); });
        run(st, spline_kernel_name(p, 1), nn * p.S * eb, "spline taps launch",
            [&] { return launch_spline(p, signal, out, workspace, st, 1); });
        if (!bare) note_use(p, st);
        return CWT_OK;
    }
    const double fb = p.precision == CWT_FP64 ? 16.0 : 8.0;
    if (!p.segs.empty()) {
        static const char *what[4] = {"local launch", "segment spectra launch", "segment reduce launch",
                                      "segment inverse launch"};
        BatchArgs a{};
        a.i0 = {signal, out, static_cast<char *>(workspace)};
        bool has_local = false, has_band = false;
        for_each_seg_launch(p, [&](const SegKernelId &id, int32_t, int64_t, double) {
            (id.kind == 0 ? has_local : has_band) = true;
        });
        SegStreams ss(st, has_local && has_band && !timing && !p.single_stream && !bare);
        for_each_seg_launch(p, [&](const SegKernelId &id, int32_t key, int64_t blocks, double bytes) {
            a.k0 = p.keys[key];
            hipStream_t ks = ss.of(id.kind);
            run(ks, seg_kernel_id_name(id), bytes, what[id.kind], [&] { return launch_seg_kernel(id, a, blocks, ks); });
        });
        ss.end();
    }
    if (p.M > 0)
        run(st, "forward", nn * sb + (double)p.M * fb, "forward launch",
            [&] { return launch_forward(p, signal, workspace, st); });
    for (auto &g : p.groups)
        run(st, local_kernel_name(p, g), nn * sb + nn * (double)g.scales.size() * eb, "local launch",
            [&] { return launch_local(p, g, signal, out, st); });
    for (auto &c : p.columns) {
        double rows = 0.0, band = 0.0;
        for (size_t i = 0; i < c.items.size(); ++i) {
            const auto &d = c.items[i];
            if (d.r0 != 0) continue;
            rows += d.sb >= 0 ? 2.0 : 1.0;
            band += (double)d.B * fb;
        }
        run(st, column_kernel_name(p, c), band + nn * rows * eb, "column launch",
            [&] { return launch_column(p, c, workspace, out, st); });
    }
    if (!bare) note_use(p, st);
    return CWT_OK;
}

}  // namespace cwt

extern "C" {

int cwt_exec(cwt_plan_t plan, const void *signal, void *out, void *workspace, void *stream) {
    return guarded([&]() -> int { return cwt::exec_impl(plan, signal, out, workspace, stream, false); });
}

}  // extern "C"

namespace cwt {

// Workspace of cwt_exec_scratch: a fixed array in the device memory of every
// GPU the library runs on, held from the library's load until the process
// ends.  Host code never uses its name as an address: the device address is
// looked up once per device (scratch_ptr) and passed to the kernels.
constexpr size_t kScratchBytes = size_t(128) << 20;
static __device__ __align__(256) char scratch[kScratchBytes];

// Device address of `scratch` on the current device, looked up on the first
// call made with that device current.
static void *scratch_ptr() {
    static std::mutex mu;
    static std::map<int, void *> ptrs;
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    std::lock_guard<std::mutex> g(mu);
    auto it = ptrs.find(dev);
    if (it != ptrs.end()) return it->second;
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
        fail(CWT_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    ptrs[dev] = ptr;
    return ptr;
}

}  // namespace cwt

extern "C" {

int cwt_exec_scratch(cwt_plan_t plan, const void *signal, void *out, void *stream) {
    return guarded([&]() -> int {
        if (!plan) cwt::fail(CWT_EINVAL, "plan is NULL");
        const size_t need = plan->p->ws_bytes;
        if (need > cwt::kScratchBytes)
            cwt::fail(CWT_EUNSUPPORTED, "plan needs " + std::to_string(need) + " bytes of workspace; the scratch "
                                        "array holds " + std::to_string(cwt::kScratchBytes));
        void *ws = need ? cwt::scratch_ptr() : nullptr;
        return cwt::exec_impl(plan, signal, out, ws, stream, true);
    });
}

size_t cwt_scratch_bytes(void) { return cwt::kScratchBytes; }

int cwt_plan_timing_enable(cwt_plan_t plan, int32_t on) {
    return guarded([&]() -> int {
        if (!plan) cwt::fail(CWT_EINVAL, "plan is NULL");
        plan->p->timing = on != 0;
        return CWT_OK;
    });
}

int cwt_plan_timing_read(cwt_plan_t plan, int32_t max_kernels, char *names, int64_t *launches, double *ms,
                         double *bytes_per_launch) {
    return guarded([&]() -> int {
        if (!plan) cwt::fail(CWT_EINVAL, "plan is NULL");
        Plan &p = *plan->p;
        std::vector<std::string> keys;
        std::vector<int64_t> cnt;
        std::vector<double> tot, byt;
        for (auto &r : p.timing_recs) {
            HIPCHK(hipEventSynchronize(r.b));
            float t = 0.f;
            HIPCHK(hipEventElapsedTime(&t, r.a, r.b));
            size_t k = 0;
            while (k < keys.size() && keys[k] != r.name) ++k;
            if (k == keys.size()) {
                keys.push_back(r.name);
                cnt.push_back(0);
                tot.push_back(0.0);
                byt.push_back(0.0);
            }
            cnt[k] += 1;
            tot[k] += t;
            byt[k] += r.bytes;
            p.event_pool.push_back(r.a);
            p.event_pool.push_back(r.b);
        }
        p.timing_recs.clear();
        int n = (int)keys.size();
        for (int k = 0; k < n && k < max_kernels; ++k) {
            if (names) {
                std::strncpy(names + 64 * k, keys[k].c_str(), 63);
                names[64 * k + 63] = 0;
            }
            if (launches) launches[k] = cnt[k];
            if (ms) ms[k] = tot[k];
            if (bytes_per_launch) bytes_per_launch[k] = byt[k] / (double)cnt[k];
        }
        return n;
    });
}

namespace cwt {

static size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Layout of a batch workspace: the plans' own workspaces one after the
// other, then the launch tables of the merged segmented launches.
struct BatchLayout {
    std::vector<size_t> ws_off;  // per instance
    size_t tables_off = 0, bytes = 0;
    // merged launches in execution order
    struct Merged {
        SegKernelId id;
        std::vector<BatchRange> ranges;
        int64_t blocks = 0;
        double bytes = 0.0;
        size_t ranges_off = 0, map_off = 0;  // within the tables
    };
    std::vector<Merged> merged;
    size_t insts_off = 0, tables_bytes = 0;
};

static bool seg_plan(const Plan &p) { return p.method == CWT_METHOD_FFT && p.fft_mode == CWT_FFT_SEGMENTED; }

static BatchLayout batch_layout(const cwt_plan_t *plans, int32_t n) {
    BatchLayout bl;
    size_t off = 0;
    bl.ws_off.resize(n);
    std::map<SegKernelId, size_t> index;
    for (int32_t i = 0; i < n; ++i) {
        const Plan &p = *plans[i]->p;
        bl.ws_off[i] = off;
        off = align256(off + p.ws_bytes);
        if (!seg_plan(p)) continue;
        for_each_seg_launch(p, [&](const SegKernelId &id, int32_t key, int64_t blocks, double bytes) {
            if (blocks <= 0) return;
            auto it = index.find(id);
            if (it == index.end()) {
                it = index.emplace(id, bl.merged.size()).first;
                bl.merged.emplace_back();
                bl.merged.back().id = id;
            }
            auto &m = bl.merged[it->second];
            m.ranges.push_back({m.blocks, p.d_keys + key, i, 0});
            m.blocks += blocks;
            m.bytes += bytes;
        });
    }
    // execution order: all local launches, then forward, reduce, inverse
    std::sort(bl.merged.begin(), bl.merged.end(),
              [](const BatchLayout::Merged &x, const BatchLayout::Merged &y) { return x.id < y.id; });
    bl.tables_off = off;
    size_t t = 0;
    bl.insts_off = t;
    t = align256(t + (size_t)n * sizeof(BatchInst));
    for (auto &m : bl.merged) {
        m.ranges_off = t;
        t = align256(t + m.ranges.size() * sizeof(BatchRange));
        m.map_off = t;
        t = align256(t + (size_t)((m.blocks + 255) / 256 + 1) * sizeof(int32_t));
    }
    bl.tables_bytes = t;
    bl.bytes = off + t;
    return bl;
}

}  // namespace cwt

size_t cwt_batch_workspace_bytes(const cwt_plan_t *plans, int32_t n) {
    if (!plans || n <= 0) return 0;
    for (int32_t i = 0; i < n; ++i)
        if (!plans[i]) return 0;
    try {
        return cwt::batch_layout(plans, n).bytes;
    } catch (...) {
        return 0;
    }
}

int cwt_exec_batch(const cwt_plan_t *plans, const void *const *signals, void *const *outs, int32_t n,
                   void *workspace, void *stream) {
    return guarded([&]() -> int {
        if (n < 0) cwt::fail(CWT_EINVAL, "n < 0");
        if (n == 0) return CWT_OK;
        if (!plans || !signals || !outs) cwt::fail(CWT_EINVAL, "NULL array");
        for (int32_t i = 0; i < n; ++i) {
            if (!plans[i]) cwt::fail(CWT_EINVAL, "plan is NULL");
            const Plan &p = *plans[i]->p;
            if (p.host_only) cwt::fail(CWT_EINVAL, "plan was built host-only");
            if (!signals[i] || !outs[i]) cwt::fail(CWT_EINVAL, "signal/out is NULL");
            const size_t ealign = p.precision == CWT_FP64 ? 8 : 4;
            if ((uintptr_t)signals[i] % ealign || (uintptr_t)outs[i] % ealign)
                cwt::fail(CWT_EINVAL, "signal/out not aligned to the element size");
        }
        if (!workspace) cwt::fail(CWT_EINVAL, "workspace is NULL");
        if ((uintptr_t)workspace % 256) cwt::fail(CWT_EINVAL, "workspace not 256-byte aligned");
        hipStream_t st = static_cast<hipStream_t>(stream);
        cwt::BatchLayout bl = cwt::batch_layout(plans, n);
        char *ws = static_cast<char *>(workspace);
        char *tables = ws + bl.tables_off;
        if (!bl.merged.empty()) {
            // launch tables, copied in one transfer (the host buffer may be
            // released once the call returns: pageable copies are staged)
            std::vector<char> host(bl.tables_bytes, 0);
            auto *insts = reinterpret_cast<cwt::BatchInst *>(host.data() + bl.insts_off);
            for (int32_t i = 0; i < n; ++i) insts[i] = {signals[i], outs[i], ws + bl.ws_off[i]};
            for (auto &m : bl.merged) {
                std::memcpy(host.data() + m.ranges_off, m.ranges.data(), m.ranges.size() * sizeof(cwt::BatchRange));
                // coarse[c]: the range holding block 256 c (the last range past the end)
                auto *coarse = reinterpret_cast<int32_t *>(host.data() + m.map_off);
                const int64_t nc = (m.blocks + 255) / 256 + 1;
                size_t r = 0;
                for (int64_t c = 0; c < nc; ++c) {
                    const int64_t b = std::min<int64_t>(c * 256, m.blocks - 1);
                    while (r + 1 < m.ranges.size() && m.ranges[r + 1].block0 <= b) ++r;
                    coarse[c] = (int32_t)r;
                }
            }
            HIPCHK(hipMemcpyAsync(tables, host.data(), host.size(), hipMemcpyHostToDevice, st));
            Plan &tp = *plans[0]->p;  // timing records go to the first plan
            bool has_local = false, has_band = false;
            for (auto &m : bl.merged) (m.id.kind == 0 ? has_local : has_band) = true;
            cwt::SegStreams ss(st, has_local && has_band && !tp.timing && !tp.single_stream);
            for (auto &m : bl.merged) {
                cwt::BatchArgs a{};
                a.ranges = reinterpret_cast<const cwt::BatchRange *>(tables + m.ranges_off);
                a.coarse = reinterpret_cast<const int32_t *>(tables + m.map_off);
                a.insts = reinterpret_cast<const cwt::BatchInst *>(tables + bl.insts_off);
                a.nranges = (int32_t)m.ranges.size();
                hipStream_t ks = ss.of(m.id.kind);
                cwt::timed(tp, ks, cwt::seg_kernel_id_name(m.id), m.bytes, "batched segment launch",
                           [&] { return cwt::launch_seg_kernel(m.id, a, m.blocks, ks); });
            }
            ss.end();
            // one event after the merged launches orders the release of every
            // segmented plan of the batch
            if (!cwt::capturing(st)) {
                const auto ev = cwt::record_use(st);
                for (int32_t i = 0; i < n; ++i)
                    if (cwt::seg_plan(*plans[i]->p)) cwt::note_use(*plans[i]->p, st, ev);
            }
        }
        for (int32_t i = 0; i < n; ++i) {
            if (cwt::seg_plan(*plans[i]->p)) continue;
            int rc = cwt_exec(plans[i], signals[i], outs[i], ws + bl.ws_off[i], stream);
            if (rc != CWT_OK) return rc;
        }
        return CWT_OK;
    });
}

int64_t cwt_plan_fft_len(cwt_plan_t plan) { return plan ? plan->p->M : -1; }

int cwt_plan_spline_delta(cwt_plan_t plan, int32_t *delta) {
    if (!plan || !delta) return CWT_EINVAL;
    const Plan &p = *plan->p;
    for (int j = 0; j < p.S; ++j) delta[j] = p.method != CWT_METHOD_FFT ? p.spl_delta[j] : 0;
    return CWT_OK;
}

int cwt_plan_spline_taps(cwt_plan_t plan, int32_t *taps) {
    if (!plan || !taps) return CWT_EINVAL;
    const Plan &p = *plan->p;
    for (int j = 0; j < p.S; ++j) taps[j] = p.method != CWT_METHOD_FFT ? p.spl_ntaps[j] : 0;
    return CWT_OK;
}

double cwt_plan_spline_hstar(cwt_plan_t plan) { return plan ? plan->p->hstar : 0.0; }

int cwt_plan_describe(cwt_plan_t plan, char *buf, size_t size) {
    if (!plan || (!buf && size)) return CWT_EINVAL;
    const Plan &p = *plan->p;
    std::string s;
    char line[256];
    auto add = [&](const char *fmt, auto... a) {
        std::snprintf(line, sizeof line, fmt, a...);
        s += line;
    };
    add("N=%lld S=%d method=%s precision=%s workspace=%zu tables=%zu\n", (long long)p.N, p.S,
        p.method == CWT_METHOD_SPLINE ? "spline"
        : p.method == CWT_METHOD_A19 ? "a19"
        : p.method == CWT_METHOD_V97 ? "v97"
                                     : (p.fft_mode == CWT_FFT_WHOLE ? "fft-whole" : "fft-segmented"),
        p.precision == CWT_FP64 ? "fp64" : "fp32", p.ws_bytes, p.table_bytes);
    for (const auto &g : p.segs)
        add("%s L=%d P=%d B=%d Tg=%lld V=%lld nseg=%lld nchunk=%d iters=%d scales=%zu%s%s\n",
            g.kind == cwt::SegGroup::LOCAL ? "local" : "band", g.L, g.P, g.B, (long long)g.Tg, (long long)g.V,
            (long long)g.nseg, g.nchunk, g.iters, g.scales.size(), g.colpair ? " colpair=1" : "",
            g.cshift ? " shift=1" : "");
    for (const auto &l : p.seg_launches)
        add("launch P=%d groups=%zu forward=%zu reduce=%zu inverse=%zu\n", l.P, l.gdev.size(), l.fwd.size(),
            l.red.size(), l.inv.size());
    if (p.method != CWT_METHOD_FFT) {
        add("spline h*=%.6f E=%lld tiles=%zu\n", p.hstar, (long long)p.spl_E, p.spl_work.size());
        for (int j = 0; j < p.S; ++j)
            add("spline scale=%d delta=%d R=%d I=%d taps=%d exact=%d\n", j, p.spl[j].delta, p.spl[j].R, p.spl[j].I,
                p.spl_ntaps[j], p.spl[j].mode);
    }
    if (size) {
        const size_t n = std::min(size - 1, s.size());
        std::memcpy(buf, s.data(), n);
        buf[n] = 0;
    }
    return (int)std::min<size_t>(s.size(), 0x7fffffff);
}

int cwt_plan_scale_path(cwt_plan_t plan, int32_t *path) {
    if (!plan || !path) return CWT_EINVAL;
    for (int j = 0; j < plan->p->S; ++j) path[j] = plan->p->path[j];
    return CWT_OK;
}

const char *cwt_last_error(void) { return cwt::g_err.c_str(); }

}  // extern "C"

// ---------------------------------------------------------------------------
// statistics epilogue (Sec. 5): environment-dependent and global wavelet
// power spectra of a segmented FFT plan, reduced in the output kernels

namespace cwt {

static bool wps_plan_ok(const Plan &p) {
    return p.method == CWT_METHOD_FFT && p.fft_mode == CWT_FFT_SEGMENTED && !p.segs.empty() && p.psi_mode == CWT_PSI_ALIASED;
}
static size_t wps_part_bytes(const Plan &p) {
    return align256((size_t)(p.wps_base.empty() ? 0 : p.wps_base.back()) * kWpsMaxBins * sizeof(double));
}
static size_t wps_ws_bytes(const Plan &p) {
    return align256(p.ws_bytes) + wps_part_bytes(p) + align256((size_t)kWpsCountBlocks * kWpsMaxBins * sizeof(uint64_t));
}

static int exec_wps_impl(cwt_plan_t plan, const void *signal, const void *env, const double *thr, int32_t nthr,
                         double *wps, int64_t *counts, void *workspace, void *stream) {
    if (!plan) fail(CWT_EINVAL, "plan is NULL");
    Plan &p = *plan->p;
    if (!wps_plan_ok(p))
        fail(CWT_EUNSUPPORTED, "power spectra need a segmented FFT plan with the aliased spectrum (the default)");
    if (p.host_only) fail(CWT_EINVAL, "plan was built host-only");
    if (!signal || !wps) fail(CWT_EINVAL, "signal/wps is NULL");
    if (!workspace) fail(CWT_EINVAL, "workspace is NULL");
    if (nthr < 0 || nthr > kWpsMaxBins - 1)
        fail(CWT_EINVAL, "between 0 and " + std::to_string(kWpsMaxBins - 1) + " thresholds");
    if (nthr > 0 && !thr) fail(CWT_EINVAL, "thresholds is NULL");
    for (int32_t k = 0; k < nthr; ++k) {
        if (!std::isfinite(thr[k])) fail(CWT_EINVAL, "thresholds must be finite");
        if (k > 0 && !(thr[k] > thr[k - 1])) fail(CWT_EINVAL, "thresholds must be strictly ascending");
    }
    if (!env) env = signal;
    const size_t ealign = p.precision == CWT_FP64 ? 8 : 4;
    if ((uintptr_t)signal % ealign || (uintptr_t)env % ealign || (uintptr_t)wps % 8 || (uintptr_t)counts % 8)
        fail(CWT_EINVAL, "signal/env/wps/counts not aligned to their element size");
    if ((uintptr_t)workspace % 256) fail(CWT_EINVAL, "workspace not 256-byte aligned");
    hipStream_t st = static_cast<hipStream_t>(stream);
    char *ws = static_cast<char *>(workspace);
    double *part = reinterpret_cast<double *>(ws + align256(p.ws_bytes));
    uint64_t *cpart = reinterpret_cast<uint64_t *>(ws + align256(p.ws_bytes) + wps_part_bytes(p));
    BatchArgs a{};
    a.i0 = {signal, nullptr, ws, env, part};
    a.wps.nbin = nthr + 1;
    for (int32_t k = 0; k < nthr; ++k) a.wps.thr[k] = thr[k];
    const bool fp64 = p.precision == CWT_FP64;
    const double nn = (double)p.N, sb = fp64 ? 8.0 : 4.0;
    auto run = [&](hipStream_t ks, const std::string &name, double bytes, const char *what, auto &&launch) {
        if (p.timing) {
            timed(p, ks, name, bytes, what, launch);
            return;
        }
        const hipError_t e = launch();
        if (e != hipSuccess) fail(CWT_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
    };
    run(st, "wps_count_kernel", nn * sb, "power spectrum count launch",
        [&] { return launch_wps_count(env, p.N, fp64, a.wps, cpart, st); });
    bool has_local = false, has_band = false;
    for_each_seg_launch(p, [&](const SegKernelId &id, int32_t, int64_t, double) {
        (id.kind == 0 ? has_local : has_band) = true;
    });
    static const char *what[4] = {"local launch", "segment spectra launch", "segment reduce launch",
                                  "segment inverse launch"};
    SegStreams ss(st, has_local && has_band && !p.timing && !p.single_stream);
    for_each_seg_launch(p, [&](const SegKernelId &id, int32_t key, int64_t blocks, double bytes) {
        a.k0 = p.keys[key];
        hipStream_t ks = ss.of(id.kind);
        // the output kernels read the signal (or band spectra) and env, and
        // write one slot of sums per scale and workgroup
        double b = bytes;
        if (id.kind == 0) b = 2.0 * nn * sb;
        for (auto &l : p.seg_launches)
            if (id.kind == 3 && l.key[2] == key) {
                b = nn * sb;
                for (auto &gd : l.gdev) b += (double)gd.nseg * gd.B * 16.0;
            }
        run(ks, seg_kernel_id_name(id, id.kind == 0 || id.kind == 3), b, what[id.kind],
            [&] { return launch_seg_kernel_wps(id, a, blocks, ks); });
    });
    ss.end();
    run(st, "wps_finalize_kernel", (double)p.wps_base.back() * a.wps.nbin * 8.0, "power spectrum finalize launch",
        [&] {
            return launch_wps_finalize(part, p.d_wps_base, p.S, a.wps, cpart, p.N, wps, counts, st);
        });
    note_use(p, st);
    return CWT_OK;
}

}  // namespace cwt

extern "C" {

int cwt_global_wps(cwt_plan_t plan, const void *signal, double *wps, void *workspace, void *stream) {
    return guarded([&]() -> int {
        if (!plan) cwt::fail(CWT_EINVAL, "plan is NULL");
        if (!signal || !wps || !workspace) cwt::fail(CWT_EINVAL, "signal/wps/workspace is NULL");
        cwt::Plan &p = *plan->p;
        if (!p.spec_ok)
            cwt::fail(CWT_EUNSUPPORTED, "cwt_global_wps needs a periodic plan of the FFT method with fft_mode WHOLE, "
                                        "psi_mode ALIASED, a band-limited wavelet and N of the form 2^a * {1,3,5,9}, "
                                        "2^a >= 64, with at least one scale on the whole-signal spectrum");
        if (p.host_only) cwt::fail(CWT_EINVAL, "plan was built host-only");
        if (p.S > 65535) cwt::fail(CWT_EUNSUPPORTED, "cwt_global_wps takes at most 65535 scales");
        const size_t ealign = p.precision == CWT_FP64 ? 8 : 4;
        if ((uintptr_t)signal % ealign || (uintptr_t)wps % 8) cwt::fail(CWT_EINVAL, "signal/wps misaligned");
        if ((uintptr_t)workspace % 256) cwt::fail(CWT_EINVAL, "workspace not 256-byte aligned");
        hipStream_t st = static_cast<hipStream_t>(stream);
        hipError_t e = cwt::launch_forward(p, signal, workspace, st);
        if (e != hipSuccess) cwt::fail(CWT_EDEVICE, std::string("forward launch: ") + hipGetErrorString(e));
        char *w = static_cast<char *>(workspace);
        e = cwt::launch_parseval_wps(p.spec_w, w + p.ws_F_off, p.M, p.d_scales64, p.S,
                                     reinterpret_cast<double *>(w + p.ws_pars_off), wps, p.precision == CWT_FP64, st);
        if (e != hipSuccess) cwt::fail(CWT_EDEVICE, std::string("Parseval launch: ") + hipGetErrorString(e));
        cwt::note_use(p, st);
        return CWT_OK;
    });
}

size_t cwt_wps_workspace_bytes(cwt_plan_t plan) {
    if (!plan || !cwt::wps_plan_ok(*plan->p)) return 0;
    return cwt::wps_ws_bytes(*plan->p);
}

int cwt_exec_wps(cwt_plan_t plan, const void *signal, const void *env, const double *thresholds, int32_t nthr,
                 double *wps, int64_t *counts, void *workspace, void *stream) {
    return guarded([&]() -> int {
        return cwt::exec_wps_impl(plan, signal, env, thresholds, nthr, wps, counts, workspace, stream);
    });
}

}  // extern "C"
