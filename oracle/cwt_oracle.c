/*
 * cwt_oracle.c -- plain, slow FP64 CPU oracle for the multi-scale 1D CWT.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code, header, table or constant generator
 * with the HIP library.
 *
 * What it computes
 * ----------------
 * (1) The canonical transform, as the unit-step Riemann sum of
 *         W(s,b) = (1/s) * integral f(x) conj(psi((x-b)/s)) dx
 *     over the samples (Sec. 3, Eq. discreteCWT, re-normalised to the
 *     1/s correlation form):
 *         W[j,b] = (1/s_j) * sum_{t=-T..T} f_ext[b+t] * conj(psi(t/s_j))
 *     f_ext is the periodic extension (periodic boundary) or the zero
 *     extension (zero boundary).  T = floor(chi * s_j), where chi is the
 *     radius beyond which |psi| < rel * max|psi| (Table 2 truncates the
 *     non-compact wavelets the same way, at a fixed small level).  psi is
 *     evaluated in the time domain with libm exp/cos/sin.  Each output is a
 *     pairwise sum, so the rounding error grows like log2(2T+1).
 *
 * (2) The exact target of the spline method (Sec. 3.3, Eqs. beta3_signal
 *     and beta3_wavelet_approx_m02): with f_c = sum_n c[n] beta3(u-n) the
 *     cubic-spline interpolant of the signal and
 *     psi_h(y) = sum_k d[k] beta3(y/h - k) the spline approximation of the
 *     wavelet at step h,
 *         W_spl(s,x) = (1/s) * integral f_c(u) conj(psi_h((u-x)/s)) du.
 *     The knots of f_c are the integers and those of psi_h((u-x)/s) are
 *     x + s h k, k integer.  Between two consecutive knots of the merged set
 *     the integrand is a polynomial of degree 6, so 4-point Gauss-Legendre
 *     quadrature on each such piece is exact.  oracle_spline_target takes
 *     an integer knot step s h = delta (every knot an integer, one piece per
 *     unit interval); oracle_spline_target_step takes any real step s h.
 *
 * Wavelets (unit L2 norm; FT convention psi^(w) = int psi(x) e^{-iwx} dx):
 *   kind 0  Morlet(w0): C (e^{i w0 x} - e^{-w0^2/2}) e^{-x^2/2},
 *           C = pi^{-1/4} (1 + e^{-w0^2} - 2 e^{-3 w0^2/4})^{-1/2}.
 *           The subtracted constant makes psi^(0) = 0, as in the corrected
 *           Morlet wavelet of Table 2 (there with w0 = 4, conjugated because
 *           the paper's FT uses e^{+ikx}).
 *   kind 1  DOG(m): (-1)^{m+1} Gamma(m+1/2)^{-1/2} d^m/dx^m e^{-x^2/2}
 *           = -He_m(x) e^{-x^2/2} / sqrt(Gamma(m+1/2)), He_m the
 *           probabilists' Hermite polynomial.  m = 2 is the Mexican hat.
 *   The wavelets of Table 2 (the MW there is kind 0 with w0 = -4):
 *   kind 2  CBSW   sqrt(30/31) (2 beta3(x) - beta3(x+1) - beta3(x-1))
 *   kind 3  GDW    (18 pi)^{-1/4} (2 - x^2) e^{-x^2/4}
 *   kind 4  CW-GDW sqrt(8/(1+5e)) pi^{-1/4} ((1-x^2) cos x - x sin x)
 *                  e^{(1-x^2)/2}
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_MORLET 0
#define ORC_DOG 1
#define ORC_CBSW 2
#define ORC_GDW 3
#define ORC_CWGDW 4
#define ORC_PERIODIC 0
#define ORC_ZERO 1

static double beta3(double x);

/* Mother wavelet in the time domain. */
static void psi_eval(int kind, double p, double x, double *re, double *im) {
    if (kind == ORC_CBSW) {
        *re = sqrt(30.0 / 31.0) * (2.0 * beta3(x) - beta3(x + 1.0) - beta3(x - 1.0));
        *im = 0.0;
        return;
    }
    if (kind == ORC_GDW) {
        *re = pow(18.0 * M_PI, -0.25) * (2.0 - x * x) * exp(-0.25 * x * x);
        *im = 0.0;
        return;
    }
    if (kind == ORC_CWGDW) {
        *re = sqrt(8.0 / (1.0 + 5.0 * exp(1.0))) * pow(M_PI, -0.25) *
              ((1.0 - x * x) * cos(x) - x * sin(x)) * exp(0.5 * (1.0 - x * x));
        *im = 0.0;
        return;
    }
    if (kind == ORC_MORLET) {
        double w0 = p;
        double C = pow(M_PI, -0.25) /
                   sqrt(1.0 + exp(-w0 * w0) - 2.0 * exp(-0.75 * w0 * w0));
        double g = exp(-0.5 * x * x);
        *re = C * (cos(w0 * x) - exp(-0.5 * w0 * w0)) * g;
        *im = C * sin(w0 * x) * g;
    } else {
        int m = (int)p;
        double hm1 = 1.0, h = x; /* He_0, He_1 */
        if (m == 0) h = 1.0;
        for (int n = 1; n < m; ++n) {
            double hn = x * h - n * hm1; /* He_{n+1} = x He_n - n He_{n-1} */
            hm1 = h;
            h = hn;
        }
        *re = -h * exp(-0.5 * x * x) / sqrt(tgamma(m + 0.5));
        *im = 0.0;
    }
}

/* Second derivative of the smooth wavelets (kinds 0, 1, 3, 4), written out
 * by differentiating the forms above twice:
 *   Morlet: C e^{-x^2/2} [e^{i w0 x}(x^2 - 2 i w0 x - w0^2 - 1) - e^{-w0^2/2}(x^2 - 1)]
 *   DOG(m): -Gamma(m+1/2)^{-1/2} He_{m+2}(x) e^{-x^2/2}
 *   GDW:    C e^{-x^2/4} [2 x^2 - 2 - (x^2 - 2)^2 / 4]
 *   CW-GDW: C e^{(1-x^2)/2} [q2 - 2 x q1 + (x^2 - 1) q0] with
 *           q0 = (1 - x^2) cos x - x sin x, q1 = -3 x cos x - (2 - x^2) sin x,
 *           q2 = (x^2 - 5) cos x + 5 x sin x */
static void psi2_eval(int kind, double p, double x, double *re, double *im) {
    *im = 0.0;
    if (kind == ORC_MORLET) {
        double w0 = p;
        double C = pow(M_PI, -0.25) /
                   sqrt(1.0 + exp(-w0 * w0) - 2.0 * exp(-0.75 * w0 * w0));
        double g = exp(-0.5 * x * x), k = exp(-0.5 * w0 * w0);
        double ar = x * x - w0 * w0 - 1.0, ai = -2.0 * w0 * x;
        double c = cos(w0 * x), s = sin(w0 * x);
        *re = C * g * (c * ar - s * ai - k * (x * x - 1.0));
        *im = C * g * (c * ai + s * ar);
    } else if (kind == ORC_GDW) {
        double u = x * x - 2.0;
        *re = pow(18.0 * M_PI, -0.25) * exp(-0.25 * x * x) * (2.0 * x * x - 2.0 - 0.25 * u * u);
    } else if (kind == ORC_CWGDW) {
        double c = cos(x), s = sin(x);
        double q0 = (1.0 - x * x) * c - x * s;
        double q1 = -3.0 * x * c - (2.0 - x * x) * s;
        double q2 = (x * x - 5.0) * c + 5.0 * x * s;
        *re = sqrt(8.0 / (1.0 + 5.0 * exp(1.0))) * pow(M_PI, -0.25) * exp(0.5 * (1.0 - x * x)) *
              (q2 - 2.0 * x * q1 + (x * x - 1.0) * q0);
    } else if (kind == ORC_DOG) {
        int m = (int)p + 2;
        double hm1 = 1.0, h = x;
        for (int n = 1; n < m; ++n) {
            double hn = x * h - n * hm1;
            hm1 = h;
            h = hn;
        }
        *re = -h * exp(-0.5 * x * x) / sqrt(tgamma(p + 0.5));
    } else {
        *re = NAN;
    }
}

int oracle_psi2(int kind, double p, const double *x, long n, double *re, double *im) {
    for (long i = 0; i < n; ++i) psi2_eval(kind, p, x[i], &re[i], &im[i]);
    return 0;
}

int oracle_psi(int kind, double p, const double *x, long n, double *re,
               double *im) {
    for (long i = 0; i < n; ++i) psi_eval(kind, p, x[i], &re[i], &im[i]);
    return 0;
}

/* Radius chi such that |psi(x)| < rel * max|psi| for every |x| > chi.
 * Scans a 1/4096 grid on [0, 64]; all supported wavelets are symmetric in
 * modulus and decay like a Gaussian, so the last grid point above the
 * level plus one grid step bounds the radius. */
double oracle_chi(int kind, double p, double rel) {
    const double step = 1.0 / 4096.0;
    const long n = 64 * 4096;
    double mx = 0.0, re, im;
    for (long i = 0; i <= n; ++i) {
        psi_eval(kind, p, i * step, &re, &im);
        double a = hypot(re, im);
        if (a > mx) mx = a;
    }
    double last = 0.0;
    for (long i = 0; i <= n; ++i) {
        psi_eval(kind, p, i * step, &re, &im);
        if (hypot(re, im) >= rel * mx) last = i * step;
    }
    return last + step;
}

static double pw_sum(const double *a, long n) {
    if (n <= 16) {
        double s = 0.0;
        for (long i = 0; i < n; ++i) s += a[i];
        return s;
    }
    long h = n / 2;
    return pw_sum(a, h) + pw_sum(a + h, n - h);
}

static long wrap(long i, long N) {
    long r = i % N;
    return r < 0 ? r + N : r;
}

typedef struct {
    long T;
    double *kr, *ki; /* conj(psi(t/s))/s for t in [-T, T], index t+T */
} scale_kernel;

static void make_kernel(scale_kernel *k, int kind, double p, double s,
                        double chi) {
    k->T = (long)floor(chi * s);
    long L = 2 * k->T + 1;
    k->kr = (double *)malloc(sizeof(double) * L);
    k->ki = (double *)malloc(sizeof(double) * L);
    for (long t = -k->T; t <= k->T; ++t) {
        double re, im;
        psi_eval(kind, p, (double)t / s, &re, &im);
        k->kr[t + k->T] = re / s;
        k->ki[t + k->T] = -im / s;
    }
}

/* One output W[s,b] from a precomputed kernel; bufr/bufi hold 2T+1 doubles. */
static void one_output(const double *f, long N, int boundary,
                       const scale_kernel *k, long b, double *bufr,
                       double *bufi, double *wr, double *wi) {
    long L = 2 * k->T + 1;
    for (long t = -k->T; t <= k->T; ++t) {
        long i = b + t;
        double v;
        if (boundary == ORC_PERIODIC)
            v = f[wrap(i, N)];
        else
            v = (i >= 0 && i < N) ? f[i] : 0.0;
        bufr[t + k->T] = v * k->kr[t + k->T];
        bufi[t + k->T] = v * k->ki[t + k->T];
    }
    *wr = pw_sum(bufr, L);
    *wi = pw_sum(bufi, L);
}

/* Full transform: out_re/out_im are [S][N] row-major (out_im may be NULL
 * for a real wavelet).  rel is the truncation level for chi. */
int oracle_cwt(const double *f, long N, int boundary, int kind, double p,
               const double *scales, int S, double rel, double *out_re,
               double *out_im, int nthreads) {
    double chi = oracle_chi(kind, p, rel);
    scale_kernel *ks = (scale_kernel *)malloc(sizeof(scale_kernel) * S);
    long Tmax = 0;
    for (int j = 0; j < S; ++j) {
        make_kernel(&ks[j], kind, p, scales[j], chi);
        if (ks[j].T > Tmax) Tmax = ks[j].T;
    }
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel
    {
        double *br = (double *)malloc(sizeof(double) * (2 * Tmax + 1));
        double *bi = (double *)malloc(sizeof(double) * (2 * Tmax + 1));
#pragma omp for schedule(dynamic, 64)
        for (long o = 0; o < (long)S * N; ++o) {
            int j = (int)(o / N);
            long b = o % N;
            double wr, wi;
            one_output(f, N, boundary, &ks[j], b, br, bi, &wr, &wi);
            out_re[o] = wr;
            if (out_im) out_im[o] = wi;
        }
        free(br);
        free(bi);
    }
    for (int j = 0; j < S; ++j) {
        free(ks[j].kr);
        free(ks[j].ki);
    }
    free(ks);
    return 0;
}

/* Selected outputs: W[scale_idx[i], pos[i]] for i < npts. */
int oracle_cwt_points(const double *f, long N, int boundary, int kind,
                      double p, const double *scales, int S, double rel,
                      const int *scale_idx, const long *pos, long npts,
                      double *out_re, double *out_im, int nthreads) {
    double chi = oracle_chi(kind, p, rel);
    scale_kernel *ks = (scale_kernel *)calloc(S, sizeof(scale_kernel));
    char *used = (char *)calloc(S, 1);
    for (long i = 0; i < npts; ++i) used[scale_idx[i]] = 1;
    long Tmax = 0;
    for (int j = 0; j < S; ++j) {
        if (!used[j]) continue;
        make_kernel(&ks[j], kind, p, scales[j], chi);
        if (ks[j].T > Tmax) Tmax = ks[j].T;
    }
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel
    {
        double *br = (double *)malloc(sizeof(double) * (2 * Tmax + 1));
        double *bi = (double *)malloc(sizeof(double) * (2 * Tmax + 1));
#pragma omp for schedule(dynamic, 16)
        for (long i = 0; i < npts; ++i) {
            double wr, wi;
            one_output(f, N, boundary, &ks[scale_idx[i]], pos[i], br, bi, &wr,
                       &wi);
            out_re[i] = wr;
            if (out_im) out_im[i] = wi;
        }
        free(br);
        free(bi);
    }
    for (int j = 0; j < S; ++j) {
        if (!used[j]) continue;
        free(ks[j].kr);
        free(ks[j].ki);
    }
    free(ks);
    free(used);
    return 0;
}

/* ---------------------------------------------------------------------- */
/* Spline-method exact target.                                             */

/* Cubic B-spline (App. B, Eq. betan with n = 3): support [-2, 2]. */
static double beta3(double x) {
    double a = fabs(x);
    if (a >= 2.0) return 0.0;
    if (a >= 1.0) {
        double u = 2.0 - a;
        return u * u * u / 6.0;
    }
    return 2.0 / 3.0 - a * a + 0.5 * a * a * a;
}

/* c[n] for n in [c0, c0 + nc), zero outside. */
static double coef(const double *c, long c0, long nc, long n) {
    long i = n - c0;
    return (i >= 0 && i < nc) ? c[i] : 0.0;
}

/*
 * W_spl(s, x) for the positions x[i] (integers).  c: spline coefficients of
 * the signal on [c0, c0+nc) (the caller extends them periodically when the
 * boundary is periodic).  d_re/d_im: wavelet spline coefficients d[k] for
 * k in [-Nd, Nd].  delta = s*h (a positive integer).
 */
int oracle_spline_target(const double *c, long c0, long nc,
                         const double *d_re, const double *d_im, long Nd,
                         long delta, double s, const long *x, long nx,
                         double *out_re, double *out_im, int nthreads) {
    static const double gx[4] = {-0.8611363115940526, -0.3399810435848563,
                                 0.3399810435848563, 0.8611363115940526};
    static const double gw[4] = {0.3478548451374538, 0.6521451548625461,
                                 0.6521451548625461, 0.3478548451374538};
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
    long half = (Nd + 2) * delta; /* support radius of psi_h((u-x)/s) */
    long nint = 2 * half;
#pragma omp parallel
    {
        double *tr = (double *)malloc(sizeof(double) * nint * 4);
        double *ti = (double *)malloc(sizeof(double) * nint * 4);
#pragma omp for schedule(dynamic, 8)
        for (long i = 0; i < nx; ++i) {
            long xi = x[i];
            long cnt = 0;
            /* coordinates relative to the output: v = u - x, so that no
             * large position enters a spline argument */
            for (long n = -half; n < half; ++n) {
                for (int q = 0; q < 4; ++q) {
                    double v = n + 0.5 * (1.0 + gx[q]);
                    /* f_c(x + v): c[x + m] beta3(v - m), m in [n-1, n+2] */
                    double fc = 0.0;
                    for (long m = n - 1; m <= n + 2; ++m)
                        fc += coef(c, c0, nc, xi + m) * beta3(v - (double)m);
                    /* psi_h(v/s) = sum_k d[k] beta3(v/delta - k) */
                    double y = v / (double)delta;
                    long k0 = (long)floor(y) - 1;
                    double pr = 0.0, pi = 0.0;
                    for (long k = k0; k <= k0 + 3; ++k) {
                        if (k < -Nd || k > Nd) continue;
                        double b = beta3(y - (double)k);
                        pr += d_re[k + Nd] * b;
                        pi += d_im[k + Nd] * b;
                    }
                    double w = 0.5 * gw[q] / s;
                    /* f_c * conj(psi_h) */
                    tr[cnt] = w * fc * pr;
                    ti[cnt] = -w * fc * pi;
                    ++cnt;
                }
            }
            out_re[i] = pw_sum(tr, cnt);
            out_im[i] = pw_sum(ti, cnt);
        }
        free(tr);
        free(ti);
    }
    return 0;
}

/*
 * W_spl(s, x) for a real knot step `step` = s h of the wavelet spline (any
 * step > 0, in samples).  Arguments as for oracle_spline_target.  For each
 * output the integration range |u - x| <= (Nd + 2) step is cut at the
 * integers and at the points x + step k; every piece gets 4-point
 * Gauss-Legendre nodes, and the two cubic splines are evaluated there from
 * the knot interval that holds the piece's midpoint.
 */
int oracle_spline_target_step(const double *c, long c0, long nc,
                              const double *d_re, const double *d_im, long Nd,
                              double step, double s, const long *x, long nx,
                              double *out_re, double *out_im, int nthreads) {
    static const double gx[4] = {-0.8611363115940526, -0.3399810435848563,
                                 0.3399810435848563, 0.8611363115940526};
    static const double gw[4] = {0.3478548451374538, 0.6521451548625461,
                                 0.6521451548625461, 0.3478548451374538};
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
    const double half = (double)(Nd + 2) * step; /* support radius */
    const long maxpieces = 2 * (long)ceil(half) + 2 * (Nd + 2) + 8;
#pragma omp parallel
    {
        double *tr = (double *)malloc(sizeof(double) * maxpieces * 4);
        double *ti = (double *)malloc(sizeof(double) * maxpieces * 4);
#pragma omp for schedule(dynamic, 8)
        for (long i = 0; i < nx; ++i) {
            /* coordinates relative to the output, v = u - x (x is an
             * integer, so the integer knots stay integers) */
            const long xi = x[i];
            const double lo = -half, hi = half;
            /* two sorted knot sequences: integers in (lo, hi), and
             * step k for k = -(Nd+2)..Nd+2 (the first and last are lo and
             * hi themselves) */
            long nint = (long)floor(lo) + 1; /* next integer above lo */
            long k = -(Nd + 2) + 1;
            double a = lo;
            long cnt = 0;
            while (a < hi) {
                double bi = (double)nint;
                double bk = (k <= Nd + 2) ? step * (double)k : hi;
                double b = bi < bk ? bi : bk;
                if (b > hi) b = hi;
                if (bi <= b) ++nint;
                if (bk <= b) ++k;
                if (b > a) {
                    const double mid = 0.5 * (a + b), hw = 0.5 * (b - a);
                    const long nf = (long)floor(mid);
                    const long kf = (long)floor(mid / step);
                    for (int q = 0; q < 4; ++q) {
                        const double v = mid + hw * gx[q];
                        double fc = 0.0;
                        for (long m = nf - 1; m <= nf + 2; ++m)
                            fc += coef(c, c0, nc, xi + m) * beta3(v - (double)m);
                        const double y = v / step;
                        double pr = 0.0, pi = 0.0;
                        for (long kk = kf - 1; kk <= kf + 2; ++kk) {
                            if (kk < -Nd || kk > Nd) continue;
                            const double bb = beta3(y - (double)kk);
                            pr += d_re[kk + Nd] * bb;
                            pi += d_im[kk + Nd] * bb;
                        }
                        const double wq = hw * gw[q] / s;
                        tr[cnt] = wq * fc * pr;
                        ti[cnt] = -wq * fc * pi;
                        ++cnt;
                    }
                }
                a = b;
            }
            out_re[i] = pw_sum(tr, cnt);
            out_im[i] = pw_sum(ti, cnt);
        }
        free(tr);
        free(ti);
    }
    return 0;
}

/*
 * CWT of the spline interpolant f_c with a piecewise-cubic wavelet given on
 * np pieces of width dy starting at y0: on piece k (y in [y0 + k dy,
 * y0 + (k+1) dy), t = y - y0 - k dy) the wavelet is sum_i a[4k+i] t^i
 * (complex: a_re, a_im), zero outside.  W(s, x) = (1/s) int f_c(x + v)
 * conj(psi(v/s)) dv over the merged knots (integers and s (y0 + k dy)),
 * 4-point Gauss-Legendre per piece, in coordinates relative to the output.
 */
int oracle_pp_target(const double *c, long c0, long nc, const double *a_re,
                     const double *a_im, long np, double y0, double dy,
                     double s, const long *x, long nx, double *out_re,
                     double *out_im, int nthreads) {
    static const double gx[4] = {-0.8611363115940526, -0.3399810435848563,
                                 0.3399810435848563, 0.8611363115940526};
    static const double gw[4] = {0.3478548451374538, 0.6521451548625461,
                                 0.6521451548625461, 0.3478548451374538};
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
    const double lo = s * y0, hi = s * (y0 + dy * (double)np);
    const long maxpieces = (long)ceil(hi - lo) + np + 8;
#pragma omp parallel
    {
        double *tr = (double *)malloc(sizeof(double) * maxpieces * 4);
        double *ti = (double *)malloc(sizeof(double) * maxpieces * 4);
#pragma omp for schedule(dynamic, 8)
        for (long i = 0; i < nx; ++i) {
            const long xi = x[i];
            long nint = (long)floor(lo) + 1;
            long k = 1; /* next wavelet knot: s (y0 + k dy) */
            double a = lo;
            long cnt = 0;
            while (a < hi) {
                double bi = (double)nint;
                double bk = (k < np) ? s * (y0 + dy * (double)k) : hi;
                double b = bi < bk ? bi : bk;
                if (b > hi) b = hi;
                if (bi <= b) ++nint;
                if (bk <= b) ++k;
                if (b > a) {
                    const double mid = 0.5 * (a + b), hw = 0.5 * (b - a);
                    const long nf = (long)floor(mid);
                    long kp = (long)floor((mid / s - y0) / dy);
                    if (kp < 0) kp = 0;
                    if (kp >= np) kp = np - 1;
                    for (int q = 0; q < 4; ++q) {
                        const double v = mid + hw * gx[q];
                        double fc = 0.0;
                        for (long m = nf - 1; m <= nf + 2; ++m)
                            fc += coef(c, c0, nc, xi + m) * beta3(v - (double)m);
                        const double t = v / s - y0 - dy * (double)kp;
                        const double *ar = a_re + 4 * kp, *ai = a_im + 4 * kp;
                        const double pr = ((ar[3] * t + ar[2]) * t + ar[1]) * t + ar[0];
                        const double pi = ((ai[3] * t + ai[2]) * t + ai[1]) * t + ai[0];
                        const double wq = hw * gw[q] / s;
                        tr[cnt] = wq * fc * pr;
                        ti[cnt] = -wq * fc * pi;
                        ++cnt;
                    }
                }
                a = b;
            }
            out_re[i] = pw_sum(tr, cnt);
            out_im[i] = pw_sum(ti, cnt);
        }
        free(tr);
        free(ti);
    }
    return 0;
}

/*
 * W[b] = sum_{t=-T..T} f_ext[b + t] k[t + T] at the positions pos[i]: a
 * direct sum with given kernel taps (complex: kr, ki), f_ext the periodic or
 * zero extension.  Pairwise summation, as for the transform above.
 */
int oracle_kernel_sum(const double *f, long N, int boundary, const double *kr,
                      const double *ki, long T, const long *pos, long npos,
                      double *out_re, double *out_im, int nthreads) {
    scale_kernel k;
    k.T = T;
    k.kr = (double *)kr;
    k.ki = (double *)ki;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel
    {
        double *br = (double *)malloc(sizeof(double) * (2 * T + 1));
        double *bi = (double *)malloc(sizeof(double) * (2 * T + 1));
#pragma omp for schedule(dynamic, 16)
        for (long i = 0; i < npos; ++i)
            one_output(f, N, boundary, &k, pos[i], br, bi, &out_re[i], &out_im[i]);
        free(br);
        free(bi);
    }
    return 0;
}
