/*
 * cwt.h -- C ABI of the MI355X (gfx950) multi-scale 1D continuous wavelet
 * transform library (libcwt.so).
 *
 * The transform (Sec. 2, Eq. CWT, in the 1/s correlation form) is
 *
 *     W(s, b) = (1/s) * integral f(x) conj(psi((x - b)/s)) dx,
 *
 * evaluated on the samples as the unit-step sum (Sec. 3, Eq. discreteCWT):
 *
 *     W[j, b] = (1/s_j) * sum_t f_ext[b + t] * conj(psi(t / s_j)),
 *
 * b = 0..N-1, with f_ext the periodic extension (CWT_PERIODIC) or the zero
 * extension (CWT_ZERO) of the signal.  Scales s_j and positions b are in
 * samples.  Four methods are offered:
 *
 *   CWT_METHOD_FFT    -- FFTCWT (Sec. 3.1, Eqs. FT_signal and
 *                        discrete_CWT_conv): one FFT of the signal, then per
 *                        scale a spectral multiply by the conjugate of the
 *                        sampled wavelet's spectrum and an inverse FFT.  The
 *                        result equals the sum above up to rounding and the
 *                        truncation level of the plan's precision.
 *   CWT_METHOD_SPLINE -- the O(N)-per-scale spline method of Sec. 3.3 (Eqs.
 *                        beta3_wavelet_approx_m02, beta3_signal, m02_cwt,
 *                        cumsum4_coeffs): the exact CWT of the cubic-spline
 *                        interpolant of the samples with the cubic-spline
 *                        approximation of the wavelet at step h_s <= h*, h*
 *                        the step where the approximation error of Eq.
 *                        m02cwt_error is 5e-4 (Sec. 3.6, Table 3; the
 *                        wavelet's truncation radius taken where |psi| falls
 *                        below 1e-14 of its maximum).  Where h* s >= 1,
 *                        h_s = delta_s / s with the whole-sample knot
 *                        spacing delta_s = floor(h* s), and the tap sum runs
 *                        on the running sums of Eq. cumsum4_coeffs, taken
 *                        exactly (128-bit fixed point); where h* s < 1,
 *                        h_s = h* (knots between samples) and the output is
 *                        a sum of exact taps over the interpolant's
 *                        coefficients.  The wavelet coefficients d_s
 *                        interpolate psi(h_s k), |k| <= N_d with N_d =
 *                        ceil(chi / h_s - 2) + 2, chi at 1e-17.  The result
 *                        matches that exact spline CWT to FP64 rounding at
 *                        any N; the output is FP64 or FP32 (precision), the
 *                        arithmetic FP64.
 *
 *   CWT_METHOD_A19    -- the A19CWT of Sec. 3.4 (Eqs. a19cwt_01 - a19cwt_04):
 *                        the wavelet approximated by piecewise cubics on
 *                        uniform knots whose third derivative on each piece
 *                        is the difference quotient of psi'' between the
 *                        knots (Eq. 3rd_derivative_wavelet).  Undoing the
 *                        integration by parts of Eq. a19cwt_03, the method
 *                        computes the CWT of the cubic-spline interpolant of
 *                        the samples with that C^2 piecewise cubic, whose B-
 *                        spline coefficients are h^2 times the double running
 *                        sum of psi''(h k).  The knot step is chi / N_chi, N_chi
 *                        the smallest count whose interpolating cubic meets
 *                        AE_A = 5e-4 (Eq. a19cwt_error, Sec. 3.6), chi where
 *                        |psi| falls below 1e-14 of its maximum, and per scale
 *                        the step follows the spline method's rule (whole-sample
 *                        knots where h s >= 1, exact taps below); the same
 *                        kernels run it, with the same exactness.
 *   CWT_METHOD_V97    -- the V97CWT of Sec. 3.2 (Eqs. beta3_wavelet_approx -
 *                        fir_filter_qi): the unit-step sum with the wavelet
 *                        at scale s = 2^i r / w~_max (1 <= r < 2) replaced by
 *                        sum_k p_r(k) beta3(t / 2^i - k), p_r = q_r * q12,
 *                        q_r(k) the integral of psi(w~_max y / r) over the cell
 *                        [k - 1/2, k + 1/2] (Eq. qj) and q12 the inverse filter
 *                        of the sampled quartic B-spline (Eq. q_12), w~_max =
 *                        1.34 c_w (Table 3); computed as the filter chain of
 *                        Eqs. fir_filter_beta - fir_filter_qi per octave level
 *                        i.  Scales below 1 / w~_max are rejected
 *                        (CWT_EUNSUPPORTED); arithmetic FP64.
 *
 * Wavelets (unit L2 norm, psi^(w) = int psi(x) e^{-iwx} dx):
 *   CWT_MORLET(w0): C (e^{i w0 x} - e^{-w0^2/2}) e^{-x^2/2} (complex output;
 *                   the corrected Morlet wavelet of Table 2, conjugated)
 *   CWT_MEXHAT:     DOG(2) (real output)
 *   CWT_DOG(m):     (-1)^{m+1} Gamma(m+1/2)^{-1/2} d^m/dx^m e^{-x^2/2} (real)
 *
 * Conventions for every entry point:
 *   - Return 0 on success or a negative CWT_E* code; no C++ exception ever
 *     crosses this interface.  cwt_last_error() returns a thread-local text
 *     for the last failure of the calling thread.
 *   - Device pointers are HIP device allocations on the current device.
 *     The caller owns signal, output and workspace memory; the library owns
 *     only the plan's small constant tables (allocated by cwt_plan, freed by
 *     cwt_destroy).
 *   - `stream` is a hipStream_t (NULL = the default stream).  Execution is
 *     asynchronous on that stream; buffers must stay alive until the stream
 *     has finished the work.
 *   - A plan is immutable after creation and may be used concurrently from
 *     several streams, provided each concurrent call gets its own workspace.
 */
#ifndef CWT_H
#define CWT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CWT_OK 0
#define CWT_EINVAL (-1)       /* invalid argument */
#define CWT_EUNSUPPORTED (-2) /* valid but outside this library's limits */
#define CWT_ENOMEM (-3)       /* host or device allocation failed */
#define CWT_EDEVICE (-4)      /* HIP runtime error */

#define CWT_PERIODIC 0
#define CWT_ZERO 1

#define CWT_MORLET 0
#define CWT_MEXHAT 1
#define CWT_DOG 2
/* The four wavelets of Table 2 (unit L2 norm, real ones even):
 *   CWT_CBSW   cubic B-spline wavelet  C_N (2 beta3(x) - beta3(x+1) - beta3(x-1)),
 *              C_N = sqrt(30/31); its spectrum 64 C_N sin^6(u/2)/u^4 is not
 *              band-limited, so the FFT method takes it only with
 *              CWT_FFT_WHOLE and CWT_PSI_ANALYTIC, and the spline method not
 *              at all (CWT_EUNSUPPORTED)
 *   CWT_GDW    Gaussian-derived wavelet C_N (2 - x^2) e^{-x^2/4}
 *   CWT_CWGDW  cosine-weighted GDW      C_N ((1-x^2) cos x - x sin x) e^{(1-x^2)/2}
 *   CWT_MW     Morlet wavelet           C_N (e^{-4ix} - e^{-8}) e^{-x^2/2}
 *              (complex output; CWT_MORLET with omega0 = -4)
 * `param` is ignored for these four. */
#define CWT_CBSW 3
#define CWT_GDW 4
#define CWT_CWGDW 5
#define CWT_MW 6

#define CWT_FP64 0 /* FP64 signal, FP64 output, FP64 arithmetic */
#define CWT_FP32 1 /* FP32 signal and output; FP32 inverse FFTs and products;
                      FP64 forward transform of the whole signal, FP64
                      twiddles and wavelet spectra, FP64 spline sums */

#define CWT_METHOD_FFT 0
#define CWT_METHOD_SPLINE 1
#define CWT_METHOD_A19 2
#define CWT_METHOD_V97 3

/* How the FFT method organises the transform:
 *   CWT_FFT_SEGMENTED -- overlap-save segments of L samples per group of
 *                        scales (L = 2^l about 8x the wavelet half-support, or
 *                        for the larger scales the length c 2^k, c odd, that
 *                        computes the fewest positions); each
 *                        segment's spectrum is taken once per group, only on
 *                        the band the group's wavelets occupy, and inverted
 *                        per scale with short band-limited FFTs.
 *   CWT_FFT_WHOLE     -- the transform as written in Sec. 3.1: one FFT of
 *                        the whole (zero- or wrap-padded) signal, then per
 *                        scale a band-limited inverse of length M. */
#define CWT_FFT_SEGMENTED 0
#define CWT_FFT_WHOLE 1

/* Which spectrum of the wavelet the FFT method multiplies by:
 *   CWT_PSI_ALIASED  -- Psi_s(w) = sum_q psi^(s (w + 2 pi q)), the transform of
 *                       the sampled wavelet: the result is the unit-step sum
 *                       of Sec. 3, Eq. discreteCWT (the library's transform);
 *   CWT_PSI_ANALYTIC -- psi^(s w) alone at every DFT bin w = 2 pi m / M,
 *                       |m| <= M/2: Eq. discrete_CWT_conv as written in
 *                       Sec. 3.1.  It differs from the sum by the aliasing
 *                       images, large at small scales.  FFT method with
 *                       CWT_FFT_WHOLE only (every scale is a band-limited
 *                       inverse of length M, M = N for a periodic signal of
 *                       a supported length, else the zero- or wrap-padded
 *                       length), FP64 or FP32. */
#define CWT_PSI_ALIASED 0
#define CWT_PSI_ANALYTIC 1

typedef struct cwt_plan_s *cwt_plan_t;

typedef struct {
    int32_t kind;  /* CWT_MORLET, CWT_MEXHAT, CWT_DOG, or a Table 2 wavelet
                      (CWT_CBSW, CWT_GDW, CWT_CWGDW, CWT_MW) */
    double param;  /* omega0 > 0 for Morlet; integer order m >= 1 for DOG;
                      ignored for the Mexican hat */
} cwt_wavelet;

typedef struct {
    int32_t precision; /* CWT_FP64 (default) or CWT_FP32 */
    int32_t method;    /* CWT_METHOD_FFT (default), CWT_METHOD_SPLINE,
                          CWT_METHOD_A19 or CWT_METHOD_V97 */
    int64_t fft_len;   /* 0: the library picks the length of the whole-signal
                          FFT; otherwise a length >= the minimum the plan
                          needs, of the form 2^a * {1,3,5,9}, 2^a >= 64 */
    int32_t host_only; /* 1: build the plan on the host only (no device
                          allocation, no device needed); it can be queried
                          but cwt_exec rejects it with CWT_EINVAL */
    int32_t fft_mode;  /* FFT method only: CWT_FFT_SEGMENTED (default) or
                          CWT_FFT_WHOLE; both give the same transform up to
                          rounding */
    int32_t single_stream; /* 1: every launch of a call stays on the
                              caller's stream (no second stream for the
                              local-group kernels); same results */
    int32_t psi_mode;  /* CWT_PSI_ALIASED (default) or CWT_PSI_ANALYTIC */
    int32_t reserved[4];
} cwt_opts;

/*
 * cwt_plan -- build a plan for signals of N samples and the S scales in
 * `scales` (host array of S doubles, copied).  Output row j belongs to
 * scales[j].  `opts` may be NULL (FP64, FFT method).
 * What is planned: Sec. 3.1 (FFTCWT: the signal transform of Eq. FT_signal
 * and, per scale, the product and inverse of Eq. discrete_CWT_conv, with
 * the wavelet spectrum evaluated once here) or Sec. 3.3 (M02CWT: h*, the
 * per-scale steps and the coefficients d_s of Eq.
 * beta3_wavelet_approx_m02, chosen by Eq. m02cwt_error as in Sec. 3.6).
 * Errors: CWT_EINVAL for N < 2, S < 1, a scale that is not finite and > 0,
 * omega0 <= 0 or not finite, a DOG order that is not an integer in [1, 16],
 * an unknown kind/boundary/precision/method/psi_mode, CWT_PSI_ANALYTIC
 * without CWT_METHOD_FFT and CWT_FFT_WHOLE, out == NULL or scales == NULL;
 * CWT_EUNSUPPORTED for CWT_CBSW other than whole-signal analytic;
 * CWT_EUNSUPPORTED for N > 2^26, S > 65536, an fft_len that is too short or
 * not of the supported form, or (spline method) a knot spacing delta_s
 * above about 2^18.4 (the 128-bit running sums then keep fewer than 40
 * fixed-point bits), more than 3601 wavelet coefficients at one scale, or
 * N + 2 E above 2^27 with E = max over the scales of (N_d + 3) delta_s + 16
 * (the tap kernel addresses the running sums with 32-bit byte offsets);
 * CWT_ENOMEM / CWT_EDEVICE on allocation or HIP failures.
 * On failure *out is set to NULL.
 */
int cwt_plan(cwt_plan_t *out, int64_t N, int32_t boundary, cwt_wavelet wavelet,
             const double *scales, int32_t S, const cwt_opts *opts);

/* Destroys a plan (NULL is accepted).  Work of the plan that is still
 * queued is not disturbed: the plan's device tables are released in stream
 * order after the last cwt_exec / cwt_exec_batch call enqueued with the
 * plan on each stream (tables allocated outside the stream-ordered arena
 * are released after a host wait for those calls).  Calls captured into a
 * HIP graph are not tracked: keep the plan alive while such a graph may be
 * launched. */
int cwt_destroy(cwt_plan_t plan);

/* 1 if the output is complex (Morlet), 0 if real; negative on error. */
int cwt_out_is_complex(cwt_plan_t plan);

/* Number of output values S*N (complex values count once); -1 on error. */
int64_t cwt_out_elems(cwt_plan_t plan);

/* Bytes of one output element: 16/8 (complex FP64/FP32) or 8/4 (real). */
int32_t cwt_out_elem_bytes(cwt_plan_t plan);

/* Bytes of device workspace cwt_exec needs (0 is possible). */
size_t cwt_workspace_bytes(cwt_plan_t plan);

/* Device bytes one execution holds: signal + output + workspace + the
 * plan's own tables.  Used for admission by device-memory footprint. */
size_t cwt_footprint_bytes(cwt_plan_t plan);

/*
 * cwt_exec -- enqueue the transform on `stream`: the signal's spectrum, the
 * per-scale spectral products and their inverses (Sec. 3.1, Eqs. FT_signal
 * and discrete_CWT_conv, in overlap-save segments or on the whole signal),
 * or the spline method's prefilter (Eq. interp_coeffs), running sums (Eq.
 * cumsum4_coeffs) and tap sums (Eq. m02_cwt) (Sec. 3.3).
 *   signal:    device, N values, double (CWT_FP64) or float (CWT_FP32).
 *   out:       device, [S][N] row-major; complex values interleaved
 *              (re, im) for Morlet; element type double or float as above.
 *              Stores are laid out for an output that starts on a 128-byte
 *              boundary (any element-aligned output gives the same result).
 *   workspace: device, at least cwt_workspace_bytes(plan) bytes, 256-byte
 *              aligned; may be NULL when that size is 0.
 * Errors: CWT_EINVAL for a NULL plan/signal/out, a NULL workspace when one is
 * needed, or a pointer not aligned to its element size; CWT_EDEVICE when a
 * launch fails.  NaN/Inf in the signal propagate; they are not checked.
 * The call only enqueues kernels and event dependencies (no allocation, no
 * host copy), so it may be captured into a HIP graph.  Part of the work may
 * run on a second stream paired with `stream` (one per calling thread,
 * device and caller stream), forked from `stream` and joined back into it
 * before the call returns; that stream and its two events are created on
 * the first call with that caller stream, so run one call before
 * capturing.  The plan is only read, so calls on different streams with
 * different workspaces may overlap entirely.  Outside graph capture the
 * call also records an event on `stream` that orders the plan's release
 * (cwt_destroy).
 */
int cwt_exec(cwt_plan_t plan, const void *signal, void *out, void *workspace,
             void *stream);

/*
 * cwt_exec_scratch -- cwt_exec without allocating anything, for callers that
 * cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation).  The workspace is a
 * fixed array of cwt_scratch_bytes() bytes (128 MiB) in the device memory of
 * every GPU the library runs on, reserved when the library loads and held
 * until the process ends; its device address is looked up once per device
 * on the first call with that device current.  signal, out and stream as
 * for cwt_exec.  Every launch stays on `stream` (no second stream), and no
 * event is recorded: keep the plan alive until the call's work has finished.
 * All calls on one GPU share that GPU's array and leave their contents in
 * it: calls that overlap in time on one GPU (different streams, or
 * different threads) race and give wrong results; serialise them.  No
 * kernel relies on the array's earlier contents.
 * Errors: as cwt_exec; CWT_EUNSUPPORTED when cwt_workspace_bytes(plan)
 * exceeds cwt_scratch_bytes() (nothing is launched).
 */
int cwt_exec_scratch(cwt_plan_t plan, const void *signal, void *out, void *stream);
size_t cwt_scratch_bytes(void);

/*
 * cwt_exec_wps -- wavelet power spectra of the signal instead of its
 * coefficients (Sec. 5): per scale, the environment-dependent power spectrum
 * (Eq. env_wps) -- the mean of |W(s, x)|^2 over the positions x whose
 * environment value env[x] falls in a bin -- and the global one (Eq.
 * global_wps), the mean over all N positions.  The bins split the real line
 * at nthr thresholds: position x is in bin k = #{i : env[x] >= thresholds[i]}
 * (k = 0 .. nthr), so every position is in exactly one bin and
 * global = sum_k (N_k / N) env_k (Eq. global_wps_env_wps); a NaN env value
 * falls in bin 0.  The paper's split into underdense and overdense
 * positions is nthr = 1, thresholds = {0}, env = the density contrast.
 * W is the transform cwt_exec computes; its squares are added up inside the
 * output kernels (FP64 sums of FP32 or FP64 values, in a fixed order), so
 * the S x N coefficients are never written.
 *   signal:     device, N values of the plan's precision.
 *   env:        device, N values of the plan's precision, or NULL for the
 *               signal itself.
 *   thresholds: host, nthr strictly ascending finite values, 0 <= nthr <= 3.
 *   wps:        device, [S][nthr + 2] doubles: columns 0..nthr the
 *               environment-dependent spectra of bins 0..nthr (NaN for an
 *               empty bin), column nthr + 1 the global spectrum.
 *   counts:     device, nthr + 1 int64 bin sizes N_k, or NULL.
 *   workspace:  device, cwt_wps_workspace_bytes(plan) bytes, 256-byte aligned
 *               (the plan's workspace plus per-workgroup partial sums).
 * Supported for segmented FFT plans (method CWT_METHOD_FFT, fft_mode
 * CWT_FFT_SEGMENTED, psi_mode CWT_PSI_ALIASED: the defaults) and otherwise
 * CWT_EUNSUPPORTED; cwt_wps_workspace_bytes returns 0 for the others.
 * Errors: CWT_EINVAL for NULL plan/signal/wps/workspace, bad thresholds or
 * misaligned pointers; CWT_EDEVICE when a launch fails.  Streams, events and
 * graph capture as for cwt_exec; the result does not depend on scheduling.
 */
size_t cwt_wps_workspace_bytes(cwt_plan_t plan);
int cwt_exec_wps(cwt_plan_t plan, const void *signal, const void *env, const double *thresholds, int32_t nthr,
                 double *wps, int64_t *counts, void *workspace, void *stream);

/*
 * cwt_global_wps -- the global wavelet power spectrum (Sec. 5, Eq.
 * global_wps), P(s) = (1/N) sum_b |W(s, b)|^2, of a periodic signal without
 * the transform: by Parseval's identity for the circular correlation of Eq.
 * discrete_CWT_conv (aliased spectrum), P(s) = (1/N^2) sum_m |F[m]|^2
 * Psi_s(omega_m)^2 with F the N-point DFT of the period, summed over the bins
 * of each scale's band (FP64 sums in a fixed order).  The same quantity as
 * column nthr + 1 of cwt_exec_wps, at the cost of one forward FFT.  The
 * plan's workspace (cwt_workspace_bytes) includes the per-chunk sums.
 *   signal:    device, N values of the plan's precision.
 *   wps:       device, S doubles.
 *   workspace: device, cwt_workspace_bytes(plan) bytes, 256-byte aligned.
 * Supported for plans of the FFT method with fft_mode CWT_FFT_WHOLE, periodic
 * boundary, psi_mode CWT_PSI_ALIASED, a band-limited wavelet (not CBSW) and
 * N = 2^a * {1,3,5,9}, 2^a >= 64 (the FFT length is then N), with at least
 * one scale that uses the whole-signal spectrum; otherwise CWT_EUNSUPPORTED.
 * Errors: CWT_EINVAL for NULL or misaligned pointers or a host-only plan;
 * CWT_EDEVICE when a launch fails.  Streams and events as for cwt_exec.
 */
int cwt_global_wps(cwt_plan_t plan, const void *signal, double *wps, void *workspace, void *stream);

/*
 * cwt_exec_batch -- transform n independent signals, each with its own plan
 * (lengths, scales, wavelets, boundaries and precisions may differ), in one
 * enqueue on `stream`.  signals[i], outs[i] as for cwt_exec with plans[i].
 * workspace: at least cwt_batch_workspace_bytes(plans, n) bytes.  Every
 * result is bit-identical to cwt_exec of the same plan and signal.  The
 * launch tables are copied from host memory at call time, so this call must
 * not be captured into a HIP graph.
 */
size_t cwt_batch_workspace_bytes(const cwt_plan_t *plans, int32_t n);
int cwt_exec_batch(const cwt_plan_t *plans, const void *const *signals,
                   void *const *outs, int32_t n, void *workspace, void *stream);

/*
 * Plan queries used by tests and schedulers.
 *   cwt_plan_fft_len:      length of the whole-signal FFT (0 if the plan
 *                          never needs it).
 *   cwt_plan_spline_delta: fills delta[j] (S entries) with the integer knot
 *                          spacing delta_j of the spline method, 0 where the
 *                          knots fall between samples (h* s < 1) and for
 *                          plans of the FFT method.
 *   cwt_plan_spline_taps:  fills taps[j] with the taps per output of scale
 *                          j: 2 N_d + 1 wavelet coefficients d_s on the
 *                          running sums, or 2 T + 1 exact taps on the
 *                          interpolant's coefficients, T = ceil((N_d + 2)
 *                          s h*) + 2 (0 for the FFT method).
 *   cwt_plan_spline_hstar: h* of the plan's wavelet (0 for the FFT method).
 *   cwt_plan_scale_path:   fills path[j] with how scale j is computed:
 *                          0 = segmented FFT (overlap-save), 1 = band-limited
 *                          inverse of the whole-signal spectrum, 2 = spline
 *                          on the running sums, 3 = spline with exact taps
 *                          (h* s < 1).
 */
int64_t cwt_plan_fft_len(cwt_plan_t plan);
int cwt_plan_spline_delta(cwt_plan_t plan, int32_t *delta);
int cwt_plan_spline_taps(cwt_plan_t plan, int32_t *taps);
double cwt_plan_spline_hstar(cwt_plan_t plan);
int cwt_plan_scale_path(cwt_plan_t plan, int32_t *path);

/*
 * cwt_plan_describe -- a text summary of the plan (one line per segment
 * group: local or band, segment length L, band transform size P, band bins
 * B, halo, outputs per segment, segments, column chunks, scales; one line
 * per band launch with its work item counts; for the spline method one line
 * per scale: knot spacing, tile columns R and rows I, taps, exact taps).  Writes at most size bytes
 * including the terminating NUL into buf (host memory, owned by the
 * caller); returns the full length of the text, or CWT_EINVAL for a NULL
 * plan or a NULL buf with size > 0.
 */
int cwt_plan_describe(cwt_plan_t plan, char *buf, size_t size);

/*
 * Launch timing for benchmarks.  While enabled on a plan, every cwt_exec of
 * that plan brackets each kernel launch with HIP events recorded on the
 * launch stream.  cwt_plan_timing_read waits for those events and reports,
 * per kernel (aggregated over all recorded launches): a name (at most 63
 * chars + NUL, in names[i*64]), the number of launches, the summed elapsed
 * milliseconds and the algorithmic bytes per launch (signal, whole-signal
 * spectrum and output bytes the launch must read or write at least once).
 * It returns the number of kernels (at most max_kernels are written) and
 * clears the records.  Not thread-safe with respect to concurrent cwt_exec
 * calls on the same plan; enabling costs two event records per launch.
 * Without timing, the local-group kernels of a segmented plan run on a
 * second stream of the calling thread, beside the band kernels on the
 * caller's stream (forked after, and joined back into, the caller's
 * stream).  With timing on, every launch of the call stays on the caller's
 * stream, so each recorded duration is that kernel's alone.  For
 * cwt_exec_batch the first plan's setting applies.
 */
int cwt_plan_timing_enable(cwt_plan_t plan, int32_t on);
int cwt_plan_timing_read(cwt_plan_t plan, int32_t max_kernels, char *names,
                         int64_t *launches, double *ms, double *bytes_per_launch);

/* Thread-local text describing the last error of this thread ("" if none). */
const char *cwt_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* CWT_H */
