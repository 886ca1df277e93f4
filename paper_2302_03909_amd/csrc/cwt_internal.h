// cwt_internal.h -- plan layout and kernel launchers shared by the host
// plan code (cwt_plan.cpp) and the device code (cwt_fft.hip, cwt_spline.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <memory>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

namespace cwt {

enum LoadMode : int32_t {
    LOAD_ZERO = 0,      // x[n] = f[n] for n < N, 0 beyond (zero boundary)
    LOAD_PERIODIC = 1,  // x[n] = f[n mod N] (FFT length == N)
    LOAD_WRAP = 2,      // x[n] = f[n mod N] for n < N + T, f[(n - M) mod N] for
                        // n >= M - T, 0 between (periodic, FFT length != N)
};

enum ScalePath : int32_t { PATH_LOCAL = 0, PATH_COLUMN = 1, PATH_SPLINE = 2, PATH_SPLINE_DIRECT = 3 };

// One overlap-save group: scales that share the segment FFT length L and the
// halo Tg; V = L - 2 Tg outputs per segment.
struct LocalGroup {
    int32_t L = 0;
    int64_t Tg = 0, V = 0, nseg = 0;
    std::vector<int32_t> scales;  // scale indices
    int64_t tab_off = 0;          // offset (elements) into the plan's spectrum table
    int32_t *d_scales = nullptr;  // device copy of `scales`
};

// Work item of the band-limited inverse kernel: G consecutive columns of one
// scale (or of a pair of scales sharing the transform, real wavelets).
struct ColumnDesc {
    int32_t sa, sb;      // output rows (sb = -1: none)
    int32_t pad0, pad1;
    int64_t r0;          // first column
    int64_t mlo, B;      // band: signed bins [mlo, mlo + B)
    int64_t Q;           // number of columns M / P
    int64_t taba, tabb;  // offsets of the spectrum samples of sa / sb
};

// A group of scales transformed with the same segment length: L = 2^lgL
// (LOCAL), or L = cL 2^lgL with cL odd (BAND).
//   LOCAL: full L-point spectrum, fused kernel (NCOL segments per workgroup)
//   BAND:  spectrum needed on [klo, klo + B) only, B <= P, L = P * Q
struct SegGroup {
    enum Kind { LOCAL = 0, BAND = 1 };
    int32_t kind = LOCAL;
    int32_t L = 0, lgL = 0, P = 0, cL = 1;
    int64_t Tg = 0, V = 0, nseg = 0;
    int64_t klo = 0;
    int32_t B = 0, nchunk = 1, iters = 1;
    std::vector<int32_t> scales;  // scale indices (LOCAL: table rows in order)
    int64_t tab_off = 0;          // LOCAL: offset (elements) of the L-point tables
    int32_t *d_scales = nullptr;
    int64_t twl_off = -1;  // LOCAL: per-pass LDS twiddle table of size L, bytes
    int64_t gtw_off = -1;  // BAND: column factors (w_L^{m g}, or column pairs), g < 16, m in band, bytes
    int32_t colpair = 0;   // BAND, real output: complex column g holds columns 2g, 2g + 1 of one scale
    int32_t cshift = 0;    // BAND: some unit's columns are shifted (SegUnit::dsh)
    int32_t colodd = 0;    // BAND, column pairs of an odd-length signal: pairs may straddle a row or window edge
    size_t ws_xp_off = 0, ws_x_off = 0;
    int32_t unit0 = 0, nunits = 0;  // BAND: range in Plan::units
    int32_t key = -1;               // LOCAL: index of its KeyDesc
    int64_t blocks = 0;             // LOCAL: workgroups of its launch
};

// device copy of a BAND group's parameters
struct SegGroupDev {
    int32_t lgL, B, nchunk, iters;  // lgL: k of the segment length L = c 2^k
    int32_t unit0, nunits;
    int32_t colpair, cshift;
    int32_t colodd, inv0;   // inv0: index of the group's first inverse work item
    int64_t V, Tg, klo, nseg;
    int64_t xp_off, x_off;  // workspace byte offsets of the partial and reduced band spectra
    int64_t gtw_off;        // byte offset of the column factors in the twiddle allocation
    int64_t L, Q;           // segment length and column count L / P
    int64_t wsm_off;        // c > 1: byte offset of w_L^z, z < c, in the twiddle allocation
    int32_t cL, pad2;       // odd factor c of L
};

// one output unit of a BAND group: a scale, or a pair of real-wavelet scales
// sharing one complex transform (sb = -1: none; always none in a column-pair
// group)
struct SegUnit {
    int32_t sa, sb;
    // offsets of their spectrum samples in the spectrum table; a single-row
    // unit (sb < 0) of a shifted group has kb = its complex samples with the
    // shift phase w_L^{-m dsh} folded in
    int64_t ka, kb;
    // single-row units: the work item of first column r0 computes columns
    // r0 - dsh .. (modulo the segment), so that the row's store runs start on
    // 128-byte lines
    int32_t dsh, pad;
};

// one workgroup of a fused launch: group g, segment seg, and idx = column
// chunk (forward), 16-bin block (reduce) or first column r0 (inverse); pad =
// number of consecutive segments (forward and reduce)
struct SegWork {
    int32_t g, seg, idx, pad;
};

// all BAND groups that share P, launched together
struct SegLaunch {
    int32_t P = 0;
    int64_t twl_off = -1;  // per-pass twiddle table of size P, bytes
    std::vector<int32_t> groups;  // indices into Plan::segs
    std::vector<SegGroupDev> gdev;
    std::vector<SegWork> fwd, red, inv;
    SegGroupDev *d_groups = nullptr;
    SegWork *d_fwd = nullptr, *d_red = nullptr, *d_inv = nullptr;
    double out_rows = 0.0;  // output rows written by the launch (for timing)
    int32_t key[3] = {-1, -1, -1};  // KeyDesc of the forward, reduce and inverse launches
};

// Launch key of the segmented FFT method, static and device resident (built
// with the plan): everything a workgroup needs besides the caller's buffers.
//   LOCAL group: one key (local2 kernel), work items = segment blocks.
//   SegLaunch:   three keys (forward, reduce, inverse), work items = `work`.
struct KeyDesc {
    int64_t N;
    int32_t periodic, cph;
    const SegGroupDev *groups;
    const SegUnit *units;
    const SegWork *work;
    const void *ktab;      // spectrum samples, plan precision (LOCAL: this group's L-point tables)
    const char *twbase;    // the plan's twiddle allocation
    const void *twl;       // per-pass LDS twiddle table of the key's transform size
    const double2 *whi, *wlo;  // FP64 w_{2^23} = hi[x >> 11] lo[x & 2047]
    int64_t Tg, V, nseg;   // LOCAL group
    int32_t nscale, pad;
    const int32_t *scale_ids;
    const int64_t *wps_base;  // statistics epilogue: first slot of each scale (plan-wide table)
};

// caller buffers of one transform
struct BatchInst {
    const void *f;
    void *out;
    char *ws;
    const void *env;  // statistics epilogue: environment values (plan precision)
    double *part;     // statistics epilogue: per-slot partial sums
};

// Statistics epilogue (Sec. 5, Eqs. env_wps and global_wps): instead of the
// coefficients, the two output kernels add up |W|^2 per scale and
// environment bin.  Bin of position x: the number of thresholds thr[k]
// (k < nbin - 1, ascending) with env[x] >= thr[k]; every position falls in
// one bin.  Each workgroup writes its sums to its own slot:
// part[(wps_base[scale] + slot) * nbin + bin], slot = the workgroup's index
// within the scale's group (local block, or inverse work item - inv0).
constexpr int kWpsMaxBins = 4;
struct WpsArgs {
    double thr[kWpsMaxBins - 1];
    int32_t nbin, pad;
};

// blocks [block0, next range's block0) of a merged launch run key `key` on
// instance `inst`, local block = blockIdx.x - block0
struct BatchRange {
    int64_t block0;
    const KeyDesc *key;
    int32_t inst, pad;
};

// kernel argument of every segmented kernel.  nranges == 0: one transform,
// key and buffers by value (k0, i0); else block b belongs to the last range
// with block0 <= b, which lies between ranges coarse[b / 256] and
// coarse[b / 256 + 1] (the ranges holding blocks 256 (b / 256) and
// 256 (b / 256 + 1), or the last one).
struct BatchArgs {
    const BatchRange *ranges;
    const int32_t *coarse;
    const BatchInst *insts;
    int32_t nranges, pad;
    KeyDesc k0;
    BatchInst i0;
    WpsArgs wps;  // read by the statistics variants only
};

// Plan-time evaluation of sampled wavelet spectra on the device
// (cwt_tables.hip).  SpecWavelet: the wavelet's spectral amplitude and the
// band [ulo, uhi] outside which it is negligible.
struct SpecWavelet {
    int32_t kind, m;
    double w0, cmor, kappa, gnorm, cn, ulo, uhi;
};
// count entries at tab[off..]: Psi_s(2 pi m / L) / L for m = m0 + e (full:
// the signed bin of e in [0, L)); shift >= 0: count complex entries (re, im
// at off + 2e, off + 2e + 1), each sample times w_L^{-m shift}.  The job's
// workgroups start at block0.
struct SpecJob {
    int64_t off, m0, count, L, block0;
    double s;
    int32_t full, shift;
};
hipError_t launch_spectrum_tables(const SpecWavelet &w, const SpecJob *jobs, int njobs, int64_t blocks, void *tab,
                                  bool fp64, hipStream_t st);
// global power spectrum of a periodic signal by Parseval from its M-point
// DFT F (plan precision, natural order): wps[j] = sum_m |F[m]|^2
// Psi_{s_j}(omega_m)^2 / M^2, from per-chunk sums part[j][c] (S x
// parseval_chunks(M) doubles of workspace) added in a fixed order
constexpr int64_t kParsevalChunk = 16384;  // signed bins per workgroup
inline int parseval_chunks(int64_t M) { return (int)((M + kParsevalChunk - 1) / kParsevalChunk); }
hipError_t launch_parseval_wps(const SpecWavelet &w, const void *F, int64_t M, const double *scales, int S,
                               double *part, double *wps, bool fp64, hipStream_t st);

struct ColumnLaunch {
    int32_t P = 0, G = 0;
    std::vector<ColumnDesc> items;
    ColumnDesc *d_items = nullptr;
};

// Bytes of LDS the band inverse kernel stages spectrum samples in (the plan
// sizes band groups to fit): with the P = 256 transform buffer it keeps three
// workgroups per compute unit.
constexpr int kSegKlsBytes = 14336;

// Spline method (Sec. 3.3, see cwt_spline.hip).  Per scale, a tap sum
// W[x] = sum_n d'[n] S[x + (n - nd) delta] with the tile shape R columns
// (consecutive positions) x I rows (stride delta):
//   mode 0 (integer knot spacing delta): S the exact box sums of the running
//     sums, d'[n] = conj(d[n - nd]) / (5040 s delta^3), 2 nd + 1 taps;
//   mode 1 (knots between samples, delta = 1): S = c, the spline
//     coefficients, d'[n] = Omega_s(n - nd), the exact taps, 2 nd + 1 taps.
// Taps are zero-padded to ntap, a multiple of 8.
struct SplineScaleDev {
    int32_t delta, nd, ntap, R, I, mode;
    int64_t d_off;  // complex FP64 elements into the plan's coefficient table
};

// one workgroup of the tap-sum launch: scale j, rows [i0, i0 + I), columns
// [r0, r0 + R) of the (row = x / delta, column = x mod delta) view of x
struct SplineWork {
    int32_t j, r0, R, pad;
    int64_t i0;
};

// an event owned by every plan whose last call on a stream it follows
struct UseEvent {
    hipEvent_t ev = nullptr;
    UseEvent() {
        if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) ev = nullptr;
    }
    ~UseEvent() {
        if (ev) (void)hipEventDestroy(ev);
    }
    UseEvent(const UseEvent &) = delete;
    UseEvent &operator=(const UseEvent &) = delete;
};

struct Plan {
    // problem
    int64_t N = 0;
    int32_t boundary = 0, kind = 0, precision = 0, method = 0;
    bool host_only = false;
    bool single_stream = false;  // keep every launch on the caller's stream
    int32_t psi_mode = 0;        // CWT_PSI_ALIASED or CWT_PSI_ANALYTIC (whole-signal FFT only)
    double param = 0.0;
    int32_t S = 0;
    std::vector<double> scales;
    bool cplx_out = false;
    int32_t cph = 0;  // conj(phase of psi^) = i^cph
    double rel = 0.0, chi = 0.0;
    std::vector<int64_t> T;
    std::vector<int32_t> path;

    // FFT method
    int64_t M = 0;  // whole-signal FFT length (0: not needed)
    int32_t M1 = 0, M2 = 0;
    int32_t load_mode = 0;
    int64_t Twrap = 0;
    std::vector<LocalGroup> groups;
    std::vector<ColumnLaunch> columns;
    std::vector<SegGroup> segs;
    std::vector<SegLaunch> seg_launches;
    std::vector<SegUnit> units;
    SegUnit *d_units = nullptr;
    std::vector<KeyDesc> keys;  // host copy (device pointers inside)
    KeyDesc *d_keys = nullptr;
    int32_t fft_mode = 0;  // 0 segmented, 1 whole signal
    int64_t w23_hi_off = -1, w23_lo_off = -1;  // FP64 w_{2^23} tables, bytes
    bool pair_real = false;
    // statistics epilogue slots (segmented plans): scale j owns slots
    // [wps_base[j], wps_base[j + 1]), one per workgroup of its group
    std::vector<int64_t> wps_base;
    int64_t *d_wps_base = nullptr;

    // spline method
    double hstar = 0.0;
    std::vector<SplineScaleDev> spl;
    std::vector<SplineWork> spl_work;
    std::vector<int32_t> spl_delta;  // delta per scale, 0 where the knots fall between samples
    std::vector<int32_t> spl_ntaps;  // taps per output per scale (2 N_d + 1, or the exact-tap count)
    bool spl_direct = false;         // some scale runs exact taps on c (workspace holds c)
    int64_t spl_E = 0;      // the running sums cover positions [-E, N + E)
    int64_t spl_len = 0;    // N + 2E
    int32_t spl_qbits = 0;  // bits of the fixed-point coefficients
    int32_t spl_nb0 = 0;    // blocks of the max|f| reduction
    int32_t spl_nblk = 0;   // blocks of the running sums
    int64_t spl_lds_bytes = 0;  // LDS of the tap-sum launch (largest tile plus its taps)
    SplineScaleDev *d_spl = nullptr;
    SplineWork *d_spl_work = nullptr;

    // V97 method (Sec. 3.2): the launch sequence.  kind 0: f_0 = beta3 * f
    // into buffer dst; 1: f_{a+1} = f_a * [h] upsampled by 2^a, src -> dst;
    // 2: F_a = f_a * [q12] upsampled by 2^a, src -> the F array; 3: tap sums
    // of the scales of level a, work items [w0, w1) of spl_work
    struct V97Step {
        int32_t kind, a, src, dst, w0, w1;
    };
    std::vector<V97Step> v97_steps;
    double v97_wmax = 0.0;      // w~_max = 1.34 c_w (Table 3)
    int32_t v97_nq12 = 0;       // q12 taps on each side
    int64_t v97_flen = 0;       // length of the f buffers (N periodic, N + 2E zero boundary)
    double *d_v97_q12 = nullptr;
    size_t ws_fa_off = 0, ws_fb_off = 0;
    size_t ws_maxp_off = 0, ws_fx_off = 0, ws_state_off = 0, ws_carry_off = 0, ws_H_off = 0, ws_C_off = 0;

    // device tables (owned).  Segmented plans keep all of them in one
    // allocation, d_arena; the pointers below then point into it.
    void *d_arena = nullptr;
    void *d_tab = nullptr;  // spectrum samples, plan precision (real)
    int64_t tab_elems = 0;
    void *d_tw_all = nullptr;  // all twiddle tables (one allocation); offsets in bytes
    std::vector<std::pair<int32_t, int64_t>> tw_off;    // (P, byte offset) plan precision
    std::vector<std::pair<int32_t, int64_t>> tw64_off;  // (P, byte offset) FP64
    int64_t twM_hi_off = -1, twM_lo_off = -1;           // plan precision, bytes
    int64_t twM64_hi_off = -1, twM64_lo_off = -1;       // FP64, bytes
    void *d_dtab = nullptr;                             // spline d_s (complex FP64)
    std::vector<void *> d_extra;                        // other owned allocations
    // periodic whole-signal plans with M = N (cwt_global_wps): the wavelet's
    // spectral amplitude and band, and the scales on the device
    SpecWavelet spec_w{};
    bool spec_ok = false;
    const double *d_scales64 = nullptr;
    size_t ws_pars_off = 0;  // per-chunk sums of cwt_global_wps in the workspace

    // launch timing (benchmarks only)
    struct TimingRec {
        std::string name;
        hipEvent_t a, b;
        double bytes;
    };
    bool timing = false;
    std::vector<TimingRec> timing_recs;
    std::vector<hipEvent_t> event_pool;

    // release ordering: per stream, an event recorded after the plan's last
    // call enqueued on it (calls under graph capture are not recorded); one
    // batched call shares one event among all its plans
    std::mutex use_mu;
    std::vector<std::pair<hipStream_t, std::shared_ptr<UseEvent>>> last_use;

    size_t ws_bytes = 0;
    size_t ws_F_off = 0, ws_Y_off = 0;  // workspace layout (FFT method)
    size_t table_bytes = 0;
};

// Segmented FFT kernels.  A launch is identified by its instantiation:
//   kind 0: local2 (size = L), 1: forward (size = P), 2: reduce, 3: inverse (size = P)
// and runs `blocks` workgroups described by `a`.
struct SegKernelId {
    int32_t kind, size, precision, cplx;  // cplx: complex output (else real pairs)
    bool operator<(const SegKernelId &o) const {
        if (kind != o.kind) return kind < o.kind;
        if (size != o.size) return size < o.size;
        if (precision != o.precision) return precision < o.precision;
        return cplx < o.cplx;
    }
};
hipError_t launch_seg_kernel(const SegKernelId &id, const BatchArgs &a, int64_t blocks, hipStream_t st);
// the statistics variants of kinds 0 and 3 (cwt_wps.hip); kinds 1 and 2 as above
hipError_t launch_seg_kernel_wps(const SegKernelId &id, const BatchArgs &a, int64_t blocks, hipStream_t st);
std::string seg_kernel_id_name(const SegKernelId &id, bool wps = false);
// statistics epilogue: bin counts of env (partials per workgroup, kWpsCountBlocks
// workgroups) and the final division (one workgroup per scale)
constexpr int kWpsCountBlocks = 512;
hipError_t launch_wps_count(const void *env, int64_t N, bool fp64, const WpsArgs &w, uint64_t *cpart, hipStream_t st);
hipError_t launch_wps_finalize(const double *part, const int64_t *base, int S, const WpsArgs &w,
                               const uint64_t *cpart, int64_t N, double *wps, int64_t *counts, hipStream_t st);
bool local2_size_ok(int L, int precision);
bool seg_size_ok(int P, int precision);
int local2_segs_per_block(int L, bool pair, bool fp64);

// names of the kernel instantiations a launch uses (timing labels)
std::string local_kernel_name(const Plan &p, const LocalGroup &g);
std::string column_kernel_name(const Plan &p, const ColumnLaunch &c);

// ---- launchers (device code) -------------------------------------------------
hipError_t launch_forward(const Plan &p, const void *signal, void *ws, hipStream_t st);
hipError_t launch_local(const Plan &p, const LocalGroup &g, const void *signal, void *out,
                        hipStream_t st);
hipError_t launch_column(const Plan &p, const ColumnLaunch &c, const void *ws, void *out,
                         hipStream_t st);
// phase 0: fixed-point running sums of the spline coefficients, 1: tap sums
hipError_t launch_spline(const Plan &p, const void *signal, void *out, void *ws, hipStream_t st, int phase);
std::string spline_kernel_name(const Plan &p, int phase);
// step k of Plan::v97_steps
hipError_t launch_v97(const Plan &p, size_t k, const void *signal, void *out, void *ws, hipStream_t st);
std::string v97_kernel_name(const Plan &p, size_t k);

// supported sizes
bool local_size_ok(int L, int precision);
bool column_size_ok(int P, int precision);
bool fwd_size_ok(int P);
int column_g(int P, int precision);
int column_nt(int P, int precision);

// twiddle table e^{+2 pi i j/P}: forward_list selects the FP64 tables of the
// whole-signal transform, otherwise the plan-precision tables
template <typename T> inline const T *tw_ptr(const Plan &p, int P, bool forward_list) {
    const auto &v = forward_list ? p.tw64_off : p.tw_off;
    for (auto &e : v)
        if (e.first == P) return reinterpret_cast<const T *>(static_cast<const char *>(p.d_tw_all) + e.second);
    return nullptr;
}

template <typename T> inline const T *tw_at(const Plan &p, int64_t byte_off) {
    return byte_off < 0 ? nullptr
                        : reinterpret_cast<const T *>(static_cast<const char *>(p.d_tw_all) + byte_off);
}

}  // namespace cwt
