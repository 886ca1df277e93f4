"""The C ABI: the library loads, exports every entry point the header
declares, and rejects invalid arguments before touching a device.  Host-only
plans check the plan logic (paths, FFT length, workspace) without a GPU."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

import paper_2302_03909_amd as cwt

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    src = open(os.path.join(ROOT, "include", "cwt.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(cwt_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_function():
    lib = cwt.load()
    names = header_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(cwt.EXPORTS) == names


def _plan_rc(n=64, bc=0, kind=0, param=6.0, scales=(2.0,), opts=None):
    lib = cwt.load()
    h = ctypes.c_void_p()
    sc = np.asarray(scales, dtype=np.float64)
    o = opts if opts is not None else cwt._Opts(0, 0, 0, 1)
    rc = lib.cwt_plan(ctypes.byref(h), n, bc, cwt._Wavelet(kind, param),
                      sc.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if sc.size else None,
                      sc.size, ctypes.byref(o))
    if rc == 0:
        lib.cwt_destroy(h)
    return rc


@pytest.mark.parametrize("kw", [dict(n=1), dict(n=0), dict(scales=()), dict(scales=(0.0,)),
                                dict(scales=(-1.0,)), dict(scales=(float("nan"),)),
                                dict(scales=(float("inf"),)), dict(bc=7), dict(kind=9),
                                dict(kind=0, param=0.0), dict(kind=0, param=float("nan")),
                                dict(kind=2, param=0.0), dict(kind=2, param=2.5),
                                dict(kind=2, param=17.0)])
def test_invalid_arguments(kw):
    assert _plan_rc(**kw) == -1
    assert cwt.load().cwt_last_error().decode() != ""


def test_unsupported_arguments():
    assert _plan_rc(n=(1 << 26) + 1) == -2
    assert _plan_rc(opts=cwt._Opts(0, 0, 1000, 1)) in (0, -2)  # only if a column path needs it


def test_bad_precision_and_method():
    assert _plan_rc(opts=cwt._Opts(5, 0, 0, 1)) == -1
    assert _plan_rc(opts=cwt._Opts(0, 5, 0, 1)) == -1


def test_null_arguments():
    lib = cwt.load()
    assert lib.cwt_plan(None, 64, 0, cwt._Wavelet(0, 6.0), None, 1, None) == -1
    assert lib.cwt_exec(None, None, None, None, None) == -1
    assert lib.cwt_destroy(None) == 0
    assert lib.cwt_out_elems(None) == -1


def test_host_only_plan_segmented_paths():
    # default (segmented) mode: small scales full-spectrum segments, the rest band-limited
    scales = np.geomspace(2, 2 ** 16, 128)
    p = cwt.Plan(1 << 22, "zero", "morlet", scales, param=6.0, precision="fp32", host_only=True)
    path = p.scale_path()
    assert path[0] == cwt.PATH_LOCAL and path[-1] == cwt.PATH_COLUMN
    assert np.all(np.diff(path) >= 0)  # monotone in scale
    assert p.fft_len == 0
    assert 0 < p.workspace_bytes < 256 << 20


def test_unknown_fft_mode_rejected():
    o = cwt._Opts(0, 0, 0, 1, 7)
    assert _plan_rc(opts=o) == -1


def test_host_only_plan_fft_paths():
    scales = np.geomspace(2, 2 ** 16, 128)
    p = cwt.Plan(1 << 22, "zero", "morlet", scales, param=6.0, precision="fp32", host_only=True,
                 fft_mode="whole")
    path = p.scale_path()
    assert set(path.tolist()) <= {cwt.PATH_LOCAL, cwt.PATH_COLUMN}
    assert path[0] == cwt.PATH_LOCAL and path[-1] == cwt.PATH_COLUMN
    # zero boundary: M >= N + T(s_max) and of the form 2^a * {1,3,5,9}
    m = p.fft_len
    assert m >= (1 << 22) + math.ceil(6.4 * 2 ** 16)
    odd = m // (m & -m)
    assert odd in (1, 3, 5, 9)
    assert p.workspace_bytes >= m * 8
    assert p.is_complex
    # host-only plans cannot run
    rc = cwt.load().cwt_exec(p.handle, ctypes.c_void_p(8), ctypes.c_void_p(8), ctypes.c_void_p(256), None)
    assert rc == -1


def test_host_only_periodic_smooth_uses_n():
    p = cwt.Plan(4096 * 9, "periodic", "mexhat", [2.0, 900.0, 3000.0], host_only=True, fft_mode="whole")
    assert p.fft_len == 4096 * 9
    q = cwt.Plan(5000, "periodic", "mexhat", [2.0, 900.0], host_only=True, fft_mode="whole")
    assert q.fft_len >= 5000 + 2 * math.ceil(8 * 900)


def test_batch_workspace_layout_host_only():
    # the batch workspace holds every plan's own workspace (256-aligned) plus
    # the launch tables of the merged launches
    plans = [cwt.Plan(n, "zero", "morlet", [2.0, 30.0, 500.0], param=6.0, precision="fp32", host_only=True)
             for n in (1000, 5000, 20000)]
    total = sum((p.workspace_bytes + 255) // 256 * 256 for p in plans)
    wb = cwt.batch_workspace_bytes(plans)
    assert wb > total
    assert cwt.batch_workspace_bytes(plans[:1]) <= wb
    assert cwt.batch_workspace_bytes([]) == 0


def _groups(plan):
    """(kind, L, P, B, Tg, V, nseg, nchunk, iters, scales) of every segment
    group in a plan's summary."""
    out = []
    for line in plan.describe().splitlines():
        parts = line.split()
        if parts and parts[0] in ("local", "band"):
            kv = dict(x.split("=") for x in parts[1:])
            out.append((parts[0],) + tuple(int(kv[k]) for k in
                                           ("L", "P", "B", "Tg", "V", "nseg", "nchunk", "iters", "scales")))
    return out


def test_segment_groups_of_the_headline_plan():
    scales = np.geomspace(2, 2 ** 16, 128)
    p = cwt.Plan(1 << 22, "zero", "morlet", scales, param=6.0, precision="fp32", host_only=True)
    g = _groups(p)
    local = [x for x in g if x[0] == "local"]
    band = [x for x in g if x[0] == "band"]
    # long FP32 signal: every local scale in one group of 2048-sample segments
    assert len(local) == 1 and local[0][1] == 2048
    assert sum(x[9] for x in g) == 128
    for kind, L, P, B, Tg, V, nseg, nchunk, iters, s in g:
        assert Tg % 16 == 0 and V == L - 2 * Tg and V > 0
        assert nseg * V >= (1 << 22) > (nseg - 1) * V
        if kind == "band":
            assert B <= P <= L // 16
            # each forward chunk reads at least two 16-column blocks
            assert iters * nchunk * 16 == L // P
            assert nchunk == 1 or iters >= 2


def test_column_pairs_only_for_real_fp32_output():
    scales = np.geomspace(2, 2 ** 16, 128)

    def band(n, wav, par, precision):
        p = cwt.Plan(n, "zero", wav, scales, param=par, precision=precision, host_only=True)
        return [(int(ln.split("L=")[1].split()[0]), int(ln.split("P=")[1].split()[0]), "colpair=1" in ln)
                for ln in p.describe().splitlines() if ln.startswith("band")]

    # real output, FP32, even N: every band group whose rows hold >= 32 columns
    g = band(1 << 22, "dog", 2.0, "fp32")
    assert g and all(cp == (L // P >= 32) for L, P, cp in g)
    assert any(cp for _, _, cp in g) and not all(cp for _, _, cp in g)
    # odd N: the same groups as the even N next to it (pairs that straddle a
    # row or window edge are stored as two single outputs)
    assert band((1 << 22) - 1, "dog", 2.0, "fp32") == band((1 << 22) - 2, "dog", 2.0, "fp32")
    # complex output or FP64: scale pairs (or single scales) only
    assert not any(cp for _, _, cp in band(1 << 22, "morlet", 6.0, "fp32"))
    assert not any(cp for _, _, cp in band(1 << 20, "dog", 2.0, "fp64"))


def test_shifted_units_only_where_rows_start_inside_a_line():
    scales = np.geomspace(2, 2 ** 16, 128)

    def flags(n, wav, par, precision):
        p = cwt.Plan(n, "zero", wav, scales, param=par, precision=precision, host_only=True)
        return [("colpair=1" in ln, "shift=1" in ln) for ln in p.describe().splitlines() if ln.startswith("band")]

    # rows of 2^22 elements start on lines: no shift
    assert not any(sh for _, sh in flags(1 << 22, "morlet", 6.0, "fp32"))
    assert not any(sh for _, sh in flags(1 << 22, "dog", 2.0, "fp32"))
    # complex rows off the line grid: band groups with shifted units (a group
    # whose rows all start on lines has none)
    g = flags((1 << 22) - 3, "morlet", 6.0, "fp32")
    assert sum(sh for _, sh in g) >= len(g) - 2
    assert any(sh for _, sh in flags((1 << 20) - 4, "morlet", 6.0, "fp64"))
    # real output: column-pair groups shift (N not a multiple of 32, odd N
    # included); scale-pair groups never do
    for n in ((1 << 22) - 2, (1 << 22) - 1):
        g = flags(n, "dog", 2.0, "fp32")
        assert all(sh == cp for cp, sh in g) and any(cp for cp, _ in g)


def test_segment_groups_not_merged_for_fp64_or_short_signals():
    scales = np.geomspace(2, 2 ** 12, 48)
    p = cwt.Plan(1 << 20, "zero", "morlet", scales, param=6.0, precision="fp64", host_only=True)
    local = [x for x in _groups(p) if x[0] == "local"]
    assert len(local) > 1 and len({x[1] for x in local}) == len(local)
    # segments of at least 256 samples for a long signal
    assert min(x[1] for x in local) >= 256
    # a short signal keeps single segments just long enough for it
    q = cwt.Plan(700, "zero", "mexhat", [2.0, 8.0, 30.0], precision="fp32", host_only=True)
    for x in _groups(q):
        assert x[1] <= 2048 and x[6] >= 1


def test_analytic_mode_rejections():
    # psi_mode ANALYTIC needs the whole-signal FFT (Sec. 3.1 form), a
    # periodic length the FFT takes as it is; the CBSW only in that form
    import paper_2302_03909_amd as cwt
    with pytest.raises(cwt.CwtError) as e:
        cwt.Plan(512, "periodic", "gdw", [2.0], psi_mode="analytic", host_only=True)
    assert e.value.code == cwt.CWT_EINVAL
    with pytest.raises(cwt.CwtError) as e:
        cwt.Plan(512, "periodic", "cbsw", [2.0], fft_mode="whole", host_only=True)
    assert e.value.code == cwt.CWT_EUNSUPPORTED
    with pytest.raises(cwt.CwtError) as e:
        cwt.Plan(512, "periodic", "cbsw", [2.0], method="spline", host_only=True)
    assert e.value.code == cwt.CWT_EUNSUPPORTED
    with pytest.raises(cwt.CwtError) as e:
        cwt.Plan(4800, "periodic", "gdw", [2.0], fft_mode="whole", psi_mode="analytic", host_only=True)
    assert e.value.code == cwt.CWT_EUNSUPPORTED
    p = cwt.Plan(512, "periodic", "cbsw", [2.0, 300.0], fft_mode="whole", psi_mode="analytic", host_only=True)
    assert p.fft_len == 512 and p.scale_path().tolist() == [cwt.PATH_COLUMN] * 2


def test_wps_workspace_and_rejections_host_only():
    # statistics epilogue (Sec. 5): workspace = the plan's own plus one slot of
    # partial sums per workgroup and scale and the bin-count partials;
    # rejected before any device work for host-only or non-segmented plans
    lib = cwt.load()
    sc = np.geomspace(2.0, 65536.0, 128)
    p = cwt.Plan(1 << 22, "periodic", "cwgdw", sc, precision="fp32", host_only=True)
    wb = cwt.wps_workspace_bytes(p)
    assert wb > p.workspace_bytes
    # at most 4 bins of 8 bytes per workgroup and scale: bounded by the plan size
    assert wb - p.workspace_bytes < 64 << 20
    thr = (ctypes.c_double * 1)(0.0)
    rc = lib.cwt_exec_wps(p.handle, None, None, thr, 1, None, None, None, None)
    assert rc == cwt.CWT_EINVAL
    sp = cwt.Plan(4096, "zero", "mexhat", [3.0, 30.0], method="spline", host_only=True)
    assert cwt.wps_workspace_bytes(sp) == 0
    assert lib.cwt_exec_wps(sp.handle, None, None, thr, 1, None, None, None, None) == cwt.CWT_EUNSUPPORTED
    wp = cwt.Plan(4096, "periodic", "morlet", [3.0, 30.0], fft_mode="whole", host_only=True)
    assert cwt.wps_workspace_bytes(wp) == 0
    assert lib.cwt_exec_wps(None, None, None, thr, 1, None, None, None, None) == cwt.CWT_EINVAL


def test_band_lengths_never_compute_more_positions_than_the_power_of_two():
    # a band group's length is c 2^k (c odd, at most 15; 2^k >= 32 P when
    # c > 1), chosen only where nseg L is below the power of two's count
    scales = np.geomspace(2, 2 ** 16, 128)
    seen_odd = False
    for n, bc, wav, par in [(1 << 22, "zero", "morlet", 6.0), ((1 << 22) - 3, "periodic", "dog", 2.0),
                            (123457, "zero", "morlet", 6.0), (20000, "zero", "dog", 2.0)]:
        p = cwt.Plan(n, bc, wav, scales[scales < n / 4], param=par, precision="fp32", host_only=True)
        for ln in p.describe().splitlines():
            if not ln.startswith("band"):
                continue
            kv = {k: int(v) for k, v in (t.split("=") for t in ln.split()[1:] if "=" in t)}
            L, P, Tg, V, nseg = kv["L"], kv["P"], kv["Tg"], kv["V"], kv["nseg"]
            c = L // (L & -L)
            assert c % 2 == 1 and c <= 15
            assert nseg * V >= n > (nseg - 1) * V
            if c == 1:
                continue
            seen_odd = True
            assert (L // c) >= 32 * P and (L // P) % 32 == 0
            L2 = 1 << (L - 1).bit_length()
            if nseg == 1 and Tg == 0:
                continue  # single zero-boundary segment: the power of two is longer
            nseg2 = -(-n // (L2 - 2 * Tg))
            assert nseg * L <= nseg2 * L2
    assert seen_odd


def test_global_wps_rejections_host_only():
    # Parseval's global spectrum needs a periodic whole-signal plan whose FFT
    # is the period's DFT; everything else is rejected before device work
    lib = cwt.load()
    dummy = ctypes.c_void_p(256)
    sc = np.geomspace(2.0, 4096.0, 24)
    ok = cwt.Plan(1 << 16, "periodic", "morlet", sc, fft_mode="whole", host_only=True)
    assert ok.fft_len == 1 << 16
    assert lib.cwt_global_wps(ok.handle, dummy, dummy, dummy, None) == cwt.CWT_EINVAL  # host-only
    assert lib.cwt_global_wps(ok.handle, None, dummy, dummy, None) == cwt.CWT_EINVAL
    assert lib.cwt_global_wps(None, dummy, dummy, dummy, None) == cwt.CWT_EINVAL
    for p in (cwt.Plan(1 << 16, "periodic", "morlet", sc, host_only=True),                    # segmented
              cwt.Plan(1 << 16, "zero", "morlet", sc, fft_mode="whole", host_only=True),      # zero boundary
              cwt.Plan(1000, "periodic", "morlet", sc[:10], fft_mode="whole", host_only=True),  # N not 2^a*{1,3,5,9}
              cwt.Plan(1 << 16, "periodic", "morlet", sc, fft_mode="whole", psi_mode="analytic", host_only=True),
              cwt.Plan(1 << 16, "periodic", "mexhat", sc, method="spline", host_only=True)):
        assert lib.cwt_global_wps(p.handle, dummy, dummy, dummy, None) == cwt.CWT_EUNSUPPORTED
