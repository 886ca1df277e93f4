#!/usr/bin/env python3
"""Benchmark of the multi-scale 1D CWT on one MI355X.

One step = one full transform of one synthetic signal whose samples already
sit in device memory (every kernel of the method, all scales).  Workloads:

  --method fft (default): N = 2^22 samples of a zero-boundary lognormal
      field, complex Morlet (omega0 = 6) or DOG(2), 128 log-spaced scales
      2..2^16, FP32 form (FP64 forward sums, FP32 output).
  --method spline: N = 2^20 samples of a zero-boundary lognormal field,
      Mexican hat (or Morlet(6)), 64 log-spaced scales 2..2^14, FP64.

Prints one JSON line (fields below), with a roofline entry for the kernel
that takes most of the step and the FP64 oracle timed on the host cores.

* Warm-up: W steps and at least 200 ms.
* K steps are timed as a caller runs them (value, ms_per_step; wall clock
  with a synchronisation on both sides), with an event on the caller's
  stream between steps (whole_step.ms_median / ms_min).
* FFT method: K steps of the same plan with every launch on the caller's
  stream (whole_step.single_stream), against the default, which runs the
  local kernels on a second stream beside the band kernels.
* K more steps with a HIP event pair around every kernel launch give the
  per-kernel durations (roofline, whole_step.kernels).  Under launch timing
  every launch stays on one stream, so each duration is that kernel's alone;
  that region's step time is reported on its own
  (whole_step.ms_per_step_with_kernel_events).
* roofline is the dominant kernel's (algorithmic bytes or flops per launch
  over its mean launch time); whole_step gives the whole transform's output
  write rate against the published 8 TB/s and against the measured copy and
  store rates of this GPU (measured_peaks).
* per_scale_error: the output of the last timed step against the FP64
  oracle at sampled positions of every scale.

    python bench.py [--steps K] [--warmup W] [--method fft|spline]
                    [--wavelet morlet|dog2|mexhat] [--boundary zero|periodic]
                    [--no-cpu-baseline] [--no-error-table] [--copy-calibration]
                    [--batch COUNT] [--serve]

--batch COUNT times cwt_exec_batch over COUNT uneven instances instead (4096
is the batched workload).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

HBM_PEAK_GBS = 8000.0      # MI355X HBM3E, published
FP64_PEAK_TFS = 78.6       # MI355X FP64 vector, published
FP32_PEAK_TFS = 157.3      # MI355X FP32 vector, published


def kernel_source_hash() -> str:
    """Hash of every kernel and plan source: counter figures taken on other
    sources are not reported."""
    h = hashlib.sha256()
    d = os.path.join(HERE, "paper_2302_03909_amd", "csrc")
    for f in sorted(os.listdir(d)):
        if f.endswith((".hip", ".h", ".cpp")):
            h.update(f.encode())
            h.update(open(os.path.join(d, f), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch from committed counter runs, if they were taken
    on the current kernel sources; else None."""
    p = os.path.join(HERE, "profiles", "traffic.json")
    if not os.path.exists(p):
        return None
    try:
        d = json.load(open(p))
    except Exception:
        return None
    e = d.get(workload, {}).get(kernel)
    if not e or e.get("source_hash") != kernel_source_hash():
        return None
    return e.get("hbm_bytes_per_launch")


def host_info():
    """Host CPU as the oracle leg sees it: the model, nproc and the cores
    this process may run on."""
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        allowed = len(os.sched_getaffinity(0))
    except AttributeError:
        allowed = os.cpu_count() or 1
    return {"cpu_model": model, "nproc": os.cpu_count() or 1, "allowed_cpus": allowed}


def oracle_threads():
    """Threads for the oracle: every core this process may use, capped by
    OMP_NUM_THREADS when the environment sets it (the machine's CPU share)."""
    info = host_info()
    n = info["allowed_cpus"]
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit() and int(env) > 0:
        n = min(n, int(env))
    return max(1, n)


def _timed_sample(run, seconds):
    count = 2000
    while True:
        t = run(count)
        if t >= seconds:
            return count, t
        count = int(count * min(8.0, max(1.5, 1.2 * seconds / max(t, 1e-3))))


def cpu_baseline_fft(f, boundary, wavelet, param, scales, seconds=10.0, one_core_seconds=4.0):
    """The FP64 direct-sum oracle on a uniform random sample of the
    workload's outputs (scale, position), on all the cores this process may
    use, then on one core."""
    import numpy as np
    import oracle
    threads = oracle_threads()
    n, s = f.size, len(scales)
    rng = np.random.default_rng(123)
    f64 = f.astype(np.float64)

    def run_with(th):
        def run(count):
            si = rng.integers(0, s, count)
            ps = rng.integers(0, n, count)
            t0 = time.perf_counter()
            oracle.cwt_points(f64, boundary, wavelet, scales, si, ps, param=param, nthreads=th)
            return time.perf_counter() - t0
        return run

    count, t = _timed_sample(run_with(threads), seconds)
    c1, t1 = _timed_sample(run_with(1), one_core_seconds)
    info = host_info()
    return {"value": count / t, "unit": "coefficients/s", "cores": threads, "kind": "oracle",
            "sample": f"{count} outputs drawn uniformly over the {s} x {n} outputs of the workload "
                      f"(FP64 direct sum), {t:.1f} s on {threads} threads",
            "one_core_value": c1 / t1, "one_core_sample": f"{c1} outputs, {t1:.1f} s on 1 thread",
            **info}


def cpu_baseline_spline(f, boundary, wavelet, param, scales, hstar, seconds=10.0):
    """The oracle's exact spline target (Gauss-Legendre over the merged
    knots) on random positions of 8 scales spread over the scale range."""
    import numpy as np
    import oracle
    threads = oracle_threads()
    n = f.size
    rng = np.random.default_rng(321)
    pick = np.linspace(0, len(scales) - 1, 8).round().astype(int)
    f64 = f.astype(np.float64)

    def run(count):
        per = max(1, count // len(pick))
        t0 = time.perf_counter()
        for j in pick:
            oracle.spline_target_scale(f64, boundary, wavelet, float(scales[j]), hstar,
                                       rng.integers(0, n, per), param=param, nthreads=threads)
        return time.perf_counter() - t0

    count, t = _timed_sample(run, seconds)
    count = max(1, count // len(pick)) * len(pick)
    return {"value": count / t, "unit": "coefficients/s", "cores": threads, "kind": "oracle",
            "sample": f"{count} outputs, equal numbers at 8 of the {len(scales)} scales (spread over the "
                      f"range), random positions of N = {n} (exact spline target), {t:.1f} s",
            **host_info()}


def warm_up(step, count, min_ms=200.0):
    """At least `count` steps and at least min_ms of wall time (synchronised
    at the end).  Returns (steps, milliseconds)."""
    import torch
    t0 = time.perf_counter()
    k = 0
    while k < count or (time.perf_counter() - t0) * 1e3 < min_ms:
        step()
        k += 1
        if k % 8 == 0:
            torch.cuda.synchronize()
    torch.cuda.synchronize()
    return k, (time.perf_counter() - t0) * 1e3


def timed_steps(step, steps):
    """K steps bracketed by a synchronisation on both sides (wall clock ->
    ms per step), with an event recorded on the caller's stream between
    steps (per-step milliseconds)."""
    import torch
    st = torch.cuda.current_stream()
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    evs[0].record(st)
    for k in range(steps):
        step()
        evs[k + 1].record(st)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    return (t1 - t0) * 1e3 / steps, [evs[k].elapsed_time(evs[k + 1]) for k in range(steps)]


def measured_peaks(torch, dev, gib=2):
    """Achievable HBM rates on this GPU: a device-to-device copy of `gib` GiB
    (reads + writes) and a fill of `gib` GiB (writes only), best of 5."""
    nbytes = gib << 30
    a = torch.empty(nbytes // 4, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    a.fill_(1.0)
    torch.cuda.synchronize()
    best_copy = best_fill = 0.0
    for _ in range(5):
        e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        e0.record()
        b.copy_(a)
        e1.record()
        a.fill_(2.0)
        e2.record()
        torch.cuda.synchronize()
        best_copy = max(best_copy, 2 * nbytes / (e0.elapsed_time(e1) * 1e-3) / 1e9)
        best_fill = max(best_fill, nbytes / (e1.elapsed_time(e2) * 1e-3) / 1e9)
    del a, b
    torch.cuda.empty_cache()
    return {"copy_gbs": round(best_copy, 1), "store_gbs": round(best_fill, 1),
            "how": f"torch copy_ and fill_ of {gib} GiB float32, best of 5 (copy counts reads and writes)"}


def error_table(plan, out, f, boundary, wav, par, scales, method, npos=96):
    """Per-scale relative L2 error (floor 1e-3 of the largest row norm) of
    the output against the FP64 oracle on the same input (FP32-rounded for
    the FP32 form), at the first and last positions and npos - 2 random ones
    of every scale: the direct sum for the FFT method, the exact spline
    target for the spline method."""
    import numpy as np
    import torch
    import oracle
    n = f.size
    rng = np.random.default_rng(77)
    pos = np.unique(np.concatenate([[0, n - 1], rng.integers(0, n, npos - 2)]))
    got = out[:, torch.as_tensor(pos, device=out.device)].cpu().numpy()
    f64 = f.astype(np.float64)
    th = oracle_threads()
    t0 = time.perf_counter()
    if method == "fft":
        si = np.repeat(np.arange(len(scales)), pos.size)
        ps = np.tile(pos, len(scales))
        ref = oracle.cwt_points(f64, boundary, wav, scales, si, ps, param=par, nthreads=th)
        ref = ref.reshape(len(scales), pos.size)
        what = "FP64 direct sum"
    else:
        hs = plan.spline_hstar()
        ref = np.stack([oracle.spline_target_scale(f64, boundary, wav, float(s), hs, pos, param=par, nthreads=th)
                        for s in scales])
        what = "exact spline target"
    got = got.astype(ref.dtype)
    nrm = np.linalg.norm(ref, axis=1)
    e = np.linalg.norm(got - ref, axis=1) / np.maximum(nrm, 1e-3 * nrm.max())
    return {"reference": f"{what} at {pos.size} positions per scale ({time.perf_counter() - t0:.1f} s)",
            "max": float(e.max()), "median": float(np.median(e)),
            "per_scale": [float(f"{v:.2e}") for v in e]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--method", default="fft", choices=["fft", "spline"])
    ap.add_argument("--batch", type=int, default=0,
                    help="time cwt_exec_batch on this many uneven instances instead (lengths 2^10..2^16, "
                         "16..96 scales, Morlet(6) / Mexican hat, half periodic tones, half zero-boundary "
                         "lognormal fields, FP32 form); 4096 is the batched workload")
    ap.add_argument("--serve", action="store_true",
                    help="served form instead: Poisson request streams (2^12..2^22 samples, 32..256 scales, "
                         "Morlet(6) / Mexican hat / DOG(4), FP32) at 0.5, 0.8 and 0.95 of the plain-batched "
                         "capacity, continuous batching against plain batching, p50 / p99 latency")
    ap.add_argument("--wps", action="store_true",
                    help="statistics epilogue instead (Sec. 5): env-WPS (split at delta = 0) and global WPS "
                         "of a periodic 1D Zel'dovich field (theta = 100), N = 2^22, 128 log scales 2..2^16, "
                         "CW-GDW, FP32 form, against the plain transform of the same field")
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--serve-warmup", type=int, default=200)
    ap.add_argument("--serve-loads", default="0.5,0.8,0.95",
                    help="offered loads, as fractions of the plain-batched capacity")
    ap.add_argument("--wavelet", default=None, choices=["morlet", "dog2", "mexhat", "cwgdw"])
    ap.add_argument("--thresholds", default="0",
                    help="--wps: comma-separated environment thresholds (empty: one bin)")
    ap.add_argument("--boundary", default="zero", choices=["zero", "periodic"])
    ap.add_argument("--fft-mode", default="segmented", choices=["segmented", "whole"],
                    help="FFT method layout: overlap-save segments (default) or one FFT of the whole "
                         "signal (Fig. fftCWT's form), for comparison")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-error-table", action="store_true")
    ap.add_argument("--mfma-probe", action="store_true",
                    help="measurement probe instead: a 16-point FP32 DFT of 2^20 columns as the radix-16 "
                         "butterfly on the vector ALUs against the same DFT as 16x16 matrix products on "
                         "the matrix cores (libcwt_probe.so), points per second of each")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="after the timed region, copy 1 GiB device-to-device 3 times (a plain copy "
                         "kernel of known size, for scaling HBM byte counters)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this build runs on one GPU only; the transform shards by scale "
                                   "(see the design notes), but no multi-GPU path is provided"}))
        sys.exit(2)

    if args.mfma_probe:
        return probe_dft16()

    import numpy as np
    import torch
    import paper_2302_03909_amd as cwt
    import synth

    if args.batch > 0:
        return bench_batch(args)
    if args.serve:
        return bench_serve(args)
    if args.wps:
        return bench_wps(args)
    if args.method == "fft":
        n, nscales, smax, precision = 1 << 22, 128, 2.0 ** 16, "fp32"
        seed, nname = synth.SEED_FIELD_4M, "2^22"
        wavelet = args.wavelet or "morlet"
    else:
        n, nscales, smax, precision = 1 << 20, 64, 2.0 ** 14, "fp64"
        seed, nname = synth.SEED_FIELD_1M, "2^20"
        wavelet = args.wavelet or "mexhat"
    wav, par = {"morlet": ("morlet", 6.0), "dog2": ("dog", 2.0), "mexhat": ("mexhat", None),
                "cwgdw": ("cwgdw", None)}[wavelet]
    scales = synth.log_scales(2.0, smax, nscales)
    dt = np.float32 if precision == "fp32" else np.float64
    f = synth.lognormal_field(n, seed=seed).astype(dt)

    dev = torch.device("cuda", 0)
    print(f"bench: {args.method} {wav} N={n} S={nscales} {precision}", file=sys.stderr, flush=True)
    plan = cwt.Plan(n, args.boundary, wav, scales, param=par, precision=precision, method=args.method,
                    fft_mode=args.fft_mode)
    x = torch.as_tensor(f, device=dev)
    out = plan.empty_output(dev)
    ws = plan.empty_workspace(dev)
    torch.cuda.synchronize()

    warm = warm_up(lambda: plan(x, out, ws), args.warmup)
    # timed region: K steps as a caller runs them (value, ms_per_step), with
    # an event on the caller's stream between steps (median and min)
    ms, per_step = timed_steps(lambda: plan(x, out, ws), args.steps)
    # the same plan with every launch on the caller's stream (no second
    # stream for the local kernels), for the choice of the default
    alt = None
    if args.method == "fft" and args.fft_mode == "segmented":
        plan1 = cwt.Plan(n, args.boundary, wav, scales, param=par, precision=precision, single_stream=True)
        warm_up(lambda: plan1(x, out, ws), 3)
        ms1, per1 = timed_steps(lambda: plan1(x, out, ws), args.steps)
        alt = {"ms_per_step": round(ms1, 4), "ms_median": round(float(np.median(per1)), 4),
               "ms_min": round(float(np.min(per1)), 4)}
        del plan1
    # second timed region: K more steps with a HIP event pair around every
    # kernel launch (per-kernel durations, roofline); launches then stay on
    # one stream and the events add a few microseconds each, so this step
    # time is reported on its own
    plan.timing(True)
    ms_ev, _ = timed_steps(lambda: plan(x, out, ws), args.steps)
    plan.timing(False)
    kern = plan.timing_read()
    coeffs = n * nscales
    value = coeffs / (ms * 1e-3)
    out_bytes = coeffs * (4 if precision == "fp32" else 8) * (2 if plan.is_complex else 1)
    # per-scale error of the last step's output against the FP64 oracle on
    # the same (FP32-rounded) input, at sampled positions of every scale
    err = None
    if not args.no_error_table:
        err = error_table(plan, out, f, args.boundary, wav, par, scales, args.method)

    wname = f"{wav}({par:g})" if par is not None else wav
    workload = (f"lognormal field N={nname} {args.boundary} boundary, {wname}, "
                f"{nscales} log scales 2..2^{int(np.log2(smax))}, "
                f"{'fp32 form' if precision == 'fp32' else 'fp64'}"
                + (", spline method" if args.method == "spline" else "")
                + (", whole-signal FFT" if args.fft_mode == "whole" else ""))

    # dominant kernel: largest total time over the timed region
    name, (cnt, tot_ms, bpl) = max(kern.items(), key=lambda kv: kv[1][1])
    avg_s = tot_ms / cnt * 1e-3
    peaks = measured_peaks(torch, dev)
    if name.startswith("spl_tap"):
        # FP64 fused multiply-adds of the tap sums: one per tap and output
        # (two for complex taps), 2 flops per FMA
        taps = plan.spline_taps().astype(np.float64)
        flops = 2.0 * n * taps.sum() * (2.0 if plan.is_complex else 1.0)
        achieved = flops / avg_s / 1e12
        roof = {"bound": "alu", "achieved": round(achieved, 2), "peak": FP64_PEAK_TFS, "unit": "TFLOP/s",
                "frac": round(achieved / FP64_PEAK_TFS, 4), "traffic": measured_traffic(name, workload),
                "kernel": name, "avg_launch_ms": round(tot_ms / cnt, 4),
                "algorithmic_flops_per_launch": flops, "output_write_gbs": round(bpl / avg_s / 1e9, 1)}
        if roof["traffic"]:
            # the counted HBM bytes (running sums read, outputs written) over
            # this run's launch time: the rate that bounds the kernel
            roof["traffic_gbs"] = round(roof["traffic"] / avg_s / 1e9, 1)
            roof["traffic_frac_of_hbm_peak"] = round(roof["traffic"] / avg_s / 1e9 / HBM_PEAK_GBS, 4)
    else:
        achieved = bpl / avg_s / 1e9
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(name, workload),
                "kernel": name, "avg_launch_ms": round(tot_ms / cnt, 4),
                "algorithmic_bytes_per_launch": bpl,
                "frac_of_measured_store_peak": round(achieved / peaks["store_gbs"], 4)}
    step_gbs = out_bytes / (ms * 1e-3) / 1e9
    # the whole step beside the dominant kernel: output bytes over ms_per_step
    roof["whole_step_output_gbs"] = round(step_gbs, 1)
    roof["whole_step_frac"] = round(step_gbs / HBM_PEAK_GBS, 4)
    whole = {"output_bytes": out_bytes,
             "output_write_gbs": round(step_gbs, 1),
             "hbm_frac_of_spec": round(step_gbs / HBM_PEAK_GBS, 4),
             "hbm_frac_of_measured_store_peak": round(step_gbs / peaks["store_gbs"], 4),
             "hbm_frac_of_measured_copy_peak": round(step_gbs / peaks["copy_gbs"], 4),
             "ms_median": round(float(np.median(per_step)), 4), "ms_min": round(float(np.min(per_step)), 4),
             "warmup_steps": warm[0], "warmup_ms": round(warm[1], 1),
             "single_stream": alt,
             "ms_per_step_with_kernel_events": round(ms_ev, 4),
             "kernels": {k: {"launches": v[0], "ms_per_step": round(v[1] / args.steps, 4),
                             "bytes_per_launch": v[2]} for k, v in kern.items()}}

    if args.copy_calibration:
        src = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    cpu = None
    if not args.no_cpu_baseline:
        print("bench: timing the oracle on the host", file=sys.stderr, flush=True)
        if args.method == "fft":
            cpu = cpu_baseline_fft(f, args.boundary, wav, par, scales)
        else:
            cpu = cpu_baseline_spline(f, args.boundary, wav, par, scales, plan.spline_hstar())

    line = {"metric": "CWT coefficients/sec (N x scales) and % HBM peak at N=2^22, 128 scales",
            "value": value, "unit": "coefficients/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32" if precision == "fp32" else "f64", "data": "synthetic",
            "config": {"workload": workload, "method": args.method, "n": n, "scales": nscales,
                       "scale_range": [2, int(smax)], "boundary": args.boundary, "wavelet": wname,
                       "precision": precision},
            "roofline": roof, "whole_step": whole, "measured_peaks": peaks, "per_scale_error": err,
            "cpu_baseline": cpu}
    print(json.dumps(line), flush=True)


def probe_dft16():
    """One radix-16 stage, butterfly on the vector ALUs against matrix products."""
    import ctypes
    path = os.path.join(HERE, "paper_2302_03909_amd", "libcwt_probe.so")
    if not os.path.exists(path):
        raise SystemExit(f"{path} is not built: run paper_2302_03909_amd/build.py")
    lib = ctypes.CDLL(path)
    lib.cwt_probe_dft16.argtypes = [ctypes.POINTER(ctypes.c_double)] * 3
    lib.cwt_probe_dft16.restype = ctypes.c_int
    valu, mfma, diff = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    rc = lib.cwt_probe_dft16(ctypes.byref(valu), ctypes.byref(mfma), ctypes.byref(diff))
    if rc != 0:
        raise SystemExit(f"cwt_probe_dft16 failed ({rc})")
    simd_cycles = 256 * 4 * 2.4e9    # SIMDs x clock: SIMD cycles per second at the rated clock
    print(json.dumps({
        "probe": "dft16: 2^20 columns of 16 complex FP32 points, 256 in-register stages per column",
        "valu_points_per_s": valu.value, "mfma_points_per_s": mfma.value,
        "valu_over_mfma": round(valu.value / mfma.value, 3),
        "valu_simd_cycles_per_point": round(simd_cycles / valu.value, 4),
        "mfma_simd_cycles_per_point": round(simd_cycles / mfma.value, 4),
        "one_stage_max_rel_diff": diff.value}))
    if not diff.value < 1e-5:
        raise SystemExit("matrix-core DFT disagrees with the butterfly")


def fft_flops(plan, kernel):
    """FFT flops of one launch of an output kernel, 5 L log2 L per complex
    L-point inverse it takes (the usual count), from the plan's segment
    groups: local2_kernel<..,L,..> takes G-column blocks of L points per
    scale (or real-scale pair), seg_inverse_kernel<..,P,..> 16 P-point
    columns per work item and unit."""
    import re
    m = re.match(r"(local2_kernel|seg_inverse_kernel)<f(32|64),(\d+),", kernel)
    if not m:
        return None
    size, fp64 = int(m.group(3)), m.group(2) == "64"
    cplx = plan.is_complex
    total = 0.0
    for line in plan.describe().splitlines():
        g = dict(kv.split("=") for kv in line.split()[1:] if "=" in kv)
        if line.startswith("local ") and m.group(1) == "local2_kernel" and int(g["L"]) == size:
            L, k = int(g["L"]), int(g["scales"])
            ncol = max((2048 if fp64 else 4096) // L, 1)
            units = k if cplx else (k + 1) // 2
            total += -(-int(g["nseg"]) // ncol) * ncol * units * 5.0 * L * math.log2(L)
        if line.startswith("band ") and m.group(1) == "seg_inverse_kernel" and int(g["P"]) == size:
            L, P, k = int(g["L"]), int(g["P"]), int(g["scales"])
            cp = g.get("colpair") == "1"
            cols = 32 if cp else 16
            units = k if (cplx or cp) else (k + 1) // 2
            total += int(g["nseg"]) * -(-(L // P) // cols) * 16 * units * 5.0 * P * math.log2(P)
    return total


def bench_wps(args):
    """One step = one cwt_exec_wps call: the environment-dependent and global
    wavelet power spectra of the field, with the coefficients reduced inside
    the output kernels (nothing of size S x N is written)."""
    import numpy as np
    import torch
    import paper_2302_03909_amd as cwt
    import synth

    n, nscales, smax = 1 << 22, 128, 2.0 ** 16
    wav, par = "cwgdw", None
    scales = synth.log_scales(2.0, smax, nscales)
    f = synth.zeldovich_field(n).astype(np.float32)
    dev = torch.device("cuda", 0)
    print(f"bench: power spectra, CW-GDW N={n} S={nscales} fp32 periodic", file=sys.stderr, flush=True)
    plan = cwt.Plan(n, "periodic", wav, scales, param=par, precision="fp32")
    x = torch.as_tensor(f, device=dev)
    ws = torch.empty(cwt.wps_workspace_bytes(plan), dtype=torch.uint8, device=dev)
    thr = tuple(float(t) for t in args.thresholds.split(",") if t.strip())

    def step():
        return cwt.exec_wps(plan, x, None, thr, workspace=ws, with_counts=False)

    warm = warm_up(step, args.warmup)
    ms, per_step = timed_steps(step, args.steps)
    # the plain transform of the same field (coefficients written)
    out = plan.empty_output(dev)
    wsp = plan.empty_workspace(dev)
    warm_up(lambda: plan(x, out, wsp), 3)
    ms_plain, per_plain = timed_steps(lambda: plan(x, out, wsp), args.steps)
    del out
    plan.timing(True)
    ms_ev, _ = timed_steps(step, args.steps)
    plan.timing(False)
    kern = plan.timing_read()
    wps, _ = step()
    torch.cuda.synchronize()
    wps = wps.cpu().numpy()
    # the global spectrum alone by Parseval (cwt_global_wps, whole-signal plan):
    # one forward FFT and a band sum per scale instead of the transform
    wplan = cwt.Plan(n, "periodic", wav, scales, param=par, precision="fp32", fft_mode="whole")
    wws = wplan.empty_workspace(dev)
    warm_up(lambda: cwt.global_wps(wplan, x, wws), 3)
    ms_pars, per_pars = timed_steps(lambda: cwt.global_wps(wplan, x, wws), args.steps)
    g_pars = cwt.global_wps(wplan, x, wws).cpu().numpy()
    del wws, wplan
    name, (cnt, tot_ms, bpl) = max(kern.items(), key=lambda kv: kv[1][1])
    avg_s = tot_ms / cnt * 1e-3
    flops = fft_flops(plan, name)
    achieved = flops / avg_s / 1e12
    coeffs = n * nscales
    workload = ("power spectra (env-WPS split at delta = 0, global WPS) of a periodic 1D Zel'dovich field "
                "theta = 100, N=2^22, CW-GDW, 128 log scales 2..2^16, fp32 form")
    line = {"metric": "CWT coefficients reduced to power spectra per second (N x scales)",
            "value": coeffs / (ms * 1e-3), "unit": "coefficients/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": workload, "n": n, "scales": nscales, "thresholds": list(thr)},
            "roofline": {"bound": "alu", "achieved": round(achieved, 2), "peak": FP32_PEAK_TFS, "unit": "TFLOP/s",
                         "frac": round(achieved / FP32_PEAK_TFS, 4), "traffic": None, "kernel": name,
                         "avg_launch_ms": round(tot_ms / cnt, 4), "fft_flops_per_launch": flops},
            "whole_step": {"ms_median": round(float(np.median(per_step)), 4),
                           "ms_min": round(float(np.min(per_step)), 4),
                           "warmup_steps": warm[0],
                           "plain_transform_ms": round(ms_plain, 4),
                           "plain_transform_ms_median": round(float(np.median(per_plain)), 4),
                           "speedup_vs_plain": round(ms_plain / ms, 3),
                           "ms_per_step_with_kernel_events": round(ms_ev, 4),
                           "kernels": {k: {"launches": v[0], "ms_per_step": round(v[1] / args.steps, 4),
                                           "bytes_per_launch": v[2]} for k, v in kern.items()},
                           "global_by_parseval": {
                               "ms": round(ms_pars, 4), "ms_median": round(float(np.median(per_pars)), 4),
                               "max_rel_diff_vs_epilogue": float(np.max(np.abs(g_pars - wps[:, -1]) / wps[:, -1]))},
                           "env_over_global_first_last_scale": [
                               [round(float(wps[0, b] / wps[0, -1]), 4) for b in range(len(thr) + 1)],
                               [round(float(wps[-1, b] / wps[-1, -1]), 4) for b in range(len(thr) + 1)]]},
            "cpu_baseline": None}
    print(json.dumps(line), flush=True)


def bench_batch(args):
    """One step = one cwt_exec_batch call over every instance (signals and
    outputs resident in device memory)."""
    import numpy as np
    import torch
    import paper_2302_03909_amd as cwt
    import synth

    dev = torch.device("cuda", 0)
    print(f"bench: drawing {args.batch} instances", file=sys.stderr, flush=True)
    insts = synth.batch_specs(count=args.batch)
    t0 = time.perf_counter()
    plans, sigs, outs = [], [], []
    for k, inst in enumerate(insts):
        if k % 512 == 0:
            print(f"bench: planning instance {k} of {len(insts)}", file=sys.stderr, flush=True)
        par = 6.0 if inst.wavelet == "morlet" else None
        plans.append(cwt.Plan(inst.n, inst.boundary, inst.wavelet, inst.scales, param=par, precision="fp32"))
        sigs.append(torch.as_tensor(inst.signal.astype(np.float32), device=dev))
        outs.append(plans[-1].empty_output(dev))
    plan_s = time.perf_counter() - t0
    ws = torch.empty(cwt.batch_workspace_bytes(plans), dtype=torch.uint8, device=dev)
    coeffs = sum(i.coefficients for i in insts)
    out_bytes = sum(o.numel() * o.element_size() for o in outs)
    for _ in range(args.warmup):
        cwt.exec_batch(plans, sigs, outs, ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        cwt.exec_batch(plans, sigs, outs, ws)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) * 1e3 / args.steps
    # per-kernel durations from a second timed region with kernel events
    plans[0].timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        cwt.exec_batch(plans, sigs, outs, ws)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    plans[0].timing(False)
    kern = plans[0].timing_read()
    ms_ev = (t1 - t0) * 1e3 / args.steps
    name, (cnt, tot_ms, bpl) = max(kern.items(), key=lambda kv: kv[1][1])
    avg_s = tot_ms / cnt * 1e-3
    achieved = bpl / avg_s / 1e9
    workload = (f"batch of {args.batch} uneven instances: N log-uniform 2^10..2^16, 16..96 log scales "
                f"2..min(N/8, 2^16), Morlet(6) / Mexican hat, half periodic tones, half zero-boundary "
                f"lognormal fields, fp32 form")
    line = {"metric": "CWT coefficients/sec (N x scales) and % HBM peak at N=2^22, 128 scales",
            "value": coeffs / (ms * 1e-3), "unit": "coefficients/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": workload, "instances": args.batch, "coefficients": coeffs,
                       "plan_seconds": round(plan_s, 2)},
            "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(name, workload),
                         "kernel": name, "avg_launch_ms": round(tot_ms / cnt, 4),
                         "algorithmic_bytes_per_launch": bpl},
            "whole_step": {"output_bytes": out_bytes,
                           "hbm_frac_of_output_write": round(out_bytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                           "ms_per_step_with_kernel_events": round(ms_ev, 4),
                           "kernels": {k: {"launches": v[0], "ms_per_step": round(v[1] / args.steps, 4),
                                           "bytes_per_launch": v[2]} for k, v in kern.items()}},
            "cpu_baseline": None}
    print(json.dumps(line), flush=True)


PLANNERS = 4  # host threads that build request plans beside the polling loop
IDLE_SLEEP = 20e-6  # polling loop: pause after an idle poll (lets the planner threads run)


def bench_serve(args):
    """Served form: requests take the first N samples of one of a few
    device-resident signals of 2^22 samples (periodic tones + noise for the
    periodic ones, lognormal fields for the zero-boundary ones).  Latency is
    arrival to device completion; outputs are dropped once complete."""
    import numpy as np
    import torch
    import synth
    from paper_2302_03909_amd.serve import (ContinuousScheduler, GpuExecutor, Request, StaticBatcher,
                                            latency_summary, run_open_loop)

    dev = torch.device("cuda", 0)
    print("bench: drawing signal pool", file=sys.stderr, flush=True)
    nmax = 1 << 22
    pool = {"periodic": [torch.as_tensor(synth.tones_noise(nmax, seed=s).astype(np.float32), device=dev)
                         for s in (1, 2)],
            "zero": [torch.as_tensor(synth.lognormal_field(nmax, seed=s).astype(np.float32), device=dev)
                     for s in (3, 4)]}
    torch.cuda.synchronize()
    par_of = {"morlet": 6.0, "mexhat": None, "dog": 4.0}

    def make(specs):
        out = []
        for i, d in enumerate(specs):
            sig = pool[d["boundary"]][d["seed"] % 2][:d["n"]]
            out.append(Request(i, d["n"], d["boundary"], d["wavelet"], par_of[d["wavelet"]], d["scales"], "fp32",
                               sig, arrival=d["arrival"]))
        return out

    total = args.serve_requests + args.serve_warmup
    budget = 32 << 30
    mean_coef = synth.mean_request_coefficients()
    # plain-batched capacity of the GPU: every request available at once,
    # plans built beforehand (the device's rate, not the planners')
    print("bench: measuring plain-batched capacity", file=sys.stderr, flush=True)
    specs = synth.request_specs(min(total, 600), rate_hz=1e9, seed=synth.SEED_SERVE + 1)
    ex = GpuExecutor(streams=1, keep_outputs=False, plan_cache=1 << 20, arena_bytes=budget)
    reqs = make(specs)
    for r in reqs:
        r.footprint = ex.prepare(r)
    sched = StaticBatcher(ex, max_batch=32, window=0.0, budget_bytes=budget)
    done = run_open_loop(sched, reqs)
    torch.cuda.synchronize()
    cap = latency_summary(done)["coefficients_per_s"]
    cap_rps = cap / mean_coef
    del ex, sched, reqs, done
    results = {}
    loads = [float(x) for x in args.serve_loads.split(",")]
    for load in loads:
        specs = synth.request_specs(total, rate_hz=load * cap_rps, seed=synth.SEED_SERVE)
        # cold: each request planned at arrival by the planner threads;
        # warm: plans of the stream's shapes already built (a plan cache hit)
        for plans in ("cold", "warm"):
            for mode in ("continuous", "plain"):
                print(f"bench: load {load} {mode} {plans} plans", file=sys.stderr, flush=True)
                ex = GpuExecutor(streams=2, keep_outputs=False, plan_cache=1 << 20, arena_bytes=budget)
                reqs = make(specs)
                if plans == "warm":
                    for r in reqs:
                        r.footprint = ex.prepare(r)
                sched = (ContinuousScheduler(ex, budget_bytes=budget, streams=2, planners=PLANNERS)
                         if mode == "continuous" else StaticBatcher(ex, max_batch=32, window=2e-3, planners=PLANNERS,
                                                                    budget_bytes=budget))
                done = run_open_loop(sched, reqs, idle_sleep=IDLE_SLEEP)
                sched.close()
                torch.cuda.synchronize()
                summ = latency_summary(done, skip=args.serve_warmup)
                summ["mean_batch"] = float(np.mean(sched.batches))
                summ["launch_host_s"] = round(ex.launch_s, 3)
                summ["arena_fallbacks"] = ex.arena_fallbacks
                results[f"{mode}@{load}/{plans}"] = summ
                for p_ in list(ex.plans.values()):
                    p_.close()
                del ex, sched, reqs, done
    top = results[f"continuous@{loads[-1]}/cold"]
    line = {"metric": f"served CWT coefficients/s and p50/p99 latency at {loads[-1]} x plain-batched capacity",
            "value": top["coefficients_per_s"], "unit": "coefficients/s", "n_gpus": 1,
            "steps": args.serve_requests, "warmup": args.serve_warmup, "ms_per_step": top["mean_ms"],
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
            "data": "synthetic",
            "config": {"workload": "Poisson request stream: N log-uniform 2^12..2^22, 32..256 log scales, "
                                   "Morlet(6) / Mexican hat / DOG(4), periodic or zero boundary, fp32 form",
                       "plain_batched_capacity_coef_per_s": cap, "capacity_requests_per_s": cap_rps,
                       "mean_request_coefficients": mean_coef, "budget_bytes": budget,
                       "planner_threads": PLANNERS},
            "serve": results, "roofline": None, "cpu_baseline": None}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
