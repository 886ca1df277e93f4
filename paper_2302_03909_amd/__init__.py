"""Python binding of libcwt.so, the MI355X (gfx950) multi-scale 1D CWT.

Argument marshalling only: every step of the transform runs in the HIP
kernels behind the C ABI declared in ``include/cwt.h``.  PyTorch provides the
device memory (its caching allocator) and the current HIP stream.  There is
no CPU fallback: if the library is missing, importing the binding raises.

    import torch, paper_2302_03909_amd as cwt
    plan = cwt.Plan(n, "zero", "morlet", scales, param=6.0, precision="fp32")
    W = plan(torch.as_tensor(signal, device="cuda", dtype=torch.float32))
    # W: [S, n] complex64 (Morlet) or float32 (Mexican hat / DOG)
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcwt.so")

CWT_PERIODIC, CWT_ZERO = 0, 1
CWT_MORLET, CWT_MEXHAT, CWT_DOG, CWT_CBSW, CWT_GDW, CWT_CWGDW, CWT_MW = 0, 1, 2, 3, 4, 5, 6
CWT_FP64, CWT_FP32 = 0, 1
CWT_METHOD_FFT, CWT_METHOD_SPLINE, CWT_METHOD_A19, CWT_METHOD_V97 = 0, 1, 2, 3
CWT_OK, CWT_EINVAL, CWT_EUNSUPPORTED, CWT_ENOMEM, CWT_EDEVICE = 0, -1, -2, -3, -4
PATH_LOCAL, PATH_COLUMN, PATH_SPLINE, PATH_SPLINE_DIRECT = 0, 1, 2, 3


class CwtError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"cwt error {code}: {msg}")
        self.code = code


class _Wavelet(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("param", ctypes.c_double)]


class _Opts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("method", ctypes.c_int32),
                ("fft_len", ctypes.c_int64), ("host_only", ctypes.c_int32),
                ("fft_mode", ctypes.c_int32), ("single_stream", ctypes.c_int32),
                ("psi_mode", ctypes.c_int32), ("reserved", ctypes.c_int32 * 4)]


EXPORTS = ["cwt_plan", "cwt_destroy", "cwt_out_is_complex", "cwt_out_elems", "cwt_out_elem_bytes",
           "cwt_workspace_bytes", "cwt_footprint_bytes", "cwt_exec", "cwt_batch_workspace_bytes",
           "cwt_exec_batch", "cwt_plan_fft_len", "cwt_plan_spline_delta", "cwt_plan_spline_taps", "cwt_plan_spline_hstar",
           "cwt_plan_scale_path", "cwt_plan_describe", "cwt_plan_timing_enable", "cwt_plan_timing_read", "cwt_last_error",
           "cwt_exec_scratch", "cwt_scratch_bytes", "cwt_wps_workspace_bytes", "cwt_exec_wps", "cwt_global_wps"]

_lib = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libcwt.so (built by ``paper_2302_03909_amd.build``)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_2302_03909_amd.build`")
    lib = ctypes.CDLL(path)
    vp = ctypes.c_void_p
    lib.cwt_plan.argtypes = [ctypes.POINTER(vp), ctypes.c_int64, ctypes.c_int32, _Wavelet,
                             ctypes.POINTER(ctypes.c_double), ctypes.c_int32, ctypes.POINTER(_Opts)]
    lib.cwt_plan.restype = ctypes.c_int
    lib.cwt_destroy.argtypes = [vp]
    lib.cwt_out_is_complex.argtypes = [vp]
    lib.cwt_out_elems.argtypes = [vp]
    lib.cwt_out_elems.restype = ctypes.c_int64
    lib.cwt_out_elem_bytes.argtypes = [vp]
    lib.cwt_workspace_bytes.argtypes = [vp]
    lib.cwt_workspace_bytes.restype = ctypes.c_size_t
    lib.cwt_footprint_bytes.argtypes = [vp]
    lib.cwt_footprint_bytes.restype = ctypes.c_size_t
    lib.cwt_exec.argtypes = [vp, vp, vp, vp, vp]
    lib.cwt_batch_workspace_bytes.argtypes = [ctypes.POINTER(vp), ctypes.c_int32]
    lib.cwt_batch_workspace_bytes.restype = ctypes.c_size_t
    lib.cwt_exec_batch.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp),
                                   ctypes.c_int32, vp, vp]
    lib.cwt_plan_fft_len.argtypes = [vp]
    lib.cwt_plan_fft_len.restype = ctypes.c_int64
    lib.cwt_plan_spline_delta.argtypes = [vp, ctypes.POINTER(ctypes.c_int32)]
    lib.cwt_plan_spline_taps.argtypes = [vp, ctypes.POINTER(ctypes.c_int32)]
    lib.cwt_plan_describe.argtypes = [vp, ctypes.c_char_p, ctypes.c_size_t]
    lib.cwt_plan_spline_hstar.argtypes = [vp]
    lib.cwt_plan_spline_hstar.restype = ctypes.c_double
    lib.cwt_plan_scale_path.argtypes = [vp, ctypes.POINTER(ctypes.c_int32)]
    lib.cwt_plan_timing_enable.argtypes = [vp, ctypes.c_int32]
    lib.cwt_plan_timing_read.argtypes = [vp, ctypes.c_int32, ctypes.c_char_p, ctypes.POINTER(ctypes.c_int64),
                                         ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
    lib.cwt_last_error.restype = ctypes.c_char_p
    lib.cwt_exec_scratch.argtypes = [vp, vp, vp, vp]
    lib.cwt_scratch_bytes.argtypes = []
    lib.cwt_scratch_bytes.restype = ctypes.c_size_t
    lib.cwt_wps_workspace_bytes.argtypes = [vp]
    lib.cwt_wps_workspace_bytes.restype = ctypes.c_size_t
    lib.cwt_exec_wps.argtypes = [vp, vp, vp, ctypes.POINTER(ctypes.c_double), ctypes.c_int32, vp, vp, vp, vp]
    lib.cwt_global_wps.argtypes = [vp, vp, vp, vp, vp]
    _lib = lib
    return lib


def _check(rc: int):
    if rc != 0:
        raise CwtError(rc, load().cwt_last_error().decode())


_BOUNDARY = {"periodic": CWT_PERIODIC, "zero": CWT_ZERO}
_PRECISION = {"fp64": CWT_FP64, "fp32": CWT_FP32}
_METHOD = {"fft": CWT_METHOD_FFT, "spline": CWT_METHOD_SPLINE, "a19": CWT_METHOD_A19, "v97": CWT_METHOD_V97}
_FFT_MODE = {"segmented": 0, "whole": 1}
_PSI_MODE = {"aliased": 0, "analytic": 1}


def _wavelet(name: str, param):
    n = name.lower()
    if n == "morlet":
        return CWT_MORLET, 6.0 if param is None else float(param)
    if n in ("mexhat", "mexican_hat"):
        return CWT_MEXHAT, 2.0
    if n == "dog":
        return CWT_DOG, 2.0 if param is None else float(param)
    paper = {"cbsw": CWT_CBSW, "gdw": CWT_GDW, "cwgdw": CWT_CWGDW, "cw-gdw": CWT_CWGDW, "mw": CWT_MW}
    if n in paper:
        return paper[n], 0.0
    raise ValueError(f"unknown wavelet {name!r}")


class Plan:
    """A transform plan: signal length, boundary, wavelet, scales, precision
    and method are fixed at construction; the device tables live until the
    plan is closed or garbage collected."""

    def __init__(self, n: int, boundary: str, wavelet: str, scales, param=None,
                 precision: str = "fp64", method: str = "fft", fft_len: int = 0,
                 host_only: bool = False, fft_mode: str = "segmented", single_stream: bool = False,
                 psi_mode: str = "aliased"):
        lib = load()
        kind, par = _wavelet(wavelet, param)
        sc = np.ascontiguousarray(np.asarray(scales, dtype=np.float64).ravel())
        opts = _Opts(_PRECISION[precision], _METHOD[method], int(fft_len), 1 if host_only else 0,
                     _FFT_MODE[fft_mode], 1 if single_stream else 0, _PSI_MODE[psi_mode])
        h = ctypes.c_void_p()
        _check(lib.cwt_plan(ctypes.byref(h), int(n), _BOUNDARY[boundary], _Wavelet(kind, par),
                            sc.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), sc.size,
                            ctypes.byref(opts)))
        self._h = h
        self.n = int(n)
        self.scales = sc.copy()
        self.boundary = boundary
        self.wavelet = wavelet
        self.param = par
        self.precision = precision
        self.method = method
        self.fft_mode = fft_mode
        self.is_complex = bool(lib.cwt_out_is_complex(h))
        self.workspace_bytes = int(lib.cwt_workspace_bytes(h))
        self.footprint_bytes = int(lib.cwt_footprint_bytes(h))
        self.fft_len = int(lib.cwt_plan_fft_len(h))

    @property
    def handle(self) -> ctypes.c_void_p:
        if self._h is None:
            raise ValueError("plan is closed")
        return self._h

    def close(self):
        if getattr(self, "_h", None) is not None:
            load().cwt_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def num_scales(self) -> int:
        return int(self.scales.size)

    def scale_path(self) -> np.ndarray:
        out = np.zeros(self.num_scales, dtype=np.int32)
        _check(load().cwt_plan_scale_path(self.handle, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))))
        return out

    def spline_delta(self) -> np.ndarray:
        out = np.zeros(self.num_scales, dtype=np.int32)
        _check(load().cwt_plan_spline_delta(self.handle, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))))
        return out

    def spline_taps(self) -> np.ndarray:
        out = np.zeros(self.num_scales, dtype=np.int32)
        _check(load().cwt_plan_spline_taps(self.handle, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))))
        return out

    def describe(self) -> str:
        """Text summary of the plan's segment groups and launches."""
        n = load().cwt_plan_describe(self.handle, None, 0)
        _check(n if n < 0 else 0)
        buf = ctypes.create_string_buffer(n + 1)
        load().cwt_plan_describe(self.handle, buf, n + 1)
        return buf.value.decode()

    def spline_hstar(self) -> float:
        return float(load().cwt_plan_spline_hstar(self.handle))

    def timing(self, on: bool = True):
        """Bracket every kernel launch of this plan with HIP events."""
        _check(load().cwt_plan_timing_enable(self.handle, 1 if on else 0))

    def timing_read(self):
        """Per-kernel {name: (launches, total_ms, algorithmic_bytes_per_launch)}
        of the launches recorded since the last read."""
        mx = 64
        names = ctypes.create_string_buffer(64 * mx)
        cnt = (ctypes.c_int64 * mx)()
        ms = (ctypes.c_double * mx)()
        by = (ctypes.c_double * mx)()
        n = load().cwt_plan_timing_read(self.handle, mx, names, cnt, ms, by)
        if n < 0:
            _check(n)
        out = {}
        for k in range(min(n, mx)):
            nm = names.raw[64 * k:64 * k + 64].split(b"\0", 1)[0].decode()
            out[nm] = (int(cnt[k]), float(ms[k]), float(by[k]))
        return out

    # -- torch helpers -------------------------------------------------------
    def _dtypes(self):
        import torch
        real = torch.float64 if self.precision == "fp64" else torch.float32
        cplx = torch.complex128 if self.precision == "fp64" else torch.complex64
        return real, (cplx if self.is_complex else real)

    def empty_output(self, device="cuda"):
        import torch
        _, odt = self._dtypes()
        return torch.empty((self.num_scales, self.n), dtype=odt, device=device)

    def empty_workspace(self, device="cuda"):
        import torch
        if self.workspace_bytes == 0:
            return None
        return torch.empty(self.workspace_bytes, dtype=torch.uint8, device=device)

    def __call__(self, signal, out=None, workspace=None, stream=None):
        """Run the transform on a device tensor of n values (float64 for fp64
        plans, float32 for fp32 plans).  Returns the [S, n] output tensor."""
        import torch
        sdt, _ = self._dtypes()
        if signal.dtype != sdt or signal.device.type != "cuda" or signal.numel() != self.n:
            raise ValueError(f"signal must be a cuda {sdt} tensor of {self.n} values")
        signal = signal.contiguous()
        if out is None:
            out = self.empty_output(signal.device)
        if workspace is None:
            workspace = self.empty_workspace(signal.device)
        st = stream if stream is not None else torch.cuda.current_stream(signal.device)
        _check(load().cwt_exec(self.handle, ctypes.c_void_p(signal.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                               ctypes.c_void_p(workspace.data_ptr() if workspace is not None else 0),
                               ctypes.c_void_p(st.cuda_stream)))
        return out


def wps_workspace_bytes(plan: Plan) -> int:
    return int(load().cwt_wps_workspace_bytes(plan.handle))


def exec_wps(plan: Plan, signal, env=None, thresholds=(0.0,), workspace=None, stream=None, with_counts=True):
    """``cwt_exec_wps``: wavelet power spectra (Sec. 5) of a device signal.
    Returns (wps, counts): wps a float64 [S, len(thresholds) + 2] tensor
    (environment-dependent spectra of the len(thresholds) + 1 bins, then the
    global one), counts the int64 bin sizes (None unless with_counts).
    env: device tensor of n values (the signal's dtype) or None (the signal)."""
    import torch
    sdt, _ = plan._dtypes()
    if signal.dtype != sdt or signal.device.type != "cuda" or signal.numel() != plan.n:
        raise ValueError(f"signal must be a cuda {sdt} tensor of {plan.n} values")
    signal = signal.contiguous()
    if env is not None:
        if env.dtype != sdt or env.device != signal.device or env.numel() != plan.n:
            raise ValueError(f"env must be a {sdt} tensor of {plan.n} values on the signal's device")
        env = env.contiguous()
    thr = (ctypes.c_double * max(1, len(thresholds)))(*[float(t) for t in thresholds])
    nb = len(thresholds) + 1
    wps = torch.empty((plan.num_scales, nb + 1), dtype=torch.float64, device=signal.device)
    counts = torch.empty(nb, dtype=torch.int64, device=signal.device) if with_counts else None
    if workspace is None:
        wb = wps_workspace_bytes(plan)
        workspace = torch.empty(max(wb, 1), dtype=torch.uint8, device=signal.device)
    st = stream if stream is not None else torch.cuda.current_stream(signal.device)
    _check(load().cwt_exec_wps(plan.handle, ctypes.c_void_p(signal.data_ptr()),
                               ctypes.c_void_p(env.data_ptr() if env is not None else 0), thr, len(thresholds),
                               ctypes.c_void_p(wps.data_ptr()),
                               ctypes.c_void_p(counts.data_ptr() if counts is not None else 0),
                               ctypes.c_void_p(workspace.data_ptr()), ctypes.c_void_p(st.cuda_stream)))
    return wps, counts


def global_wps(plan: Plan, signal, workspace=None, stream=None):
    """``cwt_global_wps``: the global wavelet power spectrum (Sec. 5) of a
    periodic device signal by Parseval from its DFT, for a whole-signal
    periodic plan.  Returns a float64 [S] tensor."""
    import torch
    sdt, _ = plan._dtypes()
    if signal.dtype != sdt or signal.device.type != "cuda" or signal.numel() != plan.n:
        raise ValueError(f"signal must be a cuda {sdt} tensor of {plan.n} values")
    signal = signal.contiguous()
    wps = torch.empty(plan.num_scales, dtype=torch.float64, device=signal.device)
    if workspace is None:
        workspace = plan.empty_workspace(signal.device)
    st = stream if stream is not None else torch.cuda.current_stream(signal.device)
    _check(load().cwt_global_wps(plan.handle, ctypes.c_void_p(signal.data_ptr()), ctypes.c_void_p(wps.data_ptr()),
                                 ctypes.c_void_p(workspace.data_ptr()), ctypes.c_void_p(st.cuda_stream)))
    return wps


def exec_scratch(plan: Plan, signal, out=None, stream=None):
    """``cwt_exec_scratch``: the transform with the library's fixed scratch
    array as workspace (no allocation by the library; ``out`` is allocated
    here when not given).  Calls that overlap on one GPU race."""
    import torch
    sdt, _ = plan._dtypes()
    if signal.dtype != sdt or signal.device.type != "cuda" or signal.numel() != plan.n:
        raise ValueError(f"signal must be a cuda {sdt} tensor of {plan.n} values")
    signal = signal.contiguous()
    if out is None:
        out = plan.empty_output(signal.device)
    st = stream if stream is not None else torch.cuda.current_stream(signal.device)
    _check(load().cwt_exec_scratch(plan.handle, ctypes.c_void_p(signal.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                   ctypes.c_void_p(st.cuda_stream)))
    return out


def scratch_bytes() -> int:
    return int(load().cwt_scratch_bytes())


def batch_workspace_bytes(plans) -> int:
    arr = (ctypes.c_void_p * len(plans))(*[p.handle.value for p in plans])
    return int(load().cwt_batch_workspace_bytes(arr, len(plans)))


def exec_batch(plans, signals, outs=None, workspace=None, stream=None):
    """Transform many signals (each with its own plan) in one enqueue."""
    import torch
    n = len(plans)
    if n == 0:
        return []
    if outs is None:
        outs = [p.empty_output(s.device) for p, s in zip(plans, signals)]
    if workspace is None:
        wb = batch_workspace_bytes(plans)
        workspace = torch.empty(wb, dtype=torch.uint8, device=signals[0].device) if wb else None
    st = stream if stream is not None else torch.cuda.current_stream(signals[0].device)
    hp = (ctypes.c_void_p * n)(*[p.handle.value for p in plans])
    sp = (ctypes.c_void_p * n)(*[s.data_ptr() for s in signals])
    op = (ctypes.c_void_p * n)(*[o.data_ptr() for o in outs])
    _check(load().cwt_exec_batch(hp, sp, op, n, ctypes.c_void_p(workspace.data_ptr() if workspace is not None else 0),
                                 ctypes.c_void_p(st.cuda_stream)))
    return outs
