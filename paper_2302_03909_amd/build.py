"""Build libcwt.so for gfx950 in-tree with hipcc (no JIT, no torch extension).

    python -m paper_2302_03909_amd.build        # or build() from Python

Every source is compiled with -O3 --offload-arch=gfx950 and packed FP32
instructions disabled; the objects are linked into
paper_2302_03909_amd/libcwt.so.  The measurement probe (csrc/probe_dft16.hip,
no part of the transform) becomes a library of its own, libcwt_probe.so.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libcwt.so")
PROBE_LIB = os.path.join(HERE, "libcwt_probe.so")
PROBE_SOURCES = ["probe_dft16.hip"]
ROOT = os.path.dirname(HERE)
SOURCES = ["cwt_plan.cpp", "cwt_spline_plan.cpp", "cwt_fft.hip", "cwt_seg.hip", "cwt_spline.hip", "cwt_tables.hip", "cwt_wps.hip",
           "cwt_wps_b1.hip", "cwt_wps_b2.hip", "cwt_wps_b4.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", os.path.join(ROOT, "include"), "-Wall", "-Wno-unused-function"]


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    if src.endswith(".cpp"):
        cmd = [HIPCC, *FLAGS, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = SOURCES + PROBE_SOURCES
    with cf.ThreadPoolExecutor(max_workers=min(len(srcs), os.cpu_count() or 4)) as ex:
        objs = dict(zip(srcs, ex.map(_compile, srcs)))
    for lib, names in ((LIB, SOURCES), (PROBE_LIB, PROBE_SOURCES)):
        tmp = lib + ".tmp"
        r = subprocess.run([HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp,
                            *(objs[n] for n in names)], capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"link of {os.path.basename(lib)} failed:\n{r.stderr}")
        os.replace(tmp, lib)
        if verbose:
            print("built", lib)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
