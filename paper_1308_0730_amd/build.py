"""Build libmvd.so (gfx950) in-tree with hipcc.

Three translation units compile in parallel: the HIP kernels, the HIP
runtime behind the C ABI, and the FP64 host preparation code.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libmvd.so")
BUILD = os.path.join(HERE, "_build")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = os.environ.get("MVD_ARCH", "gfx950")
# packed FP32 instructions stay off: plain float code only
GPU_FLAGS = ["--offload-arch=" + ARCH, "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
COMMON = ["-O3", "-std=c++17", "-fPIC", "-I" + INCLUDE, "-I" + CSRC]

# longest first: they compile in parallel
SOURCES = [
    ("mvd_kernels.hip", True),
    ("mvd_adjoint.hip", True),
    ("mvd_exact_class.hip", True),
    ("mvd_exact_z.hip", True),
    ("mvd_exact_zext.hip", True),
    ("mvd_exact_x_comb.hip", True),
    ("mvd_exact_x_win.hip", True),
    ("mvd_exact_x.hip", True),
    ("mvd_exact_y.hip", True),
    ("mvd_kernels_ct.hip", True),
    ("mvd_weights.hip", True),
    ("mvd_embed.hip", True),
    ("mvd_runtime.cpp", True),
    ("mvd_host.cpp", False),
]


def _compile(src, gpu):
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    path = os.path.join(CSRC, src)
    if gpu:
        cmd = [HIPCC, "-x", "hip"] + GPU_FLAGS + COMMON + ["-c", path, "-o", obj]
    else:
        # complex products without the inf/nan recovery calls (all values are finite)
        cmd = ["g++"] + COMMON + ["-fcx-limited-range", "-c", path, "-o", obj, "-pthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("compile failed: " + " ".join(cmd) + "\n" + r.stdout + r.stderr)
    return obj


def build(verbose=True):
    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(lambda s: _compile(*s), SOURCES))
    tmp = LIB + ".tmp"
    cmd = [HIPCC] + GPU_FLAGS + ["-shared", "-fPIC", "-o", tmp] + objs + [
        "-pthread", "-Wl,-rpath,/opt/rocm/lib", "-L/opt/rocm/lib", "-lamdhip64"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed: " + " ".join(cmd) + "\n" + r.stdout + r.stderr)
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build()
    sys.exit(0)
