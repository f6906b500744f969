"""Compile the HIP library (libmasw.so) for gfx950, in-tree.

Usage: python -m paper_2003_02256_amd.build   (or build() from Python)
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libmasw.so")
# test-only probe of the device special functions (tests/test_gpu_special.py)
PROBE_SRC = os.path.join(ROOT, "tests", "special_probe.hip")
PROBE_LIB = os.path.join(ROOT, "tests", "libspecial_probe.so")

SOURCES = ["masw_kernels.hip", "masw_runtime.hip", "masw_server.hip", "masw_classify.hip", "masw_noise.hip", "masw_inertia.hip",
           "masw_inertia_lone.hip", "masw_sweep_split.hip"]
HEADERS = ["masw_internal.hpp", "masw_math.hpp", "masw_special.hpp", "masw_host.hpp", "masw_pick.hpp", "masw_inertia.hpp",
           "masw_inertia_kernel.hpp", "masw_noise.hpp", "masw_sweep.hpp"]

# Packed FP32 instructions stay disabled; the compiler would otherwise form
# v_pk_* from ordinary float code.
HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
]


def hipcc() -> str:
    exe = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(exe):
        raise RuntimeError("hipcc not found")
    return exe


# roctx ranges around the library's calls and serving ticks
LIB_LIBS = ["-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx", "-Wl,-rpath,/opt/rocm/lib"]


def _compile(sources, out, verbose, libs=()):
    tmp = out + ".tmp"
    cmd = [hipcc(), *HIPCC_FLAGS, "-I", INCLUDE, "-I", CSRC, *sources, *libs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError(f"hipcc failed building {os.path.basename(out)}")
    os.replace(tmp, out)


def build(verbose: bool = False) -> str:
    """Always recompiles the library and the test probe; returns the library path."""
    _compile([os.path.join(CSRC, s) for s in SOURCES], LIB, verbose, LIB_LIBS)
    if os.path.exists(PROBE_SRC):
        _compile([PROBE_SRC], PROBE_LIB, verbose)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
