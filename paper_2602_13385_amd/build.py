"""Builds libscf.so (HIP for gfx950) in-tree with hipcc.

The library is the compiled product: every step of the hot path runs in its
kernels.  Compilation flags: -O3, gfx950 only, and packed FP32 instructions
disabled (-packed-fp32-ops target feature).
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libscf.so")
BUILD = os.path.join(ROOT, "_build")

SOURCES = ["scf_api.cpp", "scf_cadence.cpp", "scf_small.hip", "scf_select.hip", "scf_noalloc.hip",
           "scf_ceiling.hip",
           "scf_engines_f32_exact.hip", "scf_engines_f32_generic.hip",
           "scf_engines_f64_exact.hip", "scf_engines_f64_generic.hip"]
HEADERS = ["host_field.h", "scf_device.h", "scf_dual.h", "scf_internal.h", "scf_kernels.h",
           "scf_plan.h"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
COMMON = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-Wno-unused-command-line-argument"]


def _obj(src):
    return os.path.join(BUILD, os.path.splitext(src)[0] + ".o")


def _compile(src, verbose):
    cmd = [HIPCC] + COMMON + ["-c", os.path.join(CSRC, src), "-o", _obj(src)]
    if src.endswith(".cpp"):
        cmd = [HIPCC] + COMMON + ["-x", "hip", "-c", os.path.join(CSRC, src), "-o", _obj(src)]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"hipcc failed on {src}")
    return _obj(src)


def build(verbose: bool = False, jobs: int = 6) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose), SOURCES))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
