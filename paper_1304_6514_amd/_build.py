"""Build libnv.so (HIP, gfx950) in-tree with hipcc.

Every translation unit is compiled with the automatic generation of packed
FP32 instructions switched off (``-Xclang -target-feature -Xclang
-packed-fp32-ops``); the integrator is written as scalar FP32/FP64 code.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libnv.so")
OBJDIR = os.path.join(PKG, "_build")
SOURCES = ["nv_capi.hip", "build_kernels.hip", "compose_kernels.hip", "batch.hip",
           "surrogate.hip", "linear.hip", "probe.hip"]
ARCH = "gfx950"

HIPCC_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-fvisibility=hidden",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result", "-I", INCLUDE, "-I", CSRC,
]


# Per-source flags: the integrator's step loops (included by these files) run
# faster in one-wave-per-SIMD builds when each loop starts on a 64-byte line.
SOURCE_FLAGS = {"build_kernels.hip": ["-falign-loops=64"], "batch.hip": ["-falign-loops=64"]}


def _hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if cand and (os.path.sep not in cand or os.path.exists(cand)):
            return cand
    return "hipcc"


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"command failed ({r.returncode}): {' '.join(cmd)}")
    return r


def build(verbose: bool = False, save_temps: bool = False) -> str:
    """Compile every HIP source for gfx950 and link libnv.so in the package."""
    os.makedirs(OBJDIR, exist_ok=True)
    hipcc = _hipcc()
    extra = ["-save-temps=obj"] if save_temps else []

    def compile_one(src):
        obj = os.path.join(OBJDIR, os.path.splitext(src)[0] + ".o")
        _run([hipcc, *HIPCC_FLAGS, *SOURCE_FLAGS.get(src, []), *extra, "-c",
              os.path.join(CSRC, src), "-o", obj], verbose)
        return obj

    with ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(compile_one, SOURCES))
    tmp = LIB + ".tmp"
    _run([hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs], verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
