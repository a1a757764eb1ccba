"""Build libfse.so (HIP kernels for gfx950 + the C ABI) in-tree with hipcc.

Usage: python -m paper_1512_03210_amd.build  (or call build()).
Each translation unit is compiled in parallel into _build/, then linked into
paper_1512_03210_amd/libfse.so.  Always recompiles (no staleness guessing).
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.environ.get("FSE_BUILD_DIR", os.path.join(PKG, "_build"))
LIB = os.environ.get("FSE_LIB_OUT", os.path.join(PKG, "libfse.so"))

ARCH = os.environ.get("FSE_OFFLOAD_ARCH", "gfx950")
# Packed FP32 instructions are disabled for all device code.
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
COMMON = ["-std=c++17", "-O3", "-fPIC", f"--offload-arch={ARCH}", "-I", os.path.join(ROOT, "include")]
# Extra compile definitions (kernel variants for tuning), e.g. FSE_DEFINES="FSE_TWFULL FSE_PADFULL".
EXTRA = [f"-D{d}" for d in os.environ.get("FSE_DEFINES", "").split() if d]

SOURCES = [
    "fse_launch_f64.hip",
    "fse_launch_f32.hip",
    "fse_api.cpp",
    "fse_gausum.cpp",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm is required to build libfse.so)")


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [hipcc()] + COMMON + DEVICE_FLAGS + EXTRA
    if src.endswith(".cpp"):
        cmd += ["-x", "hip"]
    cmd += ["-c", os.path.join(CSRC, src), "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{res.stdout}\n{res.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(len(SOURCES), os.cpu_count() or 4)) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs + ["-lpthread"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{res.stdout}\n{res.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
