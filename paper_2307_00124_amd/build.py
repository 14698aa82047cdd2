"""Build the HIP library libbfpmg.so for gfx950 in the package directory.

Every source is compiled with hipcc (in parallel), then linked into one
shared object. Packed-FP32 instructions are disabled for all device code.
Run ``python paper_2307_00124_amd/build.py`` (by path: importing the package
loads the library) or call ``build()``.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libbfpmg.so")
OBJ = os.path.join(HERE, "_build")
# heaviest translation units first (they are compiled in parallel)
SOURCES = ["k_star_x32.hip", "k_star_x16.hip", "k_star_x8.hip", "k_transfer2d.hip",
           "k_transfer3d.hip", "k_point.hip", "k_exec.hip", "fp64mg.hip", "noalloc.hip", "k_tiles.hip", "k_band.hip", "k_vcycle.hip", "k_star.hip", "k_transfer.hip",
           "api.cpp", "mg.cpp", "server.cpp", "estimate.cpp", "fe.cpp"]
ARCH = os.environ.get("BFPMG_ARCH", "gfx950")
FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-result"]


def _hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _compile(src: str) -> str:
    obj = os.path.join(OBJ, os.path.splitext(src)[0] + ".o")
    cmd = [_hipcc(), *FLAGS, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compiling {src} failed:\n{r.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(OBJ, exist_ok=True)
    jobs = min(len(SOURCES), max(1, os.cpu_count() or 1))
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = OUT + ".tmp"
    cmd = [_hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"linking failed:\n{r.stderr}")
    os.replace(tmp, OUT)
    if verbose:
        print(f"built {OUT}")
    return OUT


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
