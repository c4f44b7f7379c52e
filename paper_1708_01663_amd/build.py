"""Build the CISOR HIP library (libcisor.so) in-tree for gfx950.

Usage: ``python -m paper_1708_01663_amd.build`` (or ``build()`` from Python).
Every call recompiles all sources.
"""

from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libcisor.so")
SOURCES = ["conv.hip", "solver.hip", "gemm.hip", "tv.hip", "fista.hip", "nn.hip", "setup.cpp", "cisor.cpp",
           "batch.cpp", "vec3d.hip", "vec3d.cpp", "apg.hip"]
# conv_p.hip holds the operator kernels of one transform length; it is built
# once per length (the list must match CISOR_FFT_SIZES in conv_cfg.hpp).
FFT_SIZES = [64, 128, 192, 256, 384, 512, 768, 1024]
ARCH = os.environ.get("CISOR_OFFLOAD_ARCH", "gfx950")
FLAGS = ["-std=c++17", "-O3", "-fPIC", f"--offload-arch={ARCH}",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-command-line-argument"]


def _hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False, jobs: int | None = None) -> str:
    hipcc = _hipcc()
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)

    def compile_one(unit):
        src, defs = unit if isinstance(unit, tuple) else (unit, [])
        obj = os.path.join(objdir, src + "".join("." + d.split("=")[-1] for d in defs) + ".o")
        dflags = [f"-D{d}" for d in defs]
        cmd = [hipcc, *FLAGS, *dflags, "-c", os.path.join(CSRC, src), "-o", obj]
        if src.endswith(".cpp"):
            cmd = [hipcc, "-x", "hip", *FLAGS, *dflags, "-c", os.path.join(CSRC, src), "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"compiling {src} failed:\n{r.stderr}")
        if verbose and r.stderr.strip():
            print(r.stderr, file=sys.stderr)
        return obj

    units = [("conv_p.hip", [f"CISOR_P={p}"]) for p in FFT_SIZES] + SOURCES
    jobs = jobs or min(len(units), os.cpu_count() or 4)
    with ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(compile_one, units))
    tmp = LIB + ".tmp"
    cmd = [hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp, "-pthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"linking libcisor.so failed:\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
