"""Build the host-orchestration harness: the library's sources compiled for
the host only (no device code) with AddressSanitizer on the host code, linked
with the host-only HIP stand-in (hip_stub.cpp) and the driver
(orchestration_driver.cpp) into one executable under _build/.

Usage: python tests/host_harness/build_harness.py  -> prints the executable path.
"""

from __future__ import annotations

import os
import re
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
CSRC = os.path.join(ROOT, "paper_1708_01663_amd", "csrc")
OUT = os.path.join(HERE, "_build")
EXE = os.path.join(OUT, "orchestration_driver")
sys.path.insert(0, os.path.join(ROOT, "paper_1708_01663_amd"))

ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
HIPCC = shutil.which("hipcc") or os.path.join(ROCM, "bin", "hipcc")
CLANGXX = os.path.join(ROCM, "llvm", "bin", "clang++")
# AddressSanitizer on the host side only (there is no device code in these objects)
HOST_FLAGS = ["-std=c++17", "-O1", "-g", "-fPIC", "-fno-omit-frame-pointer"]
HOST_ONLY = ["-x", "hip", "--offload-host-only", "-Wno-unused-command-line-argument",
             "-Xarch_host", "-fsanitize=address"]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"{' '.join(cmd)} failed:\n{r.stderr[-4000:]}")
    return r


def build() -> str:
    from build import FFT_SIZES, SOURCES   # the library's own source list
    os.makedirs(OUT, exist_ok=True)
    units = [(s, []) for s in SOURCES] + [("conv_p.hip", [f"CISOR_P={p}"]) for p in FFT_SIZES]

    def one(unit):
        src, defs = unit
        obj = os.path.join(OUT, src + "".join("." + d.split("=")[-1] for d in defs) + ".o")
        _run([HIPCC, *HOST_ONLY, *HOST_FLAGS, *[f"-D{d}" for d in defs], "-c", os.path.join(CSRC, src), "-o", obj])
        return obj

    with ThreadPoolExecutor(min(8, os.cpu_count() or 4)) as ex:
        objs = list(ex.map(one, units))
    # host-only objects refer to per-unit device images that do not exist: give
    # each an empty definition (the stand-in's registration ignores them)
    syms = set()
    for o in objs:
        out = _run(["nm", "-u", o]).stdout
        syms |= set(re.findall(r"\b(__hip_fatbin_[0-9a-f]+)\b", out))
    fat = os.path.join(OUT, "fatbin_stubs.cpp")
    with open(fat, "w") as fh:
        for s in sorted(syms):
            fh.write(f'extern "C" {{ char {s}[16] = {{0}}; }}\n')
    extra = []
    for src in (os.path.join(HERE, "hip_stub.cpp"), os.path.join(HERE, "orchestration_driver.cpp"), fat):
        obj = os.path.join(OUT, os.path.basename(src) + ".o")
        _run([CLANGXX, *HOST_FLAGS, "-fsanitize=address", "-D__HIP_PLATFORM_AMD__", f"-I{ROCM}/include",
              "-c", src, "-o", obj])
        extra.append(obj)
    _run([CLANGXX, "-fsanitize=address", *objs, *extra, "-o", EXE, "-lpthread"])
    return EXE


if __name__ == "__main__":
    print(build())
