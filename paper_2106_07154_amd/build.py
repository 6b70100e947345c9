"""Build liblts.so (HIP, gfx950) in place next to this file.

    python -m paper_2106_07154_amd.build
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "liblts.so")
SOURCES = [os.path.join(CSRC, n) for n in ("lts_api.cpp", "lts_ensemble.cpp", "lts_surrogate.cpp",
                                             "lts_kernels.hip", "lts_mpnn.hip",
                                             "lts_noalloc.hip")]
HEADERS = [os.path.join(CSRC, "lts_internal.h"), os.path.join(CSRC, "lts_host.h"),
           os.path.join(CSRC, "lts_mpnn.h"), os.path.join(ROOT, "include", "lts.h"),
           os.path.join(ROOT, "include", "lts_surrogate.h")]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
# Packed FP32 instructions are disabled for every HIP translation unit.
FLAGS = ["-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-shared",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-command-line-argument", "-I", os.path.join(ROOT, "include")]


def build_lib(verbose: bool = False) -> str:
    tmp = LIB + f".tmp{os.getpid()}"
    cmd = [HIPCC] + FLAGS + ["-o", tmp] + SOURCES
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


def stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(s) > t for s in SOURCES + HEADERS)


if __name__ == "__main__":
    print(build_lib(verbose=True))
    sys.exit(0)
