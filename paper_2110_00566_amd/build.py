"""Build libmgglam.so (gfx950) in-tree with hipcc.

    python -m paper_2110_00566_amd.build

All HIP code is compiled with packed-FP32 instructions disabled
(``-target-feature -packed-fp32-ops``).
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libmgglam.so")
SOURCES = ["mg_api.hip", "pm.hip", "fft.hip", "kmo_background.cpp"]
HEADERS = ["mg_device.h", "mg_kernels.h", "mg_tiled.h", "mg_adjoint.h", "mg_adj_tiled.h", "mg_dc.h"]
ARCH = os.environ.get("MGGLAM_ARCH", "gfx950")


def hipcc() -> str:
    for c in (os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc"), "hipcc"):
        if os.path.sep not in c or os.path.exists(c):
            return c
    return "hipcc"


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc(), "--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-shared",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-Wall", "-Wno-unused-result", "-o", tmp] + [os.path.join(CSRC, s) for s in SOURCES]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
    sys.exit(0)
