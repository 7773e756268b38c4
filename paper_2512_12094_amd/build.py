"""Builds libpp.so (the HIP library behind include/pp.h) for gfx950.

All device code is compiled for gfx950 only, with floating-point
contraction off (the gate rule's products and sums round exactly like the
plain definition) and without packed FP32 instructions."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libpp.so")
SOURCES = [os.path.join(CSRC, "pp_api.hip")]
DEPS = SOURCES + [os.path.join(CSRC, f) for f in ("pp_kernels.hpp", "pp_merge.hpp", "pp_layer.hpp", "pp_sort.hpp", "pp_types.h", "pp_fixed.h")] + \
    [os.path.join(ROOT, "include", "pp.h")]


def command(out: str):
    return ["hipcc", "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
            "-ffp-contract=off", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wall", "-Wno-unused-function",
            f"-I{os.path.join(ROOT, 'include')}", f"-I{CSRC}", "-o", out] + SOURCES


def build(force: bool = True, verbose: bool = False) -> str:
    if not force and os.path.exists(LIB) and all(
            os.path.getmtime(LIB) >= os.path.getmtime(d) for d in DEPS):
        return LIB
    tmp = LIB + f".tmp{os.getpid()}"
    cmd = command(tmp)
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(force=True, verbose=True)
    print(LIB)
    sys.exit(0)
