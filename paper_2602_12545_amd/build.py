"""Builds libfld.so (HIP, gfx950) in the package directory with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libfld.so")
SOURCES = [os.path.join(HERE, "csrc", f) for f in ("fld_host.hip", "fld_batch.hip", "fld_tune.hip", "fld_forest.hip")]
HEADERS = [os.path.join(HERE, "csrc", f) for f in ("fld_internal.hpp", "fld_kernels.hpp", "fld_line.hpp", "fld_sub.hpp", "fld_mg.hpp", "fld_dense.hpp", "fld_band.hpp", "fld_batch.hpp")] + \
          [os.path.join(ROOT, "include", "fld.h")]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # keep the compiler from forming packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
    "-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc"),
]


def build(verbose: bool = True) -> str:
    tmp = LIB + ".tmp"
    cmd = [HIPCC, *FLAGS, *SOURCES, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build()
    sys.exit(0)
