"""Build libmsp.so (HIP for gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INC = os.path.join(ROOT, "include")
OUT = os.path.join(HERE, "libmsp.so")
BUILD = os.path.join(HERE, "_build")

ARCH = "gfx950"
# packed FP32 instructions are disabled for all device code
NO_PK_F32 = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
HIPFLAGS = ["-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC", "-Wall",
            "-Wno-unused-function", *NO_PK_F32, f"-I{INC}", f"-I{CSRC}"]
HOSTFLAGS = ["-O2", "-std=c++17", "-fPIC", "-Wall", "-ffp-contract=off", f"-I{INC}", f"-I{CSRC}"]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)


def build(verbose: bool = False) -> str:
    """Compile every source and link libmsp.so (always recompiles)."""
    os.makedirs(BUILD, exist_ok=True)
    objs = []
    host = os.path.join(BUILD, "msp_host.o")
    _run(["g++", *HOSTFLAGS, "-c", os.path.join(CSRC, "msp_host.cpp"), "-o", host], verbose)
    objs.append(host)
    for src in ("msp_kernels.hip", "msp_chain.hip", "msp_api.cpp"):
        obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
        _run(["hipcc", *HIPFLAGS, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj], verbose)
        objs.append(obj)
    tmp = OUT + f".tmp{os.getpid()}"
    _run(["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs, "-pthread"],
         verbose)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    build(verbose=True)
    print(OUT)
    sys.exit(0)
