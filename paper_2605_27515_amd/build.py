"""Build the HIP library liblindblad.so for gfx950 in-tree with hipcc.

Usage: python -m paper_2605_27515_amd.build   (or build() from Python).
The host C++ MPO builder and the device kernels go into one shared library
whose exported symbols are the C ABI of include/lindblad.h.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "liblindblad.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

SOURCES = ["engine.hip", "kernels.hip", "tdvp.hip", "capi_kernels.hip", "mpo.cpp", "hostla.cpp", "serve.cpp"]
HIP_FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-pthread",
             # packed FP32 instructions stay off: some of their forms have given
             # wrong results with no error
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wno-unused-result"]


def build(verbose: bool = False) -> str:
    objs = []
    build_dir = os.path.join(HERE, "_build")
    os.makedirs(build_dir, exist_ok=True)
    for src in SOURCES:
        path = os.path.join(CSRC, src)
        obj = os.path.join(build_dir, src + ".o")
        if src.endswith(".hip"):
            cmd = [HIPCC, *HIP_FLAGS, "-c", path, "-o", obj]
        else:
            cmd = [HIPCC, "-O3", "-std=c++17", "-fPIC", "-pthread", "-c", path, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        objs.append(obj)
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-pthread", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
