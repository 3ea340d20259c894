"""Build libssmap.so in-tree with hipcc for gfx950.

The library is one shared object: host C++ (C ABI, setup, SVD, launch
sequence) plus HIP kernels. Flags: -O3, gfx950 only, packed-FP32 code
generation disabled for device code.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libssmap.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

SOURCES = ["ssmap.cpp", "server.cpp", "mask.cpp", "svd.cpp", "kernels_common.hip", "kernels_fused.hip", "kernels_gemm.hip"]
DEVICE_FLAGS = ["--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
COMMON = ["-O3", "-std=c++20", "-fPIC", "-Wall", "-Wno-unused-result", "-I", os.path.join(ROOT, "include")]


def build(verbose: bool = False) -> str:
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    objs = []
    for src in SOURCES:
        path = os.path.join(CSRC, src)
        obj = os.path.join(objdir, src + ".o")
        cmd = [HIPCC] + COMMON + ["-c", path, "-o", obj]
        cmd[1:1] = DEVICE_FLAGS   # host-only sources too: no device pass for other targets
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        objs.append(obj)
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs + ["-lpthread"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    # stand-alone read+write streaming reference used by the roofline notes
    exe = os.path.join(HERE, "copy_ceiling")
    cmd = [HIPCC] + DEVICE_FLAGS + ["-O3", "-std=c++20", os.path.join(CSRC, "copy_ceiling.hip"),
                                    "-o", exe]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
