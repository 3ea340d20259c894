"""Build libssmap.so in-tree with hipcc for gfx950.

The library is one shared object: host C++ (C ABI, setup, SVD, launch
sequence) plus HIP kernels. Flags: -O3, gfx950 only, packed-FP32 code
generation disabled for device code. Sources compile in parallel.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libssmap.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

SOURCES = ["ssmap.cpp", "server.cpp", "mask.cpp", "svd.cpp", "kernels_common.hip",
           "kernels_fused.hip", "kernels_gemm.hip", "kernels_split.hip", "libgemm.cpp"]
DEVICE_FLAGS = ["--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
COMMON = ["-O3", "-std=c++20", "-fPIC", "-Wall", "-Wno-unused-result", "-I", os.path.join(ROOT, "include")]


def _jobs() -> int:
    try:
        return max(1, min(8, int(os.environ.get("MAX_JOBS", "") or (os.cpu_count() or 1))))
    except ValueError:
        return 4


def build(verbose: bool = False, csrc: str = CSRC, out: str = LIB, objdir: str | None = None) -> str:
    objdir = objdir or os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    cmds, objs = [], []
    for src in SOURCES:
        obj = os.path.join(objdir, src + ".o")
        # host-only sources too: no device pass for other targets
        cmds.append([HIPCC] + DEVICE_FLAGS + COMMON + ["-c", os.path.join(csrc, src), "-o", obj])
        objs.append(obj)

    def run(cmd):
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)

    with ThreadPoolExecutor(_jobs()) as ex:
        for f in [ex.submit(run, c) for c in cmds]:
            f.result()
    tmp = out + ".tmp"
    run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs +
        ["-L/opt/rocm/lib", "-lhipblaslt", "-lpthread"])
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
