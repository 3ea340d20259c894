"""The library's host C++ (threaded Jacobi SVD, mask codes and the Lanczos
norm of a masked grid, brick occupancy, the serving loop's first-fit
allocator) built with g++ under AddressSanitizer and UndefinedBehaviorSanitizer
and run on the CPU (tests/sanitize/host_check.cpp). No device code is built."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2401_12890_amd", "csrc")


def test_host_code_under_sanitizers(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None or not os.path.isdir("/opt/rocm/include"):
        pytest.skip("needs g++ and the ROCm headers")
    exe = tmp_path / "host_check"
    sanitize = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                "-fno-omit-frame-pointer"]
    cmd = [gxx, "-std=c++20", "-O1", "-g", "-D__HIP_PLATFORM_AMD__", "-I", CSRC,
           "-I", os.path.join(ROOT, "include"), "-I", "/opt/rocm/include"] + sanitize + [
        os.path.join(ROOT, "tests", "sanitize", "host_check.cpp"),
        os.path.join(CSRC, "svd.cpp"), os.path.join(CSRC, "mask.cpp"),
        "-o", str(exe), "-lpthread"]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ,
               ASAN_OPTIONS="detect_leaks=1:abort_on_error=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "host checks passed" in r.stdout
