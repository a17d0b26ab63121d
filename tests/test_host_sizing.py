"""The library's host sizing and planning code built with the address and
undefined-behaviour sanitizers and run on the CPU (no GPU): drift-scan time
groups, request footprints, type-3 workspaces, matrix-core chunking, the
geometry and snapshot plans and the planned-FFT table, on the degenerate
cases (empty sky, one source, one antenna, one time, zero budget)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2506_02130_amd", "csrc")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def test_host_sizing_under_sanitizers(tmp_path):
    cxx = shutil.which("g++")
    if cxx is None or not os.path.isdir(os.path.join(ROCM, "include", "hip")):
        pytest.skip("g++ or the HIP headers are missing")
    exe = str(tmp_path / "host_sizing")
    srcs = [os.path.join(ROOT, "tests", "host_sizing_main.cpp")] + [
        os.path.join(CSRC, f) for f in ("plan.cpp", "sizing.cpp", "fft_plans.cpp")]
    cmd = [cxx, "-std=c++17", "-O1", "-g", "-ffp-contract=off", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-D__HIP_PLATFORM_AMD__",
           "-I", os.path.join(ROCM, "include"), "-I", CSRC, "-I", os.path.join(ROOT, "include"),
           *srcs, "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=120)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "all passed" in r.stdout
