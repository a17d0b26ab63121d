"""Build libfv.so (the HIP kernels and the C-ABI runtime) for gfx950 with hipcc.

Every source is compiled to an object in parallel, then linked into
``paper_2506_02130_amd/libfv.so``.  Device code is built with packed FP32
instructions disabled; host code with FMA contraction off so that host-side
grid sizes are the exact IEEE value of their expression.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libfv.so")
ARCH = os.environ.get("FV_OFFLOAD_ARCH", "gfx950")

ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
HIPCC = shutil.which("hipcc") or os.path.join(ROCM, "bin", "hipcc")
CXX = shutil.which("g++") or "g++"
COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
          "-Wno-unused-but-set-variable", f"--offload-arch={ARCH}"]
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-munsafe-fp-atomics"]
HOST_ONLY_FLAGS = ["-ffp-contract=off"]

SOURCES = ["plan.cpp", "runtime.cpp", "batch.cpp", "server.cpp", "tune.cpp", "nufft.hip", "nufft_f32_2d.hip", "nufft_f32_3d.hip",
           "nufft_f64_2d.hip", "nufft_f64_3d.hip", "direct.hip", "zz.hip", "lattice.hip", "frontend.hip",
           "drift.cpp", "beams.hip", "beams.cpp", "polar.hip", "polar.cpp",
           "basis.hip", "basis.cpp", "noalloc.hip", "fft_reg.hip", "fft_reg_cols.hip",
           "fft_plans.cpp", "sizing.cpp"]


def _compile(src: str) -> str:
    import time
    t0 = time.time()
    path = os.path.join(CSRC, src)
    obj = os.path.join(BUILD, src + ".o")
    if src.endswith(".hip"):
        cmd = [HIPCC] + COMMON + ["-x", "hip"] + DEVICE_FLAGS
    else:
        # host-only translation units: plain C++ against the HIP runtime headers
        cmd = [CXX, "-O2", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function"] + HOST_ONLY_FLAGS + [
            "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROCM, "include")]
    cmd += ["-I", CSRC, "-I", os.path.join(HERE, "..", "include"), "-c", path, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {src}\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    if r.stderr.strip():
        sys.stderr.write(r.stderr)
    if os.environ.get("FV_BUILD_TIMES"):
        print(f"  {src}: {time.time() - t0:.1f}s")
    return obj


def build(jobs: int = 8, verbose: bool = True) -> str:
    os.makedirs(BUILD, exist_ok=True)
    # the FFT plan tables are generated source (committed); regenerated when
    # the generator is newer than them (the search takes about a minute)
    gen = os.path.join(CSRC, "gen_fft_plans.py")
    incs = [os.path.join(CSRC, f"fft_plans_{k}.inc") for k in ("rows", "cols")]
    if any(not os.path.exists(f) or os.path.getmtime(f) < os.path.getmtime(gen) for f in incs):
        r = subprocess.run([sys.executable, gen], capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"FFT plan generation failed\n{r.stdout}\n{r.stderr}")
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        order = sorted(SOURCES, key=lambda f: 0 if f.startswith("fft_reg") else 1)
        done = dict(zip(order, ex.map(_compile, order)))
        objs = [done[f] for f in SOURCES]
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs + [
        "-L", os.path.join(ROCM, "lib"), "-lamdhip64", "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build()
