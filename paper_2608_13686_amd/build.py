"""Builds the HIP library ``paper_2608_13686_amd/libsfhk.so`` for gfx950.

Every source is compiled with hipcc; packed FP32 instructions are disabled
(``-packed-fp32-ops``) for every HIP translation unit.
"""
import concurrent.futures as cf
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libsfhk.so")
OBJ = os.path.join(PKG, "_build")
SOURCES = ["abi.hip", "setup_kernels.hip", "propagate_f64.hip", "propagate_mixed.hip",
           "propagate_latency.hip", "serve.hip", "serve_abi.hip", "analysis.hip"]
ARCH = os.environ.get("SFHK_OFFLOAD_ARCH", "gfx950")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CFLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-I", os.path.join(ROOT, "include"), "-I", CSRC,
          "-Wall", "-Wno-unused-function"]
# The FP64 trajectory kernels run at an occupancy fixed by their LDS (two
# wavefronts per SIMD), so the machine scheduler is asked for instruction-level
# parallelism instead of occupancy (measured 0.65% faster on N2); the latency
# form runs one or two wavefronts per SIMD, whose step latency the same
# strategy shortens (4-6% measured).
EXTRA = {src: ["-mllvm", "-amdgpu-sched-strategy=max-ilp"]
         for src in ("propagate_f64.hip", "serve.hip", "propagate_latency.hip")}


def _compile(src, verbose):
    obj = os.path.join(OBJ, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *CFLAGS, *EXTRA.get(src, []), "-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose=False):
    os.makedirs(OBJ, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose), SOURCES))
    cmd = [HIPCC, "-shared", f"--offload-arch={ARCH}", "-o", LIB + ".tmp", *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
