"""Build the HIP library libtw.so for gfx950 in-tree (hipcc cross-compiles; no GPU needed).

Usage: python -m paper_2310_07119_amd.build
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
OUT = os.path.join(PKG, "libtw.so")
EXAMPLE = os.path.join(PKG, "tw_c_example")
BUILD = os.path.join(ROOT, "_build")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
COMMON = ["-O3", f"--offload-arch={ARCH}", "-std=c++20", "-fPIC",
          # packed FP32 instructions stay off: some of their forms have given wrong results on this hardware
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-I", os.path.join(ROOT, "include")]
# The sampler must not contract a*b+c into fma: its draws are defined as a
# fixed sequence of correctly rounded operations.
PER_FILE = {"kernels_sample.hip": ["-ffp-contract=off"]}
SOURCES = ["api.hip", "tune.hip", "kernels_step.hip", "kernels_cols.hip", "kernels_slab.hip", "kernels_batch.hip",
           "kernels_sample.hip", "kernels_moments.hip", "kernels_tracers.hip", "kernels_fno.hip", "fno.hip",
           "noalloc.hip"]


def _compile(src):
    obj = os.path.join(BUILD, src.replace(".hip", ".o"))
    cmd = [HIPCC, "-c", os.path.join(CSRC, src), "-o", obj] + COMMON + PER_FILE.get(src, [])
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    return obj


def build(verbose=True):
    os.makedirs(BUILD, exist_ok=True)
    jobs = min(len(SOURCES), int(os.environ.get("MAX_JOBS", "8")))
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = OUT + ".tmp"
    cmd = [HIPCC, "-shared", "-o", tmp] + objs + [f"--offload-arch={ARCH}", "-fPIC"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, OUT)
    # a host program that uses the C ABI directly (tests/c_abi_example.cpp)
    example = os.path.join(ROOT, "tests", "c_abi_example.cpp")
    if os.path.exists(example):
        cmd = [HIPCC, "-O2", "-std=c++17", "-I", os.path.join(ROOT, "include"), example, "-o", EXAMPLE,
               "-L", PKG, "-ltw", "-Wl,-rpath,$ORIGIN"]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"C ABI example build failed:\n{r.stderr}")
    if verbose:
        print(f"built {OUT}")
    return OUT


if __name__ == "__main__":
    build()
    sys.exit(0)
