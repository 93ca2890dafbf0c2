"""Build libpic355.so (gfx950) in-tree with hipcc.

Each HIP source is compiled to an object in parallel, then linked into one
shared library next to this file.  Packed FP32 instructions are disabled
(-packed-fp32-ops): every float operation issues as a scalar VALU op.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libpic355.so")
SOURCES = ["kernels_particles.hip", "kernels_grid.hip", "capi.hip"]
MICRO_SRC = "microbench.hip"
MICRO_LIB = os.path.join(HERE, "libpic355_micro.so")
ARCH = os.environ.get("PIC355_ARCH", "gfx950")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-fvisibility=hidden",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + os.path.join(ROOT, "include"), "-I" + CSRC,
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
]


def _compile(src):
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC] + FLAGS + ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    return obj


def _link(objs, lib):
    tmp = lib + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, lib)


def build(verbose=False):
    """Compile every HIP source for the target arch and link the library
    (and the separate atomic-throughput probe the benchmark script loads)."""
    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(max_workers=len(SOURCES) + 1) as ex:
        objs = list(ex.map(_compile, SOURCES + [MICRO_SRC]))
    _link(objs[:-1], LIB)
    _link(objs[-1:], MICRO_LIB)
    if verbose:
        print("built", LIB)
        print("built", MICRO_LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
