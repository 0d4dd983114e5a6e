"""Build libhf.so (HIP for gfx950) and libhf_cpu.so (OpenMP) in-tree.

Every translation unit under csrc/ is compiled with hipcc to an object in
parallel and linked into paper_2010_10039_amd/libhf.so; cpu/hf_cpu.cpp is
compiled with g++ -fopenmp into paper_2010_10039_amd/libhf_cpu.so.  Run as
``python -m paper_2010_10039_amd.build``.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
OBJDIR = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libhf.so")
CPU_SRC = os.path.join(PKG, "cpu", "hf_cpu.cpp")
CPU_LIB = os.path.join(PKG, "libhf_cpu.so")
ARCH = "gfx950"

HIPCC_FLAGS = [
    f"--offload-arch={ARCH}",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-Wall",
    "-Wno-unused-result",
    # no packed-FP32 instructions anywhere in the library
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    f"-I{INCLUDE}",
    f"-I{CSRC}",
]


def _hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found: install ROCm or set HIPCC")


def sources() -> list[str]:
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))


def _compile(src: str) -> str:
    obj = os.path.join(OBJDIR, os.path.basename(src)[:-4] + ".o")
    cmd = [_hipcc(), *HIPCC_FLAGS, "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{r.stdout}\n{r.stderr}")
    return obj


def build_cpu(verbose: bool = False) -> str:
    """Compile the multi-core CPU baseline (cpu/hf_cpu.cpp) into libhf_cpu.so."""
    tmp = CPU_LIB + ".tmp"
    cmd = ["g++", "-O3", "-std=c++17", "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wextra", f"-I{INCLUDE}",
           CPU_SRC, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"g++ failed on {CPU_SRC}:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, CPU_LIB)
    if verbose:
        print(f"built {CPU_LIB}")
    return CPU_LIB


def build(verbose: bool = False) -> str:
    """Compile every csrc/*.hip for gfx950 and link libhf.so (and the CPU
    baseline library); returns libhf.so's path."""
    os.makedirs(OBJDIR, exist_ok=True)
    srcs = sources()
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs) + 1)) as ex:
        cpu = ex.submit(build_cpu, verbose)
        objs = list(ex.map(_compile, srcs))
        cpu.result()
    tmp = LIB + ".tmp"
    cmd = [_hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
