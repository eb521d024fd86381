"""Builds the HIP library ``librqmc.so`` for gfx950 with hipcc.

Every translation unit under ``csrc/`` is compiled in parallel and linked
into one shared library next to this file.  The build always recompiles
(it is the "does it build" check) unless ``only_if_stale`` is set.
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "librqmc.so")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
# Packed FP32 VALU forms are disabled: every FP32 operation is a plain
# single-lane instruction.
CFLAGS = ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-Wall",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-I" + INCLUDE, "-I" + CSRC]


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.cpp")))


def _compile(src: str, verbose: bool) -> str:
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    cmd = [HIPCC] + CFLAGS + ["-c", src, "-o", obj]
    if src.endswith(".cpp"):
        cmd = [HIPCC] + CFLAGS + ["-x", "hip", "-c", src, "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {os.path.basename(src)}:\n{r.stdout}\n{r.stderr}")
    return obj


def stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    deps = sources() + glob.glob(os.path.join(CSRC, "*.h")) + glob.glob(os.path.join(INCLUDE, "*.h"))
    return any(os.path.getmtime(d) > t for d in deps)


def build(verbose: bool = False, only_if_stale: bool = False, jobs: int = 8) -> str:
    if only_if_stale and not stale():
        return LIB
    os.makedirs(BUILD, exist_ok=True)
    srcs = sources()
    with cf.ThreadPoolExecutor(max_workers=min(jobs, len(srcs))) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose), srcs))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


# The CPU baseline generator (Algorithm 2, multi-core and SIMD): a host-only
# library of its own, built with g++ for x86-64-v3 (AVX2, FMA).
CSRC_CPU = os.path.join(HERE, "csrc_cpu")
LIB_CPU = os.path.join(HERE, "librqmc_cpu.so")


def build_cpu(verbose: bool = False) -> str:
    src = os.path.join(CSRC_CPU, "rq_cpu_alg2.cpp")
    cmd = ["g++", "-O3", "-std=c++17", "-fPIC", "-shared", "-fopenmp", "-march=x86-64-v3",
           "-ffp-contract=off", "-Wall", "-Wextra", "-I" + INCLUDE, src, "-o", LIB_CPU + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"g++ failed on rq_cpu_alg2.cpp:\n{r.stdout}\n{r.stderr}")
    os.replace(LIB_CPU + ".tmp", LIB_CPU)
    return LIB_CPU


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    build_cpu(verbose="-v" in sys.argv)
    print(LIB, LIB_CPU)
