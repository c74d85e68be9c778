"""Build libctaux_hip.so for gfx950 with hipcc (in-tree, no JIT cache).

Usage: python -m paper_1010_3690_amd.build [--jobs N]
"""

from __future__ import annotations

import argparse
import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIBDIR = os.path.join(HERE, "lib")
LIB = os.path.join(LIBDIR, "libctaux_hip.so")
SOURCES = ["api.hip", "k_block.hip", "k_prep.hip", "k_propose.hip", "k_skinny.hip", "k_update.hip", "k_measure.hip",
           "k_refine.hip", "k_invert.hip", "build_n.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
# Packed FP32 instructions are kept out of every kernel (plain FP32 code only).
CFLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-Xclang", "-target-feature",
          "-Xclang", "-packed-fp32-ops", "-I", os.path.join(ROOT, "include"), "-I", CSRC,
          "-Wall", "-Wno-unused-result"]


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *CFLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    warn = "\n".join(l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l and l.strip())
    if warn.strip():
        sys.stderr.write(warn + "\n")
    return obj


CPU_LIB = os.path.join(LIBDIR, "libctaux_cpu.so")
CXX = os.environ.get("CXX", "g++")
# the host library runs on other x86-64 hosts than the build's: AVX2 + FMA, no -march=native
CPU_FLAGS = ["-O3", "-std=c++17", "-fPIC", "-shared", "-mavx2", "-mfma", "-Wall", "-I", os.path.join(ROOT, "include")]


def build_cpu() -> str:
    """The host (CPU) submatrix library, libctaux_cpu.so."""
    os.makedirs(LIBDIR, exist_ok=True)
    tmp = CPU_LIB + ".tmp"
    subprocess.check_call([CXX, *CPU_FLAGS, "-o", tmp, os.path.join(CSRC, "cpu_submatrix.cpp")])
    os.replace(tmp, CPU_LIB)
    return CPU_LIB


def build(jobs: int = 8) -> str:
    os.makedirs(BUILD, exist_ok=True)
    os.makedirs(LIBDIR, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    build_cpu()
    return LIB


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=8)
    a = ap.parse_args()
    print(build(a.jobs))
