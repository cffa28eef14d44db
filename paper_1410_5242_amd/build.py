"""Build libkpm.so (HIP, gfx950) in-tree with hipcc.

Every translation unit is compiled for gfx950 only, with the packed-FP32
instruction selection disabled, then linked into one shared library next to
this file.  Run ``python -m paper_1410_5242_amd.build``.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libkpm.so")
SOURCES = ["kpm_runtime.cpp", "kpm_build.hip", "kpm_spmmv.hip", "kpm_dos.hip",
           "kpm_sweep_c128_large.hip", "kpm_sweep_c128_small.hip",
           "kpm_sweep_c64_large.hip", "kpm_sweep_c64_small.hip", "kpm_lattice.hip",
           "kpm_batched_c64.hip", "kpm_batched_c128.hip", "kpm_mlp.hip", "kpm_start.hip", "kpm_gather_c64.hip", "kpm_gather_c128.hip",
           "kpm_naive.hip", "kpm_lanczos.hip", "kpm_stream.hip", "kpm_sell.hip"]
ARCH = "gfx950"

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
]


def _compile(src: str, verbose: bool) -> str:
    obj = os.path.join(OBJ, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *FLAGS, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    return obj


def build(verbose: bool = False, jobs: int = 8) -> str:
    os.makedirs(OBJ, exist_ok=True)
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose), SOURCES))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
    sys.exit(0)
