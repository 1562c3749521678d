"""Builds libamnerf.so (the HIP kernels and the host C ABI) for gfx950, in-tree.

Usage: python paper_2310_01881_amd/build.py [-j N]   (run as a file: importing the package
loads the library this script builds)
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libamnerf.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

SOURCES = ["amnerf.cpp", "trav.hip", "scan.hip", "sort.hip", "mlp.hip", "mlp8.hip", "mlp_bwd.hip", "comp.hip",
           "train.hip", "prop.hip", "err.hip", "ess.hip", "ert.hip"]
# Packed fp32 arithmetic is disabled for all device code.
FLAGS = ["--offload-arch=gfx950", "-O3", "-fPIC", "-std=c++17", "-Wall", "-Wno-unused-function",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I" + os.path.join(ROOT, "include")]
# Kernels that post-process every matrix-core result with vector instructions keep their
# accumulators in ordinary VGPRs: in the accumulation registers each result would first be
# copied out (one v_accvgpr_read per value).
PER_FILE = {"prop.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form=1"],
            "mlp_bwd.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form=1"],
            "mlp8.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form=1"]}


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC] + FLAGS + PER_FILE.get(src, []) + ["-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s\n%s" % (" ".join(cmd), r.stdout, r.stderr))
    return obj


def build(jobs: int = 8) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed: %s\n%s" % (r.stdout, r.stderr))
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    j = 8
    if len(sys.argv) > 2 and sys.argv[1] == "-j":
        j = int(sys.argv[2])
    print(build(j))
