"""Builds libdefmm.so in-tree: the host plan builder with g++ (no FP
contraction, so traversal decisions are reproducible) and the HIP kernels and
C ABI with hipcc for gfx950."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libdefmm.so")
ARCH = os.environ.get("DEFMM_OFFLOAD_ARCH", "gfx950")

HIP_FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
             # no packed FP32 instructions anywhere in device code
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wno-unused-result"]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


def build(verbose: bool = False, jobs: int = 3) -> str:
    bdir = os.path.join(HERE, "_build")
    os.makedirs(bdir, exist_ok=True)
    objs = []
    host_obj = os.path.join(bdir, "plan_build.o")
    cmds = [["g++", "-O2", "-std=c++17", "-fPIC", "-ffp-contract=off", "-pthread", "-c",
             os.path.join(CSRC, "plan_build.cpp"), "-o", host_obj]]
    objs.append(host_obj)
    layout_obj = os.path.join(bdir, "fourier_layout.o")
    cmds.append(["g++", "-O2", "-std=c++17", "-fPIC", "-c", os.path.join(CSRC, "fourier_layout.cpp"), "-o", layout_obj])
    objs.append(layout_obj)
    for src in ("kernels.hip", "capi.hip", "build_device.hip"):
        obj = os.path.join(bdir, src.replace(".hip", ".o"))
        cmds.append(["hipcc", *HIP_FLAGS, "-c", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    procs = []
    for c in cmds:
        if verbose:
            print(" ".join(c), flush=True)
        procs.append(subprocess.Popen(c))
    rc = [p.wait() for p in procs]
    if any(rc):
        raise RuntimeError(f"compilation failed: {rc}")
    _run(["hipcc", "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-pthread", "-o", LIB + ".tmp"],
         verbose)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
