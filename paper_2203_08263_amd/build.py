"""Build libnbody_hip.so (gfx950) in-tree with hipcc.

Usage: ``python -m paper_2203_08263_amd.build``.  Every HIP source is
compiled for gfx950 only, with packed-FP32 instruction selection disabled.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libnbody_hip.so")
SOURCES = ["nbody_kernels.hip", "nbody_nearfar.hip", "nbody_f32.hip", "nbody_api.hip"]
MICROBENCH = os.path.join(HERE, "valu_microbench")
ARCH = "gfx950"

HIPCC_FLAGS = [
    "--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-shared",
    "-Wall", "-Wno-unused-function",
    # No packed FP32 (v_pk_*_f32) instruction selection.
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
]


def hipcc() -> str:
    exe = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(exe):
        raise RuntimeError("hipcc not found; ROCm is required to build")
    return exe


def build(verbose: bool = False) -> str:
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc(), *HIPCC_FLAGS, *srcs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed building libnbody_hip.so")
    os.replace(tmp, LIB)
    return LIB


def build_microbench(verbose: bool = False) -> str:
    """The VALU issue-rate microbenchmark (a standalone gfx950 executable)."""
    flags = [f for f in HIPCC_FLAGS if f not in ("-fPIC", "-shared")]
    tmp = MICROBENCH + ".tmp%d" % os.getpid()
    cmd = [hipcc(), *flags, os.path.join(CSRC, "valu_microbench.hip"), "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed building valu_microbench")
    os.replace(tmp, MICROBENCH)
    return MICROBENCH


if __name__ == "__main__":
    print(build(verbose=True))
    print(build_microbench(verbose=True))
