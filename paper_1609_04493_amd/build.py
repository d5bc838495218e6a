"""Builds libpdyn.so in-tree with hipcc for gfx950.

All HIP code is compiled with packed FP32 instructions disabled
(-packed-fp32-ops): some of their forms have produced silently wrong results
on the target machines, and the kernels are written for unpacked FP32/FP64
VALU throughput.
"""

from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libpdyn.so")
ARCH = "gfx950"

HIP_FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wno-unused-command-line-argument"]


def hipcc() -> str:
    return os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc")


def sources():
    return [os.path.join(CSRC, f) for f in sorted(os.listdir(CSRC)) if f.endswith(".hip")]


PEAKS_LIB = os.path.join(HERE, "libpdyn_peaks.so")
PEAKS_SRC = os.path.join(CSRC, "peaks", "peaks.hip")


def _hipcc_shared(out: str, srcs, verbose: bool):
    tmp = out + ".tmp"
    cmd = [hipcc(), *HIP_FLAGS, "-shared", "-o", tmp, *srcs]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"hipcc failed building {os.path.basename(out)}")
    os.replace(tmp, out)


def build(verbose: bool = False) -> str:
    """libpdyn.so (the dynamics library), then libpdyn_peaks.so (the measured roofline denominators)."""
    _hipcc_shared(LIB, sources(), verbose)
    _hipcc_shared(PEAKS_LIB, [PEAKS_SRC], verbose)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
