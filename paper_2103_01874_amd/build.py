"""Build libppe.so (HIP, gfx950) in-tree with hipcc.

Usage: python -m paper_2103_01874_amd.build   (or call build()).
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libppe.so")
HOSTCHECK = os.path.join(HERE, "libppe_hostcheck.so")

HIP_FLAGS = [
    "-O3",
    "-std=c++17",
    "--offload-arch=gfx950",
    "-fPIC",
    "-shared",
    # no packed-FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm is required to build libppe.so)")


def _compile(src: str, out: str, extra=(), verbose=False):
    tmp = out + ".tmp"
    cmd = [hipcc(), *HIP_FLAGS, *extra, "-I", os.path.join(ROOT, "include"), "-I", CSRC, src, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"hipcc failed building {os.path.basename(out)}")
    os.replace(tmp, out)


def build(verbose: bool = False) -> str:
    """Compile libppe.so (the library) and libppe_hostcheck.so (CPU test support)."""
    _compile(os.path.join(CSRC, "ppe_lib.hip"), LIB, verbose=verbose)
    _compile(os.path.join(CSRC, "hostcheck.cpp"), HOSTCHECK, extra=("-x", "hip"), verbose=verbose)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
