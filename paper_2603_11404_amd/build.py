"""Builds libtk.so (HIP for gfx950) in-tree with hipcc.

Usage: python -m paper_2603_11404_amd.build   (or call build_library()).
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libtk.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    "-ffp-contract=off",          # no implicit FMA: identical rounding in every form of the path
    "-fno-fast-math",
    "-mcode-object-version=5",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
    "-Wno-unused-function",
    "-Wno-unused-result",
]


def sources() -> list[str]:
    src = os.path.join(HERE, "csrc")
    return sorted(glob.glob(os.path.join(src, "*.hip")) + glob.glob(os.path.join(src, "*.cpp")))


def build_library(verbose: bool = False) -> str:
    """Compile every HIP/C++ source under csrc/ into paper_2603_11404_amd/libtk.so."""
    tmp = LIB + ".tmp"
    cmd = [HIPCC, *FLAGS, "-I", os.path.join(ROOT, "include"), "-o", tmp, *sources()]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed building libtk.so")
    warn = "\n".join(l for l in (res.stdout + res.stderr).splitlines() if "packed-fp32-ops" not in l)
    if verbose and warn.strip():
        sys.stderr.write(warn + "\n")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build_library(verbose=True))
