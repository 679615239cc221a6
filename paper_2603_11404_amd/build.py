"""Builds libtk.so (HIP for gfx950) in-tree with hipcc.

Usage: python -m paper_2603_11404_amd.build   (or call build_library()).
"""
from __future__ import annotations

import concurrent.futures
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
    "-ffp-contract=off",          # no implicit FMA: identical rounding in every form of the path
    "-fno-fast-math",
    "-mcode-object-version=5",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
    "-Wno-unused-function",
    "-Wno-unused-result",
    "-Rpass-analysis=kernel-resource-usage",   # per-kernel register / scratch report, checked below
]


def resource_problems(diagnostics: str) -> list[str]:
    """Kernels whose resource report shows private (scratch) memory or vector
    register spills: every kernel of the library is meant to live in registers
    and LDS (scalar spills go to vector-register lanes and are allowed)."""
    bad, name = [], None
    for line in diagnostics.splitlines():
        if "remark:" not in line:
            continue
        text = line.split("remark:", 1)[1].strip()
        if text.startswith("Function Name:"):
            name = text.split(":", 1)[1].split("[")[0].strip()
        for key in ("ScratchSize [bytes/lane]:", "VGPRs Spill:"):
            if text.startswith(key):
                value = int(text[len(key):].split("[")[0].strip())
                if value != 0:
                    bad.append(f"{name}: {key} {value}")
    return bad


# Sources compiled on their own with extra flags.  raster.hip: the chunk
# claims of its kernels are lane-0 LDS atomics whose results are read many
# instructions later; the compiler's atomic optimizer rewrites such an atomic
# into a form that waits for the result right away.
SOURCE_FLAGS = {
    "raster.hip": ["-mllvm", "-amdgpu-atomic-optimizer-strategy=None"],
}


def sources() -> list[str]:
    src = os.path.join(HERE, "csrc")
    return sorted(glob.glob(os.path.join(src, "*.hip")) + glob.glob(os.path.join(src, "*.cpp")))


def _run(cmd: list[str], verbose: bool) -> str:
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed building libtk.so")
    return res.stdout + res.stderr


def build_library(verbose: bool = False) -> str:
    """Compile every HIP/C++ source under csrc/ into paper_2603_11404_amd/libtk.so."""
    tmp = LIB + ".tmp"
    inc = ["-I", os.path.join(ROOT, "include")]
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    jobs = []
    for src in sources():
        obj = os.path.join(objdir, os.path.basename(src) + ".o")
        extra = SOURCE_FLAGS.get(os.path.basename(src), [])
        jobs.append(([HIPCC, *FLAGS, *extra, *inc, "-c", "-o", obj, src], obj))
    # one object per source, compiled side by side, then linked
    with concurrent.futures.ThreadPoolExecutor(max_workers=min(4, len(jobs))) as ex:
        diag = "".join(ex.map(lambda j: _run(j[0], verbose), jobs))
    diag += _run([HIPCC, "--offload-arch=gfx950", "-fPIC", "-shared", "-o", tmp, *[o for _, o in jobs]], verbose)
    bad = resource_problems(diag)
    if bad:
        os.remove(tmp)
        raise RuntimeError("kernels using scratch memory or spilling:\n  " + "\n  ".join(bad))
    warn = "\n".join(l for l in diag.splitlines() if "packed-fp32-ops" not in l and "remark:" not in l
                     and "Rpass-analysis" not in l and l.strip() and not l.lstrip().startswith(("|", "^")))
    if verbose and warn.strip():
        sys.stderr.write(warn + "\n")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build_library(verbose=True))
