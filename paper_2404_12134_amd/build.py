"""Build the gfx950 shared library libwetsand_mi.so from csrc/ (in-tree).

hipcc cross-compiles for gfx950 without a GPU.  Flags that matter for the
numerics: -ffp-contract=off (no FMA contraction: every fma in the kernels is
written out, so float64 results match a plain CPU evaluation bit for bit)
and no fast-math.  Packed FP32 instructions are disabled.
"""

from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libwetsand_mi.so")
OBJDIR = os.path.join(HERE, "_build")
# Per-source extra flags.  The DTW kernels never form a NaN from finite
# inputs (only +inf boundaries, sums and minima of non-negative values), so
# -fno-honor-nans lets min() map to a bare v_min_f64.
# The Soft-DTW kernels never subtract two infinities: every computed cell has
# at least one finite predecessor, so the same holds there.
SOURCES = {"wts_dtw.hip": ["-fno-honor-nans"], "wts_dtw32.hip": ["-fno-honor-nans"],
           "wts_soft.hip": ["-fno-honor-nans"], "wts_abi.hip": [], "wts_aux.hip": []}
ARCH = os.environ.get("WTS_OFFLOAD_ARCH", "gfx950")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
    "-fno-fast-math", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-command-line-argument",
]


def _compile(src: str) -> str:
    obj = os.path.join(OBJDIR, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *FLAGS, *SOURCES[src], "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed on " + src)
    return obj


# The VALU issue-rate microbenchmark behind the roofline's op counts: its own
# library, outside the C ABI of the hot path.
UBENCH_SRC = "wts_ubench.hip"
UBENCH_LIB = os.path.join(HERE, "libwts_ubench.so")


def _build_ubench() -> str:
    tmp = UBENCH_LIB + ".tmp"
    cmd = [HIPCC, *FLAGS, "-shared", os.path.join(CSRC, UBENCH_SRC), "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed on " + UBENCH_SRC)
    os.replace(tmp, UBENCH_LIB)
    return UBENCH_LIB


def build(verbose: bool = False) -> str:
    """Compile every source (always) and link the shared libraries."""
    os.makedirs(OBJDIR, exist_ok=True)
    with ThreadPoolExecutor(max_workers=len(SOURCES) + 1) as ex:
        ub = ex.submit(_build_ubench)
        objs = list(ex.map(_compile, list(SOURCES)))
        ub.result()
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("link failed")
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
