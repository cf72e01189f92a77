"""Compile the gfx950 HIP library (libhfqmc.so) in-tree with hipcc: every
source to an object in parallel, then one shared-library link."""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys
import tempfile

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libhfqmc.so")
SOURCES = ["hfqmc_sweep.hip", "hfqmc_sweep_global.hip", "hfqmc_window.hip", "hfqmc_window_mixed.hip",
           "hfqmc_window_global.hip",
           "hfqmc_lattice.hip", "hfqmc_abi.cpp"]

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC",
    # no packed-fp32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-ffp-contract=off", "-Wall", "-Wno-unused-result",
    # keep branch-selected register reads as branches: sinking them into one
    # load through a phi of pointers would demote the register tiles to scratch
    "-mllvm", "-simplifycfg-sink-common=false",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    return "hipcc"


def _jobs() -> int:
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(n, 16, len(SOURCES)))


def build(verbose: bool = False) -> str:
    """Always recompiles; returns the library path."""
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    with tempfile.TemporaryDirectory(prefix="hfqmc_build_") as tmpd:
        def compile_one(src):
            obj = os.path.join(tmpd, os.path.splitext(src)[0] + ".o")
            cmd = [hipcc(), *HIPCC_FLAGS, *inc, "-c", os.path.join(CSRC, src), "-o", obj]
            if verbose:
                print(" ".join(cmd), file=sys.stderr, flush=True)
            subprocess.check_call(cmd)
            return obj

        with cf.ThreadPoolExecutor(_jobs()) as ex:
            objs = list(ex.map(compile_one, SOURCES))
        tmp = LIB + ".tmp"
        cmd = [hipcc(), "--offload-arch=gfx950", "-fPIC", "-shared", *objs, "-o", tmp]
        if verbose:
            print(" ".join(cmd), file=sys.stderr, flush=True)
        subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
