"""Builds libplenoctree.so (host API + gfx950 HIP kernels) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libplenoctree.so")
ARCH = "gfx950"

HIP_FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # identical rounding in the forward and backward walks: no implicit FMA contraction
    "-ffp-contract=off",
    # hardware float atomics for the gradient scatter
    "-munsafe-fp-atomics",
    # no packed-FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def hipcc() -> str:
    return os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


N_PARTS = 8  # po_kernels.hip is compiled once per part (PO_PART), in parallel


def _compile_cmds():
    cmds = []
    for part in range(N_PARTS):
        obj = os.path.join(PKG, "_build", f"po_kernels.p{part}.o")
        cmds.append((obj, [hipcc(), *HIP_FLAGS, f"-DPO_PART={part}", "-I", INCLUDE, "-I", CSRC, "-c",
                           os.path.join(CSRC, "po_kernels.hip"), "-o", obj]))
    for src in ("po_api.cpp", "po_codebook.cpp"):
        obj = os.path.join(PKG, "_build", src + ".o")
        cmds.append((obj, [hipcc(), "-O2", "-std=c++17", "-fPIC", "-Wall", "-pthread", "-I", INCLUDE, "-I", CSRC,
                           "-c", os.path.join(CSRC, src), "-o", obj]))
    return cmds


def build(verbose: bool = False, jobs: int = 0) -> str:
    """Compiles every source under csrc/ into one shared library next to this
    file (the kernel parts in parallel, up to `jobs` compilers at once)."""
    os.makedirs(os.path.join(PKG, "_build"), exist_ok=True)
    cmds = _compile_cmds()
    jobs = jobs or min(len(cmds), max(1, min(16, os.cpu_count() or 1)))
    running, objs, failed = [], [], []
    pending = list(cmds)
    while pending or running:
        while pending and len(running) < jobs:
            obj, cmd = pending.pop(0)
            if verbose:
                print(" ".join(cmd), flush=True)
            running.append((obj, cmd, subprocess.Popen(cmd)))
            objs.append(obj)
        obj, cmd, p = running.pop(0)
        if p.wait() != 0:
            failed.append(" ".join(cmd))
    if failed:
        raise subprocess.CalledProcessError(1, failed[0])
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-pthread", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
