"""Compile the HIP library for gfx950 into paper_1704_04794_amd/liboi_hip.so.

    python -m paper_1704_04794_amd.build

Every translation unit is compiled with FMA contraction off (-ffp-contract=off):
the Stage-1 table, the selection thresholds and the stopping rules are fp64
expressions whose rounding is part of the sampler's specification.  Packed
fp32 instructions are disabled for device code.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "liboi_hip.so")
SOURCES = ["iicp_kernels.hip", "oi_api.cpp"]
ARCH = os.environ.get("OI_OFFLOAD_ARCH", "gfx950")


def _hipcc() -> str:
    for c in (os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc"), "hipcc"):
        if os.path.sep not in c or os.path.exists(c):
            return c
    return "hipcc"


def build(verbose: bool = False, jobs: int = 2) -> str:
    hipcc = _hipcc()
    common = ["-O3", "-std=c++17", "-fPIC", "-ffp-contract=off", "-Wall",
              "-I", os.path.join(ROOT, "include"), "-I", CSRC]
    objs = []
    procs = []
    for src in SOURCES:
        obj = os.path.join(CSRC, "_build", src + ".o")
        os.makedirs(os.path.dirname(obj), exist_ok=True)
        cmd = [hipcc, "-x", "hip", f"--offload-arch={ARCH}",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
               *common, "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append(subprocess.Popen(cmd, stderr=subprocess.PIPE, text=True))
        objs.append(obj)
    failed = False
    for pr in procs:
        _, err = pr.communicate()
        keep = [ln for ln in (err or "").splitlines() if "packed-fp32-ops" not in ln]
        if keep:
            print("\n".join(keep), file=sys.stderr)
        failed |= pr.returncode != 0
    if failed:
        raise RuntimeError("hipcc failed")
    tmp = LIB + ".tmp"
    link = [hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    if verbose:
        print(" ".join(link), flush=True)
    subprocess.run(link, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
