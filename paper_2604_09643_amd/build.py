"""Build the gfx950 HIP library ``libradiate.so`` in-tree (hipcc, no JIT cache).

Packed FP32 instructions are disabled for all device code (``-packed-fp32-ops``);
the kernels are written for the unpacked FP32 VALU.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "csrc", "radiate.hip")
HDR = os.path.join(ROOT, "include", "radiate.h")
LIB = os.path.join(HERE, "libradiate.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def hipcc_command(out: str, fast: bool = False) -> list:
    cmd = [HIPCC, "-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-shared",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-I", os.path.join(ROOT, "include"), "-o", out, SRC]
    if fast:
        cmd.insert(1, "-DRA_FAST_BUILD")
    return cmd


def build(fast: bool = False, verbose: bool = True) -> str:
    """Compile every kernel for gfx950 into paper_2604_09643_amd/libradiate.so."""
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = hipcc_command(tmp, fast=fast)
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    noise = ("is not a recognized feature for this target", "argument unused during compilation")
    err = "\n".join(l for l in res.stderr.splitlines() if not any(n in l for n in noise))
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + err)
    if err.strip() and verbose:
        print(err, file=sys.stderr)
    os.replace(tmp, LIB)
    return LIB


def is_stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(p) > t for p in (SRC, HDR))


if __name__ == "__main__":
    build(fast="--fast" in sys.argv)
