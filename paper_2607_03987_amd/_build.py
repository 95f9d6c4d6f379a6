"""Compile libpakr.so (HIP, gfx950) in-tree."""
from __future__ import annotations

import os
import shutil
import subprocess

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libpakr.so")
SOURCES = [os.path.join(CSRC, "pakr.hip")]
DEPS = SOURCES + [os.path.join(CSRC, f) for f in ("pakr_device.hpp", "pakr_kernels.hpp",
                                                  "pakr_adjoint.hpp")] + [
    os.path.join(ROOT, "include", "pakr.h")]

HIPFLAGS = [
    "-O3", "--offload-arch=gfx950", "-std=c++17", "-fPIC", "-shared",
    # contract freely, except where a pragma forbids it (the sample conversion
    # must round the product and the sum separately)
    "-ffp-contract=fast-honor-pragmas",
    # no packed FP32 (v_pk_*_f32) code generation
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
]


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found: install ROCm or set HIPCC")


def build(force: bool = True, verbose: bool = False) -> str:
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= max(
            os.path.getmtime(p) for p in DEPS):
        return LIB
    tmp = LIB + f".tmp{os.getpid()}"
    cmd = [hipcc(), *HIPFLAGS, *SOURCES, "-o", tmp]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + res.stderr[-4000:])
    if verbose:
        print(res.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=False))
