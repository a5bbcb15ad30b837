"""Builds libkgrt.so (the HIP library behind include/kgrt.h) for gfx950 with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libkgrt.so")
SOURCES = [os.path.join(CSRC, "kgrt.hip"), os.path.join(CSRC, "kgrt_mlp.hip")]
HEADERS = [os.path.join(CSRC, "kgrt_device.hpp"), os.path.join(ROOT, "include", "kgrt.h")]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # no packed FP32 instructions anywhere in this library
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
]


def hipcc() -> str:
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    return os.path.join(rocm, "bin", "hipcc")


def build(force: bool = True, verbose: bool = False, out: str = LIB, defines=()) -> str:
    """Compile the library in-tree (always, unless force=False and it is up to date).

    defines: extra preprocessor settings, e.g. ("KGRT_WAVES_TORUS=3",) for launch-shape experiments.
    """
    if not force and os.path.exists(out):
        newest = max(os.path.getmtime(p) for p in SOURCES + HEADERS)
        if os.path.getmtime(out) >= newest:
            return out
    tmp = out + ".tmp%d" % os.getpid()
    cmd = [hipcc()] + HIPCC_FLAGS + ["-D" + d for d in defines] + ["-o", tmp] + SOURCES
    if verbose:
        print(" ".join(cmd), file=sys.stderr)
    subprocess.check_call(cmd)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
