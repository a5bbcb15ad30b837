"""Builds libkgrt.so (the HIP library behind include/kgrt.h) for gfx950 with hipcc."""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
import tempfile

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libkgrt.so")
SOURCES = [os.path.join(CSRC, "kgrt.hip"), os.path.join(CSRC, "kgrt_mlp.hip"), os.path.join(CSRC, "kgrt_spectra.hip")]
HEADERS = [os.path.join(CSRC, "kgrt_device.hpp"), os.path.join(CSRC, "kgrt_mino.hpp"), os.path.join(ROOT, "include", "kgrt.h")]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # no packed FP32 instructions anywhere in this library
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
]

# Per-source flags. The integrator keeps no loop-invariant values hoisted by
# the machine-level LICM pass: in the persistent loop it hoisted 32-bit halves
# of the FP64 polynomial constants into SGPRs, which then spilled to VGPR
# lanes and came back through v_readlane on every step (measured on gfx950:
# 591 -> 251 readlanes, 205 -> 134 VGPRs for the torus kernel).
#
# It is also built without the accumulating v_fmac_f64 form, so an FP64 fused
# multiply-add whose addend is a constant reads it from an SGPR pair (set by
# scalar moves, which issue beside the vector ALU) instead of first copying it
# into the destination VGPRs with two vector moves: each Horner step of the
# polynomial approximations cost three vector instructions instead of one
# (static vector moves in the torus kernel 409 -> 183).
SOURCE_FLAGS = {"kgrt.hip": ["-mllvm", "-disable-machine-licm", "-Xclang", "-target-feature", "-Xclang", "-fmacf64-inst"]}


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
    tmpdir = tempfile.mkdtemp(prefix="kgrt_build_")
    try:
        objs = []
        for src in SOURCES:
            obj = os.path.join(tmpdir, os.path.basename(src) + ".o")
            cmd = ([hipcc()] + HIPCC_FLAGS + SOURCE_FLAGS.get(os.path.basename(src), []) +
                   ["-D" + d for d in defines] + ["-c", "-o", obj, src])
            if verbose:
                print(" ".join(cmd), file=sys.stderr)
            subprocess.check_call(cmd)
            objs.append(obj)
        tmp = out + ".tmp%d" % os.getpid()
        cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
        if verbose:
            print(" ".join(cmd), file=sys.stderr)
        subprocess.check_call(cmd)
        os.replace(tmp, out)
    finally:
        shutil.rmtree(tmpdir, ignore_errors=True)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
