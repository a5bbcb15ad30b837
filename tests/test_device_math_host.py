"""Accuracy of the integrator's light FP64 elementary functions, host build.

The per-step path uses its own bounded-range exp, expm1, log, quotient and
sin/cos (kgrt_device.hpp) in place of the general library routines. Those are
__host__ __device__ and do the same FP64 operations on the host (fused
multiply-adds included), so a host build of them, checked against
multiple-precision values (mpmath at 60 digits) over the argument ranges the
kernels use, bounds their error in ulps. The device-only reciprocal seed is
replaced by the IEEE reciprocal on the host; its two Newton steps leave
less than an ulp either way.
"""
import os
import shutil
import subprocess

import mpmath
import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1601_02063_amd", "csrc")

PROGRAM = r"""
#include "kgrt_device.hpp"
#include <cstdio>
int main() {
    char op[8];
    double x, y;
    while (scanf("%7s %la %la", op, &x, &y) == 3) {
        double s = 0.0, c = 0.0;
        switch (op[0]) {
            case 'e': printf("%a\n", kgrt::fm::exp(x)); break;
            case 'm': printf("%a\n", kgrt::fm::expm1(x)); break;
            case 'l': printf("%a\n", kgrt::fm::log(x)); break;
            case 'd': printf("%a\n", kgrt::fm::div(x, y)); break;
            case 's': kgrt::sincos_bounded(x, &s, &c); printf("%a %a\n", s, c); break;
        }
    }
    return 0;
}
"""


@pytest.fixture(scope="module")
def prog(tmp_path_factory):
    hipcc = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc")
    if not os.path.exists(hipcc) and shutil.which("hipcc") is None:
        pytest.skip("hipcc not available")
    d = tmp_path_factory.mktemp("fm")
    src, exe = d / "fm.hip", d / "fm"
    src.write_text(PROGRAM)
    subprocess.check_call([hipcc if os.path.exists(hipcc) else "hipcc", "-O2", "-std=c++17",
                           "--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                           "-I", CSRC, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                          stderr=subprocess.DEVNULL)
    return str(exe)


def run(exe, lines):
    out = subprocess.run([exe], input="\n".join(lines) + "\n", capture_output=True, text=True, check=True).stdout
    return [[float.fromhex(t) for t in l.split()] for l in out.strip().split("\n")]


def ulps(got, exact):
    """|got - exact| in units of the last place of exact (exact: an mpmath number)."""
    e = float(exact)
    ulp = np.spacing(abs(e)) if e != 0.0 else np.spacing(0.0)
    return float(abs(mpmath.mpf(got) - exact) / ulp)


mpmath.mp.dps = 60


def test_exp_expm1(prog):
    rng = np.random.default_rng(11)
    xs = np.concatenate([rng.uniform(-745.0, 709.0, 300), rng.uniform(-40.0, 40.0, 300), rng.uniform(-1, 1, 200),
                         [0.0, -0.0, 1e-300, 0.34657359, -0.34657359, 1.0, -1.0, 700.0, -700.0]])
    got = run(prog, [f"e {x.hex()} 0x0p+0" for x in xs] + [f"m {x.hex()} 0x0p+0" for x in xs if abs(x) < 40])
    n = len(xs)
    worst_e = max(ulps(g[0], mpmath.exp(mpmath.mpf(x))) for g, x in zip(got[:n], xs)
                  if float(mpmath.exp(mpmath.mpf(x))) > 2.3e-308)  # normal results
    xm = [x for x in xs if abs(x) < 40]
    worst_m = max(ulps(g[0], mpmath.expm1(mpmath.mpf(x))) for g, x in zip(got[n:], xm) if x != 0.0)
    assert worst_e <= 1.5, worst_e
    assert worst_m <= 4.0, worst_m
    # underflow and overflow ends
    assert run(prog, ["e " + (-800.0).hex() + " 0x0p+0", "e " + (710.0).hex() + " 0x0p+0"]) == [[0.0], [float("inf")]]


def test_log(prog):
    rng = np.random.default_rng(12)
    xs = np.concatenate([10.0 ** rng.uniform(-300, 300, 400), rng.uniform(0.5, 2.0, 300),
                         [1.0, 2.0, 0.5, 0.7071067811865476, 0.7071067811865475, 1e-310]])
    got = run(prog, [f"l {x.hex()} 0x0p+0" for x in xs])
    worst = max(ulps(g[0], mpmath.log(mpmath.mpf(x))) for g, x in zip(got, xs) if x != 1.0)
    assert worst <= 2.5, worst
    assert got[list(xs).index(1.0)][0] == 0.0


def test_div(prog):
    rng = np.random.default_rng(13)
    a = rng.uniform(-1, 1, 500) * 10.0 ** rng.uniform(-100, 100, 500)
    b = rng.uniform(0.1, 1, 500) * 10.0 ** rng.uniform(-100, 100, 500) * rng.choice([-1, 1], 500)
    got = run(prog, [f"d {x.hex()} {y.hex()}" for x, y in zip(a, b)])
    worst = max(ulps(g[0], mpmath.mpf(x) / mpmath.mpf(y)) for g, x, y in zip(got, a, b))
    assert worst <= 1.0, worst


def test_sincos_bounded(prog):
    rng = np.random.default_rng(14)
    xs = np.concatenate([rng.uniform(-4.0, 7.0, 400), rng.uniform(-2.0 ** 20, 2.0 ** 20, 200),
                         [0.0, np.pi / 2, np.pi, 1e-12, 3 * np.pi / 4]])
    got = run(prog, [f"s {x.hex()} 0x0p+0" for x in xs])
    for (s, c), x in zip(got, xs):
        es, ec = mpmath.sin(mpmath.mpf(x)), mpmath.cos(mpmath.mpf(x))
        # in ulps of the result; near a zero of sin or cos (|value| <= 1e-3), where the
        # reduction's error is absolute, within two ulps of 1e-3 plus one ulp of the value
        for g, e in ((s, es), (c, ec)):
            if abs(float(e)) > 1e-3:
                assert ulps(g, e) <= 2.0, (x, g, float(e))
            else:
                assert abs(mpmath.mpf(g) - e) <= 2.0 * np.spacing(1.0) * 1e-3 + np.spacing(abs(float(e))), (x, g)
    assert got[len(xs) - 5] == [0.0, 1.0]
