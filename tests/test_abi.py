"""C-ABI checks that need no GPU: the library loads, exports every declared
symbol, its struct layouts match the header, and argument validation works."""
import ctypes
import os
import re
import subprocess
import tempfile

import pytest

from tests.conftest import ROOT

HEADER = os.path.join(ROOT, "include", "kgrt.h")
LIB = os.path.join(ROOT, "paper_1601_02063_amd", "libkgrt.so")


def _declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(kgrt_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def K():
    if not os.path.exists(LIB):
        pytest.fail("libkgrt.so is not built (run __graft_entry__.build())")
    from paper_1601_02063_amd import kgrt
    return kgrt


def test_library_exports_every_declared_symbol(K):
    names = _declared_functions()
    assert len(names) >= 10
    lib = ctypes.CDLL(LIB)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_struct_layout_matches_header(K):
    probe = r'''
#include <stdio.h>
#include <stddef.h>
#include "kgrt.h"
#define P(T) printf(#T " %zu\n", sizeof(T));
#define F(T, f) printf(#T "." #f " %zu\n", offsetof(T, f));
int main(void) {
  P(kgrt_camera) P(kgrt_model) P(kgrt_integrator) P(kgrt_outputs) P(kgrt_launch) P(kgrt_adam) P(kgrt_fallback) P(kgrt_kernel_info)
  F(kgrt_camera, nx) F(kgrt_camera, x_min) F(kgrt_camera, y_max)
  F(kgrt_model, r_in) F(kgrt_model, r_emit_max) F(kgrt_integrator, max_steps) F(kgrt_integrator, flags)
  F(kgrt_outputs, tau) F(kgrt_launch, refill_min) F(kgrt_adam, eps) F(kgrt_fallback, grad_max) F(kgrt_kernel_info, waves_per_simd)
  F(kgrt_model, spot_phi0) F(kgrt_model, grid_dev) F(kgrt_model, grid_nph) F(kgrt_model, grid_r_max)
  return 0; }
'''
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "p.c")
        open(c, "w").write(probe)
        exe = os.path.join(d, "p")
        subprocess.check_call(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), c, "-o", exe])
        got = dict(line.rsplit(" ", 1) for line in subprocess.check_output([exe]).decode().split("\n") if line)
    want = {
        "kgrt_camera": ctypes.sizeof(K.CCamera), "kgrt_model": ctypes.sizeof(K.CModel),
        "kgrt_integrator": ctypes.sizeof(K.CIntegrator), "kgrt_outputs": ctypes.sizeof(K.COutputs),
        "kgrt_launch": ctypes.sizeof(K.CLaunch), "kgrt_adam": ctypes.sizeof(K.CAdam),
        "kgrt_fallback": ctypes.sizeof(K.CFallback), "kgrt_kernel_info": ctypes.sizeof(K.CKernelInfo),
        "kgrt_camera.nx": K.CCamera.nx.offset, "kgrt_camera.x_min": K.CCamera.x_min.offset,
        "kgrt_camera.y_max": K.CCamera.y_max.offset, "kgrt_model.r_in": K.CModel.r_in.offset,
        "kgrt_model.r_emit_max": K.CModel.r_emit_max.offset,
        "kgrt_integrator.max_steps": K.CIntegrator.max_steps.offset,
        "kgrt_integrator.flags": K.CIntegrator.flags.offset, "kgrt_outputs.tau": K.COutputs.tau.offset,
        "kgrt_launch.refill_min": K.CLaunch.refill_min.offset, "kgrt_adam.eps": K.CAdam.eps.offset,
        "kgrt_fallback.grad_max": K.CFallback.grad_max.offset,
        "kgrt_kernel_info.waves_per_simd": K.CKernelInfo.waves_per_simd.offset,
        "kgrt_model.spot_phi0": K.CModel.spot_phi0.offset, "kgrt_model.grid_dev": K.CModel.grid_dev.offset,
        "kgrt_model.grid_nph": K.CModel.grid_nph.offset, "kgrt_model.grid_r_max": K.CModel.grid_r_max.offset,
    }
    for k, v in want.items():
        assert int(got[k]) == v, k


def test_version_and_strerror(K):
    L = K.lib()
    assert L.kgrt_version() >= 100
    for code in (0, -1, -2, -3, -4, -5):
        assert L.kgrt_strerror(code)
    assert L.kgrt_last_error(None) == b""


def _ok_request(K):
    return K.Camera(), K.Model(kind=K.MODEL_THIN_DISK), [], K.Integrator()


@pytest.mark.parametrize("mutate", [
    lambda c, m, f, i: setattr(c, "a", 1.0),
    lambda c, m, f, i: setattr(c, "a", float("nan")),
    lambda c, m, f, i: setattr(c, "incl_deg", 0.0),
    lambda c, m, f, i: setattr(c, "incl_deg", 180.0),
    lambda c, m, f, i: setattr(c, "r_obs", 5.0),
    lambda c, m, f, i: setattr(c, "nx", -1),
    lambda c, m, f, i: setattr(c, "x_max", -20.0),
    lambda c, m, f, i: setattr(c, "y_min", float("inf")),
    lambda c, m, f, i: setattr(m, "kind", 7),
    lambda c, m, f, i: setattr(m, "r_out", -1.0),
    lambda c, m, f, i: setattr(m, "r_in", 30.0),
    lambda c, m, f, i: setattr(i, "rtol", 1e-16),
    lambda c, m, f, i: setattr(i, "rtol", 0.5),
    lambda c, m, f, i: setattr(i, "hmax_frac", 0.0),
    lambda c, m, f, i: setattr(i, "horizon_delta", 0.0),
    lambda c, m, f, i: setattr(i, "max_steps", 0),
    lambda c, m, f, i: setattr(i, "flags", 8),
])
def test_invalid_arguments_rejected(K, mutate):
    cam, mod, freqs, integ = _ok_request(K)
    assert K.check_args(cam, mod, freqs, integ) == K.OK
    mutate(cam, mod, freqs, integ)
    assert K.check_args(cam, mod, freqs, integ) == K.E_INVALID_ARG


def test_torus_frequency_checks(K):
    cam, _, _, integ = _ok_request(K)
    tor = K.Model(kind=K.MODEL_TORUS)
    assert K.check_args(cam, tor, [230e9], integ) == K.OK
    assert K.check_args(cam, tor, [], integ) == K.E_INVALID_ARG
    assert K.check_args(cam, tor, [230e9] * 17, integ) == K.E_INVALID_ARG
    assert K.check_args(cam, tor, [-1.0], integ) == K.E_INVALID_ARG
    assert K.check_args(cam, tor, [float("nan")], integ) == K.E_INVALID_ARG
    assert K.check_args(cam, K.Model(kind=K.MODEL_TORUS, T0_K=0.0), [230e9], integ) == K.E_INVALID_ARG
    # empty images are valid requests
    assert K.check_args(K.Camera(nx=0, ny=0), tor, [230e9], integ) == K.OK


def test_grid_model_checks(K):
    """The gridded-plasma model's arguments are validated on the host; the grid pointer is
    only stored, never dereferenced, so a dummy address serves here."""
    cam, _, _, integ = _ok_request(K)
    L = K.lib()

    def check(freqs=(230e9,), **kw):
        m = K.Model(kind=K.MODEL_GRID).c()
        m.grid_dev, m.grid_nr, m.grid_nth, m.grid_nph = 4096, 16, 8, 8
        m.grid_r_min, m.grid_r_max = 1.0, 1000.0
        for k, v in kw.items():
            setattr(m, k, v)
        fa, nf = K._freqs(list(freqs))
        return L.kgrt_check_args(ctypes.byref(cam.c()), ctypes.byref(m), fa, nf, ctypes.byref(integ.c()))

    assert check() == K.OK
    assert check(freqs=[86e9] * 16) == K.OK
    assert check(grid_nph=1) == K.OK
    for kw in [dict(grid_dev=None), dict(grid_nr=1), dict(grid_nth=1), dict(grid_nph=0), dict(grid_reserved=1),
               dict(grid_r_min=0.0), dict(grid_r_min=1000.0), dict(grid_r_max=float("inf")),
               dict(mbh_msun=0.0), dict(grid_nr=2048, grid_nth=1024, grid_nph=1024), dict(grid_dev=4100)]:
        assert check(**kw) == K.E_INVALID_ARG, kw
    for freqs in ([], [230e9] * 17, [0.0], [float("nan")]):
        assert check(freqs=freqs) == K.E_INVALID_ARG, freqs


def test_context_without_gpu_reports_no_device(K):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(K.KgrtError) as e:
        K.Context(0)
    assert e.value.code == K.E_NO_DEVICE


@pytest.mark.parametrize("a,inc", [(0.0, 60.0), (0.9, 60.0), (0.998, 89.0), (0.5, 5.0), (0.3, 30.0)])
def test_critical_curve_table_matches_parametrisation(K, a, inc):
    """The fallback band's table agrees with the spherical-photon-orbit curve computed
    independently in the tests (sky-plane distance of curve points to the table)."""
    import numpy as np
    from tests.helpers import critical_curve_distance
    R = K.critical_curve(a, inc)
    psi = -np.pi + (np.arange(1024) + 0.5) * 2 * np.pi / 1024
    x, y = R * np.cos(psi), R * np.sin(psi)
    # table points lie on the curve: convert (x, y) -> (xi, eta) of a ray at infinity and measure
    th = np.radians(inc)
    xi = -x * np.sin(th)
    eta = y ** 2 - a * a * np.cos(th) ** 2 + xi ** 2 / np.tan(th) ** 2
    d = critical_curve_distance(a, inc, xi, eta)
    # bins hold the largest radius in their angular range: ~dR/dpsi x half a bin (< 0.01 M),
    # against a fallback band of 0.5 M
    assert np.median(d) < 1e-2 and d.max() < 2e-2, (np.median(d), d.max())


def test_pixel_solid_angle_matches_oracle(K):
    """Host function of the library against the oracle's definition (no GPU needed)."""
    from oracle import spectra as S
    for (nx, ny, ext, m, d) in [(1024, 1024, (-20.0, 20.0, -20.0, 20.0), 4e6, 2.4687e22),
                                (64, 48, (-15.0, 15.0, -10.0, 12.0), 10.0, 3.0857e22)]:
        cam = K.Camera(a=0.5, incl_deg=30.0, nx=nx, ny=ny, x_min=ext[0], x_max=ext[1], y_min=ext[2], y_max=ext[3])
        got = K.pixel_solid_angle(cam, m, d)
        assert got == pytest.approx(S.pixel_solid_angle(nx, ny, *ext, m, d), rel=1e-15)
    bad = K.Camera(a=0.5, incl_deg=30.0, nx=0, ny=4)
    with pytest.raises(ValueError):
        K.pixel_solid_angle(bad, 4e6, 1e22)
    with pytest.raises(ValueError):
        K.pixel_solid_angle(K.Camera(a=0.5, incl_deg=30.0, nx=4, ny=4), 4e6, -1.0)


def test_image_spectra_rejects_bad_arguments(K):
    """Argument checks run on the host before any launch (no GPU needed)."""
    L = K.lib()
    dummy = ctypes.c_void_p(16)
    assert L.kgrt_image_spectra(dummy, 10, 0, dummy, dummy, 1, dummy, None) == K.E_INVALID_ARG   # nfreq < 1
    assert L.kgrt_image_spectra(dummy, -1, 1, dummy, dummy, 1, dummy, None) == K.E_INVALID_ARG   # total < 0
    assert L.kgrt_image_spectra(dummy, 10, 1, dummy, dummy, -1, dummy, None) == K.E_INVALID_ARG  # nimg < 0
    assert L.kgrt_image_spectra(dummy, 10, 1, dummy, dummy, 70000, dummy, None) == K.E_INVALID_ARG
    assert L.kgrt_image_spectra(None, 10, 1, dummy, dummy, 1, dummy, None) == K.E_INVALID_ARG    # NULL intensity
    assert L.kgrt_image_spectra(dummy, 10, 1, None, dummy, 1, dummy, None) == K.E_INVALID_ARG    # NULL offsets
    assert L.kgrt_image_spectra(dummy, 10, 1, dummy, dummy, 1, None, None) == K.E_INVALID_ARG    # NULL flux
    assert L.kgrt_image_spectra(None, 0, 1, None, None, 0, None, None) == K.OK                   # nothing to do
