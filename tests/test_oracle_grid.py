"""Pins of the oracle's gridded-plasma model (a simulation snapshot sampled along each ray).

Each check takes a route of its own:
  * sampling: scipy's RegularGridInterpolator (linear) on the same nodes, with the
    periodic azimuthal node appended, against the oracle's trilinear interpolation;
  * coefficients: the invariant transfer equation with scipy's constants and Bessel
    functions, the emitter's four-velocity normalised by the metric as a matrix;
  * a snapshot holding the torus profile (fields linear in ln r) reproduces the torus
    model's images;
  * an optically thick shell of uniform temperature moving with a gridded angular
    velocity gives g^3 B_nu(T, nu/g) at its surface.
"""
import math

import numpy as np
import pytest
from scipy.interpolate import RegularGridInterpolator

import oracle as O
from paper_1601_02063_amd import scenes
from tests.test_oracle_pins_kerr import (C_CGS, GM_SUN_CGS, MP_CGS, kerr_metric, photon_momentum, planck,
                                         synchrotron_j_per_sr)


def _interpolator(grid, r_min, r_max):
    nr, nth, nph, _ = grid.shape
    lnr = np.linspace(math.log(r_min), math.log(r_max), nr)
    th = np.linspace(0.0, math.pi, nth)
    ph = 2.0 * math.pi * np.arange(nph + 1) / nph
    data = np.concatenate([grid, grid[:, :, :1, :]], axis=2).astype(np.float64)  # periodic node
    return RegularGridInterpolator((lnr, th, ph), data, method="linear")


def _grid_scene(grid, r_min, r_max, **kw):
    return O.Scene(model=O.MODEL_GRID, grid=grid, grid_r_min=r_min, grid_r_max=r_max, **kw)


def test_grid_sample_is_trilinear_and_periodic():
    pg = scenes.plasma_grid(77, 24, 12, 10, a=0.5, r_min=1.5, r_max=200.0)
    g = pg["grid"]
    scn = _grid_scene(g, 1.5, 200.0, a=0.5)
    ip = _interpolator(g, 1.5, 200.0)
    rng = np.random.default_rng(5)
    for _ in range(300):
        r = math.exp(rng.uniform(math.log(1.9), math.log(200.0)))
        th = rng.uniform(0.0, math.pi)
        ph = rng.uniform(-25.0, 25.0)
        inside, v = O.grid_sample(scn, r, th, ph)
        assert inside
        want = ip([[math.log(r), th, ph % (2.0 * math.pi)]])[0]
        assert np.allclose(v, want, rtol=1e-12, atol=1e-12 * np.abs(want).max()), (r, th, ph, v, want)
    # nodes are reproduced (float32 values widened exactly)
    lnr = np.linspace(math.log(1.5), math.log(200.0), 24)
    for i, j, k in [(2, 0, 0), (5, 3, 9), (23, 11, 4), (12, 6, 0)]:
        inside, v = O.grid_sample(scn, math.exp(lnr[i]), j * math.pi / 11, 2 * math.pi * k / 10)
        assert np.allclose(v, g[i, j, k].astype(np.float64), rtol=1e-12, atol=1e-9)
    # theta beyond the poles is clamped to the pole nodes
    assert np.array_equal(O.grid_sample(scn, 10.0, -0.01, 1.0)[1], O.grid_sample(scn, 10.0, 0.0, 1.0)[1])
    # no plasma outside the radial range or at the capture radius
    assert not O.grid_sample(scn, 1.4999, 1.0, 0.0)[0]
    assert not O.grid_sample(scn, 200.001, 1.0, 0.0)[0]
    rcap = (1 + math.sqrt(1 - 0.25)) * (1 + 1e-3)
    scn2 = _grid_scene(g, 1.0, 200.0, a=0.5)
    assert not O.grid_sample(scn2, rcap * 0.9999, 1.0, 0.0)[0]
    assert O.grid_sample(scn2, rcap * 1.0001, 1.0, 0.0)[0]


def _redshift_with_omega(a, r, th, L_traced, omega, pr=0.0, pth=0.0):
    G = kerr_metric(a, r, th)
    k = np.array([1.0, 0.0, 0.0, omega])
    norm = k @ G @ k
    if norm < 0:
        u = k / math.sqrt(-norm)
    else:
        Ginv = np.linalg.inv(G)
        u = Ginv @ np.array([-1.0 / math.sqrt(-Ginv[0, 0]), 0.0, 0.0, 0.0])
    return 1.0 / -(photon_momentum(L_traced, pr, pth) @ u)


def test_grid_coefficients_from_invariant_transfer():
    """ln n_e, ln T_e, ln B and Omega from the snapshot; thermal synchrotron per steradian and
    Kirchhoff absorption at nu/g, with g of matter moving with the gridded Omega; per unit affine
    parameter a_lam = alpha_0 r_g/g and e_lam = g^3 j_0 r_g/g."""
    pg = scenes.plasma_grid(78, 20, 10, 8, a=0.9, r_min=1.2, r_max=300.0)
    g = pg["grid"]
    mbh = 6.5e9
    scn = _grid_scene(g, 1.2, 300.0, a=0.9, mbh_msun=mbh)
    ip = _interpolator(g, 1.2, 300.0)
    rg = GM_SUN_CGS * mbh / C_CGS ** 2
    rng = np.random.default_rng(8)
    checked = 0
    while checked < 80:
        r = math.exp(rng.uniform(math.log(2.2), math.log(300.0)))
        th = rng.uniform(0.2, math.pi - 0.2)
        ph = rng.uniform(0.0, 6.0)
        L = rng.uniform(-6.0, 6.0)
        nu = 10 ** rng.uniform(10.5, 12.5)
        ln_ne, ln_te, ln_b, om = ip([[math.log(r), th, ph]])[0]
        g_want = _redshift_with_omega(0.9, r, th, L, om)
        if not g_want > 0.0:
            continue  # no photon with this L reaches matter moving this fast
        checked += 1
        a_lam, e_lam, gg = O.grid_coeffs(scn, r, th, ph, L / -1.0, nu)
        assert gg == pytest.approx(g_want, rel=1e-12)
        nu0 = nu / g_want
        j0 = synchrotron_j_per_sr(nu0, math.exp(ln_ne), math.exp(ln_te), math.exp(ln_b))
        alpha0 = j0 / planck(nu0, math.exp(ln_te))
        assert a_lam == pytest.approx(alpha0 * rg / g_want, rel=1e-7)
        assert e_lam == pytest.approx(g_want ** 3 * j0 * rg / g_want, rel=1e-7)


def test_grid_holding_the_torus_profile_reproduces_the_torus():
    """A snapshot whose ln n_e, ln T_e and ln B are linear in ln r (the torus with an unbounded
    scale height) and whose Omega is the Keplerian 1/(r^3/2 + a) on a fine radial grid: its
    images equal the torus model's within the float32 storage and the interpolation of Omega."""
    a, r_min, r_max, nr = 0.9, 1.0, 1000.0, 8192
    torus = dict(n0_cgs=1e6, r_norm=2.0, n_index=1.1, h_over_r=1e6, T0_K=1e11, T_index=0.84, eps_B=0.1,
                 mbh_msun=4e6, r_emit_max=r_max)
    lnr = np.linspace(math.log(r_min), math.log(r_max), nr)
    r = np.exp(lnr)
    grid = np.empty((nr, 2, 1, 4), dtype=np.float32)
    ln_ne = math.log(1e6) - 1.1 * np.log(r / 2.0)
    grid[:, :, 0, 0] = ln_ne[:, None]
    grid[:, :, 0, 1] = (math.log(1e11) - 0.84 * np.log(r / 2.0))[:, None]
    grid[:, :, 0, 2] = (0.5 * (np.log(8 * math.pi * 0.1 * MP_CGS * C_CGS ** 2 / 6.0) + ln_ne - lnr))[:, None]
    grid[:, :, 0, 3] = (1.0 / (r ** 1.5 + a))[:, None]
    freqs = [86e9, 230e9, 690e9]
    common = dict(a=a, incl_deg=40.0, freqs_hz=freqs, hmax_frac=0.02)
    st = O.Scene(model=O.MODEL_TORUS, **common, **torus)
    sg = _grid_scene(grid, r_min, r_max, mbh_msun=4e6, **common)
    rt = O.trace_image(st, 9, 7, -12, 12, -10, 10).ravel()
    rgi = O.trace_image(sg, 9, 7, -12, 12, -10, 10).ravel()
    assert np.array_equal(rt["steps"], rgi["steps"])
    for f in range(3):
        assert np.all(rt["I"][:, f] > 0)
        assert np.allclose(rgi["I"][:, f], rt["I"][:, f], rtol=2e-5, atol=0)
        assert np.allclose(rgi["tau"][:, f], rt["tau"][:, f], rtol=2e-5, atol=0)


@pytest.mark.parametrize("x,y", [(3.0, 4.0), (-6.0, 1.0), (1.0, -9.0)])
def test_grid_thick_shell_moving_with_gridded_omega(x, y):
    """A shell 20 <= r <= 30 of uniform temperature, optically thick within a fraction of a step,
    rotating with a uniform gridded Omega: the emergent intensity is g^3 B_nu(T, nu/g) with g of
    that flow at the ray's first point inside."""
    T, omega = 3e10, 0.008
    grid = np.empty((3, 5, 4, 4), dtype=np.float32)
    grid[..., 0] = math.log(1e13)
    grid[..., 1] = math.log(T)
    grid[..., 2] = math.log(30.0)
    grid[..., 3] = omega
    freqs = [86e9, 230e9, 690e9]
    scn = _grid_scene(grid, 20.0, 30.0, a=0.9, incl_deg=60.0, freqs_hz=freqs, hmax_frac=0.05, mbh_msun=4e6)
    res, path = O.trace_path(scn, x, y)
    k = int(np.nonzero(path[:, 1] <= 30.0)[0][0])
    lam, r, th, ph, t, pr, pth = path[k]
    g = _redshift_with_omega(0.9, r, th, res["L"], float(np.float32(omega)), pr, pth)
    assert abs(g - 1.0) > 0.01
    for f, nu in enumerate(freqs):
        assert res["tau"][f] > 1e3
        T_stored = math.exp(float(grid[0, 0, 0, 1]))  # ln T_e as the float32 snapshot holds it
        assert res["I"][f] == pytest.approx(g ** 3 * planck(nu / g, T_stored), rel=1e-8)
