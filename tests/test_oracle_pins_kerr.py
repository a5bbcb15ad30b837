"""More pins of the CPU oracle: the Kerr crossing, the emitter's redshift off the
equator, the torus plasma and its transfer coefficients, and step underflow.

Each check takes a route of its own:
  * the crossing: Hamilton's equations of the Kerr null Hamiltonian (the metric
    of Eq. (1) written out here), differentiated by complex steps and integrated
    by scipy's DOP853 to the event cos(theta) = 0;
  * the redshift (Eq. (2)): the contraction -p.u with the metric as a 4x4
    matrix, u normalised by that matrix (Keplerian) or built from the lapse with
    the numerically inverted metric (zero-angular-momentum observer);
  * the transfer coefficients: the invariant form of the transfer equation
    (I/nu^3, j/nu^2 and nu alpha invariant, proper length per unit affine
    parameter r_g/g), scipy's physical constants and Bessel functions;
  * the thick limit of a moving emitter: I = g^3 B_nu(T, nu/g) from those routes;
  * the formal solution of the transfer equation along a straight line in
    flat space, integrated by scipy.
"""
import math

import numpy as np
import pytest
import scipy.constants as sc
from scipy.integrate import solve_ivp
from scipy.special import kv

import oracle as O

# ------------------------------------------------------------- test-side physics

# CGS from scipy's CODATA values; the solar GM is the IAU 2015 nominal value (Resolution B3)
C_CGS = sc.c * 100.0
H_CGS = sc.h * 1e7
K_CGS = sc.k * 1e7
ME_CGS = sc.m_e * 1e3
MP_CGS = sc.m_p * 1e3
E_ESU = sc.e * sc.c * 10.0
GM_SUN_CGS = 1.3271244e20 * 1e6


def kerr_metric(a, r, th, M=1.0):
    """Covariant Boyer-Lindquist metric of Eq. (1), index order (t, r, theta, phi)."""
    s, c = math.sin(th), math.cos(th)
    sig = r * r + a * a * c * c
    dl = r * r - 2 * M * r + a * a
    g = np.zeros((4, 4))
    g[0, 0] = -(1 - 2 * M * r / sig)
    g[0, 3] = g[3, 0] = -2 * M * a * r * s * s / sig
    g[1, 1] = sig / dl
    g[2, 2] = sig
    g[3, 3] = (r * r + a * a + 2 * M * a * a * r * s * s / sig) * s * s
    return g


def photon_momentum(L_traced, pr, pth):
    """Covariant momentum of the physical photon: the traced ray reversed (E_traced = -1)."""
    return np.array([-1.0, -pr, -pth, -L_traced])


def emitter_velocity(a, r, th):
    """Keplerian circular flow Omega = 1/(r^3/2 + a) when it is timelike at (r, theta),
    else the zero-angular-momentum observer. Returns (u^mu, which)."""
    G = kerr_metric(a, r, th)
    k = np.array([1.0, 0.0, 0.0, 1.0 / (r ** 1.5 + a)])
    norm = k @ G @ k
    if norm < 0:
        return k / math.sqrt(-norm), "keplerian"
    Ginv = np.linalg.inv(G)
    lapse = 1.0 / math.sqrt(-Ginv[0, 0])
    u = Ginv @ np.array([-lapse, 0.0, 0.0, 0.0])
    return u, "zamo"


def redshift_contraction(a, r, th, L_traced, pr=0.0, pth=0.0):
    """g = nu_obs/nu_emit for a static observer at infinity, Eq. (2): 1/(-p.u)."""
    u, which = emitter_velocity(a, r, th)
    return 1.0 / -(photon_momentum(L_traced, pr, pth) @ u), which


def planck(nu, T):
    return 2 * H_CGS * nu ** 3 / C_CGS ** 2 / math.expm1(H_CGS * nu / (K_CGS * T))


def synchrotron_j_per_sr(nu, ne, Te, B):
    """Thermal synchrotron emissivity (Mahadevan et al. 1996 fit, Eqs. (37)-(39)) per steradian."""
    theta = K_CGS * Te / (ME_CGS * C_CGS ** 2)
    nu_c = 3 * E_ESU * B / (4 * math.pi * ME_CGS * C_CGS) * theta ** 2
    x = nu / nu_c
    Mx = 4.0505 * x ** (-1 / 6) * (1 + 0.40 * x ** -0.25 + 0.5316 * x ** -0.5) * math.exp(-1.8899 * x ** (1 / 3))
    return nu * ne * E_ESU ** 2 / (math.sqrt(3) * C_CGS * kv(2, 1 / theta)) * Mx


def torus_plasma(scn, r, th):
    """The torus reading: density with a Gaussian scale height h r, power-law temperature and an
    equipartition-fraction field, B^2/(8 pi) = eps_B n_e m_p c^2 / (6 r)."""
    z = r * math.cos(th)
    ne = scn.n0_cgs * (r / scn.r_norm) ** -scn.n_index * math.exp(-0.5 * (z / (scn.h_over_r * r)) ** 2)
    Te = scn.T0_K * (r / scn.r_norm) ** -scn.T_index
    B = math.sqrt(8 * math.pi * scn.eps_B * ne * MP_CGS * C_CGS ** 2 / (6 * r))
    return ne, Te, B


def transfer_coefficients(scn, r, th, g, nu):
    """(d tau/d lambda, d I_obs/d lambda) from the invariant transfer equation: in the emitter's
    frame dI_0/dl = j_0 - alpha_0 I_0 at nu_0 = nu/g; I_obs = g^3 I_0; dl/dlambda = r_g/g."""
    ne, Te, B = torus_plasma(scn, r, th)
    nu0 = nu / g
    j0 = synchrotron_j_per_sr(nu0, ne, Te, B)
    alpha0 = j0 / planck(nu0, Te)
    dl_dlam = (GM_SUN_CGS * scn.mbh_msun / C_CGS ** 2) / g
    return alpha0 * dl_dlam, g ** 3 * j0 * dl_dlam


# ------------------------------------------------- crossing: Hamiltonian flow

def _kerr_hamiltonian(a, r, th, pr, pth, E, L):
    s, c = np.sin(th), np.cos(th)
    sig = r * r + a * a * c * c
    dl = r * r - 2 * r + a * a
    W = (r * r + a * a) * E - a * L
    return (dl * pr * pr + pth * pth + (L / s - a * E * s) ** 2 - W * W / dl) / (2 * sig)


_CS = 1e-30
_EYE = np.eye(6) * (1j * _CS)


def _hamilton_flow(a, E, L):
    """(r, theta, phi, t, p_r, p_theta)' from complex-step partial derivatives of H."""
    def f(lam, z):
        base = np.array([z[0], z[1], z[4], z[5], E, L], dtype=complex)
        P = base[None, :] + _EYE
        dH = _kerr_hamiltonian(a, P[:, 0], P[:, 1], P[:, 2], P[:, 3], P[:, 4], P[:, 5]).imag / _CS
        d_r, d_th, d_pr, d_pth, d_E, d_L = dH
        return [d_pr, d_pth, d_L, -d_E, -d_r, -d_th]
    return f


def _first_crossing(a, y6, c4):
    rplus = 1 + math.sqrt(1 - a * a)

    def equator(lam, z):
        return z[1] - math.pi / 2
    equator.terminal = True

    def horizon(lam, z):
        return z[0] - rplus * (1 + 1e-3)
    horizon.terminal = True

    def escape(lam, z):
        return z[0] - 1001.0
    escape.terminal = True
    sol = solve_ivp(_hamilton_flow(a, c4[0], c4[1]), (0.0, 1e5), y6, method="DOP853", rtol=1e-13, atol=1e-13,
                    events=[equator, horizon, escape])
    if len(sol.t_events[0]) == 0:
        return None
    return sol.y_events[0][0]


KERR_RAYS = [(0.9, 60.0, 5.0, 3.0), (0.9, 60.0, -4.0, -7.0), (0.9, 60.0, -3.0, 0.5), (0.998, 80.0, -6.0, 2.0),
             (0.998, 80.0, 4.5, -1.0), (0.998, 30.0, 2.0, 6.0), (0.5, 30.0, 8.0, 8.0), (0.94, 17.0, -1.0, 7.0)]


@pytest.mark.parametrize("a,inc,x,y", KERR_RAYS)
def test_kerr_first_crossing_against_hamiltonian_flow(a, inc, x, y):
    """The first equatorial crossing of a Kerr ray (radius, phi, t, redshift and disk intensity)
    against an independent integration of the same geodesic; the oracle at rtol 1e-12 and a
    ten times smaller step cap reproduces it to 1e-9, and at the production controls (rtol 1e-8,
    step cap 0.05 r) its true error stays below 2e-7 (the error the parity bars sit inside)."""
    tight = O.Scene(a=a, incl_deg=inc, model=O.MODEL_THIN_DISK, rtol=1e-12, hmax_frac=0.005)
    prod = O.Scene(a=a, incl_deg=inc, model=O.MODEL_THIN_DISK)
    ok, y6, c4 = O.initial_state(prod, x, y)
    assert ok
    ref = _first_crossing(a, y6, c4)
    rt, rp = O.trace_ray(tight, x, y), O.trace_ray(prod, x, y)
    if ref is None:
        assert not (rt["status"] & O.CROSSED) and not (rp["status"] & O.CROSSED)
        return
    assert rt["status"] & O.CROSSED and rp["status"] & O.CROSSED
    rc = ref[0]
    g_ref, which = redshift_contraction(a, rc, math.pi / 2, c4[1], ref[4], ref[5])
    assert rt["r_cross"] == pytest.approx(rc, rel=1e-9)
    assert rt["phi_cross"] == pytest.approx(ref[2], rel=1e-9, abs=1e-9)
    assert rt["t_cross"] == pytest.approx(ref[3], rel=1e-9)
    assert rt["g"] == pytest.approx(g_ref, rel=1e-9)
    on_disk = O.isco(a) <= rc <= 20.0
    assert bool(rt["status"] & O.DISK_HIT) == on_disk
    if on_disk:
        assert which == "keplerian"
        assert rt["intensity"] == pytest.approx(g_ref ** 3 / rc ** 3, rel=4e-9)
        assert rt["i_bol"] == pytest.approx(g_ref ** 4 / rc ** 3, rel=5e-9)
    # the production tolerance's true error
    assert rp["r_cross"] == pytest.approx(rc, rel=2e-7)
    assert rp["g"] == pytest.approx(g_ref, rel=2e-7)
    assert rp["phi_cross"] == pytest.approx(ref[2], rel=2e-7, abs=2e-7)


def test_production_error_shrinks_with_tolerance():
    """P14: at a = 0.9 and 0.998 the crossing radius converges as rtol falls (1e-8 -> 1e-10)."""
    for a, inc, x, y in KERR_RAYS[:5]:
        ok, y6, c4 = O.initial_state(O.Scene(a=a, incl_deg=inc), x, y)
        ref = _first_crossing(a, y6, c4)
        errs = []
        for rtol in (1e-8, 1e-10):
            r = O.trace_ray(O.Scene(a=a, incl_deg=inc, model=O.MODEL_THIN_DISK, rtol=rtol), x, y)
            errs.append(abs(r["r_cross"] - ref[0]) / ref[0])
        assert errs[1] < errs[0] / 5 or errs[0] < 1e-10, errs


# ----------------------------------------------------------- P11: redshift

@pytest.mark.parametrize("a", [0.0, 0.5, 0.9, 0.998])
def test_emitter_redshift_off_the_equator(a):
    """Eq. (2) with the emitter's four-velocity normalised by the metric itself (u.u = -1),
    at every polar angle: the Keplerian shell where its orbit is timelike, the
    zero-angular-momentum observer where it is not."""
    scn = O.Scene(a=a)
    rng = np.random.default_rng(17)
    branches = {"keplerian": 0, "zamo": 0}
    rplus = 1 + math.sqrt(1 - a * a)
    for _ in range(300):
        r = rplus * (1.001 + 9 * rng.random() ** 3)
        th = rng.uniform(0.05, math.pi - 0.05)
        xi = rng.uniform(-6, 6)
        u, which = emitter_velocity(a, r, th)
        G = kerr_metric(a, r, th)
        assert u @ G @ u == pytest.approx(-1.0, abs=1e-9)
        want, _ = redshift_contraction(a, r, th, -xi)  # the traced ray's L is -xi (E = -1)
        got = O.redshift(scn, r, th, xi)
        assert got == pytest.approx(want, rel=1e-9), (r, th, xi, which)
        branches[which] += 1
    assert branches["keplerian"] > 100
    if a > 0.4:
        assert branches["zamo"] > 10  # inside the circular-photon-orbit region


# --------------------------------------------- R19/R22: transfer coefficients

def test_torus_coefficients_from_invariant_transfer():
    """The torus plasma (density with scale height h r, temperature power law, field from
    B^2/8pi = eps_B n_e m_p c^2/(6 r)) and the redshift powers of Eqs. (30)-(31): emission
    g^2 j_0(nu/g) and absorption alpha_0(nu/g)/g per unit affine parameter."""
    scn = O.Scene(a=0.9, model=O.MODEL_TORUS, freqs_hz=[230e9], n0_cgs=3e6, r_norm=2.5, n_index=1.3,
                  h_over_r=0.4, T0_K=8e10, T_index=0.7, eps_B=0.2, mbh_msun=6.5e9, r_emit_max=500.0)
    rng = np.random.default_rng(23)
    for _ in range(60):
        r = rng.uniform(2.5, 80.0)
        th = rng.uniform(0.3, math.pi - 0.3)
        g = rng.uniform(0.3, 1.8)
        nu = 10 ** rng.uniform(10.5, 12.5)
        a_lam, e_lam = O.torus_coeffs(scn, r, th, g, nu)
        a_want, e_want = transfer_coefficients(scn, r, th, g, nu)
        assert a_lam == pytest.approx(a_want, rel=1e-7), (r, th, g, nu)  # the oracle rounds e to 9 digits
        assert e_lam == pytest.approx(e_want, rel=1e-7), (r, th, g, nu)
    # no emission or absorption at or inside the capture radius, nor beyond r_emit_max
    rcap = (1 + math.sqrt(1 - 0.81)) * (1 + 1e-3)
    assert O.torus_coeffs(scn, rcap * 0.999, 1.0, 1.0, 230e9) == (0.0, 0.0)
    assert O.torus_coeffs(scn, 500.5, 1.0, 1.0, 230e9) == (0.0, 0.0)
    assert O.torus_coeffs(scn, 499.5, 1.0, 1.0, 230e9)[1] > 0.0


@pytest.mark.parametrize("x,y", [(3.0, 4.0), (-6.0, 1.0), (1.0, -9.0), (12.0, 12.0)])
def test_thick_moving_emitter(x, y):
    """P13(iii): a medium of uniform temperature, optically thick within a fraction of one step,
    filling r <= 30 M around a spinning hole. The ray's first point inside sees the Keplerian
    shell moving with redshift g, and the emergent intensity is g^3 B_nu(T, nu/g) there."""
    T = 3e10
    freqs = [86e9, 230e9, 690e9]
    scn = O.Scene(a=0.9, incl_deg=60.0, model=O.MODEL_TORUS, freqs_hz=freqs, T0_K=T, T_index=0.0, n0_cgs=1e12,
                  n_index=0.0, h_over_r=1e6, hmax_frac=0.05, r_emit_max=30.0)
    res, path = O.trace_path(scn, x, y)
    k = int(np.nonzero(path[:, 1] <= 30.0)[0][0])
    lam, r, th, ph, t, pr, pth = path[k]
    g, which = redshift_contraction(0.9, r, th, res["L"], pr, pth)
    assert which == "keplerian"
    assert abs(math.cos(th)) > 0.05  # off the equatorial plane
    for f, nu in enumerate(freqs):
        assert res["tau"][f] > 1e3
        assert res["I"][f] == pytest.approx(g ** 3 * planck(nu / g, T), rel=1e-8)


def test_formal_solution_along_a_straight_line():
    """P13(ii) and the profile of the torus: in flat space (M = 0, a = 0, so g = 1) every ray is a
    straight line, and the transfer equation's formal solution along it, integrated here with
    the coefficients above, is what the oracle's quadrature converges to (step cap 0.0025 r), in
    the optically thin regime and with absorption."""
    base = dict(a=0.0, mass=0.0, incl_deg=50.0, model=O.MODEL_TORUS, hmax_frac=0.0025, r_norm=2.0,
                n_index=1.1, h_over_r=0.3, T0_K=1e11, T_index=0.84, eps_B=0.1, mbh_msun=4e6, r_emit_max=1000.0)
    th_o = math.radians(50.0)
    n_hat = np.array([math.sin(th_o), 0.0, math.cos(th_o)])
    e_x = np.array([0.0, 1.0, 0.0])
    e_y = np.array([-math.cos(th_o), 0.0, math.sin(th_o)])
    for n0, thin in [(1e4, True), (3e10, False)]:
        freqs = [86e9, 345e9]
        scn = O.Scene(n0_cgs=n0, freqs_hz=freqs, **base)
        for px, py in [(2.0, 3.0), (-5.0, 0.5), (0.0, -8.0)]:
            res = O.trace_ray(scn, px, py)
            assert res["status"] & O.ESCAPED
            p0 = 1000.0 * n_hat + px * e_x + py * e_y
            lam_end = res["lambda_end"]

            def f(lam, z, nu):
                p = p0 - lam * n_hat
                r = float(np.linalg.norm(p))
                if r > 1000.0:
                    return [0.0, 0.0]
                a_l, e_l = transfer_coefficients(scn, r, math.acos(p[2] / r), 1.0, nu)
                return [a_l, e_l * math.exp(-z[0])]
            for k, nu in enumerate(freqs):
                sol = solve_ivp(f, (0.0, lam_end), [0.0, 0.0], args=(nu,), method="RK45", rtol=1e-10,
                                atol=1e-40, max_step=2.0, first_step=0.5)
                tau_ref, I_ref = sol.y[:, -1]
                assert res["tau"][k] == pytest.approx(tau_ref, rel=1e-4)
                assert res["I"][k] == pytest.approx(I_ref, rel=1e-4)
                if thin:
                    assert tau_ref < 1e-2
                elif k == 0:
                    assert tau_ref > 1.0  # the absorbing case really absorbs


# ---------------------------------------------------------------- underflow

def test_step_underflow_at_the_coordinate_horizon():
    """With a capture radius of r_+(1 + 1e-12) the Boyer-Lindquist coordinate singularity at the
    horizon drives the adaptive step below 1e-12 r before the ray gets there: every ray the radial
    potential captures ends in UNDERFLOW (never CAPTURED) just outside r_+; the others escape."""
    a = 0.9
    scn = O.Scene(a=a, incl_deg=60.0, model=O.MODEL_GEODESIC, horizon_delta=1e-12)
    res = O.trace_image(scn, 6, 6, -5, 5, -5, 5).ravel()
    rplus = 1 + math.sqrt(1 - a * a)
    uf = (res["status"] & O.UNDERFLOW) != 0
    assert uf.sum() >= 20
    assert not np.any(res["status"] & O.CAPTURED)
    for ray in res[uf]:
        assert 0 <= ray["final_state"][0] - rplus < 1e-5
        assert not ray["status"] & O.ESCAPED
        xi, eta = ray["L"] / ray["E"], ray["Q"] / ray["E"] ** 2
        coeffs = [1.0, 0.0, a * a - xi * xi - eta, 2.0 * ((xi - a) ** 2 + eta), -a * a * eta]
        rts = np.roots(coeffs)
        real = rts[np.abs(rts.imag) < 1e-9].real
        assert not np.any(real > rplus)  # no radial turning point outside the horizon
    assert np.all(res["status"][~uf] & O.ESCAPED)


# ------------------------------------- higher-order images of a thick disk

def _equator_crossings(a, y6, c4, max_cross=4):
    """All equatorial crossings (state vectors) of the Hamiltonian flow before the ray is captured
    or escapes, in order."""
    rplus = 1 + math.sqrt(1 - a * a)

    def equator(lam, z):
        return z[1] - math.pi / 2

    def horizon(lam, z):
        return z[0] - rplus * (1 + 1e-3)
    horizon.terminal = True

    def escape(lam, z):
        return z[0] - 1001.0
    escape.terminal = True
    sol = solve_ivp(_hamilton_flow(a, c4[0], c4[1]), (0.0, 1e5), y6, method="DOP853", rtol=1e-13, atol=1e-13,
                    events=[equator, horizon, escape])
    rcap = rplus * (1 + 1e-3)
    return [z for z in sol.y_events[0] if z[0] > rcap][:max_cross]


DISK_IMAGE_RAYS = [(0.0, 80.0, -4.667, -7.867), (0.0, 80.0, -0.933, -5.2), (0.0, 80.0, 3.6, -3.867),
                   (0.9, 75.0, 0.933, -6.8), (0.9, 75.0, -2.267, 2.8), (0.998, 85.0, -1.467, -4.133),
                   (0.998, 85.0, -1.0, -3.6), (0.5, 40.0, -4.4, -0.933), (0.5, 40.0, 3.067, 4.667),
                   (0.9, 60.0, 5.0, 3.0), (0.0, 80.0, -5.3, 0.4), (0.998, 85.0, 2.4, 3.4)]


@pytest.mark.parametrize("a,inc,x,y", DISK_IMAGE_RAYS)
def test_disk_images_through_every_crossing(a, inc, x, y):
    """Thick thin disk seen through every crossing: the ray ends at the first equatorial crossing
    that lands on the disk [r_ISCO, 20 M], which may be its second or third (a higher-order image
    made by the hole's lensing). Crossing order, radius, redshift and intensity against the
    independent flow (to 1e-9 at rtol 1e-12); the production controls within the method's error,
    2e-7 for the direct image and about e^pi times more per extra half orbit."""
    ok, y6, c4 = O.initial_state(O.Scene(a=a, incl_deg=inc), x, y)
    zs = _equator_crossings(a, y6, c4)
    r_in = O.isco(a)
    hit = next((k for k, z in enumerate(zs) if r_in <= z[0] <= 20.0), None)
    tight = O.trace_ray(O.Scene(a=a, incl_deg=inc, model=O.MODEL_DISK_IMAGES, rtol=1e-12, hmax_frac=0.005), x, y)
    prod = O.trace_ray(O.Scene(a=a, incl_deg=inc, model=O.MODEL_DISK_IMAGES), x, y)
    if hit is None:
        assert not tight["status"] & O.DISK_HIT and not prod["status"] & O.DISK_HIT
        assert tight["n_cross"] == len(zs) and tight["intensity"] == 0.0
        return
    z = zs[hit]
    g_ref, _ = redshift_contraction(a, z[0], math.pi / 2, c4[1], z[4], z[5])
    # each half orbit near the photon sphere amplifies an error by about e^pi: the higher the
    # image order, the larger the true error of the same controls
    amp = 30.0 ** hit
    for res, tol in ((tight, 1e-9 * amp), (prod, 2e-7 * amp)):
        assert res["status"] & O.DISK_HIT and res["status"] & O.CROSSED
        assert res["n_cross"] == hit + 1
        assert res["r_cross"] == pytest.approx(z[0], rel=tol)
        assert res["phi_cross"] == pytest.approx(z[2], rel=tol)
        assert res["t_cross"] == pytest.approx(z[3], rel=tol)
        assert res["g"] == pytest.approx(g_ref, rel=tol)
        assert res["intensity"] == pytest.approx(g_ref ** 3 / z[0] ** 3, rel=5 * tol)
    # the disk absorbs the ray: it ends there, neither captured nor escaped
    assert not prod["status"] & 3


def test_disk_images_include_higher_orders_and_match_first_crossing_model():
    """Over an image, the rays whose first crossing is on the disk give exactly the first-crossing
    model's values, and some pixels show the disk only through a later crossing."""
    pts = O.pixel_points(24, 24, -9, 9, -9, 9)
    for a, inc in [(0.0, 80.0), (0.9, 75.0)]:
        one = O.trace_points(O.Scene(a=a, incl_deg=inc, model=O.MODEL_THIN_DISK), pts)
        many = O.trace_points(O.Scene(a=a, incl_deg=inc, model=O.MODEL_DISK_IMAGES), pts)
        first = (one["status"] & O.DISK_HIT) != 0
        assert np.all(many["status"][first] & O.DISK_HIT)
        assert np.all(many["n_cross"][first] == 1)
        for k in ("r_cross", "g", "phi_cross", "t_cross", "intensity", "i_bol"):
            assert np.array_equal(many[k][first], one[k][first]), k
        later = ((many["status"] & O.DISK_HIT) != 0) & ~first
        assert later.sum() >= 5, (a, inc, later.sum())
        assert np.all(many["n_cross"][later] >= 2)


# ------------------------------------------------------------- hot spot

def _spot_geometry(a, r_s, phi0, t_obs):
    om = 1.0 / (r_s ** 1.5 + a)
    Rs = math.sqrt(r_s * r_s + a * a)

    def dist(z):  # pseudo-Cartesian distance from the centre at the emission time t_obs + t
        r, th, ph, t = z[0], z[1], z[2], z[3]
        R = math.sqrt(r * r + a * a)
        p = np.array([R * math.sin(th) * math.cos(ph), R * math.sin(th) * math.sin(ph), r * math.cos(th)])
        pc = phi0 + om * (t_obs + t)
        return float(np.linalg.norm(p - np.array([Rs * math.cos(pc), Rs * math.sin(pc), 0.0])))
    return om, dist


def _spot_entry(a, y6, c4, r_s, size, phi0, t_obs):
    """First entry of the Hamiltonian flow into {z > 0, d < 4 r_spot}: the continuous function
    max(d - 4 r_spot, -z) falls through 0 there, whether through the dome or the base."""
    om, dist = _spot_geometry(a, r_s, phi0, t_obs)
    rplus = 1 + math.sqrt(1 - a * a)

    def entry(lam, z):
        return max(dist(z) - 4 * size, -z[0] * math.cos(z[1]))
    entry.terminal = True
    entry.direction = -1

    def horizon(lam, z):
        return z[0] - rplus * (1 + 1e-3)
    horizon.terminal = True

    def escape(lam, z):
        return z[0] - 1001.0
    escape.terminal = True

    def near(lam, z):  # the spot lies within r_s + 4 r_spot of the hole
        return z[0] - (r_s + 4 * size + 3.0)
    near.terminal = True
    near.direction = -1
    flow = _hamilton_flow(a, c4[0], c4[1])
    far = solve_ivp(flow, (0.0, 1e5), y6, method="DOP853", rtol=1e-13, atol=1e-13, events=[near, horizon, escape])
    if len(far.t_events[0]) == 0:
        return None
    # short steps near the spot, so that a ray grazing its surface is not stepped over
    lam0 = far.t_events[0][0]
    sol = solve_ivp(flow, (lam0, lam0 + 1e5), far.y_events[0][0], method="DOP853", rtol=1e-13, atol=1e-13,
                    max_step=0.05, events=[entry, horizon, escape])
    if len(sol.t_events[0]) == 0:
        return None
    return sol.y_events[0][0]


SPOT_RAYS = [(0.0, 60.0, 0.0, 0.0, 0.0), (0.0, 60.0, 35.0, 0.0, 0.0), (0.0, 60.0, 170.0, 40.0, 0.0),
             (0.0, 30.0, 250.0, 13.0, 0.0), (0.9, 60.0, 90.0, -20.0, 8.0), (0.9, 75.0, 300.0, 7.0, 8.0)]


@pytest.mark.parametrize("a,inc,phi0_deg,t_obs,orbit", SPOT_RAYS)
def test_hot_spot_entry_against_hamiltonian_flow(a, inc, phi0_deg, t_obs, orbit):
    """Section 4.4: rays end where they first enter the optically thick spot, evaluated at the
    emission time t_obs - Delta t; the entry point (r, phi, t), the redshift of the co-moving spot
    material and the intensity g^3 exp(-d^2/(2 r_spot^2)) against the independent flow, for pixels
    over the spot's direct and lensed images."""
    r_s = orbit if orbit > 0 else O.isco(a)
    phi0 = math.radians(phi0_deg)
    spot = dict(model=O.MODEL_HOT_SPOT, spot_r=orbit, spot_size=0.5, spot_phi0=phi0, t_obs=t_obs)
    scn = O.Scene(a=a, incl_deg=inc, rtol=1e-12, hmax_frac=0.005, **spot)
    prod = O.Scene(a=a, incl_deg=inc, **spot)
    pts = O.pixel_points(20, 20, -9, 9, -9, 9)
    coarse = O.trace_points(prod, pts)
    hits = np.nonzero((coarse["status"] & O.SPOT_HIT) != 0)[0]
    assert len(hits) >= 3
    om, dist = _spot_geometry(a, r_s, phi0, t_obs)
    checked = grazing = 0
    for i in hits[:: max(1, len(hits) // 5)]:
        x, y = pts[i]
        ok, y6, c4 = O.initial_state(scn, x, y)
        z = _spot_entry(a, y6, c4, r_s, 0.5, phi0, t_obs)
        res = O.trace_ray(scn, x, y)
        if z is None:  # the flow's event search stepped over a grazing entry
            grazing += 1
            continue
        assert res["status"] == O.SPOT_HIT
        assert res["r_cross"] == pytest.approx(z[0], rel=1e-8)
        assert res["phi_cross"] == pytest.approx(z[2], rel=1e-8, abs=1e-8)
        assert res["t_cross"] == pytest.approx(t_obs + z[3], rel=1e-8, abs=1e-8)
        # the spot material co-rotates with the centre: u = u^t (1, 0, 0, Omega_s), u.u = -1
        G = kerr_metric(a, z[0], z[1])
        k = np.array([1.0, 0.0, 0.0, om])
        assert k @ G @ k < 0  # timelike wherever the spot is
        u = k / math.sqrt(-(k @ G @ k))
        g_ref = 1.0 / -(photon_momentum(c4[1], z[4], z[5]) @ u)
        assert res["g"] == pytest.approx(g_ref, rel=1e-8)
        j = math.exp(-dist(z) ** 2 / (2 * 0.25))
        assert res["intensity"] == pytest.approx(g_ref ** 3 * j, rel=1e-6)
        assert res["i_bol"] == pytest.approx(g_ref ** 4 * j, rel=1e-6)
        checked += 1
    assert checked >= 3 and grazing <= 1


def test_hot_spot_images_repeat_after_one_orbit():
    """The spot returns after one orbital period 2 pi / Omega_s: images at t_obs and t_obs + T agree."""
    a = 0.0
    T = 2 * math.pi * (6.0 ** 1.5 + a)
    pts = O.pixel_points(24, 24, -9, 9, -9, 9)
    im = [O.trace_points(O.Scene(a=a, incl_deg=60.0, model=O.MODEL_HOT_SPOT, t_obs=t), pts) for t in (30.0, 30.0 + T)]
    hit0, hit1 = (im[0]["status"] & O.SPOT_HIT) != 0, (im[1]["status"] & O.SPOT_HIT) != 0
    assert hit0.sum() > 5 and np.array_equal(hit0, hit1)
    np.testing.assert_allclose(im[1]["intensity"][hit0], im[0]["intensity"][hit0], rtol=1e-6)
    np.testing.assert_allclose(im[1]["t_cross"][hit0] - T, im[0]["t_cross"][hit0], rtol=1e-9)


def test_hot_spot_approaching_side_brightest():
    """Over one orbit the observed flux peaks while the spot approaches the observer (g > 1 then)."""
    a, inc = 0.0, 60.0
    T = 2 * math.pi * 6.0 ** 1.5
    pts = O.pixel_points(32, 32, -9, 9, -9, 9)
    flux, gmax = [], []
    for k in range(8):
        r = O.trace_points(O.Scene(a=a, incl_deg=inc, model=O.MODEL_HOT_SPOT, t_obs=k * T / 8), pts)
        hit = (r["status"] & O.SPOT_HIT) != 0
        flux.append(r["i_bol"].sum())
        gmax.append(r["g"][hit].max())
    k = int(np.argmax(flux))
    assert gmax[k] > 1.0
    assert max(flux) > 3 * min(flux)
