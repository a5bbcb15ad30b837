"""Pins of the oracle's spectra (flux density per image and frequency, section 4).

The sum is checked against closed forms a plausible slip would break: a
separable geometric image (a wrong index, a dropped or extra pixel, an image
range shifted by one, frequencies and images swapped all change it), a
constant image, linearity, and the solid-angle bookkeeping (the pixels of an
image add up to the solid angle of the whole image plane)."""
import math

import numpy as np
import pytest

from oracle import spectra as S


def geometric_batch(dims, freqs_scale, r=0.93, q=0.71):
    """Images of nx x ny pixels with I[f][j nx + i] = c_f r^i q^j, concatenated."""
    parts, offsets = [], [0]
    for nx, ny in dims:
        i = np.arange(nx)[None, :]
        j = np.arange(ny)[:, None]
        img = (r ** i) * (q ** j)
        parts.append(img.ravel())
        offsets.append(offsets[-1] + nx * ny)
    base = np.concatenate(parts) if parts else np.zeros(0)
    I = np.stack([c * base for c in freqs_scale])
    return I, offsets


def geometric_sum(nx, ny, r=0.93, q=0.71):
    return (1 - r ** nx) / (1 - r) * (1 - q ** ny) / (1 - q)


def test_geometric_images_closed_form():
    dims = [(7, 5), (0, 0), (1, 1), (31, 17), (12, 40)]
    cs = [1.0, 2.5e-3, 7.0e4]
    I, off = geometric_batch(dims, cs)
    dom = [1.0, 2.0, 3.0, 0.5, 1e-20]
    F = S.image_spectra(I, off, dom)
    assert F.shape == (len(dims), len(cs))
    for k, (nx, ny) in enumerate(dims):
        for f, c in enumerate(cs):
            want = dom[k] * c * geometric_sum(nx, ny) if nx * ny else 0.0
            assert F[k, f] == pytest.approx(want, rel=1e-14, abs=0.0), (k, f)


def test_constant_image_and_linearity():
    rng = np.random.Generator(np.random.PCG64(5))
    n = 10000
    I = np.full((2, n), 3.0)
    F = S.image_spectra(I, [0, n], [0.25])
    assert F[0, 0] == 0.25 * 3.0 * n and F[0, 1] == F[0, 0]
    A = rng.uniform(0, 1, (3, 5000))
    B = rng.uniform(0, 1, (3, 5000))
    off, dom = [0, 1234, 5000], [1.0, 1.0]
    FA, FB, FAB = (S.image_spectra(X, off, dom) for X in (A, B, 2 * A + B))
    assert np.allclose(FAB, 2 * FA + FB, rtol=1e-14, atol=0)
    # images are disjoint: the spectra of a batch add up to the spectrum of all rays
    assert math.isclose(FA[:, 1].sum(), math.fsum(A[1]), rel_tol=1e-15)


def test_pixel_solid_angles_cover_the_image_plane():
    nx, ny, ext = 1024, 768, (-20.0, 20.0, -15.0, 15.0)
    mbh, dist = 4e6, 8.0 * 3.0856775814913673e21  # Sgr A*-like: 4e6 solar masses (section 4.5) at 8 kpc
    dom = S.pixel_solid_angle(nx, ny, *ext, mbh, dist)
    rg = S.gravitational_radius_cm(mbh)
    assert rg == pytest.approx(5.9065e11, rel=1e-4)  # G M / c^2 for 4e6 solar masses
    whole = (ext[1] - ext[0]) * (ext[3] - ext[2]) * (rg / dist) ** 2
    assert nx * ny * dom == pytest.approx(whole, rel=1e-14)
    # halving the pitch quarters the pixel
    assert S.pixel_solid_angle(2 * nx, 2 * ny, *ext, mbh, dist) == pytest.approx(dom / 4, rel=1e-15)


def test_spectrogram_bins_and_lightcurve():
    """Spectrogram rows (section 4.4): each ray's weight lands in the bin [e_b, e_b+1) holding its g,
    rays outside the edges are dropped, and a frame's bins add up to its lightcurve point (the
    frequency-integrated flux) whenever every g lies inside the edges."""
    edges = [0.5, 0.75, 1.0, 1.25, 1.5]
    # frame 0: g cycles through the four bins' midpoints; frame 1: a bin edge and two outsiders
    g0 = np.array([0.6, 0.8, 1.1, 1.3] * 5)
    w0 = 2.0 ** -np.arange(20)
    g1 = np.array([0.75, 1.0, 1.5, 0.49, 1.25])
    w1 = np.array([1.0, 10.0, 100.0, 1000.0, 10000.0])
    Sg = S.spot_spectrogram(np.concatenate([w0, w1]), np.concatenate([g0, g1]), [0, 20, 25], [2.0, 0.5], edges)
    want0 = [2.0 * sum(w0[b::4]) for b in range(4)]
    np.testing.assert_allclose(Sg[0], want0, rtol=1e-15)
    # 0.75 -> bin 1, 1.0 -> bin 2, 1.25 -> bin 3; 1.5 (the last edge) and 0.49 are outside
    np.testing.assert_allclose(Sg[1], [0.0, 0.5, 5.0, 5000.0], rtol=1e-15)
    lc = S.image_spectra(w0, [0, 20], [2.0])[0, 0]
    assert Sg[0].sum() == pytest.approx(lc, rel=1e-15)


# ------------------------------------------------- Novikov-Thorne disk (f2)

def _circular_orbit(a, r):
    """Omega, specific energy E and angular momentum L of prograde circular equatorial orbits (M = 1)."""
    sr = np.sqrt(r)
    den = r ** 0.75 * np.sqrt(r ** 1.5 - 3 * sr + 2 * a)
    return 1 / (r ** 1.5 + a), (r ** 1.5 - 2 * sr + a) / den, (r * r - 2 * a * sr + a * a) / den


def _page_thorne_f_quadrature(a, r):
    """f(r) of Eq. (35) from its defining integral (Page & Thorne 1974): the flux
    F = Mdot/(4 pi r) (-dOmega/dr) / (E - Omega L)^2 int_{r_ISCO}^r (E - Omega L) dL/dr' dr',
    over its Newtonian form 3 Mdot / (8 pi r^3); derivatives by complex steps, scipy quadrature."""
    from scipy.integrate import quad
    from scipy.optimize import minimize_scalar
    h = 1e-30
    dOm = lambda x: (_circular_orbit(a, x + 1j * h)[0]).imag / h
    dL = lambda x: (_circular_orbit(a, x + 1j * h)[2]).imag / h
    r_ms = minimize_scalar(lambda x: _circular_orbit(a, x)[1], bounds=(1.0 + 1e-6 + (a > 0.99) * 0.1, 10.0),
                           method="bounded", options={"xatol": 1e-12}).x
    def integrand(x):
        Om, E, L = _circular_orbit(a, x)
        return (E - Om * L) * dL(x)
    I, _ = quad(integrand, r_ms, r, epsabs=0, epsrel=1e-13, limit=200)
    Om, E, L = _circular_orbit(a, r)
    F_over_mdot = -dOm(r) / (E - Om * L) ** 2 * I / (4 * math.pi * r)
    return F_over_mdot / (3 / (8 * math.pi * r ** 3))


@pytest.mark.parametrize("a", [0.0, 0.5, 0.9, 0.998])
def test_novikov_thorne_factor_closed_form_vs_integral(a):
    """Page & Thorne's closed form of f(r) equals their defining integral; f vanishes at the ISCO
    (zero torque there, section 4.3) and tends to 1 far away (the Newtonian disk)."""
    checked = 0
    for r in [1.3, 2.5, 4.0, 7.0, 12.0, 30.0, 100.0, 1e4]:
        f = float(S.novikov_thorne_f(a, r))
        if f == 0.0:
            continue  # inside the ISCO
        assert f == pytest.approx(_page_thorne_f_quadrature(a, r), rel=1e-7), (a, r)
        checked += 1
    assert checked >= 5
    assert np.all(S.novikov_thorne_f(a, np.array([0.5, 0.9])) == 0.0)
    assert abs(float(S.novikov_thorne_f(a, 1e10)) - 1.0) < 1e-4
    # vanishes at the ISCO itself
    import oracle as O
    assert abs(float(S.novikov_thorne_f(a, O.isco(a) * (1 + 1e-12)))) < 1e-5


def test_stefan_boltzmann_constant():
    """sigma from its definition agrees with the printed CODATA 2018 value (5.670374419e-8 W m^-2
    K^-4, truncated to ten digits) and with scipy's."""
    from scipy import constants as C
    assert S.SIGMA_SB == pytest.approx(5.670374419e-5, rel=2e-10)
    assert S.SIGMA_SB == pytest.approx(C.Stefan_Boltzmann * 1e3, rel=2e-10)  # W m^-2 K^-4 -> erg cm^-2 s^-1 K^-4


def test_disk_spectrum_integrates_to_redshifted_stefan_boltzmann():
    """Each disk pixel contributes g^3 B_nu(T, nu/g); over all frequencies that is g^4 sigma T^4 / pi
    (Stefan-Boltzmann with the redshift of I_nu/nu^3), so a frequency quadrature of the spectrum
    gives domega * sum g^4 sigma T_eff^4 / pi; pixels off the disk contribute nothing."""
    a, mbh, mdot = 0.9, 10.0, 1e19
    r = np.array([3.0, 5.0, 9.0, 20.0, 2.0, 40.0])
    g = np.array([1.2, 0.8, 1.05, 0.9, 0.7, 1.0])
    hit = np.array([True, True, True, True, False, True])
    nu = np.geomspace(1e14, 1e20, 6001)
    F = S.disk_spectrum(r, g, hit, [0, 6], [2.0], nu, [a], mbh, mdot)[0]
    T = S.novikov_thorne_teff(a, r[hit], mbh, mdot)
    want = 2.0 * np.sum(g[hit] ** 4 * S.SIGMA_SB * T ** 4 / math.pi)
    lnu = np.log(nu)
    got = np.sum(0.5 * (F[1:] * nu[1:] + F[:-1] * nu[:-1]) * np.diff(lnu))
    assert got == pytest.approx(want, rel=1e-5)
    # Teff from Eq. (35) in cgs: sigma T^4 = 3 G M Mdot f / (8 pi R^3)
    rg = S.gravitational_radius_cm(mbh)
    T5 = S.novikov_thorne_teff(a, 5.0, mbh, mdot)
    assert S.SIGMA_SB * T5 ** 4 == pytest.approx(
        3 * S.GM_SUN * mbh * mdot * S.novikov_thorne_f(a, 5.0) / (8 * math.pi * (5.0 * rg) ** 3), rel=1e-12)
