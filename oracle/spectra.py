"""Spectra of traced images -- TEST INFRASTRUCTURE ONLY.

Part of the FP64 CPU oracle (see the package docstring: only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
use it, and it shares no code with the GPU library).

The flux density an observer at distance D receives from an image at one
frequency (the spectra of section 4) is the integral of the observed specific
intensity over the solid angle the image subtends. The image plane of section
2.2 is flat, in units of M = r_g = G M_bh / c^2, so a pixel of dx by dy M^2
subtends dx dy (r_g / D)^2 sr, and

    F_nu = sum over the image's pixels of I_nu * dx dy (r_g / D)^2.

This module is that definition written out: one exactly rounded sum
(``math.fsum``) per image and frequency.
"""
from __future__ import annotations

import math
from typing import Sequence

import numpy as np

C_LIGHT = 2.99792458e10  # speed of light, cm s^-1 (exact)
GM_SUN = 1.3271244e26    # nominal solar GM, cm^3 s^-2 (IAU 2015 Resolution B3)


def gravitational_radius_cm(mbh_msun: float) -> float:
    """r_g = G M / c^2 in cm for a black hole of mbh_msun solar masses."""
    return GM_SUN * mbh_msun / (C_LIGHT * C_LIGHT)


def pixel_solid_angle(nx: int, ny: int, x_min: float, x_max: float, y_min: float, y_max: float,
                      mbh_msun: float, distance_cm: float) -> float:
    """Solid angle (sr) of one pixel of an nx x ny image over [x_min, x_max] x [y_min, y_max] M."""
    q = gravitational_radius_cm(mbh_msun) / distance_cm
    return ((x_max - x_min) / nx) * ((y_max - y_min) / ny) * q * q


def image_spectra(intensity, offsets: Sequence[int], domega: Sequence[float]) -> np.ndarray:
    """F[k, f] = domega[k] * sum of intensity[f, offsets[k]:offsets[k + 1]] (exactly rounded sum).

    intensity: [nfreq, total] (or [total]) observed I_nu of all images' rays, image k owning
    rays offsets[k] .. offsets[k + 1] - 1 (the layout of a batch of images)."""
    I = np.atleast_2d(np.asarray(intensity, dtype=np.float64))
    nimg = len(offsets) - 1
    F = np.zeros((nimg, I.shape[0]))
    for k in range(nimg):
        lo, hi = int(offsets[k]), int(offsets[k + 1])
        for f in range(I.shape[0]):
            F[k, f] = float(domega[k]) * math.fsum(I[f, lo:hi])
    return F


def spot_spectrogram(i_bol, g, offsets: Sequence[int], domega: Sequence[float], g_edges: Sequence[float]) -> np.ndarray:
    """S[k, b] = domega[k] * sum of i_bol over image k's rays with g_edges[b] <= g < g_edges[b + 1]
    (exactly rounded sums): the flux of a line emitted at one rest-frame energy, binned by its
    observed energy shift g, one row per frame (the spectrogram of section 4.4, Fig. 7). Summed
    over the bins it is the frame's point of the lightcurve (Fig. 8)."""
    w = np.asarray(i_bol, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    e = np.asarray(g_edges, dtype=np.float64)
    nimg, nb = len(offsets) - 1, len(e) - 1
    S = np.zeros((nimg, nb))
    for k in range(nimg):
        lo, hi = int(offsets[k]), int(offsets[k + 1])
        for b in range(nb):
            sel = (g[lo:hi] >= e[b]) & (g[lo:hi] < e[b + 1])
            S[k, b] = float(domega[k]) * math.fsum(w[lo:hi][sel])
    return S


# ----------------------------------------------------- Novikov-Thorne disk

H_PLANCK = 6.62607015e-27  # erg s (exact, SI 2019)
K_BOLTZ = 1.380649e-16     # erg K^-1 (exact, SI 2019)
# Stefan-Boltzmann constant, erg cm^-2 s^-1 K^-4: its definition 2 pi^5 k^4 / (15 h^3 c^2), exact
# with the exact h, k and c (the printed CODATA 2018 value 5.670374419e-5 is this, truncated)
SIGMA_SB = 2.0 * math.pi ** 5 * K_BOLTZ ** 4 / (15.0 * H_PLANCK ** 3 * C_LIGHT ** 2)


def novikov_thorne_f(a: float, r):
    """Correction factor f(r) of the disk flux of section 4.3 (Eq. (35)),
    F(r) = 3 Mdot M f(r) / (8 pi r^3), for a prograde disk whose stress vanishes at r_ISCO:
    the closed form of Page & Thorne (1974) in x = sqrt(r/M),

        f = x^2 / (x^3 - 3x + 2a) * [x - x0 - (3/2) a ln(x/x0)
              - sum_i 3 (x_i - a)^2 / (x_i (x_i - x_j)(x_i - x_k)) ln((x - x_i)/(x0 - x_i))],

    x0 = sqrt(r_ISCO), x_1,2,3 the roots of x^3 - 3x + 2a = 0. It is 0 at the ISCO and tends to 1
    far out. Zero inside the ISCO."""
    r = np.asarray(r, dtype=np.float64)
    z1 = 1.0 + np.cbrt(1.0 - a * a) * (np.cbrt(1.0 + a) + np.cbrt(1.0 - a))
    z2 = math.sqrt(3.0 * a * a + z1 * z1)
    r_ms = 3.0 + z2 - math.sqrt((3.0 - z1) * (3.0 + z1 + 2.0 * z2))  # Bardeen, Press & Teukolsky (1972)
    x0 = math.sqrt(r_ms)
    th = math.acos(a)
    xs = (2.0 * math.cos((th - math.pi) / 3.0), 2.0 * math.cos((th + math.pi) / 3.0), -2.0 * math.cos(th / 3.0))
    x = np.sqrt(np.maximum(r, r_ms))
    bracket = x - x0 - 1.5 * a * np.log(x / x0)
    for i in range(3):
        xi, xj, xk = xs[i], xs[(i + 1) % 3], xs[(i + 2) % 3]
        bracket = bracket - 3.0 * (xi - a) ** 2 / (xi * (xi - xj) * (xi - xk)) * np.log((x - xi) / (x0 - xi))
    f = x * x * bracket / (x ** 3 - 3.0 * x + 2.0 * a)
    return np.where(r >= r_ms, f, 0.0)


def novikov_thorne_teff(a: float, r, mbh_msun: float, mdot_gs: float):
    """Effective temperature (K) of the disk surface at r (in M), from Eq. (35):
    sigma T^4 = 3 G M Mdot f(r) / (8 pi R^3), R = r r_g."""
    rg = gravitational_radius_cm(mbh_msun)
    GM = GM_SUN * mbh_msun
    F = 3.0 * GM * mdot_gs * novikov_thorne_f(a, r) / (8.0 * math.pi * (np.asarray(r) * rg) ** 3)
    return (F / SIGMA_SB) ** 0.25


def planck(nu, T):
    """B_nu(T), erg s^-1 cm^-2 Hz^-1 sr^-1 (0 where T = 0)."""
    nu = np.asarray(nu, dtype=np.float64)
    T = np.asarray(T, dtype=np.float64)
    with np.errstate(divide="ignore", over="ignore", invalid="ignore"):
        x = H_PLANCK * nu / (K_BOLTZ * T)
        B = 2.0 * H_PLANCK * nu ** 3 / C_LIGHT ** 2 / np.expm1(x)
    return np.where(T > 0, np.nan_to_num(B, nan=0.0, posinf=0.0), 0.0)


def disk_spectrum(r_cross, g, hit, offsets: Sequence[int], domega: Sequence[float], freqs: Sequence[float],
                  spins: Sequence[float], mbh_msun: float, mdot_gs: float) -> np.ndarray:
    """F[k, f] = domega[k] * sum over image k's disk pixels of g^3 B_nu(T_eff(r_c), nu_f / g): the
    observed flux density of the Novikov-Thorne disk (section 4.3), each surface element a
    blackbody at its effective temperature, seen with the redshift g of its pixel (I_nu / nu^3
    invariant), exactly rounded sums. spins[k] is image k's a."""
    r_cross = np.asarray(r_cross, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    hit = np.asarray(hit, dtype=bool)
    nimg = len(offsets) - 1
    F = np.zeros((nimg, len(freqs)))
    for k in range(nimg):
        lo, hi = int(offsets[k]), int(offsets[k + 1])
        sel = np.nonzero(hit[lo:hi])[0] + lo
        T = novikov_thorne_teff(spins[k], r_cross[sel], mbh_msun, mdot_gs)
        for f, nu in enumerate(freqs):
            F[k, f] = float(domega[k]) * math.fsum(g[sel] ** 3 * planck(nu / g[sel], T))
    return F
