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
