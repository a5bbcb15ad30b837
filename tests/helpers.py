"""Shared test plumbing: one workload dict -> oracle scene and kgrt parameters."""
import math

import numpy as np


def oracle_scene(w, **over):
    import oracle as O
    cam, mod, integ = w["camera"], w["model"], w["integ"]
    kw = dict(a=cam["a"], incl_deg=cam["incl_deg"], phi_obs_deg=cam["phi_obs_deg"], r_obs=cam["r_obs"],
              rtol=integ["rtol"], hmax_frac=integ["hmax_frac"], horizon_delta=integ["horizon_delta"],
              max_steps=integ["max_steps"], model=mod["kind"], stop_at_crossing=bool(integ["flags"] & 1),
              freqs_hz=list(w["freqs"]))
    for k in ("r_in", "r_out", "n0_cgs", "r_norm", "n_index", "h_over_r", "T0_K", "T_index", "eps_B",
              "mbh_msun", "r_emit_max"):
        if k in mod:
            kw[k] = mod[k]
    kw.update(over)
    return O.Scene(**kw)


def kgrt_params(w):
    from paper_1601_02063_amd import kgrt as K
    cam = K.Camera(**w["camera"])
    mod = K.Model(**w["model"])
    integ = K.Integrator(**w["integ"])
    return cam, mod, list(w["freqs"]), integ


def pixel_xy(cam, idx):
    """Image-plane coordinates of pixel indices (j*nx + i), cell-centred."""
    idx = np.asarray(idx)
    i, j = idx % cam["nx"], idx // cam["nx"]
    x = cam["x_min"] + ((i + 0.5) * (cam["x_max"] - cam["x_min"])) / cam["nx"]
    y = cam["y_min"] + ((j + 0.5) * (cam["y_max"] - cam["y_min"])) / cam["ny"]
    return np.stack([x, y], axis=1)


def critical_curve_distance(a, incl_deg, xi, eta, npts=4096):
    """Distance in the plane of sky coordinates at infinity (alpha, beta) from the
    ray's (xi, eta) to the Kerr critical curve (spherical photon orbits)."""
    th = math.radians(incl_deg)
    s, c = math.sin(th), math.cos(th)
    alpha = -np.asarray(xi) / s
    b2 = np.asarray(eta) + a * a * c * c - np.asarray(xi) ** 2 * (c / s) ** 2
    beta = np.sqrt(np.maximum(b2, 0.0))  # distance is symmetric in the sign of beta
    if a < 1e-9:
        return np.abs(np.hypot(alpha, beta) - math.sqrt(27.0))
    rp_lo = 2 * (1 + math.cos(2 / 3 * math.acos(-a)))
    rp_hi = 2 * (1 + math.cos(2 / 3 * math.acos(a)))
    rp = np.linspace(rp_lo, rp_hi, npts)
    xc = -(rp ** 3 - 3 * rp ** 2 + a * a * rp + a * a) / (a * (rp - 1))
    ec = rp ** 3 * (4 * a * a - rp * (rp - 3) ** 2) / (a * a * (rp - 1) ** 2)
    bc2 = ec + a * a * c * c - xc ** 2 * (c / s) ** 2
    ok = bc2 >= 0
    ac = -xc[ok] / s
    bc = np.sqrt(bc2[ok])
    d = np.sqrt((alpha[:, None] - ac[None, :]) ** 2 + (beta[:, None] - bc[None, :]) ** 2)
    return d.min(axis=1)
