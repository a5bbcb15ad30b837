"""Shared test plumbing: one workload dict -> oracle scene and kgrt parameters."""
import math

import numpy as np


def oracle_scene(w, **over):
    import oracle as O
    cam, mod, integ = w["camera"], w["model"], w["integ"]
    kw = dict(a=cam["a"], incl_deg=cam["incl_deg"], phi_obs_deg=cam["phi_obs_deg"], r_obs=cam["r_obs"],
              rtol=integ["rtol"], hmax_frac=integ["hmax_frac"], horizon_delta=integ["horizon_delta"],
              max_steps=integ["max_steps"], model=mod["kind"], stop_at_crossing=bool(integ["flags"] & 1),
              freqs_hz=list(w["freqs"]), t_obs=cam.get("t_obs", 0.0))
    for k in ("r_in", "r_out", "n0_cgs", "r_norm", "n_index", "h_over_r", "T0_K", "T_index", "eps_B",
              "mbh_msun", "r_emit_max", "spot_r", "spot_size", "spot_phi0"):
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


def critical_curve_distance(a, incl_deg, xi, eta, npts=8192):
    """Distance in the plane of sky coordinates at infinity (alpha, beta) from the
    ray's (xi, eta) to the Kerr critical curve (spherical photon orbits).

    The visible part of the photon-orbit radii (beta^2 >= 0) is bracketed by a scan
    and bisection, then sampled with points clustered at its ends, where
    beta ~ sqrt(r - r_end) changes fastest."""
    th = math.radians(incl_deg)
    s, c = math.sin(th), math.cos(th)
    alpha = -np.atleast_1d(np.asarray(xi, dtype=float)) / s
    b2 = np.atleast_1d(np.asarray(eta, dtype=float)) + a * a * c * c - (alpha * s) ** 2 * (c / s) ** 2
    beta = np.sqrt(np.maximum(b2, 0.0))  # distance is symmetric in the sign of beta
    if a < 1e-9:
        return np.abs(np.hypot(alpha, beta) - math.sqrt(27.0))

    def curve(r):
        xc = -(r ** 3 - 3 * r ** 2 + a * a * r + a * a) / (a * (r - 1))
        ec = r ** 3 * (4 * a * a - r * (r - 3) ** 2) / (a * a * (r - 1) ** 2)
        return xc, ec + a * a * c * c - xc ** 2 * (c / s) ** 2

    r1 = 2 * (1 + math.cos(2 / 3 * math.acos(-a)))
    r2 = 2 * (1 + math.cos(2 / 3 * math.acos(a)))
    grid = np.linspace(r1, r2, 20001)
    vis = curve(grid)[1] >= 0
    if not vis.any():
        return np.full(alpha.shape, np.inf)
    i0, i1 = np.argmax(vis), len(vis) - 1 - np.argmax(vis[::-1])

    def edge(lo_in, hi_out):  # bisection for beta^2 = 0 between a visible and an invisible radius
        for _ in range(60):
            mid = 0.5 * (lo_in + hi_out)
            if curve(mid)[1] >= 0:
                lo_in = mid
            else:
                hi_out = mid
        return lo_in

    lo = grid[i0] if i0 == 0 else edge(grid[i0], grid[i0 - 1])
    hi = grid[i1] if i1 == len(grid) - 1 else edge(grid[i1], grid[i1 + 1])
    u = np.linspace(0.0, 1.0, npts)
    rp = lo + (hi - lo) * 0.5 * (1 - np.cos(np.pi * u))
    xc, bc2 = curve(rp)
    ac = -xc / s
    bc = np.sqrt(np.maximum(bc2, 0.0))
    out = np.empty(alpha.shape)
    for k in range(0, len(alpha), 256):
        da = alpha[k:k + 256, None] - ac[None, :]
        db = beta[k:k + 256, None] - bc[None, :]
        out[k:k + 256] = np.sqrt(da * da + db * db).min(axis=1)
    return out
