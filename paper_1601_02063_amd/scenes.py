"""Seeded synthetic workloads (parameters, random draws and synthetic data; no ray tracing or transfer).

Shared by the tests, the benchmark and the CPU reference runs so that both
sides see identical inputs. Values are plain dicts of floats/ints:

  * thin_disk_image  -- a = 0.9, inclination 60 deg, observer at 1000 M,
    64x64 pixels over +-15 M, Keplerian thin disk from the ISCO to 20 M with
    emissivity r^-3, relative tolerance 1e-8, step cap 0.05 r.
  * torus_image      -- a = 0.94, inclination 17 deg, n x n pixels (n = 1024 by
    default) over +-20 M, optically thin thermal-synchrotron torus at 230 GHz,
    step cap 0.02 r.
  * batch_scenes     -- 256 images with sizes drawn from {64, 128, 256, 512}^2,
    spin U[0, 0.998], inclination U[1, 89] deg (drawn in that order per image
    from numpy PCG64(seed)), torus at 8 log-spaced frequencies 86-690 GHz.
  * label_rays       -- (a, incl, x, y) with a ~ U[0, 0.998], incl ~ U[1, 89] deg,
    x, y ~ U[-15, 15] M.
  * projection_image -- the timing workload of the paper's Table 1: a = 0.95,
    inclination 60 deg, first-crossing projection, +-15 M.
  * hot_spot_frames  -- the orbiting hot spot of section 4.4: a = 0, inclination
    60 deg, spot of radius 0.5 M on the ISCO, n x n pixels over +-9 M, frames at
    observer times k dt (by default nframes frames over one orbit at r = 6 M).
  * plasma_grid      -- a GRMHD-like snapshot on a (ln r, theta, phi) grid: the torus
    workload's mean profile with seeded log-normal turbulence and a perturbed
    Keplerian flow (the data the gridded-plasma model samples);
    grid_image -- the torus camera over such a snapshot.
"""
from __future__ import annotations

import numpy as np

R_OBS = 1000.0  # observer distance used throughout the paper's section 2.2

TORUS = dict(kind=2, n0_cgs=1e6, r_norm=2.0, n_index=1.1, h_over_r=0.3, T0_K=1e11, T_index=0.84,
             eps_B=0.1, mbh_msun=4e6, r_emit_max=R_OBS)
THIN_DISK = dict(kind=1, r_in=0.0, r_out=20.0)


def batch_frequencies() -> list:
    """Eight observing frequencies log-spaced from 86 to 690 GHz."""
    return [86e9 * (690.0 / 86.0) ** (k / 7.0) for k in range(8)]


def thin_disk_image(n: int = 64, a: float = 0.9, incl_deg: float = 60.0, half: float = 15.0) -> dict:
    return dict(camera=dict(a=a, incl_deg=incl_deg, nx=n, ny=n, x_min=-half, x_max=half, y_min=-half, y_max=half,
                            r_obs=R_OBS, phi_obs_deg=0.0),
                model=dict(THIN_DISK), freqs=[],
                integ=dict(rtol=1e-8, hmax_frac=0.05, horizon_delta=1e-3, max_steps=100000, flags=0))


def torus_image(n: int = 1024, a: float = 0.94, incl_deg: float = 17.0, half: float = 20.0,
                freqs=(230e9,)) -> dict:
    return dict(camera=dict(a=a, incl_deg=incl_deg, nx=n, ny=n, x_min=-half, x_max=half, y_min=-half, y_max=half,
                            r_obs=R_OBS, phi_obs_deg=0.0),
                model=dict(TORUS), freqs=list(freqs),
                integ=dict(rtol=1e-8, hmax_frac=0.02, horizon_delta=1e-3, max_steps=100000, flags=0))


def projection_image(n: int, a: float = 0.95, incl_deg: float = 60.0, half: float = 15.0) -> dict:
    w = thin_disk_image(n, a, incl_deg, half)
    w["model"] = dict(kind=0, r_in=0.0, r_out=20.0)
    w["integ"]["flags"] = 1  # stop at the first equatorial crossing
    return w


def batch_scenes(seed: int = 1603, nimg: int = 256) -> list:
    rng = np.random.Generator(np.random.PCG64(seed))
    sizes = (64, 128, 256, 512)
    out = []
    for _ in range(nimg):
        n = int(sizes[rng.integers(0, 4)])
        a = float(rng.uniform(0.0, 0.998))
        inc = float(rng.uniform(1.0, 89.0))
        out.append(torus_image(n, a, inc, 20.0, batch_frequencies()))
    return out


def label_rays(n: int, seed: int = 1604) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    rays = np.empty((n, 4))
    rays[:, 0] = rng.uniform(0.0, 0.998, n)
    rays[:, 1] = rng.uniform(1.0, 89.0, n)
    rays[:, 2] = rng.uniform(-15.0, 15.0, n)
    rays[:, 3] = rng.uniform(-15.0, 15.0, n)
    return rays


def sample_pixels(nx: int, ny: int, k: int, seed: int) -> np.ndarray:
    """k distinct pixel indices (j*nx + i) drawn without replacement."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.sort(rng.choice(nx * ny, size=min(k, nx * ny), replace=False))


def render_scenes(seed: int = 1605, nimg: int = 64, n: int = 2048) -> list:
    """Thin-disk images for the surrogate render: (a, incl) drawn per image as for the
    training rays (a ~ U[0, 0.998], incl ~ U[1, 89] deg), n x n pixels over +-15 M."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for _ in range(nimg):
        a = float(rng.uniform(0.0, 0.998))
        inc = float(rng.uniform(1.0, 89.0))
        out.append(thin_disk_image(n, a, inc, 15.0))
    return out


def hot_spot_frames(n: int = 128, nframes: int = 32, a: float = 0.0, incl_deg: float = 60.0, half: float = 9.0,
                    spot_r: float = 0.0, spot_size: float = 0.5, spot_phi0: float = 0.0, dt: float = 0.0) -> list:
    """Frames of the hot spot (model kind 4) at observer times k * dt, k = 0 .. nframes - 1.
    dt <= 0 spreads the frames over 2 pi 6^(3/2) M, one Keplerian orbit at r = 6 M (the ISCO of
    a = 0, the paper's case)."""
    if dt <= 0.0:
        dt = 2.0 * np.pi * 6.0 ** 1.5 / nframes
    out = []
    for k in range(nframes):
        w = thin_disk_image(n, a, incl_deg, half)
        w["camera"]["t_obs"] = k * dt
        w["model"] = dict(kind=4, spot_r=spot_r, spot_size=spot_size, spot_phi0=spot_phi0)
        out.append(w)
    return out


# CGS constants of the snapshot recipe (CODATA 2018): proton mass and speed of light
_MP_CGS, _C_CGS = 1.67262192369e-24, 2.99792458e10


def _random_field(rng, lnr, th, ph, nmodes: int = 12):
    """Unit-variance smooth random field on the grid: a sum of nmodes plane waves in
    (ln r, theta, phi) with radial wavenumbers U[1, 6] per e-folding, integer polar and
    azimuthal wavenumbers (0..6, 0..8; the azimuthal ones keep it periodic) and random phases."""
    f = np.zeros(np.broadcast_shapes(lnr.shape, th.shape, ph.shape))
    for _ in range(nmodes):
        kr = rng.uniform(1.0, 6.0) * (1.0 if rng.uniform() < 0.5 else -1.0)
        lt = int(rng.integers(0, 7))
        mp = int(rng.integers(0, 9))
        psi = rng.uniform(0.0, 2.0 * np.pi)
        f = f + np.cos(kr * lnr + lt * th + mp * ph + psi)
    return f * np.sqrt(2.0 / nmodes)


def plasma_grid(seed: int = 1610, nr: int = 128, nth: int = 64, nph: int = 64, a: float = 0.94,
                r_min: float = 1.0, r_max: float = 1000.0, turbulence: float = 1.0) -> dict:
    """A GRMHD-like plasma snapshot (model kind 5): float32 [nr][nth][nph][4] of
    (ln n_e [cm^-3], ln T_e [K], ln B [G], Omega [1/M]) on the nodes
    ln r_i = ln r_min + i (ln r_max - ln r_min)/(nr - 1), theta_j = j pi/(nth - 1), phi_k = 2 pi k/nph.

    Recipe: the mean state is the torus workload's profile, n_e = 1e6 (r/2)^-1.1
    exp(-cos^2(theta)/(2 0.3^2)) cm^-3, T_e = 1e11 (r/2)^-0.84 K, B^2/(8 pi) = 0.1 n_e m_p c^2/(6 r),
    flowing with Omega = 1/(r^3/2 + a); on top of it seeded log-normal fluctuations,
    ln n_e += 0.6 t G1, ln T_e += 0.3 t G2, ln B += 0.4 t G3, and Omega *= 1 + 0.1 t G4, with G_k
    independent unit-variance smooth random fields (_random_field) and t = turbulence."""
    rng = np.random.Generator(np.random.PCG64(seed))
    lnr = np.linspace(np.log(r_min), np.log(r_max), nr)[:, None, None]
    th = np.linspace(0.0, np.pi, nth)[None, :, None]
    ph = (2.0 * np.pi * np.arange(nph) / nph)[None, None, :]
    r = np.exp(lnr)
    ln_ne = np.log(1e6) - 1.1 * np.log(r / 2.0) - np.cos(th) ** 2 / (2.0 * 0.3 ** 2)
    ln_te = np.log(1e11) - 0.84 * np.log(r / 2.0)
    ln_b = 0.5 * (np.log(8.0 * np.pi * 0.1 * _MP_CGS * _C_CGS ** 2 / 6.0) + ln_ne - np.log(r))
    omega = 1.0 / (r ** 1.5 + a)
    t = float(turbulence)
    cube = np.empty((nr, nth, nph, 4), dtype=np.float32)
    cube[..., 0] = ln_ne + 0.6 * t * _random_field(rng, lnr, th, ph)
    cube[..., 1] = ln_te + 0.3 * t * _random_field(rng, lnr, th, ph)
    cube[..., 2] = ln_b + 0.4 * t * _random_field(rng, lnr, th, ph)
    cube[..., 3] = omega * (1.0 + 0.1 * t * _random_field(rng, lnr, th, ph))
    return dict(grid=cube, grid_r_min=float(r_min), grid_r_max=float(r_max), a=float(a))


def grid_image(n: int = 1024, a: float = 0.94, incl_deg: float = 17.0, half: float = 20.0, freqs=(230e9,),
               seed: int = 1610, grid_shape=(256, 128, 128)) -> dict:
    """The torus camera and integrator over a plasma_grid snapshot of the same spin (model kind 5).
    Returns the workload dict with 'grid' (the float32 cube) and its radial range in 'model'."""
    w = torus_image(n, a, incl_deg, half, freqs)
    pg = plasma_grid(seed, *grid_shape, a=a)
    w["model"] = dict(kind=5, mbh_msun=TORUS["mbh_msun"], grid_r_min=pg["grid_r_min"], grid_r_max=pg["grid_r_max"])
    w["grid"] = pg["grid"]
    return w
