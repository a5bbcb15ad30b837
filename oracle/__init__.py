"""FP64 CPU oracle of the Kerr ray tracer -- TEST INFRASTRUCTURE ONLY.

A plain, slow, obviously-correct reference of the method of Pu, Yun, Younsi &
Yoon (2016, "Odyssey"): rays traced backwards from a flat image plane through
Kerr spacetime with an adaptive fifth-order Runge-Kutta scheme (section 2.1),
initial conditions of section 2.2, radiative transfer of section 2.3, thin
Keplerian disk (section 4.3, also optically thick through every crossing), the
orbiting hot spot (section 4.4), a thermal-synchrotron torus (section 4.5
emissivity, Eqs. (37)-(39)) and the same emissivity from a gridded plasma
snapshot of the kind GRMHD simulations produce (section 6).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package. The GPU library never does, and this
package never imports the GPU library: the two share no code.

The arithmetic lives in ``kerr_oracle.cpp`` (plain C++17, ``double``,
``-ffp-contract=off``); this module is ctypes marshalling plus the pixel-centre
rule of the image plane.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field
from typing import Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "kerr_oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")

# status bits (kerr_oracle.cpp)
CAPTURED, ESCAPED, CROSSED, DISK_HIT = 1, 2, 4, 8
MAXSTEPS, UNDERFLOW, NONFINITE, REFINE_UNCONVERGED, SPOT_HIT = 16, 32, 64, 256, 512

MODEL_GEODESIC, MODEL_THIN_DISK, MODEL_TORUS, MODEL_DISK_IMAGES, MODEL_HOT_SPOT, MODEL_GRID = 0, 1, 2, 3, 4, 5


def build(force: bool = False) -> str:
    """Compile the oracle library with g++ (no FMA contraction, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["g++", "-std=c++17", "-O2", "-ffp-contract=off", "-fno-fast-math",
               "-fPIC", "-shared", "-pthread", "-o", tmp, _SRC]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


class _Scene(ctypes.Structure):
    _fields_ = [
        ("a", ctypes.c_double), ("mass", ctypes.c_double), ("incl_deg", ctypes.c_double),
        ("phi_obs_deg", ctypes.c_double), ("r_obs", ctypes.c_double), ("rtol", ctypes.c_double),
        ("hmax_frac", ctypes.c_double), ("horizon_delta", ctypes.c_double),
        ("max_steps", ctypes.c_int32), ("model", ctypes.c_int32),
        ("stop_at_crossing", ctypes.c_int32), ("nfreq", ctypes.c_int32),
        ("freqs_hz", ctypes.c_double * 16),
        ("r_in", ctypes.c_double), ("r_out", ctypes.c_double),
        ("n0_cgs", ctypes.c_double), ("r_norm", ctypes.c_double), ("n_index", ctypes.c_double),
        ("h_over_r", ctypes.c_double), ("T0_K", ctypes.c_double), ("T_index", ctypes.c_double),
        ("eps_B", ctypes.c_double), ("mbh_msun", ctypes.c_double), ("r_emit_max", ctypes.c_double),
        ("spot_r", ctypes.c_double), ("spot_size", ctypes.c_double), ("spot_phi0", ctypes.c_double),
        ("t_obs", ctypes.c_double),
        ("pr_form", ctypes.c_int32), ("reserved", ctypes.c_int32),
        ("grid", ctypes.c_void_p),
        ("grid_nr", ctypes.c_int32), ("grid_nth", ctypes.c_int32), ("grid_nph", ctypes.c_int32),
        ("grid_reserved", ctypes.c_int32),
        ("grid_r_min", ctypes.c_double), ("grid_r_max", ctypes.c_double),
    ]


RAY_DTYPE = np.dtype([
    ("status", "<i4"), ("steps", "<i4"), ("attempts", "<i4"), ("rhs_evals", "<i4"),
    ("r_cross", "<f8"), ("g", "<f8"), ("phi_cross", "<f8"), ("t_cross", "<f8"),
    ("intensity", "<f8"), ("i_bol", "<f8"),
    ("I", "<f8", (16,)), ("tau", "<f8", (16,)),
    ("final_state", "<f8", (6,)),
    ("E", "<f8"), ("L", "<f8"), ("Q", "<f8"), ("kappa", "<f8"),
    ("max_H_rel", "<f8"), ("max_Q_rel", "<f8"), ("lambda_end", "<f8"), ("min_sin", "<f8"),
    ("n_cross", "<i4"), ("reserved", "<i4"),
])


@dataclass
class Scene:
    """Black hole, observer, emission model and integrator controls (M = 1 units)."""
    a: float = 0.9
    incl_deg: float = 60.0
    phi_obs_deg: float = 0.0
    r_obs: float = 1000.0
    mass: float = 1.0
    rtol: float = 1e-8
    hmax_frac: float = 0.05
    horizon_delta: float = 1e-3
    max_steps: int = 100000
    model: int = MODEL_THIN_DISK
    stop_at_crossing: bool = False
    freqs_hz: Sequence[float] = field(default_factory=list)
    r_in: float = 0.0
    r_out: float = 20.0
    n0_cgs: float = 1e6
    r_norm: float = 2.0
    n_index: float = 1.1
    h_over_r: float = 0.3
    T0_K: float = 1e11
    T_index: float = 0.84
    eps_B: float = 0.1
    mbh_msun: float = 4e6
    r_emit_max: float = 1000.0
    spot_r: float = 0.0      # hot spot orbit radius (<= 0: ISCO)
    spot_size: float = 0.5   # r_spot
    spot_phi0: float = 0.0   # azimuth of the spot centre at t = 0
    t_obs: float = 0.0       # observer time of the image
    pr_form: int = 0   # 0: Eq. (14) before the null condition is substituted; 1: as printed
    # gridded plasma (model 5): float32 [nr][nth][nph][4] of (ln n_e, ln T_e, ln B, Omega) on the
    # nodes ln r_i (uniform from ln grid_r_min to ln grid_r_max), theta_j = j pi/(nth - 1),
    # phi_k = 2 pi k/nph
    grid: np.ndarray | None = None
    grid_r_min: float = 1.0
    grid_r_max: float = 1000.0

    def _c(self) -> _Scene:
        if len(self.freqs_hz) > 16:
            raise ValueError("at most 16 frequencies")
        s = _Scene()
        for name, _ in _Scene._fields_:
            if name in ("freqs_hz", "nfreq", "reserved") or name.startswith("grid"):
                continue
            setattr(s, name, getattr(self, name) if name != "stop_at_crossing" else int(self.stop_at_crossing))
        s.nfreq = len(self.freqs_hz)
        for i, f in enumerate(self.freqs_hz):
            s.freqs_hz[i] = float(f)
        if self.grid is not None:
            g = self.grid
            if g.dtype != np.float32 or not g.flags.c_contiguous or g.ndim != 4 or g.shape[3] != 4:
                raise ValueError("grid must be a C-contiguous float32 array [nr][nth][nph][4]")
            if g.shape[0] < 2 or g.shape[1] < 2 or g.shape[2] < 1:
                raise ValueError("grid needs nr >= 2, nth >= 2, nph >= 1")
            s.grid = g.ctypes.data
            s.grid_nr, s.grid_nth, s.grid_nph = g.shape[:3]
            s.grid_r_min, s.grid_r_max = self.grid_r_min, self.grid_r_max
        elif self.model == MODEL_GRID:
            raise ValueError("the gridded model needs a grid")
        return s


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build())
        L = _lib
        P = ctypes.POINTER
        d, i32, i64, vp = ctypes.c_double, ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p
        L.orc_isco.argtypes, L.orc_isco.restype = [d], d
        L.orc_k2.argtypes, L.orc_k2.restype = [d], d
        L.orc_synchrotron_j.argtypes, L.orc_synchrotron_j.restype = [d, d, d, d], d
        L.orc_redshift.argtypes, L.orc_redshift.restype = [P(_Scene), d, d, d], d
        L.orc_spot_redshift.argtypes, L.orc_spot_redshift.restype = [P(_Scene), d, d, d], d
        L.orc_redshift_omega.argtypes, L.orc_redshift_omega.restype = [P(_Scene), d, d, d, d], d
        L.orc_grid_sample.argtypes, L.orc_grid_sample.restype = [P(_Scene), d, d, d, vp], ctypes.c_int
        L.orc_grid_coeffs.argtypes, L.orc_grid_coeffs.restype = [P(_Scene), d, d, d, d, d, P(d), P(d), P(d)], None
        L.orc_torus_coeffs.argtypes, L.orc_torus_coeffs.restype = [P(_Scene), d, d, d, d, P(d), P(d)], None
        L.orc_rhs.argtypes, L.orc_rhs.restype = [P(_Scene), vp, vp, vp], None
        L.orc_initial_state.argtypes, L.orc_initial_state.restype = [P(_Scene), d, d, vp, vp], ctypes.c_int
        L.orc_trace_ray.argtypes, L.orc_trace_ray.restype = [P(_Scene), d, d, vp], ctypes.c_int
        L.orc_trace_path.argtypes, L.orc_trace_path.restype = [P(_Scene), d, d, vp, vp, i64], i64
        L.orc_trace_points.argtypes, L.orc_trace_points.restype = [P(_Scene), i64, vp, vp, ctypes.c_int], ctypes.c_int
        L.orc_trace_ray_list.argtypes, L.orc_trace_ray_list.restype = [P(_Scene), i64, vp, vp, ctypes.c_int], ctypes.c_int
        assert L.orc_sizeof_scene() == ctypes.sizeof(_Scene), "scene layout mismatch"
        assert L.orc_sizeof_ray() == RAY_DTYPE.itemsize, "ray layout mismatch"
    return _lib


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


def default_threads() -> int:
    return max(1, len(os.sched_getaffinity(0)))


# ------------------------------------------------------------------ API

def pixel_points(nx: int, ny: int, x_min: float, x_max: float, y_min: float, y_max: float) -> np.ndarray:
    """Image-plane coordinates of pixel centres, row-major [j][i] (y rows, x columns).

    reading: cell-centred pixels, x_i = x_min + (i + 1/2)(x_max - x_min)/nx,
    row j has y ascending.
    """
    i = np.arange(nx, dtype=np.float64)
    j = np.arange(ny, dtype=np.float64)
    xs = x_min + (i + 0.5) * (x_max - x_min) / nx
    ys = y_min + (j + 0.5) * (y_max - y_min) / ny
    X, Y = np.meshgrid(xs, ys)
    return np.stack([X.ravel(), Y.ravel()], axis=1)


def trace_points(scene: Scene, xy: np.ndarray, nthreads: int | None = None) -> np.ndarray:
    xy = np.ascontiguousarray(xy, dtype=np.float64).reshape(-1, 2)
    out = np.zeros(len(xy), dtype=RAY_DTYPE)
    s = scene._c()
    lib().orc_trace_points(ctypes.byref(s), len(xy), _ptr(xy), _ptr(out), nthreads or default_threads())
    return out


def trace_image(scene: Scene, nx: int, ny: int, x_min: float, x_max: float, y_min: float, y_max: float,
                nthreads: int | None = None) -> np.ndarray:
    return trace_points(scene, pixel_points(nx, ny, x_min, x_max, y_min, y_max), nthreads).reshape(ny, nx)


def trace_ray_list(scene: Scene, rays4: np.ndarray, nthreads: int | None = None) -> np.ndarray:
    """rays4: (n, 4) of (a, incl_deg, x, y); other parameters from ``scene``."""
    rays4 = np.ascontiguousarray(rays4, dtype=np.float64).reshape(-1, 4)
    out = np.zeros(len(rays4), dtype=RAY_DTYPE)
    s = scene._c()
    lib().orc_trace_ray_list(ctypes.byref(s), len(rays4), _ptr(rays4), _ptr(out), nthreads or default_threads())
    return out


def trace_ray(scene: Scene, x: float, y: float) -> np.ndarray:
    out = np.zeros(1, dtype=RAY_DTYPE)
    s = scene._c()
    lib().orc_trace_ray(ctypes.byref(s), x, y, _ptr(out))
    return out[0]


def trace_path(scene: Scene, x: float, y: float, cap: int = 200000):
    """Trace one ray and return (result, path) with path rows (lambda, r, th, ph, t, p_r, p_th)."""
    out = np.zeros(1, dtype=RAY_DTYPE)
    path = np.zeros((cap, 7), dtype=np.float64)
    s = scene._c()
    n = lib().orc_trace_path(ctypes.byref(s), x, y, _ptr(out), _ptr(path), cap)
    return out[0], path[:n].copy()


def initial_state(scene: Scene, x: float, y: float):
    """Returns (ok, y6, (E, L, Q, kappa)) for the ray through image-plane point (x, y)."""
    y6 = np.zeros(6)
    c4 = np.zeros(4)
    s = scene._c()
    rc = lib().orc_initial_state(ctypes.byref(s), x, y, _ptr(y6), _ptr(c4))
    return rc == 0, y6, c4


def rhs(scene: Scene, y6, c4) -> np.ndarray:
    y6 = np.ascontiguousarray(y6, dtype=np.float64)
    c4 = np.ascontiguousarray(c4, dtype=np.float64)
    dy = np.zeros(6)
    s = scene._c()
    lib().orc_rhs(ctypes.byref(s), _ptr(y6), _ptr(c4), _ptr(dy))
    return dy


def isco(a: float) -> float:
    return lib().orc_isco(a)


def k2(x: float) -> float:
    return lib().orc_k2(x)


def synchrotron_j(nu: float, ne: float, Te: float, B: float) -> float:
    return lib().orc_synchrotron_j(nu, ne, Te, B)


def redshift(scene: Scene, r: float, th: float, xi: float) -> float:
    s = scene._c()
    return lib().orc_redshift(ctypes.byref(s), r, th, xi)


def torus_coeffs(scene: Scene, r: float, th: float, g: float, nu: float):
    s = scene._c()
    a = ctypes.c_double()
    e = ctypes.c_double()
    lib().orc_torus_coeffs(ctypes.byref(s), r, th, g, nu, ctypes.byref(a), ctypes.byref(e))
    return a.value, e.value


def spot_redshift(scene: Scene, r: float, th: float, xi: float) -> float:
    s = scene._c()
    return lib().orc_spot_redshift(ctypes.byref(s), r, th, xi)


def redshift_omega(scene: Scene, r: float, th: float, xi: float, omega: float) -> float:
    s = scene._c()
    return lib().orc_redshift_omega(ctypes.byref(s), r, th, xi, omega)


def grid_sample(scene: Scene, r: float, th: float, ph: float):
    """(inside, [ln n_e, ln T_e, ln B, Omega]) of the gridded plasma at (r, theta, phi)."""
    v = np.zeros(4)
    s = scene._c()
    ok = lib().orc_grid_sample(ctypes.byref(s), r, th, ph, _ptr(v))
    return bool(ok), v


def grid_coeffs(scene: Scene, r: float, th: float, ph: float, xi: float, nu: float):
    """(a_lambda, e_lambda, g) of the gridded plasma for a ray with xi = L/E at frequency nu."""
    s = scene._c()
    a, e, g = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    lib().orc_grid_coeffs(ctypes.byref(s), r, th, ph, xi, nu, ctypes.byref(a), ctypes.byref(e), ctypes.byref(g))
    return a.value, e.value, g.value
