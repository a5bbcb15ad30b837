"""Python binding of the kgrt C ABI (include/kgrt.h): argument marshalling only.

PyTorch provides device memory (output tensors) and streams; every step of the
ray tracing runs in the HIP kernels of ``libkgrt.so``. There is no fallback:
if the library is missing or no GPU is usable, calls raise.
"""
from __future__ import annotations

import ctypes
import os
import weakref
from dataclasses import dataclass, field, fields
from typing import Dict, Iterable, Optional, Sequence

import torch  # loads the HIP runtime first, so libkgrt.so binds to the same one

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libkgrt.so")
HEADER_PATH = os.path.join(os.path.dirname(_HERE), "include", "kgrt.h")

OK, E_INVALID_ARG, E_HIP, E_NOMEM, E_NO_DEVICE, E_UNSUPPORTED = 0, -1, -2, -3, -4, -5
CAPTURED, ESCAPED, CROSSED, DISK_HIT = 1, 2, 4, 8
MAXSTEPS, UNDERFLOW, NONFINITE, FALLBACK, REFINE_UNCONVERGED, SPOT_HIT = 16, 32, 64, 128, 256, 512
MODEL_GEODESIC, MODEL_THIN_DISK, MODEL_TORUS, MODEL_DISK_IMAGES, MODEL_HOT_SPOT, MODEL_GRID = 0, 1, 2, 3, 4, 5
# models whose outputs carry the transfer: intensity and tau are [nfreq][n]
TRANSFER_MODELS = (MODEL_TORUS, MODEL_GRID)
NOALLOC_MAX_RAYS = 262144  # KGRT_NOALLOC_MAX_RAYS
STOP_AT_CROSSING = 1


class KgrtError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"kgrt error {code}: {msg}")
        self.code = code


class CCamera(ctypes.Structure):
    _fields_ = [("a", ctypes.c_double), ("incl_deg", ctypes.c_double), ("phi_obs_deg", ctypes.c_double),
                ("r_obs", ctypes.c_double), ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("x_min", ctypes.c_double), ("x_max", ctypes.c_double),
                ("y_min", ctypes.c_double), ("y_max", ctypes.c_double), ("t_obs", ctypes.c_double)]


class CModel(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("r_in", ctypes.c_double), ("r_out", ctypes.c_double),
                ("n0_cgs", ctypes.c_double), ("r_norm", ctypes.c_double), ("n_index", ctypes.c_double),
                ("h_over_r", ctypes.c_double), ("T0_K", ctypes.c_double), ("T_index", ctypes.c_double),
                ("eps_B", ctypes.c_double), ("mbh_msun", ctypes.c_double), ("r_emit_max", ctypes.c_double),
                ("spot_r", ctypes.c_double), ("spot_size", ctypes.c_double), ("spot_phi0", ctypes.c_double),
                ("grid_dev", ctypes.c_void_p), ("grid_nr", ctypes.c_int32), ("grid_nth", ctypes.c_int32),
                ("grid_nph", ctypes.c_int32), ("grid_reserved", ctypes.c_int32),
                ("grid_r_min", ctypes.c_double), ("grid_r_max", ctypes.c_double)]


class CIntegrator(ctypes.Structure):
    _fields_ = [("rtol", ctypes.c_double), ("hmax_frac", ctypes.c_double), ("horizon_delta", ctypes.c_double),
                ("max_steps", ctypes.c_int32), ("flags", ctypes.c_uint32)]


OUTPUT_FIELDS = ("status", "steps", "attempts", "r_cross", "g", "phi_cross", "t_cross", "intensity", "i_bol", "tau",
                 "n_cross")
INT_FIELDS = ("status", "steps", "attempts", "n_cross")


class COutputs(ctypes.Structure):
    _fields_ = [(n, ctypes.c_void_p) for n in OUTPUT_FIELDS]


class CLaunch(ctypes.Structure):
    _fields_ = [("block", ctypes.c_int32), ("blocks_per_cu", ctypes.c_int32),
                ("refill_min", ctypes.c_int32), ("mode", ctypes.c_int32)]

    def as_dict(self):
        return {"block": self.block, "blocks_per_cu": self.blocks_per_cu, "refill_min": self.refill_min,
                "mode": self.mode}


class CKernelInfo(ctypes.Structure):
    _fields_ = [("vgprs", ctypes.c_int32), ("scratch_bytes", ctypes.c_int32), ("blocks_per_cu", ctypes.c_int32),
                ("waves_per_simd", ctypes.c_int32)]


class CAdam(ctypes.Structure):
    _fields_ = [("lr", ctypes.c_float), ("beta1", ctypes.c_float), ("beta2", ctypes.c_float), ("eps", ctypes.c_float)]


class CFallback(ctypes.Structure):
    _fields_ = [("p_lo", ctypes.c_float), ("p_hi", ctypes.c_float), ("crit_band", ctypes.c_float),
                ("edge_band", ctypes.c_float), ("g_tol", ctypes.c_float), ("grad_max", ctypes.c_float)]


LAUNCH_PERSISTENT, LAUNCH_ONE_RAY_PER_THREAD = 0, 1
PLAN_GRAPH = 1


# ---------------------------------------------------------------- parameters

@dataclass
class Camera:
    a: float = 0.9
    incl_deg: float = 60.0
    nx: int = 64
    ny: int = 64
    x_min: float = -15.0
    x_max: float = 15.0
    y_min: float = -15.0
    y_max: float = 15.0
    r_obs: float = 1000.0
    phi_obs_deg: float = 0.0
    t_obs: float = 0.0

    def c(self) -> CCamera:
        return CCamera(self.a, self.incl_deg, self.phi_obs_deg, self.r_obs, self.nx, self.ny,
                       self.x_min, self.x_max, self.y_min, self.y_max, self.t_obs)


@dataclass
class Model:
    kind: int = MODEL_THIN_DISK
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
    spot_r: float = 0.0       # hot spot orbit radius (<= 0: ISCO)
    spot_size: float = 0.5    # r_spot
    spot_phi0: float = 0.0    # azimuth of the spot centre at t = 0 (radians)
    # gridded plasma (MODEL_GRID): a contiguous CUDA float32 tensor [nr, nth, nph, 4] of
    # (ln n_e, ln T_e, ln B, Omega) on the (ln r, theta, phi) nodes, and its radial range
    grid: Optional[torch.Tensor] = None
    grid_r_min: float = 1.0
    grid_r_max: float = 1000.0

    def c(self) -> CModel:
        ptr, dims = None, (0, 0, 0)
        if self.grid is not None:
            g = self.grid
            if not (g.is_cuda and g.dtype == torch.float32 and g.is_contiguous() and g.dim() == 4 and g.shape[3] == 4):
                raise ValueError("grid must be a contiguous CUDA float32 tensor [nr, nth, nph, 4]")
            ptr, dims = g.data_ptr(), tuple(int(v) for v in g.shape[:3])
        return CModel(self.kind, 0, self.r_in, self.r_out, self.n0_cgs, self.r_norm, self.n_index, self.h_over_r,
                      self.T0_K, self.T_index, self.eps_B, self.mbh_msun, self.r_emit_max, self.spot_r,
                      self.spot_size, self.spot_phi0, ptr, dims[0], dims[1], dims[2], 0,
                      self.grid_r_min, self.grid_r_max)


@dataclass
class Integrator:
    rtol: float = 1e-8
    hmax_frac: float = 0.05
    horizon_delta: float = 1e-3
    max_steps: int = 100000
    flags: int = 0

    def c(self) -> CIntegrator:
        return CIntegrator(self.rtol, self.hmax_frac, self.horizon_delta, self.max_steps, self.flags)


# ---------------------------------------------------------------- library

_lib = None


def lib() -> ctypes.CDLL:
    """Loads libkgrt.so (built by ``paper_1601_02063_amd.build``); raises if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1601_02063_amd.build` "
                               "(there is no CPU fallback)")
        L = ctypes.CDLL(LIB_PATH)
        P, vp, i32, i64, d = ctypes.POINTER, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        L.kgrt_ctx_create.argtypes, L.kgrt_ctx_create.restype = [ctypes.c_int, P(vp)], ctypes.c_int
        L.kgrt_ctx_destroy.argtypes, L.kgrt_ctx_destroy.restype = [vp], ctypes.c_int
        L.kgrt_ctx_set_launch.argtypes, L.kgrt_ctx_set_launch.restype = [vp, P(CLaunch)], ctypes.c_int
        L.kgrt_ctx_num_cus.argtypes, L.kgrt_ctx_num_cus.restype = [vp], ctypes.c_int
        L.kgrt_kernel_info_get.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                           ctypes.POINTER(CKernelInfo)]
        L.kgrt_kernel_info_get.restype = ctypes.c_int
        L.kgrt_check_args.argtypes = [P(CCamera), P(CModel), P(d), i32, P(CIntegrator)]
        L.kgrt_check_args.restype = ctypes.c_int
        L.kgrt_trace.argtypes = [vp, P(CCamera), P(CModel), P(d), i32, P(CIntegrator), P(COutputs), vp]
        L.kgrt_trace.restype = ctypes.c_int
        L.kgrt_trace_noalloc.argtypes = [vp, P(CCamera), P(CModel), P(d), i32, P(CIntegrator), P(COutputs), vp]
        L.kgrt_trace_noalloc.restype = ctypes.c_int
        L.kgrt_trace_rays.argtypes = [vp, vp, i64, d, d, P(CModel), P(d), i32, P(CIntegrator), P(COutputs), vp]
        L.kgrt_trace_rays.restype = ctypes.c_int
        L.kgrt_plan_create.argtypes = [vp, vp, i32, P(CModel), P(d), i32, P(CIntegrator), P(vp)]
        L.kgrt_plan_create.restype = ctypes.c_int
        L.kgrt_plan_num_rays.argtypes, L.kgrt_plan_num_rays.restype = [vp], i64
        L.kgrt_plan_launch.argtypes, L.kgrt_plan_launch.restype = [vp, P(COutputs), ctypes.c_uint32, vp], ctypes.c_int
        L.kgrt_plan_autotune.argtypes, L.kgrt_plan_autotune.restype = [vp, P(COutputs), vp, P(CLaunch)], ctypes.c_int
        L.kgrt_plan_set_launch.argtypes, L.kgrt_plan_set_launch.restype = [vp, P(CLaunch)], ctypes.c_int
        L.kgrt_plan_destroy.argtypes, L.kgrt_plan_destroy.restype = [vp], ctypes.c_int
        L.kgrt_trace_batch.argtypes = [vp, vp, i32, P(CModel), P(d), i32, P(CIntegrator), P(COutputs), vp]
        L.kgrt_trace_batch.restype = ctypes.c_int
        fp = P(ctypes.c_float)
        L.kgrt_mlp_num_params.argtypes, L.kgrt_mlp_num_params.restype = [], i64
        L.kgrt_mlp_create.argtypes, L.kgrt_mlp_create.restype = [vp, i64, P(vp)], ctypes.c_int
        L.kgrt_mlp_destroy.argtypes, L.kgrt_mlp_destroy.restype = [vp], ctypes.c_int
        L.kgrt_mlp_last_error.argtypes, L.kgrt_mlp_last_error.restype = [vp], ctypes.c_char_p
        L.kgrt_mlp_set_params.argtypes, L.kgrt_mlp_set_params.restype = [vp, vp, i64], ctypes.c_int
        L.kgrt_mlp_get_params.argtypes, L.kgrt_mlp_get_params.restype = [vp, vp, i64], ctypes.c_int
        L.kgrt_mlp_get_adam.argtypes, L.kgrt_mlp_get_adam.restype = [vp, vp, vp, i64, vp], ctypes.c_int
        L.kgrt_mlp_set_adam.argtypes, L.kgrt_mlp_set_adam.restype = [vp, vp, vp, i64, i64], ctypes.c_int
        L.kgrt_mlp_forward.argtypes, L.kgrt_mlp_forward.restype = [vp, vp, vp, i64, vp], ctypes.c_int
        L.kgrt_mlp_loss_grads.argtypes = [vp, vp, vp, vp, i64, vp, vp, vp]
        L.kgrt_mlp_loss_grads.restype = ctypes.c_int
        L.kgrt_mlp_train_step.argtypes = [vp, vp, vp, vp, i64, P(CAdam), vp, vp]
        L.kgrt_mlp_train_step.restype = ctypes.c_int
        L.kgrt_surrogate_features.argtypes, L.kgrt_surrogate_features.restype = [vp, i64, vp, vp], ctypes.c_int
        L.kgrt_surrogate_targets.argtypes = [vp, vp, vp, vp, vp, i64, vp, vp]
        L.kgrt_surrogate_targets.restype = ctypes.c_int
        L.kgrt_surrogate_render.argtypes = [vp, vp, vp, i32, P(CModel), P(CIntegrator), P(CFallback), vp, vp, vp,
                                            vp, vp]
        L.kgrt_surrogate_render.restype = ctypes.c_int
        L.kgrt_trace_rays_dev.argtypes = [vp, vp, vp, i64, d, d, P(CModel), P(d), i32, P(CIntegrator), P(COutputs),
                                          vp]
        L.kgrt_trace_rays_dev.restype = ctypes.c_int
        L.kgrt_critical_curve.argtypes, L.kgrt_critical_curve.restype = [d, d, vp, i32], ctypes.c_int
        L.kgrt_image_spectra.argtypes = [vp, i64, i32, vp, vp, i32, vp, vp]
        L.kgrt_image_spectra.restype = ctypes.c_int
        L.kgrt_pixel_solid_angle.argtypes, L.kgrt_pixel_solid_angle.restype = [P(CCamera), d, d], d
        L.kgrt_spot_spectrogram.argtypes = [vp, vp, i64, vp, vp, i32, P(d), i32, vp, vp]
        L.kgrt_spot_spectrogram.restype = ctypes.c_int
        L.kgrt_disk_spectrum.argtypes = [vp, vp, vp, i64, vp, vp, vp, i32, d, d, P(d), i32, vp, vp]
        L.kgrt_disk_spectrum.restype = ctypes.c_int
        L.kgrt_strerror.argtypes, L.kgrt_strerror.restype = [ctypes.c_int], ctypes.c_char_p
        L.kgrt_last_error.argtypes, L.kgrt_last_error.restype = [vp], ctypes.c_char_p
        L.kgrt_version.argtypes, L.kgrt_version.restype = [], ctypes.c_int
        _lib = L
    return _lib


def _freqs(freqs: Sequence[float]):
    arr = (ctypes.c_double * max(1, len(freqs)))(*[float(f) for f in freqs])
    return arr, len(freqs)


def check_args(camera: Optional[Camera], model: Model, freqs: Sequence[float], integ: Integrator) -> int:
    """Host-side validation only (no GPU needed): returns the kgrt code."""
    fa, nf = _freqs(freqs)
    cam = ctypes.byref(camera.c()) if camera is not None else None
    return lib().kgrt_check_args(cam, ctypes.byref(model.c()), fa, nf, ctypes.byref(integ.c()))


def _stream_handle(stream) -> Optional[int]:
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


def _ptr(t: Optional[torch.Tensor], dtype: torch.dtype, n: int, device: torch.device) -> Optional[int]:
    if t is None:
        return None
    if not t.is_cuda or t.device != device:
        raise ValueError("output tensors must live on the context's GPU")
    if t.dtype != dtype or not t.is_contiguous() or t.numel() < n:
        raise ValueError(f"output tensor must be contiguous {dtype} with >= {n} elements")
    return t.data_ptr()


class Context:
    """A kgrt context on one GPU (owns the work-queue counter)."""

    def __init__(self, device: int = 0):
        self.device = torch.device("cuda", device)
        h = ctypes.c_void_p()
        rc = lib().kgrt_ctx_create(device, ctypes.byref(h))
        if rc != OK:
            raise KgrtError(rc, lib().kgrt_strerror(rc).decode())
        self._h = h
        self._plans = weakref.WeakSet()  # plans keep a pointer to this context: closed first

    def close(self):
        if getattr(self, "_h", None):
            for p in list(self._plans):
                p.close()
            lib().kgrt_ctx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc: int):
        if rc != OK:
            raise KgrtError(rc, lib().kgrt_last_error(self._h).decode())

    @property
    def num_cus(self) -> int:
        return lib().kgrt_ctx_num_cus(self._h)

    def kernel_info(self, model: int, nfreq: int = 1, block: int = 0) -> dict:
        """kgrt_kernel_info_get: VGPRs, scratch bytes per lane, blocks per CU and waves per SIMD of the
        integrator kernel for this model and number of frequencies."""
        info = CKernelInfo()
        self._check(lib().kgrt_kernel_info_get(self._h, model, nfreq, block, ctypes.byref(info)))
        return {"vgprs": info.vgprs, "scratch_bytes": info.scratch_bytes, "blocks_per_cu": info.blocks_per_cu,
                "waves_per_simd": info.waves_per_simd}

    def set_launch(self, block: int = 0, blocks_per_cu: int = 0, refill_min: int = 0, mode: int = 0):
        self._check(lib().kgrt_ctx_set_launch(self._h, ctypes.byref(CLaunch(block, blocks_per_cu, refill_min, mode))))

    def _outputs(self, outs: Dict[str, torch.Tensor], n: int, nf: int, model: Model) -> COutputs:
        o = COutputs()
        for name in OUTPUT_FIELDS:
            t = outs.get(name)
            if name in INT_FIELDS:
                setattr(o, name, _ptr(t, torch.int32, n, self.device))
            else:
                per = n * nf if (model.kind in TRANSFER_MODELS and name in ("intensity", "tau")) else n
                setattr(o, name, _ptr(t, torch.float64, per, self.device))
        return o

    def trace(self, camera: Camera, model: Model, freqs: Sequence[float], integ: Integrator,
              outs: Dict[str, torch.Tensor], stream=None):
        """kgrt_trace on caller-owned output tensors (see include/kgrt.h for layouts)."""
        n = camera.nx * camera.ny
        fa, nf = _freqs(freqs)
        o = self._outputs(outs, n, max(nf, 1), model)
        self._check(lib().kgrt_trace(self._h, ctypes.byref(camera.c()), ctypes.byref(model.c()), fa, nf,
                                     ctypes.byref(integ.c()), ctypes.byref(o), _stream_handle(stream)))

    def trace_noalloc(self, camera: Camera, model: Model, freqs: Sequence[float], integ: Integrator,
                      outs: Dict[str, torch.Tensor], stream=None):
        """kgrt_trace_noalloc: as trace, with the library's static scratch (no device allocation;
        at most NOALLOC_MAX_RAYS rays; calls overlapping on one device race)."""
        n = camera.nx * camera.ny
        fa, nf = _freqs(freqs)
        o = self._outputs(outs, n, max(nf, 1), model)
        self._check(lib().kgrt_trace_noalloc(self._h, ctypes.byref(camera.c()), ctypes.byref(model.c()), fa, nf,
                                             ctypes.byref(integ.c()), ctypes.byref(o), _stream_handle(stream)))

    def trace_rays(self, rays: torch.Tensor, model: Model, freqs: Sequence[float], integ: Integrator,
                   outs: Dict[str, torch.Tensor], r_obs: float = 1000.0, phi_obs_deg: float = 0.0, stream=None):
        """kgrt_trace_rays: rays is a contiguous float64 [n, 4] tensor of (a, incl_deg, x, y)."""
        if rays.dtype != torch.float64 or not rays.is_contiguous() or rays.dim() != 2 or rays.shape[1] != 4:
            raise ValueError("rays must be a contiguous float64 tensor of shape [n, 4]")
        if rays.device != self.device:
            raise ValueError("rays must live on the context's GPU")
        n = rays.shape[0]
        fa, nf = _freqs(freqs)
        o = self._outputs(outs, n, max(nf, 1), model)
        self._check(lib().kgrt_trace_rays(self._h, rays.data_ptr() if n else None, n, r_obs, phi_obs_deg,
                                          ctypes.byref(model.c()), fa, nf, ctypes.byref(integ.c()),
                                          ctypes.byref(o), _stream_handle(stream)))


    def trace_batch(self, cameras: Sequence[Camera], model: Model, freqs: Sequence[float], integ: Integrator,
                    outs: Dict[str, torch.Tensor], stream=None):
        """kgrt_trace_batch: images concatenated in order; waits for the stream."""
        cams = (CCamera * len(cameras))(*[c.c() for c in cameras])
        n = sum(c.nx * c.ny for c in cameras)
        fa, nf = _freqs(freqs)
        o = self._outputs(outs, n, max(nf, 1), model)
        self._check(lib().kgrt_trace_batch(self._h, cams, len(cameras), ctypes.byref(model.c()), fa, nf,
                                           ctypes.byref(integ.c()), ctypes.byref(o), _stream_handle(stream)))


class Plan:
    """kgrt_plan: many images of uneven size, spin and inclination in one persistent launch."""

    def __init__(self, ctx: Context, cameras: Sequence[Camera], model: Model, freqs: Sequence[float],
                 integ: Integrator):
        self.ctx, self.model, self.freqs = ctx, model, list(freqs)
        cams = (CCamera * len(cameras))(*[c.c() for c in cameras])
        fa, nf = _freqs(freqs)
        h = ctypes.c_void_p()
        ctx._check(lib().kgrt_plan_create(ctx._h, cams, len(cameras), ctypes.byref(model.c()), fa, nf,
                                          ctypes.byref(integ.c()), ctypes.byref(h)))
        self._h = h
        ctx._plans.add(self)
        sizes = [c.nx * c.ny for c in cameras]
        self.offsets = [0]
        for n in sizes:
            self.offsets.append(self.offsets[-1] + n)
        self.num_rays = int(lib().kgrt_plan_num_rays(h))
        assert self.num_rays == self.offsets[-1]

    def close(self):
        if getattr(self, "_h", None):
            lib().kgrt_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def alloc_outputs(self, names: Iterable[str] = OUTPUT_FIELDS):
        return alloc_outputs(self.num_rays, self.model, len(self.freqs), self.ctx.device, names)

    def launch(self, outs: Dict[str, torch.Tensor], graph: bool = False, stream=None):
        o = self.ctx._outputs(outs, self.num_rays, max(len(self.freqs), 1), self.model)
        self._keep = o
        self.ctx._check(lib().kgrt_plan_launch(self._h, ctypes.byref(o), PLAN_GRAPH if graph else 0,
                                               _stream_handle(stream)))

    def autotune(self, outs: Dict[str, torch.Tensor], stream=None) -> dict:
        o = self.ctx._outputs(outs, self.num_rays, max(len(self.freqs), 1), self.model)
        best = CLaunch()
        self.ctx._check(lib().kgrt_plan_autotune(self._h, ctypes.byref(o), _stream_handle(stream),
                                                 ctypes.byref(best)))
        return best.as_dict()

    def set_launch(self, block: int = 0, blocks_per_cu: int = 0, refill_min: int = 0, mode: int = 0):
        self.ctx._check(lib().kgrt_plan_set_launch(self._h, ctypes.byref(CLaunch(block, blocks_per_cu,
                                                                                 refill_min, mode))))

    def spectra(self, intensity: torch.Tensor, domega: torch.Tensor, stream=None) -> torch.Tensor:
        """kgrt_image_spectra over this plan's images: flux density [nimg, nfreq] (float64, device)."""
        if getattr(self, "_offsets_dev", None) is None:
            self._offsets_dev = torch.tensor(self.offsets, dtype=torch.int64, device=self.ctx.device)
        return image_spectra(intensity, self._offsets_dev, domega, stream)


def image_spectra(intensity: torch.Tensor, offsets: torch.Tensor, domega: torch.Tensor,
                  stream=None) -> torch.Tensor:
    """kgrt_image_spectra: flux[k, f] = domega[k] * sum of intensity[f, offsets[k]:offsets[k+1]].

    intensity: contiguous CUDA float64 [nfreq, total] (or [total] for one frequency); offsets:
    contiguous CUDA int64 [nimg + 1]; domega: contiguous CUDA float64 [nimg]. Returns a new
    CUDA float64 tensor [nimg, nfreq] written on `stream` (asynchronously)."""
    I = intensity.unsqueeze(0) if intensity.dim() == 1 else intensity
    if not (I.is_cuda and I.dtype == torch.float64 and I.is_contiguous() and I.dim() == 2):
        raise ValueError("intensity must be a contiguous CUDA float64 tensor [nfreq, total]")
    for t, dt, nm in ((offsets, torch.int64, "offsets"), (domega, torch.float64, "domega")):
        if not (t.is_cuda and t.dtype == dt and t.is_contiguous() and t.dim() == 1):
            raise ValueError(f"{nm} must be a contiguous 1-D CUDA {dt} tensor")
    nimg = domega.shape[0]
    if offsets.shape[0] != nimg + 1:
        raise ValueError("offsets must have nimg + 1 entries")
    nfreq, total = I.shape
    flux = torch.empty((nimg, nfreq), dtype=torch.float64, device=I.device)
    rc = lib().kgrt_image_spectra(I.data_ptr() if total else None, total, nfreq, offsets.data_ptr(),
                                  domega.data_ptr(), nimg, flux.data_ptr(), _stream_handle(stream))
    if rc != OK:
        raise KgrtError(rc, "kgrt_image_spectra failed")
    return flux


def spot_spectrogram(i_bol: torch.Tensor, g: torch.Tensor, offsets: torch.Tensor, domega: torch.Tensor,
                     g_edges: Sequence[float], stream=None) -> torch.Tensor:
    """kgrt_spot_spectrogram: out[k, b] = domega[k] * sum of i_bol over image k's rays with
    g_edges[b] <= g < g_edges[b + 1]. i_bol, g: contiguous CUDA float64 [total]; offsets: CUDA
    int64 [nimg + 1]; domega: CUDA float64 [nimg]; g_edges: host sequence of nbins + 1 edges."""
    for t, dt, nm in ((i_bol, torch.float64, "i_bol"), (g, torch.float64, "g"), (offsets, torch.int64, "offsets"),
                      (domega, torch.float64, "domega")):
        if not (t.is_cuda and t.dtype == dt and t.is_contiguous() and t.dim() == 1):
            raise ValueError(f"{nm} must be a contiguous 1-D CUDA {dt} tensor")
    if i_bol.shape != g.shape:
        raise ValueError("i_bol and g must have the same length")
    nimg = domega.shape[0]
    if offsets.shape[0] != nimg + 1:
        raise ValueError("offsets must have nimg + 1 entries")
    nbins = len(g_edges) - 1
    edges = (ctypes.c_double * max(1, nbins + 1))(*[float(e) for e in g_edges])
    out = torch.empty((nimg, max(nbins, 0)), dtype=torch.float64, device=g.device)
    total = g.shape[0]
    rc = lib().kgrt_spot_spectrogram(i_bol.data_ptr() if total else None, g.data_ptr() if total else None, total,
                                     offsets.data_ptr(), domega.data_ptr(), nimg, edges, nbins, out.data_ptr(),
                                     _stream_handle(stream))
    if rc != OK:
        raise KgrtError(rc, "kgrt_spot_spectrogram failed")
    return out


def disk_spectrum(r_cross: torch.Tensor, g: torch.Tensor, status: torch.Tensor, offsets: torch.Tensor,
                  domega: torch.Tensor, spin: torch.Tensor, mbh_msun: float, mdot_gs: float,
                  freqs: Sequence[float], stream=None) -> torch.Tensor:
    """kgrt_disk_spectrum: the Novikov-Thorne disk's flux density [nimg, nfreq] from traced images
    (r_cross, g float64 and status int32 [total]; offsets int64 [nimg + 1]; domega, spin float64
    [nimg]; all contiguous CUDA tensors)."""
    for t, dt, nm in ((r_cross, torch.float64, "r_cross"), (g, torch.float64, "g"), (status, torch.int32, "status"),
                      (offsets, torch.int64, "offsets"), (domega, torch.float64, "domega"),
                      (spin, torch.float64, "spin")):
        if not (t.is_cuda and t.dtype == dt and t.is_contiguous() and t.dim() == 1):
            raise ValueError(f"{nm} must be a contiguous 1-D CUDA {dt} tensor")
    nimg = domega.shape[0]
    if offsets.shape[0] != nimg + 1 or spin.shape[0] != nimg:
        raise ValueError("offsets must have nimg + 1 entries and spin nimg")
    fa, nf = _freqs(freqs)
    out = torch.empty((nimg, nf), dtype=torch.float64, device=g.device)
    total = g.shape[0]
    rc = lib().kgrt_disk_spectrum(r_cross.data_ptr() if total else None, g.data_ptr() if total else None,
                                  status.data_ptr() if total else None, total, offsets.data_ptr(), domega.data_ptr(),
                                  spin.data_ptr(), nimg, mbh_msun, mdot_gs, fa, nf, out.data_ptr(),
                                  _stream_handle(stream))
    if rc != OK:
        raise KgrtError(rc, "kgrt_disk_spectrum failed")
    return out


def pixel_solid_angle(camera: Camera, mbh_msun: float, distance_cm: float) -> float:
    """kgrt_pixel_solid_angle: sr subtended by one pixel of `camera` at `distance_cm`."""
    v = float(lib().kgrt_pixel_solid_angle(ctypes.byref(camera.c()), mbh_msun, distance_cm))
    if v < 0.0:
        raise ValueError("invalid camera, mass or distance")
    return v


def alloc_outputs(n: int, model: Model, nfreq: int, device, names: Iterable[str] = OUTPUT_FIELDS):
    """Allocates output tensors for n rays (torus intensity/tau are [nfreq, n])."""
    out = {}
    for name in names:
        if name == "n_cross" and model.kind != MODEL_DISK_IMAGES:
            continue
        if name in INT_FIELDS:
            out[name] = torch.empty(n, dtype=torch.int32, device=device)
        elif model.kind in TRANSFER_MODELS and name in ("intensity", "tau"):
            out[name] = torch.empty((max(nfreq, 1), n), dtype=torch.float64, device=device)
        elif model.kind not in TRANSFER_MODELS and name == "tau":
            continue
        else:
            out[name] = torch.empty(n, dtype=torch.float64, device=device)
    return out


def trace_image(ctx: Context, camera: Camera, model: Model, freqs: Sequence[float], integ: Integrator,
                names: Iterable[str] = OUTPUT_FIELDS, stream=None) -> Dict[str, torch.Tensor]:
    """Allocates outputs and traces one image (asynchronous on `stream`)."""
    out = alloc_outputs(camera.nx * camera.ny, model, len(freqs), ctx.device, names)
    ctx.trace(camera, model, freqs, integ, out, stream)
    return out


# ------------------------------------------------------------ surrogate

def _dev_check(t: torch.Tensor, dtype, shape_tail, name):
    if not t.is_cuda or t.dtype != dtype or not t.is_contiguous() or tuple(t.shape[1:]) != tuple(shape_tail):
        raise ValueError(f"{name} must be a contiguous CUDA {dtype} tensor of shape [n, {shape_tail}]")


class Mlp:
    """kgrt_mlp: the surrogate network (BF16-MFMA hidden layers, FP32 head, Adam)."""

    def __init__(self, ctx: Context, max_batch: int = 65536):
        self.ctx = ctx
        self.max_batch = max_batch
        h = ctypes.c_void_p()
        rc = lib().kgrt_mlp_create(ctx._h, max_batch, ctypes.byref(h))
        if rc != OK:
            raise KgrtError(rc, "kgrt_mlp_create failed")
        self._h = h

    @staticmethod
    def num_params() -> int:
        return int(lib().kgrt_mlp_num_params())

    def _check(self, rc):
        if rc != OK:
            raise KgrtError(rc, lib().kgrt_mlp_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_h", None):
            lib().kgrt_mlp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, params):
        import numpy as np
        p = np.ascontiguousarray(params, dtype=np.float32)
        self._check(lib().kgrt_mlp_set_params(self._h, p.ctypes.data, p.size))

    def get_params(self):
        import numpy as np
        p = np.zeros(self.num_params(), dtype=np.float32)
        self._check(lib().kgrt_mlp_get_params(self._h, p.ctypes.data, p.size))
        return p

    def get_adam(self):
        """(first moments, second moments, steps taken) of the optimiser."""
        import numpy as np
        m = np.zeros(self.num_params(), dtype=np.float32)
        v = np.zeros(self.num_params(), dtype=np.float32)
        step = ctypes.c_int64()
        self._check(lib().kgrt_mlp_get_adam(self._h, m.ctypes.data, v.ctypes.data, m.size, ctypes.byref(step)))
        return m, v, int(step.value)

    def set_adam(self, m, v, step: int):
        import numpy as np
        m = np.ascontiguousarray(m, dtype=np.float32)
        v = np.ascontiguousarray(v, dtype=np.float32)
        if m.size != self.num_params() or v.size != self.num_params():
            raise ValueError("moment vectors must have num_params entries")
        self._check(lib().kgrt_mlp_set_adam(self._h, m.ctypes.data, v.ctypes.data, m.size, int(step)))

    def forward(self, x: torch.Tensor, out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
        _dev_check(x, torch.float32, (4,), "x")
        y = out if out is not None else torch.empty((x.shape[0], 5), dtype=torch.float32, device=x.device)
        self._check(lib().kgrt_mlp_forward(self._h, x.data_ptr(), y.data_ptr(), x.shape[0], _stream_handle(stream)))
        return y

    def loss_grads(self, x: torch.Tensor, t: torch.Tensor, idx: Optional[torch.Tensor] = None,
                   n: Optional[int] = None, stream=None):
        _dev_check(x, torch.float32, (4,), "x")
        _dev_check(t, torch.float32, (6,), "t")
        n = n if n is not None else (idx.numel() if idx is not None else x.shape[0])
        loss = torch.zeros(1, dtype=torch.float32, device=x.device)
        grads = torch.empty(self.num_params(), dtype=torch.float32, device=x.device)
        self._check(lib().kgrt_mlp_loss_grads(self._h, x.data_ptr(), t.data_ptr(),
                                              idx.data_ptr() if idx is not None else None, n, loss.data_ptr(),
                                              grads.data_ptr(), _stream_handle(stream)))
        return loss, grads

    def train_step(self, x: torch.Tensor, t: torch.Tensor, idx: Optional[torch.Tensor], n: int, lr: float,
                   loss: torch.Tensor, betas=(0.9, 0.999), eps: float = 1e-8, stream=None):
        opt = CAdam(lr, betas[0], betas[1], eps)
        self._check(lib().kgrt_mlp_train_step(self._h, x.data_ptr(), t.data_ptr(),
                                              idx.data_ptr() if idx is not None else None, n, ctypes.byref(opt),
                                              loss.data_ptr(), _stream_handle(stream)))


def surrogate_features(rays: torch.Tensor, stream=None) -> torch.Tensor:
    _dev_check(rays, torch.float64, (4,), "rays")
    f = torch.empty((rays.shape[0], 4), dtype=torch.float32, device=rays.device)
    rc = lib().kgrt_surrogate_features(rays.data_ptr(), rays.shape[0], f.data_ptr(), _stream_handle(stream))
    if rc != OK:
        raise KgrtError(rc, "kgrt_surrogate_features failed")
    return f


def surrogate_targets(rays: torch.Tensor, outs: Dict[str, torch.Tensor], stream=None) -> torch.Tensor:
    _dev_check(rays, torch.float64, (4,), "rays")
    n = rays.shape[0]
    t = torch.empty((n, 6), dtype=torch.float32, device=rays.device)
    rc = lib().kgrt_surrogate_targets(rays.data_ptr(), outs["status"].data_ptr(), outs["r_cross"].data_ptr(),
                                      outs["g"].data_ptr(), outs["phi_cross"].data_ptr(), n, t.data_ptr(),
                                      _stream_handle(stream))
    if rc != OK:
        raise KgrtError(rc, "kgrt_surrogate_targets failed")
    return t


def surrogate_render(ctx: Context, mlp: Mlp, cameras: Sequence[Camera], model: Model, integ: Integrator,
                     fallback=(0.05, 0.95, 0.5, 0.25, 0.0, 0.0), stream=None):
    # (surrogate.DEFAULT_FALLBACK is the tuned policy; this default keeps the optional checks off)
    """kgrt_surrogate_render: thin-disk images from the network with FP64 fallback.

    Returns dict(intensity [total] f64, status [total] i32, flux [nimg] f64, fallback [nimg] i64)."""
    cams = (CCamera * len(cameras))(*[c.c() for c in cameras])
    total = sum(c.nx * c.ny for c in cameras)
    dev = ctx.device
    out = {"intensity": torch.empty(total, dtype=torch.float64, device=dev),
           "status": torch.empty(total, dtype=torch.int32, device=dev),
           "flux": torch.empty(len(cameras), dtype=torch.float64, device=dev),
           "fallback": torch.empty(len(cameras), dtype=torch.int64, device=dev)}
    fb = CFallback(*(tuple(fallback) + (0.0,) * (6 - len(fallback))))
    rc = lib().kgrt_surrogate_render(ctx._h, mlp._h, cams, len(cameras), ctypes.byref(model.c()),
                                     ctypes.byref(integ.c()), ctypes.byref(fb), out["intensity"].data_ptr(),
                                     out["status"].data_ptr(), out["flux"].data_ptr(), out["fallback"].data_ptr(),
                                     _stream_handle(stream))
    if rc != OK:
        raise KgrtError(rc, lib().kgrt_mlp_last_error(mlp._h).decode())
    return out


def critical_curve(a: float, incl_deg: float):
    """Radius of the critical curve on 1024 polar-angle bins starting at -pi (host, no GPU needed)."""
    import numpy as np
    R = np.zeros(1024, dtype=np.float32)
    rc = lib().kgrt_critical_curve(a, incl_deg, R.ctypes.data, 1024)
    if rc != OK:
        raise KgrtError(rc, "kgrt_critical_curve failed")
    return R
