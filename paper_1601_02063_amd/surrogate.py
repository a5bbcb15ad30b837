"""Training and evaluation of the learned surrogate (host orchestration).

Every arithmetic step runs in the library's kernels: the integrator labels
rays, feature/target kernels build the training set, kgrt_mlp_train_step does
forward, backward and Adam. This module only schedules batches (a seeded
permutation per epoch), the learning rate, validation and checkpoints.
"""
from __future__ import annotations

import json
import math
import os
import time
from typing import Dict, Optional

import numpy as np
import torch

from . import kgrt as K
from . import scenes

ARCH = ("mlp 4-256x4-5 SiLU; training: 256x256 layers in BF16 on MFMA (FP32 accumulate), FP32 input layer, "
        "head and Adam; inference: one fused MFMA kernel, input layer and head on hi+lo BF16 splits")

# The trained network shipped with the package (thin disk r_in = ISCO, r_out = 20 M,
# observer at 1000 M); its .json beside it records how it was trained and its accuracy.
DEFAULT_WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights", "thin_disk_mlp.npz")

# Fallback policy (p_lo, p_hi, crit_band, edge_band, g_tol, grad_max): the two required rules
# (capture probability band, 0.5 M critical-curve band) and a disk-edge band of 1e-4 M around
# the polished crossing radius (whose error is the integrator's own, ~1e-7 relative, so only a
# crossing that close to an edge can land on the other side of it); the g-head consistency
# check and the neighbour rule are off (they guarded the network's radius error, which the
# Mino-time polish removes).
DEFAULT_FALLBACK = (0.05, 0.95, 0.5, 1e-4, 0.0, 0.0)


LAYERS = ((4, 256), (256, 256), (256, 256), (256, 256), (256, 5))


def init_params(seed: int) -> np.ndarray:
    """Initial weights and biases ~ U(-1/sqrt(fan_in), 1/sqrt(fan_in)), layer by layer W[out][in], b[out]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for fan_in, fan_out in LAYERS:
        bound = 1.0 / math.sqrt(fan_in)
        parts.append(rng.uniform(-bound, bound, size=fan_in * fan_out))
        parts.append(rng.uniform(-bound, bound, size=fan_out))
    return np.concatenate(parts).astype(np.float32)


def label_dataset(ctx: K.Context, n: int, seed: int, chunk: int = 1 << 21):
    """Rays (a, incl, x, y) ~ U[0, 0.998] x U[1, 89] deg x U[-15, 15]^2, labelled by the
    FP64 integrator (thin-disk model). Returns (rays f64, features f32, targets f32, seconds)."""
    rays = torch.from_numpy(scenes.label_rays(n, seed)).to(ctx.device)
    model = K.Model(kind=K.MODEL_THIN_DISK)
    integ = K.Integrator()
    t = torch.empty((n, 6), dtype=torch.float32, device=ctx.device)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for lo in range(0, n, chunk):
        hi = min(n, lo + chunk)
        r = rays[lo:hi]
        out = K.alloc_outputs(hi - lo, model, 0, ctx.device, ("status", "r_cross", "g", "phi_cross"))
        ctx.trace_rays(r, model, [], integ, out)
        t[lo:hi] = K.surrogate_targets(r, out)
    x = K.surrogate_features(rays)
    torch.cuda.synchronize()
    return rays, x, t, time.perf_counter() - t0


def validation_loss(mlp: K.Mlp, x, t, chunk: int) -> float:
    n = (x.shape[0] // 32) * 32
    tot, cnt = 0.0, 0
    for lo in range(0, n, chunk):
        m = min(chunk, n - lo)
        m -= m % 32
        if m == 0:
            break
        loss, _ = mlp.loss_grads(x[lo:lo + m], t[lo:lo + m])
        tot += float(loss) * m
        cnt += m
    return tot / max(cnt, 1)


def _isco(a):
    """Prograde ISCO radius (Bardeen, Press & Teukolsky 1972), for selecting disk rays in evaluations."""
    z1 = 1 + (1 - a * a) ** (1 / 3) * ((1 + a) ** (1 / 3) + (1 - a) ** (1 / 3))
    z2 = torch.sqrt(3 * a * a + z1 * z1)
    return 3 + z2 - torch.sqrt((3 - z1) * (3 + z1 + 2 * z2))


def accuracy(mlp: K.Mlp, x, t, r_out: float = 20.0) -> Dict[str, float]:
    """Errors of the predictions on a labelled set (evaluation only): all crossing rays,
    and the rays whose first crossing lies on the disk (ISCO to r_out), which are the
    ones an image depends on."""
    y = mlp.forward(x)
    crossed = t[:, 5] > 0.5
    cap_pred = (y[:, 0] > 0).float()
    rc = torch.exp(t[:, 1].double())
    disk = crossed & (rc >= _isco(x[:, 0].double())) & (rc <= r_out)
    rel = (torch.exp(y[:, 1] - t[:, 1]) - 1.0).abs()
    gab = (y[:, 2] - t[:, 2]).abs()
    q = lambda v, p: float(torch.quantile(v[:1 << 20], p)) if v.numel() else float("nan")
    out = {"capture_accuracy": float((cap_pred == t[:, 0]).float().mean())}
    for name, m in (("", crossed), ("disk_", disk)):
        out[name + "r_c_rel_err_median"] = q(rel[m], 0.5)
        out[name + "r_c_rel_err_p99"] = q(rel[m], 0.99)
        out[name + "g_abs_err_median"] = q(gab[m], 0.5)
        out[name + "g_abs_err_p99"] = q(gab[m], 0.99)
    out["disk_fraction"] = float(disk.float().mean())
    return out


def train(ctx: K.Context, mlp: K.Mlp, x, t, xv, tv, epochs: int, batch: int = 65536, lr0: float = 1e-3,
          lr_min_frac: float = 0.02, seed: int = 1604, log=None) -> Dict:
    """Adam with a cosine learning-rate decay over all steps; one seeded permutation per epoch."""
    n = x.shape[0]
    steps_per_epoch = n // batch
    total = max(1, epochs * steps_per_epoch)
    gen = torch.Generator(device=ctx.device)
    gen.manual_seed(seed)
    loss = torch.zeros(1, dtype=torch.float32, device=ctx.device)
    hist = []
    step = 0
    train_s = 0.0
    for ep in range(epochs):
        perm = torch.randperm(n, generator=gen, device=ctx.device).to(torch.int32)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for b in range(steps_per_epoch):
            lr = lr0 * (lr_min_frac + (1 - lr_min_frac) * 0.5 * (1 + math.cos(math.pi * step / total)))
            mlp.train_step(x, t, perm[b * batch:(b + 1) * batch], batch, lr, loss)
            step += 1
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        train_s += dt
        rec = {"epoch": ep, "train_loss_last": float(loss), "val_loss": validation_loss(mlp, xv, tv, batch),
               "epoch_s": dt, "samples_per_s": steps_per_epoch * batch / dt}
        hist.append(rec)
        if log:
            log(rec)
    return {"history": hist, "steps": step, "train_seconds": train_s,
            "samples_per_s": step * batch / max(train_s, 1e-9)}


def save_checkpoint(path: str, mlp: K.Mlp, meta: Dict):
    """Parameters, the optimiser's moments and its step count (training resumes exactly)."""
    m, v, step = mlp.get_adam()
    np.savez(path, params=mlp.get_params(), adam_m=m, adam_v=v, adam_step=np.int64(step))
    with open(os.path.splitext(path)[0] + ".json", "w") as f:
        json.dump(dict(meta, arch=ARCH), f, indent=1)


def load_checkpoint(path: str, mlp: K.Mlp) -> Optional[Dict]:
    if not os.path.exists(path):
        return None
    with np.load(path, allow_pickle=False) as z:
        mlp.set_params(z["params"])
        if "adam_m" in z.files:
            mlp.set_adam(z["adam_m"], z["adam_v"], int(z["adam_step"]))
    meta_path = os.path.splitext(path)[0] + ".json"
    return json.load(open(meta_path)) if os.path.exists(meta_path) else {}


def render_errors(I_s: torch.Tensor, I_ref: torch.Tensor, offsets) -> Dict:
    """Flux error per image and per-pixel relative error (|I_s - I_ref| <= 1e-2 I_ref where
    I_ref > 0, I_s == 0 where I_ref == 0)."""
    flux_err = []
    worst, bad, n_pos = 0.0, 0, 0
    q999 = []
    for k in range(len(offsets) - 1):
        a, b = offsets[k], offsets[k + 1]
        s, r = I_s[a:b], I_ref[a:b]
        fr = float(r.sum())
        flux_err.append(abs(float(s.sum()) - fr) / fr if fr > 0 else float(s.sum() != 0))
        pos = r > 0
        rel = ((s - r).abs() / r.clamp_min(1e-300))[pos]
        n_pos += int(pos.sum())
        if rel.numel():
            worst = max(worst, float(rel.max()))
            bad += int((rel > 1e-2).sum())
            q999.append(float(torch.quantile(rel[:1 << 24].float(), 0.999)))
        bad += int(((s != 0) & ~pos).sum())
    return {"flux_rel_err_max": max(flux_err), "flux_rel_err_mean": float(np.mean(flux_err)),
            "pixel_rel_err_max": worst, "pixel_rel_err_p999_max": max(q999) if q999 else 0.0,
            "pixels_violating_1e-2": bad, "pixels_with_emission": n_pos}
