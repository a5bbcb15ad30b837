#!/usr/bin/env python3
"""Benchmark of the FP64 Kerr ray tracer with radiative transfer on one MI355X.

Default workload: the optically thin thermal-synchrotron torus image
(a = 0.94, inclination 17 deg, 1024 x 1024 rays over +-20 M, 230 GHz). One
step = one full image traced by kgrt_trace (ray start, adaptive Cash-Karp
integration, per-step transfer of tau and I_nu, writeback), inputs and
outputs resident in HBM.

Metric: ns per photon per accepted RK step = kernel time / sum of accepted
steps over the image (the paper's Table 1 quantity T/S).

Prints ONE JSON line. Other workloads (--workload):
  thin_disk, projection   the 64x64 thin-disk image; the first-crossing projection
  batch                   256 uneven torus images, 8 frequencies, one graph-replayed plan
  train                   surrogate training on integrator-labelled rays (writes a checkpoint)
  infer                   the fused surrogate network alone, 2^24 samples
  render                  64 surrogate+fallback thin-disk images of 2048^2 vs the integrator
  table1                  the paper's Table 1 sweep (projection, N = 2 ... 2048)
  grid                    the torus camera over a 256x128x128 GRMHD-like plasma snapshot (1024^2, 230 GHz)
Extra modes:
  --calibrate RAY   trace copies of one ray (no divergence) so a rocprofv3
                    --pmc run can count FP64 VALU instructions per step.
  --copy-probe      one plain 1 GiB device copy (scales HBM byte counters).
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "ns/photon/RK step; images/s surrogate+fallback vs integrator @1% flux"
FP64_VECTOR_PEAK_TFLOPS = 78.6  # 256 CU x 2.4 GHz x 128 FP64 FLOP/clk/CU

# FP64 FLOPs per attempted Cash-Karp step of the torus workload, transfer of
# the accepted steps included. "calibrated": 64 x (ADD + MUL + TRANS + 2 FMA)
# FP64 VALU instructions per attempt from rocprofv3 counters on a
# divergence-free run (every lane traces the same ray), see
# profiles/trace_kernel_flop_calibration.md (the thin-disk figure, from three disk
# rays, also serves the projection workload, which runs the same kernel; the
# batch figure is the eight-frequency torus kernel's, from the torus rays traced
# at the batch's eight frequencies; the grid figure is the gridded-plasma kernel's,
# from the torus rays traced through the 256x128x128 snapshot).
FLOPS_PER_ATTEMPT = {"torus": (1287.0, "calibrated"), "thin_disk": (852.0, "calibrated"),
                     "projection": (852.0, "calibrated"), "batch": (2173.0, "calibrated"),
                     "grid": (1356.0, "calibrated")}

# HBM bytes per launch of the dominant kernel from rocprofv3 FETCH_SIZE and
# WRITE_SIZE (scaled by a 1 GiB copy probe), see
# profiles/torus_1024_hbm_traffic.md. Valid only for the kernel sources they
# were taken on (md5 of csrc/kgrt.hip + csrc/kgrt_device.hpp); null otherwise.
# VALU lane utilisation of the dominant kernel (useful FP64 FLOPs / FP64 lane
# slots issued, rocprofv3 counters), valid for the sources it was taken on; see
# profiles/trace_kernel_flop_calibration.md.
HEAD_MD5 = "30905ad1bf94774f8d905f9cc6655a3a"
LANE_UTILISATION = {"torus": {"value": 0.940, "source_md5": HEAD_MD5},
                    "batch": {"value": 0.892, "source_md5": HEAD_MD5},
                    "thin_disk": {"value": 0.910, "source_md5": HEAD_MD5},
                    "grid": {"value": 0.939, "source_md5": HEAD_MD5}}

TRAFFIC = {"torus": {"bytes": 132671652, "source_md5": HEAD_MD5},
           # the one launch of the 256-image plan, see profiles/batch256_trace_kernel_traffic.md
           "batch": {"bytes": 22641750604, "source_md5": HEAD_MD5},
           # the 1024^2 thin-disk image, see profiles/trace_kernel_flop_calibration.md
           "thin_disk": {"bytes": 316799880, "source_md5": HEAD_MD5},
           # the 1024^2 image of the gridded snapshot, see profiles/grid_1024_kernel_trace.md
           "grid": {"bytes": 3613276482, "source_md5": HEAD_MD5}}


def kernel_source_md5() -> str:
    import hashlib
    h = hashlib.md5()
    for name in ("kgrt.hip", "kgrt_device.hpp"):
        with open(os.path.join(ROOT, "paper_1601_02063_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()

CALIBRATION_RAYS = {
    # (a, incl_deg, x, y): a captured ray, an escaping ray through the torus, a far ray
    "captured": (0.94, 17.0, 1.5, 2.0),
    "escaping": (0.94, 17.0, 7.0, -5.0),
    "far": (0.94, 17.0, 18.0, 15.0),
    # thin disk (a = 0.9, incl 60 deg, as the 64x64 disk image): a disk hit, a far ray, a captured ray
    "disk_hit": (0.9, 60.0, 6.0, 3.0),
    "disk_far": (0.9, 60.0, 14.0, 12.0),
    "disk_captured": (0.9, 60.0, 0.5, 0.5),
    # the gridded plasma (the torus camera over the 256x128x128 snapshot): the torus rays
    "grid_captured": (0.94, 17.0, 1.5, 2.0),
    "grid_escaping": (0.94, 17.0, 7.0, -5.0),
    "grid_far": (0.94, 17.0, 18.0, 15.0),
}


def workload(name: str, n: int | None):
    from paper_1601_02063_amd import scenes
    if name == "torus":
        return scenes.torus_image(n or 1024), "optically thin thermal-synchrotron torus, a=0.94, incl=17 deg, " \
            f"{n or 1024}x{n or 1024} rays over +-20 M, 230 GHz, rtol 1e-8, step cap 0.02 r"
    if name == "thin_disk":
        return scenes.thin_disk_image(n or 64), f"thin Keplerian disk ISCO-20 M, a=0.9, incl=60 deg, " \
            f"{n or 64}x{n or 64} rays over +-15 M, rtol 1e-8"
    if name == "projection":
        return scenes.projection_image(n or 1024), f"first-crossing projection, a=0.95, incl=60 deg, " \
            f"{n or 1024}x{n or 1024} rays over +-15 M, rtol 1e-8"
    if name == "grid":
        return scenes.grid_image(n or 1024), "thermal-synchrotron plasma sampled from a GRMHD-like snapshot " \
            "(256x128x128 (ln r, theta, phi) nodes over 1-1000 M, seed 1610), a=0.94, incl=17 deg, " \
            f"{n or 1024}x{n or 1024} rays over +-20 M, 230 GHz, rtol 1e-8, step cap 0.02 r"
    raise SystemExit(f"unknown workload {name}")


def cpu_model() -> str:
    """The host CPU's model name (/proc/cpuinfo), else the platform's processor string."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine()


def cpu_baseline(w, nsample: int, seed: int = 2024):
    """The CPU oracle on a seeded sample of pixels of the same workload."""
    import numpy as np

    import oracle as O
    from paper_1601_02063_amd import scenes
    cam = w["camera"]
    idx = scenes.sample_pixels(cam["nx"], cam["ny"], nsample, seed)
    xy = O.pixel_points(cam["nx"], cam["ny"], cam["x_min"], cam["x_max"], cam["y_min"], cam["y_max"])[idx]
    sc = O.Scene(a=cam["a"], incl_deg=cam["incl_deg"], r_obs=cam["r_obs"], rtol=w["integ"]["rtol"],
                 hmax_frac=w["integ"]["hmax_frac"], horizon_delta=w["integ"]["horizon_delta"],
                 max_steps=w["integ"]["max_steps"], model=w["model"]["kind"],
                 stop_at_crossing=bool(w["integ"]["flags"] & 1), freqs_hz=list(w["freqs"]), grid=w.get("grid"),
                 **{k: v for k, v in w["model"].items() if k != "kind"})
    threads = O.default_threads()
    t0 = time.perf_counter()
    res = O.trace_points(sc, xy, threads)
    dt = time.perf_counter() - t0
    steps = int(res["steps"].astype(np.int64).sum())
    # one thread on every threads-th pixel of the same sample
    sub = xy[::max(threads, 1)]
    t1 = time.perf_counter()
    res1 = O.trace_points(sc, sub, 1)
    dt1 = time.perf_counter() - t1
    steps1 = int(res1["steps"].astype(np.int64).sum())
    return {"value": dt / steps * 1e9, "unit": "ns/photon/RK step", "cores": threads, "kind": "oracle",
            "cpu_model": cpu_model(), "single_thread_value": dt1 / steps1 * 1e9,
            "sample": f"{len(idx)} seeded pixels (seed {seed}) of the same image, {steps} accepted steps, "
                      f"{dt:.2f} s wall on {threads} threads ({cpu_model()}); "
                      f"single thread: every {max(threads, 1)}th of them, {steps1} steps, {dt1:.2f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="torus",
                    choices=["torus", "thin_disk", "projection", "batch", "train", "infer", "render", "table1",
                             "grid"])
    ap.add_argument("--train-rays", type=int, default=10_000_000)
    ap.add_argument("--epochs", type=int, default=20)
    ap.add_argument("--ckpt", default=None,
                    help="train: checkpoint to write (default gpurun_out/surrogate.npz); "
                         "render: weights to use (default the package's trained network)")
    ap.add_argument("--images", type=int, default=64, help="render: number of images")
    ap.add_argument("--surrogate-images", type=int, default=64,
                    help="default workload: images of the surrogate-vs-integrator measurement (0 = skip)")
    ap.add_argument("--surrogate-n", type=int, default=2048, help="default workload: their side")
    ap.add_argument("--fallback", default=None,
                    help="render: p_lo,p_hi,crit_band,edge_band,g_tol,grad_max (default the tuned policy)")
    ap.add_argument("--seed", type=int, default=None, help="render/analysis: scene seed (default 1605)")
    ap.add_argument("--lr", type=float, default=1e-3, help="train: peak learning rate")
    ap.add_argument("--autotune", action="store_true", help="batch: autotune the launch shape first")
    ap.add_argument("--baselines", action="store_true", help="batch: also time per-image launches")
    ap.add_argument("--nfreq", type=int, default=1, help="calibration: number of frequencies (1 or 8)")
    ap.add_argument("--n", type=int, default=None, help="image side (default per workload)")
    ap.add_argument("--cpu-sample", type=int, default=400000,
                    help="pixels in the CPU-oracle sample (0 = skip); about 10 s of oracle work on 16 cores")
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--blocks-per-cu", type=int, default=0)
    ap.add_argument("--refill-min", type=int, default=0)
    ap.add_argument("--calibrate", default=None, choices=sorted(CALIBRATION_RAYS))
    ap.add_argument("--copy-probe", action="store_true",
                    help="run one plain 1 GiB device copy (scales the HBM byte counters)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this build runs on exactly one GPU (the ray tracer shards by images or rays across "
              "GPUs, but no multi-GPU path is built); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1601_02063_amd import kgrt as K

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda", 0)
    ctx = K.Context(0)
    ctx.set_launch(args.block, args.blocks_per_cu, args.refill_min)

    if args.calibrate:
        calibrate(ctx, args.calibrate, dev, args.nfreq)
        return
    if args.copy_probe:
        src = torch.ones(1 << 27, dtype=torch.float64, device=dev)  # 1 GiB
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": src.numel() * 8, "copy_probe_bytes_written": dst.numel() * 8}))
        return

    if args.workload == "batch":
        bench_batch(ctx, args, dev)
        return
    if args.workload == "train":
        bench_train(ctx, args, dev)
        return
    if args.workload == "infer":
        bench_infer(ctx, args, dev)
        return
    if args.workload == "table1":
        bench_table1(ctx, args, dev)
        return
    if args.workload == "render":
        bench_render(ctx, args, dev)
        return

    w, desc = workload(args.workload, args.n)
    cam, mod, freqs = K.Camera(**w["camera"]), K.Model(**w["model"]), list(w["freqs"])
    if "grid" in w:
        mod.grid = torch.from_numpy(w["grid"]).to(dev)
    integ = K.Integrator(**w["integ"])
    n = cam.nx * cam.ny
    out = K.alloc_outputs(n, mod, len(freqs), dev, names=("status", "steps", "attempts", "intensity", "tau",
                                                          "r_cross", "g"))
    stream = torch.cuda.current_stream()

    for _ in range(args.warmup):
        ctx.trace(cam, mod, freqs, integ, out)
    torch.cuda.synchronize()

    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    t0 = time.perf_counter()
    for s, e in ev:
        s.record(stream)
        ctx.trace(cam, mod, freqs, integ, out)
        e.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kern_ms = [s.elapsed_time(e) for s, e in ev]
    ms_mean = sum(kern_ms) / len(kern_ms)

    steps = int(out["steps"].to(torch.int64).sum())
    attempts = int(out["attempts"].to(torch.int64).sum())
    st = out["status"]
    ns_per_step = ms_mean * 1e6 / steps
    fpa, basis = FLOPS_PER_ATTEMPT.get(args.workload, (None, None))
    achieved = fpa * attempts / (ms_mean * 1e-3) / 1e12 if fpa else None
    tr = TRAFFIC.get(args.workload)
    traffic = tr["bytes"] if (tr and cam.nx == 1024 and cam.ny == 1024 and tr["source_md5"] == kernel_source_md5()) \
        else None
    lu = LANE_UTILISATION.get(args.workload)
    lane_util = lu["value"] if (lu and cam.nx == 1024 and cam.ny == 1024 and lu["source_md5"] == kernel_source_md5()) \
        else None
    kinfo = ctx.kernel_info(mod.kind, max(len(freqs), 1), args.block or 256)
    line = {
        "metric": METRIC,
        "value": round(ns_per_step, 6),
        "unit": "ns/photon/RK step",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall * 1e3 / args.steps, 4),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": desc, "rays": n, "nfreq": len(freqs), "launch": {
            "block": args.block or 256, "blocks_per_cu": args.blocks_per_cu or "occupancy",
            "refill_min": args.refill_min or (64 if len(freqs) < 8 else 1)}},
        "kernel_ms": round(ms_mean, 4),
        "kernel_ms_min": round(min(kern_ms), 4),
        "rays_per_s": round(n / (ms_mean * 1e-3), 1),
        "images_per_s": round(1.0 / (ms_mean * 1e-3), 3),
        "accepted_steps": steps,
        "attempted_steps": attempts,
        "steps_per_ray": round(steps / n, 2),
        "ns_per_attempted_step": round(ms_mean * 1e6 / attempts, 6),
        "ns_per_rhs_eval": round(ms_mean * 1e6 / (6 * attempts), 6),
        "captured_frac": round(float(((st & 1) != 0).float().mean()), 5),
        "kernel": dict(kinfo, lane_utilisation=lane_util),
        "roofline": {"bound": "alu", "achieved": round(achieved, 4) if fpa else None,
                     "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(achieved / FP64_VECTOR_PEAK_TFLOPS, 5) if fpa else None, "traffic": traffic,
                     "flops_per_attempt": fpa, "flops_basis": basis,
                     "kernel": {"torus": "trace_kernel<torus,1>", "grid": "trace_kernel<grid,1>"}.get(
                         args.workload, "trace_kernel<disk,1>")},
    }
    if args.workload == "grid":
        # one trilinear sample (8 nodes x 16 B) per accepted point, the start point included,
        # mostly served by the caches (the snapshot is 64 MiB)
        gb = 128 * (steps + n)
        line["grid_samples"] = {"bytes": gb, "node_bytes_per_sample": 128,
                                "achieved_GBs": round(gb / (ms_mean * 1e-3) / 1e9, 1),
                                "snapshot_bytes": int(w["grid"].nbytes)}
    if args.cpu_sample > 0:
        line["cpu_baseline"] = cpu_baseline(w, args.cpu_sample)
    if args.workload == "torus" and args.surrogate_images > 0:
        # the metric's second half: surrogate + fallback images/s against the integrator
        r = render_measure(ctx, args.surrogate_images, args.surrogate_n, 1605 if args.seed is None else args.seed,
                           args.ckpt, args.fallback)
        line["surrogate"] = {k: r[k] for k in ("workload", "images", "surrogate_images_per_s",
                                               "integrator_images_per_s", "speedup_vs_integrator", "speedup_reported",
                                               "flux_rel_err_max", "pixels_violating_1e-2", "pixels_with_emission",
                                               "pixel_rel_err_max", "fallback_fraction", "surrogate_ms",
                                               "integrator_ms", "fallback_policy")}
    ctx.close()
    print(json.dumps(line), flush=True)


def bench_batch(ctx, args, dev):
    """256 uneven torus images at 8 frequencies in one persistent, graph-replayed launch."""
    import torch

    from paper_1601_02063_amd import kgrt as K
    from paper_1601_02063_amd import scenes
    ws = scenes.batch_scenes(1603)
    cams = [K.Camera(**w["camera"]) for w in ws]
    mod, freqs, integ = K.Model(**ws[0]["model"]), list(ws[0]["freqs"]), K.Integrator(**ws[0]["integ"])
    plan = K.Plan(ctx, cams, mod, freqs, integ)
    out = plan.alloc_outputs(("status", "steps", "attempts", "intensity", "tau"))
    stream = torch.cuda.current_stream()
    tuned = plan.autotune(out) if args.autotune else None
    for _ in range(args.warmup):
        plan.launch(out, graph=True)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    t0 = time.perf_counter()
    for s, e in ev:
        s.record(stream)
        plan.launch(out, graph=True)
        e.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = sum(s.elapsed_time(e) for s, e in ev) / len(ev)
    steps = int(out["steps"].to(torch.int64).sum())
    attempts = int(out["attempts"].to(torch.int64).sum())
    fpa, basis = FLOPS_PER_ATTEMPT.get("batch", (None, None))
    line = {
        "metric": METRIC, "value": round(ms * 1e6 / steps, 6), "unit": "ns/photon/RK step", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(wall * 1e3 / args.steps, 3),
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "256 uneven torus images (sides 64-512, a ~ U[0,0.998], incl ~ U[1,89] deg, "
                               "seed 1603), 8 frequencies 86-690 GHz, one persistent launch replayed as a hipGraph",
                   "rays": plan.num_rays, "images": len(cams), "autotuned": tuned},
        "kernel_ms": round(ms, 3), "images_per_s": round(len(cams) / (ms * 1e-3), 3),
        "rays_per_s": round(plan.num_rays / (ms * 1e-3), 1), "accepted_steps": steps, "attempted_steps": attempts,
    }
    if fpa:
        ach = fpa * attempts / (ms * 1e-3) / 1e12
        tr = TRAFFIC.get("batch")
        line["roofline"] = {"bound": "alu", "achieved": round(ach, 4), "peak": FP64_VECTOR_PEAK_TFLOPS,
                            "unit": "TFLOP/s", "frac": round(ach / FP64_VECTOR_PEAK_TFLOPS, 5),
                            "traffic": tr["bytes"] if tr["source_md5"] == kernel_source_md5() else None,
                            "flops_per_attempt": fpa, "flops_basis": basis, "kernel": "trace_kernel<torus,8>"}
        lu = LANE_UTILISATION.get("batch")
        line["lane_utilisation"] = lu["value"] if lu["source_md5"] == kernel_source_md5() else None
    # spectra of the batch: flux density of every image at every frequency, seen from 8 kpc
    # (one read of each intensity: an HBM-bound reduction)
    dom = torch.tensor([K.pixel_solid_angle(c, mod.mbh_msun, SPECTRA_DISTANCE_CM) for c in cams],
                       dtype=torch.float64, device=dev)
    flux = plan.spectra(out["intensity"], dom, stream)
    torch.cuda.synchronize()
    sev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(20)]
    for s, e in sev:
        s.record(stream)
        flux = plan.spectra(out["intensity"], dom, stream)
        e.record(stream)
    torch.cuda.synchronize()
    sms = sum(s.elapsed_time(e) for s, e in sev) / len(sev)
    sbytes = plan.num_rays * len(freqs) * 8
    sgbs = sbytes / (sms * 1e-3) / 1e9
    line["spectra"] = {"ms": round(sms, 4), "kernel": "spectra_kernel", "bound": "hbm",
                       "achieved": round(sgbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": round(sgbs / HBM_PEAK_GBS, 4), "bytes": sbytes,
                       "total_flux_cgs": [float(v) for v in flux.sum(0).cpu()]}
    if args.baselines:
        for label, mode in (("per_image_persistent", K.LAUNCH_PERSISTENT),
                            ("per_image_one_ray_per_thread", K.LAUNCH_ONE_RAY_PER_THREAD)):
            ctx.set_launch(mode=mode)
            per = [K.alloc_outputs(c.nx * c.ny, mod, len(freqs), dev, names=tuple(out)) for c in cams]
            torch.cuda.synchronize()
            s0, s1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            s0.record(stream)
            for cam, view in zip(cams, per):
                ctx.trace(cam, mod, freqs, integ, view)
            s1.record(stream)
            torch.cuda.synchronize()
            bms = s0.elapsed_time(s1)
            line[label] = {"ms": round(bms, 3), "images_per_s": round(len(cams) / (bms * 1e-3), 3),
                           "batch_speedup": round(bms / ms, 3)}
        ctx.set_launch()
    plan.close()
    print(json.dumps(line), flush=True)


SPECTRA_DISTANCE_CM = 8.0 * 3.0856775814913673e21  # 8 kpc
HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
MLP_TRAIN_MFMA_FLOPS = 3 * 3 * 2 * 256 * 256  # per sample: forward, input- and weight-gradient of the 256x256 layers
MLP_FWD_FLOPS = 397824  # per sample, all layers
BF16_DENSE_PEAK_TFLOPS = 2500.0


def bench_train(ctx, args, dev):
    """Surrogate training: integrator-labelled rays, BF16-MFMA forward/backward, Adam, batch 65536."""
    import torch

    from paper_1601_02063_amd import kgrt as K
    from paper_1601_02063_amd import surrogate as S
    rays, x, t, label_s = S.label_dataset(ctx, args.train_rays, 1604)
    _, xv, tv, _ = S.label_dataset(ctx, 100_000, 1614)
    mlp = K.Mlp(ctx, 65536)
    mlp.set_params(S.init_params(7))
    log = lambda r: print(json.dumps({"train_epoch": r}), file=sys.stderr, flush=True)
    res = S.train(ctx, mlp, x, t, xv, tv, args.epochs, lr0=args.lr, log=log)
    acc = S.accuracy(mlp, xv, tv)
    ckpt = args.ckpt or os.path.join("gpurun_out", "surrogate.npz")
    os.makedirs(os.path.dirname(ckpt) or ".", exist_ok=True)
    S.save_checkpoint(ckpt, mlp, {"train_rays": args.train_rays, "epochs": args.epochs, "lr": args.lr,
                                       "val_loss": res["history"][-1]["val_loss"], **acc})
    sps = res["samples_per_s"]
    ach = sps * MLP_TRAIN_MFMA_FLOPS / 1e12
    line = {"metric": "surrogate training samples/s", "value": round(sps, 1), "unit": "samples/s", "n_gpus": 1,
            "higher_is_better": True, "dtype": "bf16 (fp32 accumulate)", "data": "synthetic",
            "config": {"workload": f"MLP 4-256x4-5 SiLU, batch 65536, Adam, {args.train_rays} integrator-labelled "
                                   f"rays, {args.epochs} epochs"},
            "label_rays_per_s": round(args.train_rays / label_s, 1), "train_seconds": round(res["train_seconds"], 3),
            "val_loss": res["history"][-1]["val_loss"], "accuracy": acc,
            "roofline": {"bound": "mfma", "achieved": round(ach, 3), "peak": BF16_DENSE_PEAK_TFLOPS,
                         "unit": "TFLOP/s", "frac": round(ach / BF16_DENSE_PEAK_TFLOPS, 5), "traffic": None,
                         "flops_per_sample": MLP_TRAIN_MFMA_FLOPS, "kernel": "256x256 layers (fwd+dgrad+wgrad)"}}
    mlp.close()
    print(json.dumps(line), flush=True)


def bench_table1(ctx, args, dev):
    """The paper's Table 1 measurement on MI355X: first-crossing projection images (a = 0.95,
    incl 60 deg, observer 1000 M, +-15 M, rtol 1e-8) of N x N pixels, N = 2 ... 2048; run time T of
    one launch (after a warm-up, median of args.steps), total accepted RK steps S, and T/S."""
    import torch

    from paper_1601_02063_amd import kgrt as K
    from paper_1601_02063_amd import scenes
    stream = torch.cuda.current_stream()
    rows = []
    for p in range(1, 12):
        N = 2 ** p
        w = scenes.projection_image(N)
        cam, mod, integ = K.Camera(**w["camera"]), K.Model(**w["model"]), K.Integrator(**w["integ"])
        out = K.alloc_outputs(N * N, mod, 0, dev, names=("status", "steps", "attempts", "r_cross", "g"))
        ctx.trace(cam, mod, [], integ, out)
        torch.cuda.synchronize()
        ts = []
        for _ in range(max(3, args.steps)):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            ctx.trace(cam, mod, [], integ, out)
            e1.record(stream)
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        T = sorted(ts)[len(ts) // 2]
        S = int(out["steps"].to(torch.int64).sum())
        rows.append({"N": N, "T_ms": round(T, 4), "S": S, "steps_per_photon": round(S / (N * N), 1),
                     "ns_per_photon_step": round(T * 1e6 / S, 5), "photon_steps_per_s": round(S / (T * 1e-3), 1)})
        print(json.dumps({"table1_row": rows[-1]}), file=sys.stderr, flush=True)
    print(json.dumps({"metric": "Table 1 analogue: ns per photon per RK step (T/S), projection a=0.95 incl 60",
                      "unit": "ns/photon/RK step", "higher_is_better": False, "n_gpus": 1, "dtype": "f64",
                      "data": "synthetic", "rows": rows}), flush=True)


MLP_INFER_MFMA_FLOPS = 3 * 2 * 256 * 256  # per sample: the three 256x256 layers


def bench_infer(ctx, args, dev):
    """Surrogate inference alone (kgrt_mlp_forward, the fused kernel): 2^24 samples per step,
    features drawn as the training rays' (seeded), initial weights (the cost does not depend
    on their values)."""
    import numpy as np
    import torch

    from paper_1601_02063_amd import kgrt as K
    from paper_1601_02063_amd import scenes
    from paper_1601_02063_amd import surrogate as S
    n = 1 << 24
    rays = scenes.label_rays(n, 1617)
    feat = np.stack([rays[:, 0], np.cos(np.radians(rays[:, 1])), rays[:, 2] / 15, rays[:, 3] / 15], 1)
    x = torch.from_numpy(feat.astype(np.float32)).to(dev)
    y = torch.empty((n, 5), dtype=torch.float32, device=dev)
    mlp = K.Mlp(ctx, 65536)
    mlp.set_params(S.init_params(7))
    stream = torch.cuda.current_stream()
    for _ in range(max(1, args.warmup)):
        mlp.forward(x, out=y)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.steps):
        mlp.forward(x, out=y)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    sps = n / (ms * 1e-3)
    ach = sps * MLP_INFER_MFMA_FLOPS / 1e12
    line = {"metric": "surrogate inference samples/s", "value": round(sps, 1), "unit": "samples/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True,
            "dtype": "bf16 (fp32 accumulate)", "data": "synthetic",
            "config": {"workload": f"MLP 4-256x4-5 SiLU forward, {n} samples per step"},
            "roofline": {"bound": "mfma", "achieved": round(ach, 3), "peak": BF16_DENSE_PEAK_TFLOPS,
                         "unit": "TFLOP/s", "frac": round(ach / BF16_DENSE_PEAK_TFLOPS, 5), "traffic": None,
                         "flops_per_sample": MLP_INFER_MFMA_FLOPS, "kernel": "mlp_infer_rows"}}
    mlp.close()
    print(json.dumps(line), flush=True)


def render_measure(ctx, nimg: int, n: int, seed: int, ckpt=None, fallback=None, per_image_log=False) -> dict:
    """Surrogate + fallback thin-disk images against the full FP64 integrator on the same GPU and
    images (config 5 at its defaults): both timed with HIP events on the stream they run on,
    flux and per-pixel errors of every image. The speedup counts only when every image is within
    1% in flux and every emitting pixel within 1e-2 (zero where the integrator's is zero)."""
    import torch

    from paper_1601_02063_amd import kgrt as K
    from paper_1601_02063_amd import scenes
    from paper_1601_02063_amd import surrogate as S
    ws = scenes.render_scenes(seed, nimg, n)
    cams = [K.Camera(**w["camera"]) for w in ws]
    mod, integ = K.Model(**ws[0]["model"]), K.Integrator(**ws[0]["integ"])
    mlp = K.Mlp(ctx, 1 << 20)
    meta = S.load_checkpoint(ckpt or S.DEFAULT_WEIGHTS, mlp)
    if meta is None:
        raise SystemExit(f"no surrogate checkpoint at {ckpt}: run --workload train first")
    stream = torch.cuda.current_stream()
    # reference: every ray through the integrator (one persistent plan, graph replay)
    plan = K.Plan(ctx, cams, mod, [], integ)
    ref = plan.alloc_outputs(("status", "intensity"))
    plan.launch(ref, graph=True)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    plan.launch(ref, graph=True)
    e1.record(stream)
    torch.cuda.synchronize()
    t_int = e0.elapsed_time(e1)
    fb = tuple(float(v) for v in fallback.split(",")) if fallback else S.DEFAULT_FALLBACK
    out = K.surrogate_render(ctx, mlp, cams, mod, integ, fb)  # warm-up
    torch.cuda.synchronize()
    e0.record(stream)
    out = K.surrogate_render(ctx, mlp, cams, mod, integ, fb)
    e1.record(stream)
    torch.cuda.synchronize()
    t_sur = e0.elapsed_time(e1)
    err = S.render_errors(out["intensity"], ref["intensity"], plan.offsets)
    nfb = int(out["fallback"].sum())
    if per_image_log:
        for k, c in enumerate(cams):
            a, b = plan.offsets[k], plan.offsets[k + 1]
            fr = float(ref["intensity"][a:b].sum())
            print(json.dumps({"image": k, "a": c.a, "incl_deg": c.incl_deg,
                              "flux_rel_err": (float(out["intensity"][a:b].sum()) - fr) / fr if fr > 0 else None,
                              "fallback_fraction": int(out["fallback"][k]) / (b - a)}), file=sys.stderr, flush=True)
    both_bars = err["flux_rel_err_max"] <= 1e-2 and err["pixels_violating_1e-2"] == 0
    res = {"workload": f"{len(cams)} thin-disk images {cams[0].nx}x{cams[0].ny} over +-15 M, (a, incl) seeded "
                       f"{seed}, disk ISCO-20 M", "images": len(cams),
           "surrogate_images_per_s": round(len(cams) / (t_sur * 1e-3), 3),
           "integrator_images_per_s": round(len(cams) / (t_int * 1e-3), 3),
           "speedup_vs_integrator": round(t_int / t_sur, 3) if both_bars else None,
           "speedup_reported": both_bars,
           "speedup_measured": round(t_int / t_sur, 3),
           "flux_rel_err_max": err["flux_rel_err_max"], "pixels_violating_1e-2": err["pixels_violating_1e-2"],
           "pixels_with_emission": err["pixels_with_emission"], "pixel_rel_err_max": err["pixel_rel_err_max"],
           "fallback_fraction": round(nfb / plan.num_rays, 5), "surrogate_ms": round(t_sur, 3),
           "integrator_ms": round(t_int, 3), "fallback_policy": fb, "checkpoint": meta, "errors": err}
    plan.close()
    mlp.close()
    return res


def bench_render(ctx, args, dev):
    """Surrogate + fallback thin-disk images vs the full FP64 integrator on the same GPU."""
    seed = 1605 if args.seed is None else args.seed
    r = render_measure(ctx, args.images, args.n or 2048, seed, args.ckpt, args.fallback, per_image_log=True)
    line = {"metric": METRIC, "value": r["surrogate_images_per_s"], "unit": "images/s",
            "n_gpus": 1, "higher_is_better": True, "dtype": "bf16 surrogate + f64 fallback", "data": "synthetic",
            "config": {"workload": r["workload"], "fallback": r["fallback_policy"], "checkpoint": r["checkpoint"]},
            "surrogate_ms": r["surrogate_ms"], "integrator_ms": r["integrator_ms"],
            "integrator_images_per_s": r["integrator_images_per_s"],
            "speedup_vs_integrator": r["speedup_vs_integrator"], "speedup_measured": r["speedup_measured"],
            "both_bars_hold": r["speedup_reported"], "flux_within_1pct": r["flux_rel_err_max"] <= 1e-2,
            "fallback_fraction": r["fallback_fraction"], "errors": r["errors"]}
    print(json.dumps(line), flush=True)


def calibrate(ctx, which: str, dev, nfreq: int = 1):
    """Traces N identical copies of one ray: every wave runs converged, so the
    FP64 VALU instruction counters divided by the attempted steps give the
    arithmetic per step without divergence."""
    import torch

    from paper_1601_02063_amd import kgrt as K
    from paper_1601_02063_amd import scenes
    if which.startswith("disk_"):
        w = scenes.thin_disk_image(16)
    elif which.startswith("grid_"):
        w = scenes.grid_image(16, freqs=(230e9,) if nfreq == 1 else scenes.batch_frequencies())
    else:
        w = scenes.torus_image(16, freqs=(230e9,) if nfreq == 1 else scenes.batch_frequencies())
    mod, freqs, integ = K.Model(**w["model"]), list(w["freqs"]), K.Integrator(**w["integ"])
    if "grid" in w:
        mod.grid = torch.from_numpy(w["grid"]).to(dev)
    nrays = 256 * 1024
    ray = torch.tensor(CALIBRATION_RAYS[which], dtype=torch.float64, device=dev)
    rays = ray.repeat(nrays, 1).contiguous()
    out = K.alloc_outputs(nrays, mod, len(freqs), dev, names=("status", "steps", "attempts", "intensity", "tau",
                                                              "r_cross", "g"))
    ctx.trace_rays(rays, mod, freqs, integ, out)
    torch.cuda.synchronize()
    att = out["attempts"]
    assert int(att.min()) == int(att.max()), "copies of one ray must take identical step sequences"
    print(json.dumps({"calibration_ray": which, "nfreq": len(freqs), "ray": CALIBRATION_RAYS[which], "rays": nrays,
                      "status": int(out["status"][0]),
                      "attempts_per_ray": int(att[0]), "steps_per_ray": int(out["steps"][0]),
                      "total_attempts": int(att.to(torch.int64).sum())}), flush=True)


if __name__ == "__main__":
    main()
