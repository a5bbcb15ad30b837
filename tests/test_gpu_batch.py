"""Batched scenes (one plan, many uneven images) on the GPU, through the C ABI.

Each ray is integrated alone, so a batch must reproduce the single-image
traces bit for bit, whatever the launch shape (persistent or one ray per
thread, autotuned), and every hipGraph replay must equal the eager launch.
The full 256-image batch is compared with the oracle on sampled rays.
"""
import numpy as np
import pytest

from paper_1601_02063_amd import scenes
from tests.helpers import kgrt_params, oracle_scene

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_1601_02063_amd import kgrt as K
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = K.Context(0)
    yield c
    c.close()


def uneven_batch(model="torus"):
    shapes = [(17, 13, 0.3, 40.0), (32, 32, 0.9, 17.0), (1, 1, 0.5, 60.0), (0, 0, 0.2, 30.0),
              (40, 25, 0.998, 85.0), (8, 64, 0.0, 5.0)]
    ws = []
    for nx, ny, a, inc in shapes:
        if model == "torus":
            w = scenes.torus_image(max(nx, 1), a, inc, freqs=(86e9, 230e9, 690e9))
        else:
            w = scenes.thin_disk_image(max(nx, 1), a, inc)
        w["camera"]["nx"], w["camera"]["ny"] = nx, ny
        ws.append(w)
    return ws


def host(out):
    return {k: v.cpu().numpy() for k, v in out.items()}


def singles(ctx, ws):
    import torch
    from paper_1601_02063_amd import kgrt as K
    res = []
    for w in ws:
        cam, mod, freqs, integ = kgrt_params(w)
        n = cam.nx * cam.ny
        out = K.alloc_outputs(max(n, 1), mod, len(freqs), ctx.device)
        if n:
            ctx.trace(cam, mod, freqs, integ, out)
        torch.cuda.synchronize()
        res.append({k: v.cpu().numpy()[..., :n] for k, v in out.items()})
    return res


def split(plan, g, names):
    parts = []
    for k in range(len(plan.offsets) - 1):
        lo, hi = plan.offsets[k], plan.offsets[k + 1]
        parts.append({name: g[name][..., lo:hi] for name in names})
    return parts


@pytest.mark.parametrize("model", ["torus", "disk"])
def test_batch_equals_single_images_every_launch_mode(ctx, model):
    import torch
    from paper_1601_02063_amd import kgrt as K
    ws = uneven_batch(model)
    ref = singles(ctx, ws)
    params = [kgrt_params(w) for w in ws]
    _, mod, freqs, integ = params[0]
    plan = K.Plan(ctx, [p[0] for p in params], mod, freqs, integ)
    out = plan.alloc_outputs()
    names = list(out)

    def check(tag):
        torch.cuda.synchronize()
        got = split(plan, host(out), names)
        for k, (gpart, rpart) in enumerate(zip(got, ref)):
            for name in names:
                assert np.array_equal(gpart[name], rpart[name]), (tag, k, name)

    for t in out.values():
        t.fill_(-7)
    plan.launch(out)
    check("eager")
    for rep in range(3):  # graph replays interleaved with unrelated eager work
        for t in out.values():
            t.fill_(-7)
        torch.ones(1 << 20, device=ctx.device).sum()
        plan.launch(out, graph=True)
        check(f"graph replay {rep}")
    best = plan.autotune(out)
    assert best["block"] in (64, 128, 256)
    plan.launch(out, graph=True)
    check("autotuned graph")
    plan.set_launch(mode=K.LAUNCH_ONE_RAY_PER_THREAD)
    plan.launch(out)
    check("one ray per thread")
    plan.close()
    # the one-shot entry point gives the same again
    out2 = plan.alloc_outputs()
    ctx.trace_batch([p[0] for p in params], mod, freqs, integ, out2)
    got = split(plan, host(out2), names)
    for gpart, rpart in zip(got, ref):
        for name in names:
            assert np.array_equal(gpart[name], rpart[name])


def test_full_scene_batch_sampled_against_oracle(ctx):
    """The 256-image batch of uneven scenes at 8 frequencies, in its benchmark launch shape
    (autotuned, graph replay). A seeded 1/64 of every image's pixels is recomputed by the
    oracle: capture flags identical except within 1e-6 M of the critical curve, I_nu and tau_nu
    within 1e-6 on every sampled ray. Rays passing within sin(theta) < 1e-6 of the pole, where
    the clamp of section 2.1 amplifies last-ulp differences, may exceed that bar only in
    bounded number and never beyond 1e-4."""
    import time
    import torch
    import oracle as O
    from paper_1601_02063_amd import kgrt as K
    from tests.helpers import critical_curve_distance
    ws = scenes.batch_scenes(1603)
    params = [kgrt_params(w) for w in ws]
    _, mod, freqs, integ = params[0]
    plan = K.Plan(ctx, [p[0] for p in params], mod, freqs, integ)
    out = plan.alloc_outputs(("status", "steps", "attempts", "intensity", "tau"))
    for t in out.values():
        t.fill_(-7)
    plan.autotune(out)
    plan.launch(out, graph=True)
    torch.cuda.synchronize()
    g = host(out)
    assert not np.any(g["status"] == -7)
    assert np.all((g["status"] & 3) != 0)
    rng = np.random.Generator(np.random.PCG64(5))
    sel, rays = [], []
    for k, w in enumerate(ws):
        cam = w["camera"]
        n = cam["nx"] * cam["ny"]
        idx = np.sort(rng.choice(n, size=n // 64, replace=False))
        xy = O.pixel_points(cam["nx"], cam["ny"], cam["x_min"], cam["x_max"], cam["y_min"], cam["y_max"])[idx]
        rays.append(np.column_stack([np.full(len(idx), cam["a"]), np.full(len(idx), cam["incl_deg"]), xy]))
        sel.append(plan.offsets[k] + idx)
    rays = np.concatenate(rays)
    gi = np.concatenate(sel)
    t0 = time.time()
    o = O.trace_ray_list(oracle_scene(ws[0]), rays)
    print(f"oracle: {len(gi)} sampled rays at 8 frequencies in {time.time() - t0:.1f} s", flush=True)
    st_g = g["status"][gi]
    same = (g["steps"][gi] == o["steps"]) & (g["attempts"][gi] == o["attempts"])
    regular = o["min_sin"] >= 1e-6
    assert same[regular].mean() >= 0.999, same[regular].mean()
    assert np.array_equal(st_g[same], o["status"][same])
    bad = np.nonzero((st_g & 1) != (o["status"] & 1))[0]
    for b in bad:
        xi, eta = o["L"][b] / o["E"][b], o["Q"][b] / o["E"][b] ** 2
        assert critical_curve_distance(rays[b, 0], rays[b, 1], [xi], [eta])[0] < 1e-6, b
    over = np.zeros(len(gi), dtype=bool)
    for f in range(8):
        I_o, I_g = o["I"][:, f], g["intensity"][f, gi]
        scale = max(np.abs(g["intensity"][f]).max(), 1e-300)
        err = np.abs(I_g - I_o) / np.maximum(np.abs(I_o), 1e-12 * scale)
        terr = np.abs(g["tau"][f, gi] - o["tau"][:, f]) / np.maximum(np.abs(o["tau"][:, f]), 1e-30)
        assert np.all(err <= 1e-4) and np.all(terr <= 1e-4), (f, err.max(), terr.max())
        over |= (err > 1e-6) | (terr > 1e-6)
    print(f"batch sample: {len(gi)} rays, identical steps {same.mean():.6f}, near-pole {int((~regular).sum())}, "
          f"over 1e-6 {int(over.sum())}, capture flips {len(bad)}", flush=True)
    assert not np.any(over & regular), np.nonzero(over & regular)[0][:10]
    assert over.sum() <= max(8, len(gi) // 20000), int(over.sum())
    assert (~regular).sum() <= len(gi) // 100
    plan.close()
