"""GPU (HIP, through the C ABI) versus the CPU oracle on the same seeded inputs.

Bars (FP64 integrator): capture classification identical except rays within
1e-6 M of the critical curve in the sky plane; first-crossing radius and
redshift within 1e-9 relative; intensities and optical depths within 1e-6
relative. Both sides run the same algorithm, so the step counts must agree
for nearly every ray; a ray whose accept/reject sequence flipped on a
last-ulp difference is listed and compared at the method's own error
(1e-6) instead.
"""
import numpy as np
import pytest

import oracle as O
from paper_1601_02063_amd import scenes
from tests.helpers import critical_curve_distance, kgrt_params, oracle_scene

pytestmark = pytest.mark.gpu

REL_GEOM = 1e-9
REL_RT = 1e-6


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_1601_02063_amd import kgrt as K
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = K.Context(0)
    yield c
    c.close()


def run_gpu(ctx, w, sentinel=True):
    import torch
    from paper_1601_02063_amd import kgrt as K
    cam, mod, freqs, integ = kgrt_params(w)
    out = K.alloc_outputs(cam.nx * cam.ny, mod, len(freqs), ctx.device)
    if sentinel:
        for k, t in out.items():
            t.fill_(-7)
    ctx.trace(cam, mod, freqs, integ, out)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


def rel(a, b):
    a, b = np.asarray(a, float), np.asarray(b, float)
    den = np.maximum(np.abs(b), 1e-300)
    return np.where((a == b), 0.0, np.abs(a - b) / den)


POLE_SIN = 1e-6  # rays passing closer to the pole run into the clamp sin(theta) >= 1e-8


def compare_disk(w, g, o, label, order_amp=False):
    """Compare GPU outputs g (dict) with oracle rays o (structured, flat).

    Strict set: rays with identical step sequences that neither pass within
    sin(theta) < 1e-6 of the pole (where the pole clamp of section 2.1 breaks the
    Hamiltonian form and amplifies last-ulp differences) nor lie within 1e-6 M of
    the critical curve. On it, disk hits agree to 1e-9 in r_c and g. Every other
    crossing is compared at the method's own accuracy, 1e-6 (g relative to
    max(g, 1e-3): g -> 0 at the photon orbit, where it is ill-conditioned).

    order_amp: the bars of a ray that hits the disk at its n-th crossing are multiplied by
    30^(n - 1) (each half orbit near the photon sphere amplifies a difference by about e^pi)."""
    cam = w["camera"]
    st_o = o["status"]
    st_g = g["status"]
    assert not np.any(st_g == -7), "some ray was never written"
    xi = o["L"] / o["E"]
    eta = o["Q"] / o["E"] ** 2
    dcrit = critical_curve_distance(cam["a"], cam["incl_deg"], xi, eta)
    near_crit = dcrit < 1e-6
    near_pole = o["min_sin"] < POLE_SIN
    ident = (g["steps"] == o["steps"]) & (g["attempts"] == o["attempts"])
    regular = ~near_crit & ~near_pole
    # capture classification
    cap_mismatch = ((st_g & 1) != (st_o & 1)) & ~near_crit
    assert not cap_mismatch.any(), (label, np.nonzero(cap_mismatch)[0][:10])
    # step sequences: identical for (nearly) every regular ray
    frac = ident[regular].mean() if regular.any() else 1.0
    assert frac >= 0.999, (label, frac, np.nonzero(regular & ~ident)[0][:10])
    assert np.array_equal(st_g[ident], st_o[ident]), label
    both = ((st_g & 4) != 0) & ((st_o & 4) != 0)
    disk = both & ((st_o & 8) != 0) & ((st_g & 8) != 0)
    strict = disk & ident & regular
    amp = 30.0 ** np.maximum(o["n_cross"] - 1, 0) if order_amp else np.ones(len(st_o))
    for k in ("r_cross", "g", "t_cross"):
        e = (rel(g[k][strict], o[k][strict]) / amp[strict]).max(initial=0)
        assert e <= REL_GEOM, (label, k, e)
    # phi is an angle with an arbitrary origin (phi_obs = 0): its error in radians, relative to
    # max(|phi|, 1) (a relative error of a crossing near phi = 0 says nothing)
    e = (np.abs(g["phi_cross"][strict] - o["phi_cross"][strict]) / np.maximum(np.abs(o["phi_cross"][strict]), 1.0)
         / amp[strict]).max(initial=0)
    assert e <= REL_GEOM, (label, "phi_cross", e)
    for k in ("intensity", "i_bol"):  # g^3 r^-3 and g^4 r^-3 amplify the geometric error a few times
        e = (rel(g[k][strict], o[k][strict]) / amp[strict]).max(initial=0)
        assert e <= 10 * REL_GEOM, (label, k, e)
    loose = both & ~strict
    assert (rel(g["r_cross"][loose], o["r_cross"][loose]) / amp[loose]).max(initial=0) <= REL_RT, label
    gerr = np.abs(g["g"][loose] - o["g"][loose]) / np.maximum(np.abs(o["g"][loose]), 1e-3) / amp[loose]
    assert gerr.max(initial=0) <= REL_RT, (label, gerr.max(initial=0))
    assert np.array_equal((st_g & 4)[regular], (st_o & 4)[regular]), label
    # intensity on every ray: equal where both hit the disk (the method's accuracy off the
    # strict set), zero where neither does; a disk-hit flip only for a crossing within
    # 1e-6 of a disk edge, where a last-ulp difference moves r_c across it
    hit_g, hit_o = (st_g & 8) != 0, (st_o & 8) != 0
    both_hit = hit_g & hit_o
    for k in ("intensity", "i_bol"):
        e = (rel(g[k][both_hit], o[k][both_hit]) / amp[both_hit]).max(initial=0)
        assert e <= 10 * REL_RT, (label, k, e)
    neither = ~hit_g & ~hit_o
    assert np.all(g["intensity"][neither] == 0.0) and np.all(o["intensity"][neither] == 0.0), label
    flips = np.nonzero(hit_g != hit_o)[0]
    if len(flips):
        r_in = w["model"]["r_in"] if w["model"]["r_in"] > 0 else O.isco(cam["a"])
        rc = o["r_cross"][flips]
        edge = np.minimum(np.abs(rc - r_in), np.abs(rc - w["model"]["r_out"])) <= 1e-6 * rc
        assert edge.all(), (label, flips[~edge][:10])
    assert len(flips) <= max(1, len(st_o) // 10000), (label, len(flips))
    # the near-pole exemption covers few rays (at 1 degree inclination, the 4% of the image
    # around its centre)
    assert near_pole.sum() <= max(4, len(st_o) // 20), (label, int(near_pole.sum()))
    return frac


# ------------------------------------------------------------ thin disk

def test_thin_disk_image_matches_oracle(ctx):
    import oracle as O
    w = scenes.thin_disk_image(64)
    g = run_gpu(ctx, w)
    o = O.trace_image(oracle_scene(w), 64, 64, -15, 15, -15, 15).ravel()
    frac = compare_disk(w, g, o, "thin disk 64^2")
    print(f"thin disk 64^2: identical step sequences {frac:.5f}")
    assert ((g["status"] & 8) != 0).sum() > 2000


@pytest.mark.parametrize("a,incl,n,half", [(0.0, 60.0, 37, 12.0), (0.998, 89.0, 41, 10.0),
                                           (0.5, 1.0, 23, 15.0), (0.9, 30.0, 1, 15.0)])
def test_thin_disk_other_geometries(ctx, a, incl, n, half):
    import oracle as O
    w = scenes.thin_disk_image(n, a, incl, half)
    w["camera"]["ny"] = n + 6 if n > 1 else 1  # ragged, non-square
    w["camera"]["y_max"] = half * 0.9
    g = run_gpu(ctx, w)
    cam = w["camera"]
    o = O.trace_image(oracle_scene(w), cam["nx"], cam["ny"], cam["x_min"], cam["x_max"], cam["y_min"],
                      cam["y_max"]).ravel()
    compare_disk(w, g, o, f"a={a} incl={incl}")


@pytest.mark.parametrize("a,incl,n", [(0.0, 80.0, 64), (0.9, 75.0, 61), (0.998, 85.0, 48)])
def test_disk_images_through_every_crossing(ctx, a, incl, n):
    """The thick disk seen through every equatorial crossing (direct and higher-order images):
    the same bars as the first-crossing disk on the emitting crossing, and the same crossing
    count wherever the step sequences agree."""
    w = scenes.thin_disk_image(n, a, incl, 9.0)
    w["model"]["kind"] = 3
    w["camera"]["ny"] = n - 5
    w["camera"]["y_max"] = 8.0
    g = run_gpu(ctx, w)
    cam = w["camera"]
    o = O.trace_image(oracle_scene(w), cam["nx"], cam["ny"], cam["x_min"], cam["x_max"], cam["y_min"],
                      cam["y_max"]).ravel()
    compare_disk(w, g, o, f"disk images a={a} incl={incl}", order_amp=True)
    ident = (g["steps"] == o["steps"]) & (g["attempts"] == o["attempts"])
    assert np.array_equal(g["n_cross"][ident], o["n_cross"][ident])
    hit = (g["status"] & 8) != 0
    higher = hit & (g["n_cross"] >= 2)
    print(f"disk images a={a} incl={incl}: {int(hit.sum())} disk pixels, {int(higher.sum())} of them "
          f"higher-order, max order {int(g['n_cross'][hit].max()) - 1}", flush=True)
    assert higher.sum() >= 20
    assert not np.any(g["status"][hit] & 3)  # the disk ends the ray


def test_projection_stop_at_crossing(ctx):
    """The timing workload: geometry only, stop at the first equatorial crossing."""
    import oracle as O
    w = scenes.projection_image(32)
    g = run_gpu(ctx, w)
    o = O.trace_image(oracle_scene(w), 32, 32, -15, 15, -15, 15).ravel()
    compare_disk(w, g, o, "projection")
    crossed = (g["status"] & 4) != 0
    assert crossed.sum() > 500
    assert np.all(g["intensity"][crossed] == 0.0)


def test_step_cap_and_empty_image(ctx):
    import oracle as O
    import torch
    from paper_1601_02063_amd import kgrt as K
    w = scenes.thin_disk_image(16)
    w["integ"]["max_steps"] = 40
    g = run_gpu(ctx, w)
    o = O.trace_image(oracle_scene(w), 16, 16, -15, 15, -15, 15).ravel()
    assert np.all((g["status"] & 16) != 0)
    assert np.array_equal(g["status"], o["status"])
    assert np.array_equal(g["steps"], o["steps"])
    # an empty image is a no-op
    cam, mod, freqs, integ = kgrt_params(scenes.thin_disk_image(0))
    out = K.alloc_outputs(1, mod, 0, ctx.device)
    out["status"].fill_(-7)
    ctx.trace(cam, mod, freqs, integ, out)
    torch.cuda.synchronize()
    assert int(out["status"][0]) == -7


def test_step_underflow_matches_oracle(ctx):
    """A capture radius of r_+(1 + 1e-12) lies where the horizon's coordinate singularity drives the
    step below 1e-12 r: every ray the oracle ends in UNDERFLOW ends so on the GPU, never CAPTURED."""
    w = scenes.thin_disk_image(12, 0.9, 60.0, 6.0)
    w["integ"]["horizon_delta"] = 1e-12
    g = run_gpu(ctx, w)
    o = O.trace_image(oracle_scene(w), 12, 12, -6, 6, -6, 6).ravel()
    uf_g, uf_o = (g["status"] & 32) != 0, (o["status"] & 32) != 0
    assert uf_o.sum() >= 40
    assert np.array_equal(uf_g, uf_o)
    assert not np.any(g["status"] & 1)
    assert np.array_equal(g["status"] & ~0x100, o["status"] & ~0x100)
    # the crossings recorded before the ray stalls agree as elsewhere
    both = ((g["status"] & 8) != 0) & ((o["status"] & 8) != 0)
    assert both.sum() > 20
    assert rel(g["r_cross"][both], o["r_cross"][both]).max() <= REL_RT


# ---------------------------------------------------------------- torus

def assert_capture_classification(st_g, o, a, incl_deg, label):
    """Capture flags agree on every ray except within 1e-6 M of the critical curve (sky-plane
    distance from the ray's exact xi, eta); the distance is computed for the disagreeing rays."""
    bad = np.nonzero((st_g & 1) != (o["status"] & 1))[0]
    if len(bad):
        xi = o["L"][bad] / o["E"][bad]
        eta = o["Q"][bad] / o["E"][bad] ** 2
        d = critical_curve_distance(a, incl_deg, xi, eta)
        assert np.all(d < 1e-6), (label, bad[d >= 1e-6][:10], d.max())
    return len(bad)


def compare_torus(g, o, nf, label, cam=None, bar=None):
    """bar: optional per-ray relative bars (arrays [n]) replacing 1e-6 where they are larger."""
    st_o, st_g = o["status"], g["status"]
    bar = REL_RT if bar is None else np.maximum(REL_RT, bar)
    assert not np.any(st_g == -7), "some ray was never written"
    same = (g["steps"] == o["steps"]) & (g["attempts"] == o["attempts"])
    assert same.mean() >= 0.995, (label, same.mean())
    assert np.array_equal(st_g[same], st_o[same])
    if cam is not None:
        assert_capture_classification(st_g, o, cam["a"], cam["incl_deg"], label)
    for f in range(nf):
        I_g, I_o = g["intensity"][f], o["I"][:, f]
        t_g, t_o = g["tau"][f], o["tau"][:, f]
        scale = max(I_o.max(), 1e-300)
        # relative bar, with an absolute floor far below the image's dynamic range
        err = np.abs(I_g - I_o) / np.maximum(np.abs(I_o), 1e-12 * scale)
        assert np.all(err <= bar), (label, f, err.max(), np.argmax(err))
        terr = np.abs(t_g - t_o) / np.maximum(np.abs(t_o), 1e-30)
        assert np.all(terr <= bar), (label, f, terr.max())
    return same.mean()


def test_torus_image_matches_oracle(ctx):
    import oracle as O
    w = scenes.torus_image(48)
    g = run_gpu(ctx, w)
    o = O.trace_image(oracle_scene(w), 48, 48, -20, 20, -20, 20).ravel()
    frac = compare_torus(g, o, 1, "torus 48^2", w["camera"])
    print(f"torus 48^2: identical step sequences {frac:.5f}")
    assert g["intensity"][0].max() > 0


def test_torus_multifrequency_ragged(ctx):
    import oracle as O
    w = scenes.torus_image(19, a=0.5, incl_deg=70.0, freqs=scenes.batch_frequencies())
    w["camera"]["ny"] = 29
    g = run_gpu(ctx, w)
    o = O.trace_image(oracle_scene(w), 19, 29, -20, 20, -20, 20).ravel()
    compare_torus(g, o, 8, "torus 8 freqs", w["camera"])


@pytest.mark.parametrize("nf", [2, 3, 6, 12])
def test_torus_frequency_counts(ctx, nf):
    """Every compiled frequency width (2, 4, 8 and 16 slots, partly filled) against the oracle."""
    import oracle as O
    freqs = [86e9 * (690.0 / 86.0) ** (k / max(nf - 1, 1)) for k in range(nf)]
    w = scenes.torus_image(11, a=0.9, incl_deg=40.0, freqs=freqs)
    w["camera"]["ny"] = 7
    g = run_gpu(ctx, w)
    o = O.trace_image(oracle_scene(w), 11, 7, -20, 20, -20, 20).ravel()
    compare_torus(g, o, nf, f"torus {nf} freqs", w["camera"])


def test_torus_full_resolution_every_pixel(ctx):
    """The benchmark configuration (1024^2 torus at 230 GHz) in its launch shape, every pixel
    recomputed by the oracle: capture flags, I_nu and tau_nu on all 1,048,576 rays."""
    import time
    w = scenes.torus_image(1024)
    g = run_gpu(ctx, w)
    t0 = time.time()
    o = O.trace_image(oracle_scene(w), 1024, 1024, -20, 20, -20, 20).ravel()
    print(f"oracle: 1024^2 torus in {time.time() - t0:.1f} s on {O.default_threads()} threads", flush=True)
    gs = {k: (v.reshape(1, -1) if k in ("intensity", "tau") else v) for k, v in g.items()}
    frac = compare_torus(gs, o, 1, "torus 1024^2", w["camera"])
    print(f"torus 1024^2: identical step sequences {frac:.6f}", flush=True)
    assert np.all((g["status"] & 3) != 0)  # every ray ended by capture or escape


# ------------------------------------------------------------- ray list

def test_ray_list_matches_oracle(ctx):
    import oracle as O
    import torch
    from paper_1601_02063_amd import kgrt as K
    rays = scenes.label_rays(3000, seed=99)
    w = scenes.thin_disk_image(1)
    cam, mod, freqs, integ = kgrt_params(w)
    out = K.alloc_outputs(len(rays), mod, 0, ctx.device)
    for t in out.values():
        t.fill_(-7)
    ctx.trace_rays(torch.from_numpy(rays).to(ctx.device), mod, freqs, integ, out)
    torch.cuda.synchronize()
    g = {k: v.cpu().numpy() for k, v in out.items()}
    o = O.trace_ray_list(oracle_scene(w), rays)
    assert not np.any(g["status"] == -7)
    regular = o["min_sin"] >= POLE_SIN
    ident = (g["steps"] == o["steps"]) & (g["attempts"] == o["attempts"])
    assert ident[regular].mean() >= 0.999
    assert np.array_equal(g["status"][ident], o["status"][ident])
    strict = ((g["status"] & 8) != 0) & ((o["status"] & 8) != 0) & ident & regular
    assert strict.sum() > 500
    for k in ("r_cross", "g", "phi_cross"):
        assert rel(g[k][strict], o[k][strict]).max() <= REL_GEOM, k
    crossed = ((g["status"] & 4) != 0) & ((o["status"] & 4) != 0)
    assert rel(g["r_cross"][crossed], o["r_cross"][crossed]).max() <= REL_RT


def test_ray_list_invalid_rays_flagged(ctx):
    import torch
    from paper_1601_02063_amd import kgrt as K
    rays = torch.tensor([[1.2, 60.0, 1.0, 1.0], [0.5, 0.0, 1.0, 1.0], [0.5, 60.0, float("nan"), 1.0],
                         [0.5, 60.0, 3.0, 2.0]], dtype=torch.float64, device=ctx.device)
    mod = K.Model(kind=K.MODEL_THIN_DISK)
    out = K.alloc_outputs(4, mod, 0, ctx.device)
    ctx.trace_rays(rays, mod, [], K.Integrator(), out)
    torch.cuda.synchronize()
    st = out["status"].cpu().numpy()
    assert list(st[:3]) == [64, 64, 64]
    assert st[3] & 3


# ------------------------------------------------------------ scheduler

def test_results_independent_of_launch_shape(ctx):
    """Each ray is computed alone, so the outputs are bitwise identical for any
    block size, residency or refill granularity, and every ray is written once."""
    w = scenes.torus_image(40, a=0.9, incl_deg=50.0)
    ref = run_gpu(ctx, w)
    try:
        for block, per_cu, refill in [(64, 1, 1), (128, 2, 8), (256, 1, 32), (256, 0, 64)]:
            ctx.set_launch(block, per_cu, refill)
            g = run_gpu(ctx, w)
            for k in ref:
                assert np.array_equal(g[k], ref[k]), (block, per_cu, refill, k)
    finally:
        ctx.set_launch()


def test_eight_frequency_results_independent_of_launch_shape(ctx):
    """The eight-frequency kernel keeps each thread's sums in LDS slots indexed by
    the block size: every block size and residency gives bitwise identical outputs,
    and they match the oracle."""
    import oracle as O
    w = scenes.torus_image(24, a=0.7, incl_deg=35.0, freqs=scenes.batch_frequencies())
    w["camera"]["ny"] = 17
    ref = run_gpu(ctx, w)
    o = O.trace_image(oracle_scene(w), 24, 17, -20, 20, -20, 20).ravel()
    compare_torus(ref, o, 8, "torus 8 freqs, default launch", w["camera"])
    try:
        for block, per_cu, refill in [(64, 0, 1), (64, 3, 4), (128, 0, 8), (128, 1, 1), (256, 2, 16)]:
            ctx.set_launch(block, per_cu, refill)
            g = run_gpu(ctx, w)
            for k in ref:
                assert np.array_equal(g[k], ref[k]), (block, per_cu, refill, k)
    finally:
        ctx.set_launch()