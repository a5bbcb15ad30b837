"""Spectra (flux density per image and frequency, section 4) on the GPU against
the oracle: the reduction on seeded intensities of uneven images (empty, one
pixel, ragged, the largest batch image), its repeatability, the clamping of
image ranges, and end to end on a small torus batch traced by both sides."""
import numpy as np
import pytest

from paper_1601_02063_amd import scenes
from tests.helpers import kgrt_params, oracle_scene

pytestmark = pytest.mark.gpu

# Positive terms: the GPU's strided partial sums and fixed tree (at most ~2e3
# additions deep for 2^18 terms) stay within a few hundred ulps of the exactly
# rounded sum.
REL_SUM = 1e-12


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_1601_02063_amd import kgrt as K
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = K.Context(0)
    yield c
    c.close()


def dev(a, dtype):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype).cuda()


@pytest.mark.parametrize("nfreq", [1, 3, 8])
def test_spectra_match_oracle(ctx, nfreq):
    import torch
    from oracle import spectra as S
    from paper_1601_02063_amd import kgrt as K
    rng = np.random.Generator(np.random.PCG64(1606 + nfreq))
    sizes = [0, 1, 37, 4096, 512 * 512, 5, 2049, 0, 64 * 64]
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    total = int(off[-1])
    # intensities spanning several decades, as a torus image does
    I = rng.uniform(0.0, 1.0, (nfreq, total)) * 10.0 ** rng.uniform(-6, 0, (nfreq, total))
    dom = rng.uniform(0.5, 2.0, len(sizes)) * 1e-22
    print(f"spectra nfreq={nfreq} total={total}", flush=True)
    F = K.image_spectra(dev(I, torch.float64), dev(off, torch.int64), dev(dom, torch.float64))
    torch.cuda.synchronize()
    got = F.cpu().numpy()
    want = S.image_spectra(I, off, dom)
    assert got.shape == (len(sizes), nfreq)
    assert np.all(got[np.array(sizes) == 0] == 0.0)
    nz = want != 0
    assert np.max(np.abs(got[nz] - want[nz]) / want[nz]) <= REL_SUM
    # same launch, same order of additions: bitwise repeatable
    F2 = K.image_spectra(dev(I, torch.float64), dev(off, torch.int64), dev(dom, torch.float64))
    torch.cuda.synchronize()
    assert np.array_equal(F2.cpu().numpy(), got)


def test_spectra_clamp_image_ranges(ctx):
    """Ranges outside [0, total] are clamped on the device; reversed ranges sum to 0."""
    import torch
    from oracle import spectra as S
    from paper_1601_02063_amd import kgrt as K
    rng = np.random.Generator(np.random.PCG64(1607))
    total = 3000
    I = rng.uniform(0.0, 1.0, (2, total))
    off = np.array([-50, 10, 10, 2500, 1000, total + 4096], dtype=np.int64)
    dom = np.ones(5)
    print("spectra clamp", flush=True)
    got = K.image_spectra(dev(I, torch.float64), dev(off, torch.int64), dev(dom, torch.float64)).cpu().numpy()
    lo = np.clip(off[:-1], 0, total)
    hi = np.clip(off[1:], 0, total)
    hi = np.maximum(hi, lo)
    want = np.stack([S.image_spectra(I, [a, b], [1.0])[0] for a, b in zip(lo, hi)])
    assert np.allclose(got, want, rtol=REL_SUM, atol=0.0)
    assert np.all(got[3] == 0.0)  # reversed range 2500 -> 1000


def test_torus_batch_spectra_match_oracle(ctx):
    """A small uneven torus batch at three frequencies: GPU plan + GPU spectra against
    oracle images + oracle spectra, to the intensity bar of the integrator (1e-6)."""
    import torch
    import oracle as O
    from oracle import spectra as S
    from paper_1601_02063_amd import kgrt as K
    freqs = [86e9, 230e9, 690e9]
    ws = [scenes.torus_image(12, a=0.5, incl_deg=30.0, freqs=freqs), scenes.torus_image(7, a=0.9, incl_deg=75.0,
                                                                                       freqs=freqs)]
    ws[0]["camera"]["ny"] = 9
    ws.insert(1, scenes.torus_image(0, a=0.2, incl_deg=50.0, freqs=freqs))
    cams = [kgrt_params(w)[0] for w in ws]
    _, mod, _, integ = kgrt_params(ws[0])
    plan = K.Plan(ctx, cams, mod, freqs, integ)
    out = plan.alloc_outputs(["status", "intensity"])
    print("spectra torus batch", flush=True)
    plan.launch(out)
    mbh, dist = mod.mbh_msun, 2.4687e22  # 8 kpc
    dom_h = [K.pixel_solid_angle(c, mbh, dist) if c.nx * c.ny else 0.0 for c in cams]
    F = plan.spectra(out["intensity"], dev(dom_h, torch.float64))
    torch.cuda.synchronize()
    got = F.cpu().numpy()
    plan.close()
    I_o, off = [], [0]
    for w in ws:
        cm = w["camera"]
        n = cm["nx"] * cm["ny"]
        if n:
            o = O.trace_image(oracle_scene(w), cm["nx"], cm["ny"], cm["x_min"], cm["x_max"], cm["y_min"],
                              cm["y_max"]).ravel()
            I_o.append(o["I"][:, :len(freqs)].T)  # the oracle returns 16 frequency slots
        off.append(off[-1] + n)
    I_o = np.concatenate(I_o, axis=1)
    dom_o = [S.pixel_solid_angle(w["camera"]["nx"], w["camera"]["ny"], w["camera"]["x_min"], w["camera"]["x_max"],
                                 w["camera"]["y_min"], w["camera"]["y_max"], mbh, dist)
             if w["camera"]["nx"] * w["camera"]["ny"] else 0.0 for w in ws]
    want = S.image_spectra(I_o, off, dom_o)
    assert np.all(got[1] == 0.0)
    nz = want != 0
    assert nz.sum() == 6
    assert np.max(np.abs(got[nz] - want[nz]) / want[nz]) <= 1e-6


def test_novikov_thorne_disk_spectrum(ctx):
    """The Novikov-Thorne disk spectrum (section 4.3, Eq. (35)) of traced thin-disk images: the GPU
    reduction against the exact-sum oracle on the same per-pixel (r_c, g), then end to end
    against the oracle's own traced images (whose r_c and g agree with the GPU's to the parity
    bars, so the flux densities agree to 1e-6)."""
    import torch
    import oracle as O
    from oracle import spectra as S
    from paper_1601_02063_amd import kgrt as K
    ws = [scenes.thin_disk_image(48, a, inc, 25.0) for a, inc in ((0.999, 85.0), (0.5, 40.0), (0.0, 70.0))]
    for w in ws:
        w["model"]["r_out"] = 50.0
    cams = [K.Camera(**w["camera"]) for w in ws]
    mod, integ = K.Model(**ws[0]["model"]), K.Integrator(**ws[0]["integ"])
    plan = K.Plan(ctx, cams, mod, [], integ)
    out = plan.alloc_outputs(("status", "steps", "attempts", "r_cross", "g"))
    plan.launch(out)
    offs = torch.tensor(plan.offsets, dtype=torch.int64, device=ctx.device)
    mbh, mdot, D = 10.0, 1e19, 10 * 3.0857e21
    dom = torch.tensor([K.pixel_solid_angle(c, mbh, D) for c in cams], dtype=torch.float64, device=ctx.device)
    spin = torch.tensor([c.a for c in cams], dtype=torch.float64, device=ctx.device)
    freqs = list(np.geomspace(1e15, 3e18, 24))  # 4 eV .. 12 keV
    F = K.disk_spectrum(out["r_cross"], out["g"], out["status"], offs, dom, spin, mbh, mdot, freqs)
    F2 = K.disk_spectrum(out["r_cross"], out["g"], out["status"], offs, dom, spin, mbh, mdot, freqs)
    torch.cuda.synchronize()
    F, F2 = F.cpu().numpy(), F2.cpu().numpy()
    assert np.array_equal(F, F2)
    g = {k: v.cpu().numpy() for k, v in out.items()}
    hit = (g["status"] & 8) != 0
    ref = S.disk_spectrum(g["r_cross"], g["g"], hit, plan.offsets, dom.cpu().numpy(), freqs,
                          [c.a for c in cams], mbh, mdot)
    assert np.all(ref[:, :12] > 0)
    np.testing.assert_allclose(F, ref, rtol=1e-11, atol=1e-300)
    # end to end: the oracle's images
    for k, w in enumerate(ws):
        cam = w["camera"]
        o = O.trace_image(oracle_scene(w), cam["nx"], cam["ny"], cam["x_min"], cam["x_max"], cam["y_min"],
                          cam["y_max"]).ravel()
        Fo = S.disk_spectrum(o["r_cross"], o["g"], (o["status"] & 8) != 0, [0, len(o)], [float(dom[k])], freqs,
                             [cam["a"]], mbh, mdot)[0]
        big = Fo > 1e-6 * Fo.max()  # the Wien tail beyond the hottest pixel is all rounding
        np.testing.assert_allclose(F[k][big], Fo[big], rtol=1e-6)
    plan.close()


def test_novikov_thorne_spectrum_rejects_bad_arguments(ctx):
    import torch
    from paper_1601_02063_amd import kgrt as K
    z = torch.zeros(4, dtype=torch.float64, device=ctx.device)
    st = torch.zeros(4, dtype=torch.int32, device=ctx.device)
    offs = torch.tensor([0, 4], dtype=torch.int64, device=ctx.device)
    one = torch.ones(1, dtype=torch.float64, device=ctx.device)
    for args in (dict(mbh_msun=-1.0, mdot_gs=1e19, freqs=[1e17]), dict(mbh_msun=10.0, mdot_gs=1e19, freqs=[]),
                 dict(mbh_msun=10.0, mdot_gs=1e19, freqs=[1e17] * 33),
                 dict(mbh_msun=10.0, mdot_gs=float("nan"), freqs=[1e17])):
        with pytest.raises(K.KgrtError):
            K.disk_spectrum(z, z, st, offs, one, one, args["mbh_msun"], args["mdot_gs"], args["freqs"])
