"""Surrogate render with fallback (through the C ABI): mechanics and consistency.

With every ray sent to the fallback the render reproduces the integrator's
images; with the default policy, fallback pixels carry integrator values,
the rest follow the decode rule applied to the network's own outputs (the
Keplerian g of section 4.3 at the predicted radius, from the oracle), and the
per-image flux and fallback counts agree with the images."""
import numpy as np
import pytest

from paper_1601_02063_amd import scenes
from tests.helpers import oracle_scene

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def setup():
    import torch
    from paper_1601_02063_amd import kgrt as K
    from paper_1601_02063_amd import surrogate as S
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ctx = K.Context(0)
    ws = scenes.render_scenes(77, nimg=3, n=96)
    ws[1]["camera"]["nx"], ws[1]["camera"]["ny"] = 80, 112  # ragged
    cams = [K.Camera(**w["camera"]) for w in ws]
    mod, integ = K.Model(**ws[0]["model"]), K.Integrator(**ws[0]["integ"])
    # a briefly trained network (its accuracy is not under test here)
    rays, x, t, _ = S.label_dataset(ctx, 1 << 16, 5)
    mlp = K.Mlp(ctx, 8192)
    mlp.set_params(S.init_params(3))
    S.train(ctx, mlp, x, t, x[:4096], t[:4096], epochs=4, batch=8192)
    plan = K.Plan(ctx, cams, mod, [], integ)
    ref = plan.alloc_outputs(("status", "intensity"))
    plan.launch(ref)
    torch.cuda.synchronize()
    yield ctx, mlp, cams, mod, integ, plan, {k: v.cpu().numpy() for k, v in ref.items()}
    plan.close()
    mlp.close()
    ctx.close()


def test_all_fallback_reproduces_integrator(setup):
    import torch
    from paper_1601_02063_amd import kgrt as K
    ctx, mlp, cams, mod, integ, plan, ref = setup
    out = K.surrogate_render(ctx, mlp, cams, mod, integ, fallback=(0.0, 1.0, 0.0, 0.0))
    torch.cuda.synchronize()
    I, st = out["intensity"].cpu().numpy(), out["status"].cpu().numpy()
    assert np.all(st & K.FALLBACK)
    err = np.abs(I - ref["intensity"]) / np.maximum(np.abs(ref["intensity"]), 1e-300)
    assert np.all((I == ref["intensity"]) | (err <= 1e-9))
    assert np.array_equal(st & 3, ref["status"] & 3)
    assert list(out["fallback"].cpu().numpy()) == [c.nx * c.ny for c in cams]
    # one image alone (its ray list starts at pixel 0 of the output)
    lo, hi = plan.offsets[1], plan.offsets[2]
    one = K.surrogate_render(ctx, mlp, cams[1:2], mod, integ, fallback=(0.0, 1.0, 0.0, 0.0))
    torch.cuda.synchronize()
    assert np.array_equal(one["intensity"].cpu().numpy(), I[lo:hi])
    assert np.array_equal(one["status"].cpu().numpy(), st[lo:hi])


def test_default_policy_consistency(setup):
    import torch
    import oracle as O
    from paper_1601_02063_amd import kgrt as K
    ctx, mlp, cams, mod, integ, plan, ref = setup
    # a policy that splits this (briefly trained) network's rays into both paths
    for policy in ((0.05, 0.95, 0.5, 0.25, 0.05, 3.0), (0.3, 0.7, 0.25, 0.1, 0.1, 6.0), (0.49, 0.51, 0.0, 0.0, 0.0, 0.0)):
        out = K.surrogate_render(ctx, mlp, cams, mod, integ, fallback=policy)
        torch.cuda.synchronize()
        I, st = out["intensity"].cpu().numpy(), out["status"].cpu().numpy()
        fb = (st & K.FALLBACK) != 0
        if 0 < fb.sum() < len(fb):
            break
    assert 0 < fb.sum() < len(fb)
    p_lo, p_hi, crit, edge, g_tol, grad_max = policy
    err = np.abs(I - ref["intensity"]) / np.maximum(np.abs(ref["intensity"]), 1e-300)
    assert np.all((I[fb] == ref["intensity"][fb]) | (err[fb] <= 1e-9))
    # non-fallback pixels: decode rule on the network's own outputs
    off = plan.offsets
    for k, cam in enumerate(cams):
        lo, hi = off[k], off[k + 1]
        xy = np.stack(np.meshgrid(cam.x_min + (np.arange(cam.nx) + 0.5) * (cam.x_max - cam.x_min) / cam.nx,
                                  cam.y_min + (np.arange(cam.ny) + 0.5) * (cam.y_max - cam.y_min) / cam.ny), -1)
        xy = xy.reshape(-1, 2)
        feat = np.stack([np.full(len(xy), cam.a), np.full(len(xy), np.cos(np.radians(cam.incl_deg))),
                         xy[:, 0] / 15, xy[:, 1] / 15], 1).astype(np.float32)
        y = mlp.forward(torch.from_numpy(feat).to(ctx.device)).cpu().numpy()
        pcap = 1 / (1 + np.exp(-y[:, 0].astype(np.float64)))
        rc = np.exp(y[:, 1].astype(np.float64))
        g = y[:, 2].astype(np.float64)
        z1 = 1 + np.cbrt(1 - cam.a ** 2) * (np.cbrt(1 + cam.a) + np.cbrt(1 - cam.a))
        rin = 3 + np.sqrt(3 * cam.a ** 2 + z1 ** 2) - np.sqrt((3 - z1) * (3 + z1 + 2 * np.sqrt(3 * cam.a ** 2 + z1 ** 2)))
        nf = ~fb[lo:hi]
        # every kept ray is outside the probability and edge bands (small float slack)
        assert np.all((pcap[nf] < p_lo + 1e-5) | (pcap[nf] > p_hi - 1e-5))
        assert np.all(np.abs(rc[nf] - rin) > edge - 1e-4) and np.all(np.abs(rc[nf] - 20.0) > edge - 1e-4)
        # the critical-curve band, from the host table: kept rays lie outside it, and rays
        # that only it can explain lie inside it
        tab = K.critical_curve(cam.a, cam.incl_deg).astype(np.float64)
        nb = len(tab)
        u = (np.arctan2(xy[:, 1], xy[:, 0]) + np.pi) * (nb / (2 * np.pi)) - 0.5
        j0 = np.floor(u).astype(np.int64)
        w = u - j0
        j0 %= nb
        Rc = (1 - w) * tab[j0] + w * tab[(j0 + 1) % nb]
        dcrit = np.abs(np.hypot(xy[:, 0], xy[:, 1]) - Rc)
        assert np.all(dcrit[nf] > crit - 1e-3)
        others = ((pcap >= p_lo - 1e-5) & (pcap <= p_hi + 1e-5)) | (np.abs(rc - rin) < edge + 1e-4) | \
            (np.abs(rc - 20.0) < edge + 1e-4) | ~np.isfinite(y[:, :3]).all(1)
        if g_tol > 0:
            others |= (rc >= rin - edge - 1e-4) & (rc <= 20.0 + edge + 1e-4)  # the g check may apply
        if grad_max > 0:
            # steepest change of the predicted ln r_c toward a 4-neighbour, one of the pair near the disk
            lr_ = y[:, 1].astype(np.float64).reshape(cam.ny, cam.nx)
            lo_r, hi_r = np.log(max(rin - edge, 1e-3)), np.log(20.0 + edge)
            near = (lr_ >= lo_r) & (lr_ <= hi_r)
            grad = np.zeros_like(lr_)
            for ax, pitch in ((1, (cam.x_max - cam.x_min) / cam.nx), (0, (cam.y_max - cam.y_min) / cam.ny)):
                dd = np.abs(np.diff(lr_, axis=ax)) / pitch
                nn = near[:, 1:] | near[:, :-1] if ax == 1 else near[1:, :] | near[:-1, :]
                dd = np.where(nn, dd, 0.0)
                if ax == 1:
                    grad[:, 1:] = np.maximum(grad[:, 1:], dd)
                    grad[:, :-1] = np.maximum(grad[:, :-1], dd)
                else:
                    grad[1:, :] = np.maximum(grad[1:, :], dd)
                    grad[:-1, :] = np.maximum(grad[:-1, :], dd)
            grad = grad.ravel()
            assert np.all(grad[nf] <= grad_max * (1 + 1e-4) + 1e-3)
            others |= grad >= grad_max * (1 - 1e-4) - 1e-3
        only_crit = fb[lo:hi] & ~others
        assert np.all(dcrit[only_crit] < crit + 1e-3)
        # Keplerian g at the predicted radius for kept rays near the disk (oracle: xi = L/E)
        sc = oracle_scene(dict(camera=dict(a=cam.a, incl_deg=cam.incl_deg, phi_obs_deg=cam.phi_obs_deg,
                                           r_obs=cam.r_obs), model=scenes.THIN_DISK, freqs=[],
                               integ=scenes.thin_disk_image()["integ"]))
        gk = np.zeros(len(rc))
        near = nf & (rc >= rin - edge) & (rc <= 20.0 + edge)
        for q in np.flatnonzero(near):
            ok, _, c4 = O.initial_state(sc, float(xy[q, 0]), float(xy[q, 1]))
            assert ok
            gk[q] = O.redshift(sc, float(rc[q]), np.pi / 2, c4[1] / c4[0])
        if g_tol > 0:
            assert np.all(np.abs(gk[near] - g[near]) <= g_tol + 1e-4)
        want = np.where((rc >= rin) & (rc <= 20.0) & (gk > 0), gk ** 3 / rc ** 3, 0.0)
        np.testing.assert_allclose(I[lo:hi][nf], want[nf], rtol=2e-5, atol=1e-12)
        assert abs(float(out["flux"][k]) - I[lo:hi].sum()) <= 1e-9 * max(abs(I[lo:hi].sum()), 1e-30)
        assert int(out["fallback"][k]) == int(fb[lo:hi].sum())
