"""The surrogate network's GPU kernels versus the FP64 reference network.

The GPU runs the three 256x256 layers in BF16 with FP32 accumulation, so it is
compared with the reference evaluated on the same BF16-rounded weights and
inputs, within 2e-2 relative (Frobenius norm per output column or per
parameter tensor).
"""
import numpy as np
import pytest

import oracle.mlp as M

pytestmark = pytest.mark.gpu

REL = 2e-2


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_1601_02063_amd import kgrt as K
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = K.Context(0)
    yield c
    c.close()


def bf16_round(a):
    import torch
    return torch.from_numpy(np.asarray(a, dtype=np.float32)).to(torch.bfloat16).to(torch.float32).numpy()


def reference_params(seed):
    """Initial parameters with W2..W4 rounded to BF16 (what the GPU multiplies with)."""
    p = M.init_params(seed).astype(np.float32)
    offs = np.cumsum([0] + [i * o + o for i, o in M.LAYERS])
    for li in (1, 2, 3):
        i, o = M.LAYERS[li]
        p[offs[li]:offs[li] + i * o] = bf16_round(p[offs[li]:offs[li] + i * o])
    return p


def rel_fro(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)


def test_forward_matches_reference(ctx):
    import torch
    from paper_1601_02063_amd import kgrt as K
    p = reference_params(11)
    rng = np.random.Generator(np.random.PCG64(2))
    x = rng.uniform(-1, 1, size=(1000, 4)).astype(np.float32)  # not a multiple of 16: ragged tail
    mlp = K.Mlp(ctx, max_batch=512)  # several chunks
    mlp.set_params(p)
    xd = torch.from_numpy(x).to(ctx.device)
    y = mlp.forward(xd).cpu().numpy()
    ref, _ = M.forward(p.astype(np.float64), x.astype(np.float64))
    for j in range(5):
        assert rel_fro(y[:, j], ref[:, j]) <= REL, (j, rel_fro(y[:, j], ref[:, j]))
    # rows are independent: a prefix evaluated alone gives the same bits
    y2 = mlp.forward(xd[:300].contiguous()).cpu().numpy()
    assert np.array_equal(y2, y[:300])
    # a single row and a tile that is mostly empty
    for m in (1, 17):
        assert np.array_equal(mlp.forward(xd[:m].contiguous()).cpu().numpy(), y[:m])
    assert np.array_equal(mlp.get_params(), p)
    mlp.close()


@pytest.mark.parametrize("n", [512, 12832])
def test_gradients_match_reference(ctx, n):
    """A gathered batch against the FP64 reference; n = 12832 is 101 blocks of 128 rows, the last
    one of 32 rows (two tiles), and a half-filled last 64-row step of the weight-gradient products."""
    import torch
    from paper_1601_02063_amd import kgrt as K
    p = reference_params(5)
    rng = np.random.Generator(np.random.PCG64(8))
    x = rng.uniform(-1, 1, size=(n + 100, 4)).astype(np.float32)
    t = np.zeros((n + 100, 6), dtype=np.float32)
    t[:, 0] = rng.integers(0, 2, n + 100)
    t[:, 1:5] = rng.normal(size=(n + 100, 4))
    t[:, 5] = rng.integers(0, 2, n + 100)
    idx = rng.permutation(n + 100)[:n].astype(np.int32)  # gathered batch
    mlp = K.Mlp(ctx, max_batch=max(1024, n))
    mlp.set_params(p)
    loss, g = mlp.loss_grads(torch.from_numpy(x).to(ctx.device), torch.from_numpy(t).to(ctx.device),
                             torch.from_numpy(idx).to(ctx.device))
    torch.cuda.synchronize()
    lref, gref = M.loss_and_grads(p.astype(np.float64), x[idx].astype(np.float64), t[idx].astype(np.float64))
    assert abs(float(loss) - lref) <= REL * abs(lref)
    g = g.cpu().numpy()
    k = 0
    for li, (i, o) in enumerate(M.LAYERS):
        for name, size in (("W", i * o), ("b", o)):
            e = rel_fro(g[k:k + size], gref[k:k + size])
            assert e <= REL, (li + 1, name, e)
            k += size
    mlp.close()


def test_gradients_partial_tile_no_gather(ctx):
    """n = 96 rows: one whole 64-row tile and half of another, no index gather."""
    import torch
    from paper_1601_02063_amd import kgrt as K
    p = reference_params(9)
    rng = np.random.Generator(np.random.PCG64(12))
    n = 96
    x = rng.uniform(-1, 1, size=(n, 4)).astype(np.float32)
    t = np.zeros((n, 6), dtype=np.float32)
    t[:, 0] = rng.integers(0, 2, n)
    t[:, 1:5] = rng.normal(size=(n, 4))
    t[:, 5] = rng.integers(0, 2, n)
    mlp = K.Mlp(ctx, max_batch=112)  # not a multiple of 64 either
    mlp.set_params(p)
    loss, g = mlp.loss_grads(torch.from_numpy(x).to(ctx.device), torch.from_numpy(t).to(ctx.device))
    torch.cuda.synchronize()
    lref, gref = M.loss_and_grads(p.astype(np.float64), x.astype(np.float64), t.astype(np.float64))
    assert abs(float(loss) - lref) <= REL * abs(lref)
    g = g.cpu().numpy()
    k = 0
    for li, (i, o) in enumerate(M.LAYERS):
        for name, size in (("W", i * o), ("b", o)):
            e = rel_fro(g[k:k + size], gref[k:k + size])
            assert e <= REL, (li + 1, name, e)
            k += size
    mlp.close()


def test_features_and_targets_kernels(ctx):
    import torch
    from paper_1601_02063_amd import kgrt as K
    from paper_1601_02063_amd import scenes
    rays = scenes.label_rays(2000, seed=31)
    rd = torch.from_numpy(rays).to(ctx.device)
    f = K.surrogate_features(rd).cpu().numpy()
    want = np.stack([rays[:, 0], np.cos(np.radians(rays[:, 1])), rays[:, 2] / 15, rays[:, 3] / 15], 1)
    np.testing.assert_allclose(f, want.astype(np.float32), rtol=1e-6, atol=1e-7)
    mod = K.Model(kind=K.MODEL_THIN_DISK)
    out = K.alloc_outputs(len(rays), mod, 0, ctx.device)
    ctx.trace_rays(rd, mod, [], K.Integrator(), out)
    t = K.surrogate_targets(rd, out).cpu().numpy()
    st = out["status"].cpu().numpy()
    crossed = (st & K.CROSSED) != 0
    rplus = 1 + np.sqrt(1 - rays[:, 0] ** 2)
    np.testing.assert_array_equal(t[:, 0], ((st & K.CAPTURED) != 0).astype(np.float32))
    np.testing.assert_array_equal(t[:, 5], crossed.astype(np.float32))
    rc = out["r_cross"].cpu().numpy()
    np.testing.assert_allclose(t[:, 1], np.log(np.where(crossed, rc, rplus)).astype(np.float32), rtol=1e-6)
    np.testing.assert_allclose(t[crossed, 2], out["g"].cpu().numpy()[crossed].astype(np.float32), rtol=1e-6)
    assert np.all(t[~crossed, 2] == 0)


def test_training_reduces_loss(ctx):
    import torch
    from paper_1601_02063_amd import kgrt as K
    from paper_1601_02063_amd import scenes
    rays = torch.from_numpy(scenes.label_rays(16384, seed=41)).to(ctx.device)
    mod = K.Model(kind=K.MODEL_THIN_DISK)
    out = K.alloc_outputs(rays.shape[0], mod, 0, ctx.device)
    ctx.trace_rays(rays, mod, [], K.Integrator(), out)
    x = K.surrogate_features(rays)
    t = K.surrogate_targets(rays, out)
    mlp = K.Mlp(ctx, max_batch=4096)
    mlp.set_params(M.init_params(1))
    loss = torch.zeros(1, dtype=torch.float32, device=ctx.device)
    gen = torch.Generator(device="cpu").manual_seed(0)
    losses = []
    for step in range(120):
        idx = torch.randperm(rays.shape[0], generator=gen)[:4096].to(torch.int32).to(ctx.device)
        mlp.train_step(x, t, idx, 4096, 1e-3, loss)
        if step % 20 == 0 or step == 119:
            losses.append(float(loss))
    assert all(np.isfinite(losses))
    assert losses[-1] < 0.1 * losses[0], losses
    mlp.close()


def _bf16_activation_bound(p, x):
    """Per-element bound on the outputs' deviation caused by rounding the hidden activations
    h_1..h_3 (the inputs of the three 256x256 layers) to BF16: first-order propagation of a
    relative error of 2^-8 (twice BF16's unit roundoff, for the second-order terms and the
    kernel's SiLU approximations) on every activation, |dy_i| <= 2^-8 sum_l,k |dy_i/dh_lk| |h_lk|."""
    layers = M.unpack(p.astype(np.float64))
    _, (hs, zs) = M.forward(p.astype(np.float64), x.astype(np.float64))
    n = x.shape[0]
    bound = np.zeros((n, 5))
    for i in range(5):
        dh = np.tile(layers[4][0][i], (n, 1))          # dy_i/dh_4
        for l in (4, 3, 2):                              # to dy_i/dh_{l-1} through layer l
            dz = dh * M.silu_grad(zs[l - 1])
            dh = dz @ layers[l - 1][0]
            bound[:, i] += np.sum(np.abs(dh) * np.abs(hs[l - 1]), axis=1)
    return 2.0 ** -8 * bound


def test_forward_elementwise_within_bf16_bound(ctx):
    """Every output element of the fused inference kernel lies within the first-order BF16 bound
    of the reference evaluated on the same BF16 weights (plus a floor of 1e-4 of the column's
    RMS for the FP32 input layer and head), on a ragged 1000-row batch."""
    import torch
    from paper_1601_02063_amd import kgrt as K
    p = reference_params(13)
    rng = np.random.Generator(np.random.PCG64(4))
    x = rng.uniform(-1, 1, size=(1000, 4)).astype(np.float32)
    mlp = K.Mlp(ctx, max_batch=1024)
    mlp.set_params(p)
    y = mlp.forward(torch.from_numpy(x).to(ctx.device)).cpu().numpy().astype(np.float64)
    ref, _ = M.forward(p.astype(np.float64), x.astype(np.float64))
    bound = _bf16_activation_bound(p, x) + 1e-4 * np.sqrt(np.mean(ref ** 2, axis=0))
    excess = np.abs(y - ref) / bound
    print(f"forward: max |dy|/bound {excess.max():.3f}, median {np.median(excess):.4f}", flush=True)
    assert np.all(excess <= 1.0), (np.unravel_index(np.argmax(excess), excess.shape), excess.max())
    mlp.close()


def test_gradients_match_reference_at_production_batch(ctx):
    """The training batch of the surrogate (65536 gathered rows, so the weight gradients are
    summed over all 64 split-K chunks of 1024 rows) against the FP64 reference on the same BF16
    weights: loss and every parameter tensor within 2e-2 (Frobenius)."""
    import torch
    from paper_1601_02063_amd import kgrt as K
    p = reference_params(17)
    rng = np.random.Generator(np.random.PCG64(18))
    n, pool = 65536, 70000
    x = rng.uniform(-1, 1, size=(pool, 4)).astype(np.float32)
    t = np.zeros((pool, 6), dtype=np.float32)
    t[:, 0] = rng.integers(0, 2, pool)
    t[:, 1:5] = rng.normal(size=(pool, 4))
    t[:, 5] = rng.integers(0, 2, pool)
    idx = rng.permutation(pool)[:n].astype(np.int32)
    mlp = K.Mlp(ctx, max_batch=n)
    mlp.set_params(p)
    loss, g = mlp.loss_grads(torch.from_numpy(x).to(ctx.device), torch.from_numpy(t).to(ctx.device),
                             torch.from_numpy(idx).to(ctx.device))
    torch.cuda.synchronize()
    lref, gref = M.loss_and_grads(p.astype(np.float64), x[idx].astype(np.float64), t[idx].astype(np.float64))
    assert abs(float(loss) - lref) <= REL * abs(lref)
    g = g.cpu().numpy()
    k = 0
    worst = 0.0
    for li, (i, o) in enumerate(M.LAYERS):
        for name, size in (("W", i * o), ("b", o)):
            e = rel_fro(g[k:k + size], gref[k:k + size])
            worst = max(worst, e)
            assert e <= REL, (li + 1, name, e)
            k += size
    print(f"gradients at n = {n}: worst tensor error {worst:.2e}", flush=True)
    mlp.close()


def test_adam_steps_match_reference(ctx):
    """Two kgrt_mlp_train_step calls against the FP64 Adam of Kingma & Ba applied to the GPU's own
    gradients at the same parameters: parameters, moments and step count, element by element."""
    import torch
    from paper_1601_02063_amd import kgrt as K
    p = reference_params(23)
    rng = np.random.Generator(np.random.PCG64(24))
    n = 2048
    x = torch.from_numpy(rng.uniform(-1, 1, size=(n, 4)).astype(np.float32)).to(ctx.device)
    tt = np.zeros((n, 6), dtype=np.float32)
    tt[:, 0] = rng.integers(0, 2, n)
    tt[:, 1:5] = rng.normal(size=(n, 4))
    tt[:, 5] = rng.integers(0, 2, n)
    t = torch.from_numpy(tt).to(ctx.device)
    lr, b1, b2, eps = 3e-3, 0.9, 0.999, 1e-8
    mlp = K.Mlp(ctx, max_batch=n)
    mlp.set_params(p)
    loss = torch.zeros(1, dtype=torch.float32, device=ctx.device)
    P = p.astype(np.float64)
    m = np.zeros_like(P)
    v = np.zeros_like(P)
    for step in (1, 2):
        _, g = mlp.loss_grads(x, t)
        g = g.cpu().numpy().astype(np.float64)
        P_ref, m, v = M.adam_step(P, m, v, g, step, lr, b1, b2, eps)
        mlp.train_step(x, t, None, n, lr, loss, (b1, b2), eps)
        P = mlp.get_params().astype(np.float64)
        gm, gv, gstep = mlp.get_adam()
        assert gstep == step
        # the step's gradient recomputed by loss_grads (every sum is taken in a fixed order, so
        # it is the same gradient); FP32 rounding of the update against the FP64 reference
        np.testing.assert_allclose(P, P_ref, rtol=3e-7, atol=1e-3 * lr)
        np.testing.assert_allclose(gm, m, rtol=1e-4, atol=1e-7 * np.abs(g).max())
        np.testing.assert_allclose(gv, v, rtol=1e-4, atol=1e-9 * (g ** 2).max())
        m, v = gm.astype(np.float64), gv.astype(np.float64)
    # the state round-trips through the checkpoint accessors
    mlp.set_params(p)
    mlp.set_adam(gm, gv, 2)
    gm2, gv2, s2 = mlp.get_adam()
    assert s2 == 2 and np.array_equal(gm2, gm) and np.array_equal(gv2, gv)
    mlp.close()


def test_train_step_fragments_match_repack(ctx):
    """After Adam steps the fragments written parameter by parameter at the end of each step are
    the ones a full repack of the same parameters writes: the inference outputs, the loss and the
    gradient are bit-identical before and after set_params(get_params()); two gradient calls on
    the same batch are bit-identical too (no order-dependent sums)."""
    import torch
    from paper_1601_02063_amd import kgrt as K
    p = reference_params(29)
    rng = np.random.Generator(np.random.PCG64(30))
    n = 4096
    x = torch.from_numpy(rng.uniform(-1, 1, size=(n, 4)).astype(np.float32)).to(ctx.device)
    tt = np.zeros((n, 6), dtype=np.float32)
    tt[:, 0] = rng.integers(0, 2, n)
    tt[:, 1:5] = rng.normal(size=(n, 4))
    tt[:, 5] = rng.integers(0, 2, n)
    t = torch.from_numpy(tt).to(ctx.device)
    xq = torch.from_numpy(rng.uniform(-1, 1, size=(1000, 4)).astype(np.float32)).to(ctx.device)
    mlp = K.Mlp(ctx, max_batch=n)
    mlp.set_params(p)
    loss = torch.zeros(1, dtype=torch.float32, device=ctx.device)
    for _ in range(3):
        mlp.train_step(x, t, None, n, 3e-3, loss)
    y1 = mlp.forward(xq).cpu().numpy()
    l1, g1 = mlp.loss_grads(x, t)
    l1, g1 = float(l1), g1.cpu().numpy()
    l1b, g1b = mlp.loss_grads(x, t)
    assert float(l1b) == l1 and np.array_equal(g1b.cpu().numpy(), g1)
    P = mlp.get_params()
    gm, gv, gstep = mlp.get_adam()
    assert not np.array_equal(P, p)
    mlp.set_params(P)
    mlp.set_adam(gm, gv, gstep)
    y2 = mlp.forward(xq).cpu().numpy()
    l2, g2 = mlp.loss_grads(x, t)
    assert np.array_equal(y1, y2)
    assert float(l2) == l1
    assert np.array_equal(g2.cpu().numpy(), g1)
    mlp.close()
