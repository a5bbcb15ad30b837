"""Pins of the FP64 reference MLP: its backpropagation equals central finite
differences of its loss, and its loss has the stated closed form."""
import numpy as np

import oracle.mlp as M


def _data(n, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    x = rng.uniform(-1, 1, size=(n, 4))
    t = np.zeros((n, 6))
    t[:, 0] = rng.integers(0, 2, n)
    t[:, 1:5] = rng.normal(size=(n, 4))
    t[:, 5] = rng.integers(0, 2, n)
    return x, t


def test_parameter_count():
    assert M.num_params() == 199941


def test_backprop_matches_finite_differences():
    p = M.init_params(3).astype(np.float64)
    x, t = _data(7, 4)
    _, g = M.loss_and_grads(p, x, t)
    rng = np.random.Generator(np.random.PCG64(9))
    offsets = np.cumsum([0] + [i * o + o for i, o in M.LAYERS])
    picks = list(rng.choice(len(p), 40, replace=False)) + [offsets[k] for k in range(5)] + [len(p) - 1]
    eps = 1e-6
    for i in picks:
        q = p.copy()
        q[i] += eps
        lp = M.loss(q, x, t)
        q[i] -= 2 * eps
        lm = M.loss(q, x, t)
        fd = (lp - lm) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-7 + 1e-6 * abs(fd), (i, fd, g[i])


def test_loss_closed_form_for_zero_network():
    """All-zero parameters give outputs 0: BCE = log 2, MSE terms = weighted squared targets."""
    p = np.zeros(M.num_params())
    x, t = _data(5, 1)
    want = np.mean(np.log(2.0) + 10 * t[:, 1] ** 2 + 10 * t[:, 2] ** 2 + t[:, 5] * (t[:, 3] ** 2 + t[:, 4] ** 2))
    assert abs(M.loss(p, x, t) - want) < 1e-12


def test_adam_first_step_closed_form():
    """From zero moments the bias corrections make the first step lr g / (|g| + eps) per parameter
    (the moments are (1 - beta1) g and (1 - beta2) g^2 before correction)."""
    rng = np.random.Generator(np.random.PCG64(21))
    p0 = rng.normal(size=1000)
    g = rng.normal(size=1000) * 10.0 ** rng.uniform(-9, 2, size=1000)
    lr, b1, b2, eps = 1e-3, 0.9, 0.999, 1e-8
    p, m, v = M.adam_step(p0, np.zeros(1000), np.zeros(1000), g, 1, lr, b1, b2, eps)
    np.testing.assert_allclose(p0 - p, lr * g / (np.abs(g) + eps), rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(m, 0.1 * g, rtol=1e-14)
    np.testing.assert_allclose(v, 0.001 * g * g, rtol=1e-12)


def test_adam_constant_gradient_moves_at_lr():
    """Under a constant gradient the bias-corrected moments are g and g^2 at every step, so every
    step moves each parameter by lr g / (|g| + eps): a missing or misplaced correction drifts."""
    g = np.array([3.0, -0.5, 1e-4, -2e-7])
    p = np.zeros(4)
    m = np.zeros(4)
    v = np.zeros(4)
    lr, eps = 2e-3, 1e-8
    for t in range(1, 60):
        q, m, v = M.adam_step(p, m, v, g, t, lr, 0.9, 0.999, eps)
        np.testing.assert_allclose(p - q, lr * g / (np.abs(g) + eps), rtol=1e-9)
        p = q


def test_adam_minimises_a_quadratic():
    """Adam's steps on f = sum c_i x_i^2 / 2 bring every coordinate from 1 to within a few lr of 0."""
    c = np.array([1e-2, 1.0, 1e2, 1e4])
    p = np.ones(4)
    m = np.zeros(4)
    v = np.zeros(4)
    for t in range(1, 4001):
        p, m, v = M.adam_step(p, m, v, c * p, t, 1e-2)
    assert np.all(np.abs(p) < 0.05), p
