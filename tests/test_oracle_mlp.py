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
