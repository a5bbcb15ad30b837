"""FP64 reference of the surrogate network -- TEST INFRASTRUCTURE ONLY.

The surrogate is a multilayer perceptron 4 -> 256 -> 256 -> 256 -> 256 -> 5
with SiLU activations (z * sigmoid(z)) on the four hidden layers and a linear
output. It maps ray features (a, cos(inclination), x/15, y/15) to
(capture logit, log r_c, g, sin phi_c, cos phi_c).

Parameters are one flat float vector, layer by layer, each layer its weight
matrix W[out][in] (row-major) followed by its bias b[out].

Loss of one sample with targets t = (capture, log r_c, g, sin phi, cos phi,
phi_valid):
    BCE-with-logits(o0, t0) + 10 (o1 - t1)^2 + 10 (o2 - t2)^2
                            + t5 ((o3 - t3)^2 + (o4 - t4)^2),
averaged over the batch. Plain numpy in float64; no blocking or fusion.
"""
from __future__ import annotations

import numpy as np

LAYERS = ((4, 256), (256, 256), (256, 256), (256, 256), (256, 5))
W_CAP, W_LOGR, W_G, W_PHI = 1.0, 10.0, 10.0, 1.0


def num_params() -> int:
    return sum(i * o + o for i, o in LAYERS)


def unpack(params: np.ndarray):
    params = np.asarray(params, dtype=np.float64)
    out, k = [], 0
    for i, o in LAYERS:
        W = params[k:k + i * o].reshape(o, i)
        k += i * o
        b = params[k:k + o]
        k += o
        out.append((W, b))
    assert k == len(params)
    return out


def init_params(seed: int) -> np.ndarray:
    """Uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) for weights and biases."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for i, o in LAYERS:
        bound = 1.0 / np.sqrt(i)
        parts.append(rng.uniform(-bound, bound, size=i * o))
        parts.append(rng.uniform(-bound, bound, size=o))
    return np.concatenate(parts).astype(np.float32)


def sigmoid(z):
    return 1.0 / (1.0 + np.exp(-z))


def silu(z):
    return z * sigmoid(z)


def silu_grad(z):
    s = sigmoid(z)
    return s * (1.0 + z * (1.0 - s))


def forward(params, x):
    """Returns (outputs [n, 5], cache of pre-activations and activations)."""
    layers = unpack(params)
    h = np.asarray(x, dtype=np.float64)
    hs, zs = [h], []
    for li, (W, b) in enumerate(layers):
        z = h @ W.T + b
        zs.append(z)
        h = silu(z) if li < len(layers) - 1 else z
        hs.append(h)
    return h, (hs, zs)


def loss(params, x, t):
    o, _ = forward(params, x)
    return _loss_from_outputs(o, np.asarray(t, dtype=np.float64))


def _loss_from_outputs(o, t):
    bce = np.logaddexp(0.0, o[:, 0]) - t[:, 0] * o[:, 0]
    l = (W_CAP * bce + W_LOGR * (o[:, 1] - t[:, 1]) ** 2 + W_G * (o[:, 2] - t[:, 2]) ** 2
         + W_PHI * t[:, 5] * ((o[:, 3] - t[:, 3]) ** 2 + (o[:, 4] - t[:, 4]) ** 2))
    return float(l.mean())


def loss_and_grads(params, x, t):
    """Loss and its gradient with respect to the flat parameter vector (backpropagation)."""
    t = np.asarray(t, dtype=np.float64)
    layers = unpack(params)
    o, (hs, zs) = forward(params, x)
    n = len(o)
    d = np.zeros_like(o)
    d[:, 0] = W_CAP * (sigmoid(o[:, 0]) - t[:, 0]) / n
    d[:, 1] = 2.0 * W_LOGR * (o[:, 1] - t[:, 1]) / n
    d[:, 2] = 2.0 * W_G * (o[:, 2] - t[:, 2]) / n
    d[:, 3] = 2.0 * W_PHI * t[:, 5] * (o[:, 3] - t[:, 3]) / n
    d[:, 4] = 2.0 * W_PHI * t[:, 5] * (o[:, 4] - t[:, 4]) / n
    grads = [None] * len(layers)
    dz = d
    for li in range(len(layers) - 1, -1, -1):
        W, _ = layers[li]
        grads[li] = (dz.T @ hs[li], dz.sum(axis=0))
        if li > 0:
            dz = (dz @ W) * silu_grad(zs[li - 1])
    flat = np.concatenate([np.concatenate([gW.ravel(), gb]) for gW, gb in grads])
    return _loss_from_outputs(o, t), flat


def adam_step(params, m, v, grads, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One step of Adam (Kingma & Ba 2015, Algorithm 1) in float64.

    t is the index of this step, counted from 1. Returns the new (params, m, v):
      m_t = beta1 m_{t-1} + (1 - beta1) g,   v_t = beta2 v_{t-1} + (1 - beta2) g^2,
      params_t = params_{t-1} - lr * (m_t / (1 - beta1^t)) / (sqrt(v_t / (1 - beta2^t)) + eps).
    """
    g = np.asarray(grads, dtype=np.float64)
    m = beta1 * np.asarray(m, dtype=np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, dtype=np.float64) + (1.0 - beta2) * g * g
    m_hat = m / (1.0 - beta1 ** t)
    v_hat = v / (1.0 - beta2 ** t)
    p = np.asarray(params, dtype=np.float64) - lr * m_hat / (np.sqrt(v_hat) + eps)
    return p, m, v
