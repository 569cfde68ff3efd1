"""Float64 numpy MLP oracle -- TEST INFRASTRUCTURE ONLY.

The (alpha, omega) predictor is a fully connected network
    8 -> 64 -> 64 -> 2, ReLU after the two hidden layers, linear output,
trained on mean squared error with Adam.  This file writes the forward pass,
the hand-derived backward pass and the Adam update out plainly so the GPU
kernels can be checked against them; the tests pin these against central
finite differences and Adam's closed-form first step.

Parameter layout (one flat float vector, row-major weights):
    W1[64, 8], b1[64], W2[64, 64], b2[64], W3[2, 64], b3[2]   (4866 values)
"""
from __future__ import annotations

import numpy as np

SIZES = (8, 64, 64, 2)


def layout():
    """List of (name, shape) in flat order."""
    out = []
    for li in range(3):
        fan_in, fan_out = SIZES[li], SIZES[li + 1]
        out.append((f"W{li + 1}", (fan_out, fan_in)))
        out.append((f"b{li + 1}", (fan_out,)))
    return out


def n_params() -> int:
    return int(sum(np.prod(s) for _, s in layout()))


def unpack(theta: np.ndarray) -> dict:
    p, off = {}, 0
    for name, shape in layout():
        k = int(np.prod(shape))
        p[name] = theta[off:off + k].reshape(shape)
        off += k
    return p


def init(seed: int = 0) -> np.ndarray:
    """He-uniform weights, zero biases, from numpy's PCG64 with `seed`."""
    rng = np.random.default_rng(seed)
    chunks = []
    for name, shape in layout():
        if name.startswith("W"):
            bound = np.sqrt(6.0 / shape[1])
            chunks.append(rng.uniform(-bound, bound, size=shape).ravel())
        else:
            chunks.append(np.zeros(shape))
    return np.concatenate(chunks)


def forward(theta, X):
    """Returns (Y, cache) for inputs X[B, 8]."""
    p = unpack(np.asarray(theta, dtype=np.float64))
    X = np.asarray(X, dtype=np.float64)
    z1 = X @ p["W1"].T + p["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ p["W2"].T + p["b2"]
    h2 = np.maximum(z2, 0.0)
    y = h2 @ p["W3"].T + p["b3"]
    return y, (X, z1, h1, z2, h2)


def loss(theta, X, Y) -> float:
    y, _ = forward(theta, X)
    d = y - np.asarray(Y, dtype=np.float64)
    return float(np.mean(d * d))


def loss_grad(theta, X, Y):
    """MSE over all B*2 outputs and its gradient with respect to theta."""
    p = unpack(np.asarray(theta, dtype=np.float64))
    y, (X, z1, h1, z2, h2) = forward(theta, X)
    Y = np.asarray(Y, dtype=np.float64)
    B = X.shape[0]
    d = y - Y
    L = float(np.mean(d * d))
    gy = 2.0 * d / (B * y.shape[1])              # dL/dy
    gW3 = gy.T @ h2
    gb3 = gy.sum(axis=0)
    gh2 = gy @ p["W3"]
    gz2 = gh2 * (z2 > 0.0)
    gW2 = gz2.T @ h1
    gb2 = gz2.sum(axis=0)
    gh1 = gz2 @ p["W2"]
    gz1 = gh1 * (z1 > 0.0)
    gW1 = gz1.T @ X
    gb1 = gz1.sum(axis=0)
    g = np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3.ravel(), gb3])
    return L, g


def adam_step(theta, g, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba); t is the 1-based step number.
    Returns new (theta, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def standardise_fit(F):
    """Column mean and scale of a feature matrix; zero-variance columns get scale 1."""
    F = np.asarray(F, dtype=np.float64)
    mu = F.mean(axis=0)
    sd = F.std(axis=0)
    sd = np.where(sd > 1e-12 * np.maximum(1.0, np.abs(mu)), sd, 1.0)
    return mu, sd
