"""FP64 reference for the warm-start network and its inputs.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

degree_features  f1 = log(1 + in-degree), f2 = log(1 + out-degree),
                 f3 = mean over in-neighbours u of log(1 + out-degree(u)) (0 without in-neighbours)
forward/backward 3 -> 64 -> 64 -> 1 multilayer perceptron, exact GELU
                 (x * Phi(x), Hendrycks & Gimpel 2016), mean squared error
adam             Kingma & Ba (2015), bias-corrected
start_vector     r0 = exp(y) / sum(exp(y)) (the network predicts log(V * r))

Parameter vector layout (4481 values): W1[64][3], b1[64], W2[64][64] (row j =
output j), b2[64], w3[64], b3.
"""
from __future__ import annotations

import math

import numpy as np

H = 64
OFF_W1, OFF_B1, OFF_W2, OFF_B2, OFF_W3, OFF_B3 = 0, 192, 256, 4352, 4416, 4480
NPARAM = 4481


def degree_features(g):
    indeg = np.diff(g.in_offsets).astype(np.float64)
    outdeg = g.out_degree.astype(np.float64)
    lo = np.log1p(outdeg)
    f3 = np.zeros(g.V)
    for v in range(g.V):
        a, b = g.in_offsets[v], g.in_offsets[v + 1]
        if b > a:
            f3[v] = lo[g.in_sources[a:b]].sum() / (b - a)
    return np.stack([np.log1p(indeg), lo, f3], axis=1)


def degree_features_fast(g):
    """Same definition, vectorized (for large graphs)."""
    indeg = np.diff(g.in_offsets).astype(np.int64)
    lo = np.log1p(g.out_degree.astype(np.float64))
    s = np.add.reduceat(lo[g.in_sources], g.in_offsets[:-1][indeg > 0]) if g.E else np.zeros(0)
    f3 = np.zeros(g.V)
    f3[indeg > 0] = s / indeg[indeg > 0]
    return np.stack([np.log1p(indeg.astype(np.float64)), lo, f3], axis=1)


def unpack(p):
    p = np.asarray(p, dtype=np.float64)
    return (p[OFF_W1:OFF_B1].reshape(H, 3), p[OFF_B1:OFF_W2], p[OFF_W2:OFF_B2].reshape(H, H),
            p[OFF_B2:OFF_W3], p[OFF_W3:OFF_B3], p[OFF_B3])


def init_params(seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    p = np.zeros(NPARAM)
    p[OFF_W1:OFF_B1] = rng.normal(0, 1 / math.sqrt(3), 192)
    p[OFF_W2:OFF_B2] = rng.normal(0, 1 / math.sqrt(H), H * H)
    p[OFF_W3:OFF_B3] = rng.normal(0, 1 / math.sqrt(H), H)
    return p


def _erf(x):
    return np.vectorize(math.erf)(x)


def gelu(x):
    return 0.5 * x * (1.0 + _erf(x / math.sqrt(2.0)))


def gelu_grad(x):
    return 0.5 * (1.0 + _erf(x / math.sqrt(2.0))) + x * np.exp(-0.5 * x * x) / math.sqrt(2.0 * math.pi)


def forward(p, X, mean, std):
    """y for each row of X; also returns the intermediates (Z, z1, h1, z2, h2)."""
    W1, b1, W2, b2, w3, b3 = unpack(p)
    Z = (np.asarray(X, dtype=np.float64) - mean) / std
    z1 = Z @ W1.T + b1
    h1 = gelu(z1)
    z2 = h1 @ W2.T + b2
    h2 = gelu(z2)
    y = h2 @ w3 + b3
    return y, (Z, z1, h1, z2, h2)


def loss_and_grad(p, X, t, mean, std):
    """Mean squared error over the rows and its gradient (FP64)."""
    W1, b1, W2, b2, w3, b3 = unpack(p)
    y, (Z, z1, h1, z2, h2) = forward(p, X, mean, std)
    n = len(y)
    r = y - t
    loss = float((r * r).sum() / n)
    dy = 2.0 * r / n
    g = np.zeros(NPARAM)
    g[OFF_W3:OFF_B3] = h2.T @ dy
    g[OFF_B3] = dy.sum()
    dz2 = np.outer(dy, w3) * gelu_grad(z2)
    g[OFF_W2:OFF_B2] = (dz2.T @ h1).ravel()
    g[OFF_B2:OFF_W3] = dz2.sum(axis=0)
    dz1 = (dz2 @ W2) * gelu_grad(z1)
    g[OFF_W1:OFF_B1] = (dz1.T @ Z).ravel()
    g[OFF_B1:OFF_W2] = dz1.sum(axis=0)
    return loss, g


def adam(p, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def start_vector(y):
    y = np.asarray(y, dtype=np.float64)
    e = np.exp(y - y.max())
    return e / e.sum()
