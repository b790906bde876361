"""Collaborative filtering on the rating graph: plain numpy, FP64.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Reading of the paper (Section 4 programming interface: the edge update may read
the old value of the destination, named for collaborative filtering; Section 6
applications; no algorithm is printed): gradient-descent matrix factorization.
Every vertex v (user or item) has a latent vector x_v of K values; every rating
r between u and v is an edge in both directions. One synchronous step:

    g_v   = sum over in-edges u -> v of (r_uv - <x_u, x_v>) * x_u   (EdgeUpdate, summed by Merge)
    x_v' = x_v + gamma * (g_v - lambda * x_v)                      (VertexUpdate)

which is gradient descent on F(X) = 1/2 sum_ratings (r - <x_u, x_i>)^2
+ lambda/2 sum_v |x_v|^2, since dF/dx_v = -g_v + lambda * x_v.
"""
from __future__ import annotations

import numpy as np


def _dst(g):
    return np.repeat(np.arange(g.V, dtype=np.int64), np.diff(g.in_offsets.astype(np.int64)))


def gradient(g, vals, X, chunk: int = 1 << 18):
    """(g_v for every v as [V, K], sum over in-edges of the squared error)."""
    X = np.asarray(X, dtype=np.float64)
    vals = np.asarray(vals, dtype=np.float64)
    dst = _dst(g)
    src = g.in_sources.astype(np.int64)
    G = np.zeros_like(X)
    sq = 0.0
    for a in range(0, g.E, chunk):
        b = min(a + chunk, g.E)
        xu, xv = X[src[a:b]], X[dst[a:b]]
        err = vals[a:b] - np.einsum("ek,ek->e", xu, xv)
        sq += float(err @ err)
        np.add.at(G, dst[a:b], err[:, None] * xu)
    return G, sq


def step(g, vals, X, gamma: float, lam: float):
    """One gradient step; returns (X', sum of squared errors over in-edges at X)."""
    G, sq = gradient(g, vals, X)
    X = np.asarray(X, dtype=np.float64)
    return X + gamma * (G - lam * X), sq


def objective(g, vals, X, lam: float) -> float:
    """F(X): every rating appears as two in-edges, hence the factor 1/4."""
    _, sq = gradient(g, vals, X)
    X = np.asarray(X, dtype=np.float64)
    return 0.25 * sq + 0.5 * lam * float((X * X).sum())


def init_factors(V: int, K: int, seed: int, scale: float = 0.1) -> np.ndarray:
    """Seeded uniform start in [0, scale) (same values on every side)."""
    rng = np.random.default_rng(seed)
    return (rng.random((V, K)) * scale).astype(np.float32)
