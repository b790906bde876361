"""Pins for the FP64 warm-start reference: central finite differences for every
parameter group, the GELU closed forms, features against brute force."""
import math

import numpy as np
import pytest

import graphgen
from oracle import mlp


def test_gelu_values():
    # GELU(x) = x * Phi(x); Phi(0) = 1/2, Phi(1) = 0.8413447460685429, symmetric derivative
    assert mlp.gelu(np.array([0.0]))[0] == 0.0
    assert abs(mlp.gelu(np.array([1.0]))[0] - 0.8413447460685429) < 1e-15
    assert abs(mlp.gelu(np.array([-1.0]))[0] + 1 - 0.8413447460685429) < 1e-15
    x = np.linspace(-4, 4, 41)
    h = 1e-6
    fd = (mlp.gelu(x + h) - mlp.gelu(x - h)) / (2 * h)
    assert np.max(np.abs(fd - mlp.gelu_grad(x))) < 1e-8


@pytest.mark.parametrize("seed", [0, 1])
def test_gradient_matches_finite_differences(seed):
    rng = np.random.default_rng(seed)
    p = mlp.init_params(seed) + rng.normal(0, 0.05, mlp.NPARAM)
    X = rng.normal(0, 1, (37, 3)) * [2, 1, 0.5] + [3, 2, 1]
    t = rng.normal(0, 1, 37)
    mean, std = X.mean(axis=0), X.std(axis=0)
    _, g = mlp.loss_and_grad(p, X, t, mean, std)
    idx = np.concatenate([rng.choice(np.arange(a, b), size=min(6, b - a), replace=False)
                          for a, b in [(0, 192), (192, 256), (256, 4352), (4352, 4416), (4416, 4480), (4480, 4481)]])
    h = 1e-6
    for i in idx:
        e = np.zeros(mlp.NPARAM)
        e[i] = h
        fd = (mlp.loss_and_grad(p + e, X, t, mean, std)[0] - mlp.loss_and_grad(p - e, X, t, mean, std)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])), (i, fd, g[i])


def test_adam_first_step_moves_by_lr():
    p = np.zeros(4)
    g = np.array([1.0, -2.0, 0.5, 0.0])
    p1, m, v = mlp.adam(p, g, np.zeros(4), np.zeros(4), 1, lr=0.01)
    # bias correction makes the first step lr * sign(g) (up to eps)
    assert np.allclose(p1, [-0.01, 0.01, -0.01, 0.0], atol=1e-8)


def test_features_bruteforce():
    g = graphgen.rmat_graph(9, 8, 3)
    F = mlp.degree_features(g)
    assert np.allclose(F, mlp.degree_features_fast(g), rtol=1e-14, atol=1e-15)
    v = int(np.argmax(np.diff(g.in_offsets)))
    us = g.in_sources[g.in_offsets[v]:g.in_offsets[v + 1]]
    want = sum(math.log(1 + g.out_degree[u]) for u in us) / len(us)
    assert abs(F[v, 2] - want) < 1e-12 and abs(F[v, 0] - math.log(1 + len(us))) < 1e-15


def test_start_vector_is_softmax():
    y = np.array([0.0, math.log(2.0), math.log(3.0)])
    assert np.allclose(mlp.start_vector(y), [1 / 6, 2 / 6, 3 / 6], atol=1e-15)
