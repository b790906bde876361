"""Pins for the collaborative-filtering oracle: a hand-worked step, the
gradient against central finite differences of the objective, descent for a
small step, and the graph generator's symmetry."""
import numpy as np
import pytest

import graphgen
from oracle import cf


def tiny():
    # user 0 rated item 1 with 3 and item 2 with 1 (edges in both directions)
    g = graphgen.from_edge_list(3, [(0, 1), (1, 0), (0, 2), (2, 0)])
    dst = np.repeat(np.arange(g.V), np.diff(g.in_offsets))
    r = {(0, 1): 3.0, (0, 2): 1.0}
    vals = np.array([r[(min(u, v), max(u, v))] for u, v in zip(g.in_sources, dst)])
    X = np.array([[1.0, 0.0], [1.0, 1.0], [0.0, 2.0]])
    return g, vals, X


def test_hand_step():
    g, vals, X = tiny()
    G, sq = cf.gradient(g, vals, X)
    # errors: rating (0,1): 3 - <x0, x1> = 2; rating (0,2): 1 - <x0, x2> = 1
    assert np.allclose(G, [[2.0 * 1 + 1.0 * 0, 2.0 * 1 + 1.0 * 2], [2.0, 0.0], [1.0, 0.0]])
    assert sq == pytest.approx(2 * (2.0 ** 2 + 1.0 ** 2))
    X1, _ = cf.step(g, vals, X, gamma=0.1, lam=0.5)
    assert np.allclose(X1, [[1.15, 0.4], [1.15, 0.95], [0.1, 1.9]])
    assert cf.objective(g, vals, X, 0.0) == pytest.approx(0.5 * (4.0 + 1.0))


def test_gradient_matches_finite_differences():
    g, vals, U, I = graphgen.bipartite_ratings(7, 4, 6, 3)
    X = cf.init_factors(g.V, 5, 1, scale=0.6).astype(np.float64)
    lam = 0.05
    G, _ = cf.gradient(g, vals, X)
    rng = np.random.default_rng(0)
    h = 1e-5
    for _ in range(40):
        v, j = int(rng.integers(g.V)), int(rng.integers(5))
        Xp, Xm = X.copy(), X.copy()
        Xp[v, j] += h
        Xm[v, j] -= h
        fd = (cf.objective(g, vals, Xp, lam) - cf.objective(g, vals, Xm, lam)) / (2 * h)
        assert fd == pytest.approx(-G[v, j] + lam * X[v, j], rel=1e-6, abs=1e-7)


def test_small_steps_descend():
    g, vals, U, I = graphgen.bipartite_ratings(8, 5, 8, 4)
    X = cf.init_factors(g.V, 8, 2).astype(np.float64)
    f = [cf.objective(g, vals, X, 0.01)]
    for _ in range(5):
        X, _ = cf.step(g, vals, X, gamma=1e-3, lam=0.01)
        f.append(cf.objective(g, vals, X, 0.01))
    assert all(b < a for a, b in zip(f, f[1:]))


def test_rating_graph_is_bipartite_and_symmetric():
    g, vals, U, I = graphgen.bipartite_ratings(9, 5, 8, 7)
    dst = np.repeat(np.arange(g.V), np.diff(g.in_offsets))
    assert np.all((g.in_sources < U) != (dst < U))
    fwd = {(int(u), int(v)): float(x) for u, v, x in zip(g.in_sources, dst, vals)}
    assert all(fwd[(v, u)] == x for (u, v), x in fwd.items())
    assert set(np.unique(vals).tolist()) <= {1.0, 2.0, 3.0, 4.0, 5.0}
