"""Pins for the FP64 PageRank oracle against closed forms and dense linear algebra.

None of these re-type the oracle's loop: they use aggregated-state recursions
for symmetric graphs, the dense Google matrix (matrix power and linear solve),
and invariants (mass conservation, the contraction bound).
"""
import numpy as np
import pytest

import graphgen
import oracle

D = 0.85


def cycle(n):
    return graphgen.from_edge_list(n, [(i, (i + 1) % n) for i in range(n)])


def complete(n):
    return graphgen.from_edge_list(n, [(i, j) for i in range(n) for j in range(n) if i != j])


def bistar(n):
    # hub 0 <-> leaves 1..n
    return graphgen.from_edge_list(n + 1, [(0, i) for i in range(1, n + 1)] + [(i, 0) for i in range(1, n + 1)])


def instar(n):
    # leaves 1..n -> hub 0; hub has no out-edges (dangling)
    return graphgen.from_edge_list(n + 1, [(i, 0) for i in range(1, n + 1)])


def google_matrix(g, d=D):
    V = g.V
    A = np.zeros((V, V))  # A[v,u] = 1/outdeg(u) for u->v
    for v in range(V):
        for u in g.in_sources[g.in_offsets[v]:g.in_offsets[v + 1]]:
            A[v, u] = 1.0 / g.out_degree[u]
    dang = (g.out_degree == 0).astype(np.float64)
    return d * (A + np.outer(np.ones(V), dang) / V) + (1 - d) / V * np.ones((V, V)), A, dang


@pytest.mark.parametrize("n", [2, 3, 7, 64])
def test_cycle_and_complete_uniform(n):
    for g in (cycle(n), complete(n)):
        r, res = oracle.pagerank(g, iters=20)
        assert np.max(np.abs(r - 1.0 / n)) < 1e-15
        assert np.all(res < 64 * 2.3e-16)


@pytest.mark.parametrize("n", [1, 2, 5, 40])
def test_bidirectional_star(n):
    g = bistar(n)
    V = n + 1
    # two-state recursion (hub h, each leaf l), uniform start
    h, l = 1.0 / V, 1.0 / V
    for _ in range(20):
        h, l = (1 - D) / V + D * n * l, (1 - D) / V + D * h / n
    r, _ = oracle.pagerank(g, iters=20)
    assert abs(r[0] - h) < 1e-14
    assert np.max(np.abs(r[1:] - l)) < 1e-14
    # fixed point: hub = (1 + d n) / ((n+1)(1+d))
    r_inf, res = oracle.pagerank(g, iters=2000, tol=1e-15)
    assert abs(r_inf[0] - (1 + D * n) / (V * (1 + D))) < 1e-12
    assert np.max(np.abs(r_inf[1:] - (1 - r_inf[0]) / n)) < 1e-12


@pytest.mark.parametrize("n", [1, 3, 10])
def test_instar_dangling_hub(n):
    g = instar(n)
    V = n + 1
    h, l = 1.0 / V, 1.0 / V
    for _ in range(20):
        h, l = (1 - D) / V + D * (n * l + h / V), (1 - D) / V + D * h / V
    r, _ = oracle.pagerank(g, iters=20)
    assert abs(r[0] - h) < 1e-14 and np.max(np.abs(r[1:] - l)) < 1e-14
    r_inf, _ = oracle.pagerank(g, iters=5000, tol=1e-16)
    hub = ((1 - D) / V + D) / (1 + D - D / V)
    assert abs(r_inf[0] - hub) < 1e-12
    if n == 1:
        assert abs(r_inf[0] - 0.649122807017544) < 1e-12
        assert abs(r_inf[1] - 0.350877192982456) < 1e-12


@pytest.mark.parametrize("seed", range(12))
def test_dense_matrix_power_and_solve(seed):
    rng = np.random.default_rng(seed)
    V = int(rng.integers(2, 13))
    m = int(rng.integers(1, 3 * V))
    g = graphgen.random_graph(V, m, seed)
    G, A, dang = google_matrix(g)
    r = np.full(V, 1.0 / V)
    rs = [r]
    for _ in range(20):
        r = G @ r
        rs.append(r)
    ro, res = oracle.pagerank(g, iters=20)
    assert np.max(np.abs(ro - rs[-1])) < 1e-14
    want_res = [np.abs(rs[t + 1] - rs[t]).sum() for t in range(20)]
    assert np.max(np.abs(res - want_res)) < 1e-14
    # fixed point by a dense solve
    M = np.eye(V) - D * A - (D / V) * np.outer(np.ones(V), dang)
    rstar = np.linalg.solve(M, (1 - D) / V * np.ones(V))
    rinf, _ = oracle.pagerank(g, iters=3000, tol=1e-16)
    assert np.max(np.abs(rinf - rstar)) < 1e-12


def test_mass_conservation_with_dangling():
    g = graphgen.rmat_graph(12, 8, 11)
    assert (g.out_degree == 0).sum() > 0
    r = None
    for t in range(1, 21):
        r, _ = oracle.pagerank(g, iters=t)
        assert abs(r.sum() - 1.0) < 1e-12
    assert np.all(r > 0)


def test_contraction_bound_any_start():
    # ||r_t - r*||_1 <= d/(1-d) * ||r_t - r_{t-1}||_1 for the stochastic Google matrix
    g = graphgen.rmat_graph(11, 8, 5)
    rstar, _ = oracle.pagerank(g, iters=400, tol=1e-15)
    rng = np.random.default_rng(0)
    r0 = rng.random(g.V)
    r0 /= r0.sum()
    for t in (3, 8, 15):
        rt, res = oracle.pagerank(g, iters=t, r0=r0)
        assert np.abs(rt - rstar).sum() <= D / (1 - D) * res[-1] * (1 + 1e-9) + 1e-15


def test_paper_mode_equals_scaled_normalized():
    for g in (cycle(9), complete(5), bistar(6)):
        R = oracle.pagerank_paper_mode(g, 20)
        r, _ = oracle.pagerank(g, iters=20)
        assert np.max(np.abs(R - g.V * r)) < 1e-12


def test_step_at_matches_full_step():
    g = graphgen.rmat_graph(12, 16, 3)
    rng = np.random.default_rng(1)
    r = rng.random(g.V)
    r /= r.sum()
    vs = rng.integers(0, g.V, 200).astype(np.int32)
    # consistency of the spot-check entry point with one full step from the same vector
    full, _ = oracle.pagerank(g, iters=1, r0=r)
    assert np.max(np.abs(oracle.pagerank_step_at(g, r, vs) - full[vs])) < 1e-17 + 1e-15 * full[vs].max()


def test_thread_count_invariance():
    g = graphgen.rmat_graph(14, 8, 9)
    r1, res1 = oracle.pagerank(g, iters=5, threads=1)
    r4, res4 = oracle.pagerank(g, iters=5, threads=4)
    assert np.array_equal(r1, r4) and np.array_equal(res1, res4)


@pytest.mark.parametrize("seed", range(6))
def test_ppr_dense_solve(seed):
    rng = np.random.default_rng(100 + seed)
    V = int(rng.integers(2, 12))
    g = graphgen.random_graph(V, int(rng.integers(1, 3 * V)), 100 + seed)
    s = int(rng.integers(0, V))
    _, A, dang = google_matrix(g)
    e = np.zeros(V)
    e[s] = 1.0
    # r = (1-d) e + d (A r + (dang.r) e), exact 20 steps and the fixed point
    M = D * (A + np.outer(e, dang))
    r = e.copy()
    for _ in range(20):
        r = (1 - D) * e + M @ r
    assert np.max(np.abs(oracle.ppr(g, s, 20) - r)) < 1e-14
    rstar = np.linalg.solve(np.eye(V) - M, (1 - D) * e)
    assert np.max(np.abs(oracle.ppr(g, s, 400) - rstar)) < 1e-12
