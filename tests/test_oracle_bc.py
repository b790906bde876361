"""Pins for the betweenness-centrality oracle: the definition by brute force
(all-pairs BFS path counts, sigma_st(v) = sigma_sv * sigma_vt on shortest
paths), closed forms on paths and stars, and path counts on a grid."""
import itertools
from math import comb

import numpy as np
import pytest

import graphgen
from oracle import bc


def bfs_counts(adj, s, V):
    depth = [-1] * V
    sig = [0] * V
    depth[s], sig[s] = 0, 1
    frontier = [s]
    while frontier:
        nxt = []
        for u in frontier:
            for w in adj[u]:
                if depth[w] < 0:
                    depth[w] = depth[u] + 1
                    nxt.append(w)
                if depth[w] == depth[u] + 1:
                    sig[w] += sig[u]
        frontier = nxt
    return depth, sig


def brute_force(edges, V, sources):
    adj = [[] for _ in range(V)]
    for u, v in edges:
        adj[u].append(v)
    D, S = {}, {}
    for x in range(V):
        D[x], S[x] = bfs_counts(adj, x, V)
    out = np.zeros(V)
    for s in sources:
        for t in range(V):
            if t == s or D[s][t] < 0:
                continue
            for v in range(V):
                if v in (s, t) or D[s][v] < 0 or D[v][t] < 0:
                    continue
                if D[s][v] + D[v][t] == D[s][t]:
                    out[v] += S[s][v] * S[v][t] / S[s][t]
    return out


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_definition_by_brute_force(seed):
    g = graphgen.random_graph(24, 70, seed)
    dst = np.repeat(np.arange(g.V), np.diff(g.in_offsets))
    edges = list(zip(g.in_sources.tolist(), dst.tolist()))
    sources = [0, 5, 11, 17]
    assert np.allclose(bc.betweenness(g, sources), brute_force(edges, g.V, sources), rtol=1e-12, atol=1e-12)


def test_directed_path_and_star():
    n = 7
    path = graphgen.from_edge_list(n, [(i, i + 1) for i in range(n - 1)])
    # from start 0 every inner vertex v lies on the paths to the n-1-v vertices after it
    assert np.allclose(bc.betweenness(path, [0]), [0] + [n - 1 - v for v in range(1, n - 1)] + [0])
    star = graphgen.from_edge_list(6, [(i, 0) for i in range(1, 6)] + [(0, i) for i in range(1, 6)])
    # the centre lies on the one shortest path between every ordered pair of leaves
    assert bc.betweenness(star, range(6))[0] == pytest.approx(5 * 4)


def test_grid_path_counts():
    # directed 4 x 5 grid, edges right and down: sigma from the corner is a binomial
    R, C = 4, 5
    idx = lambda r, c: r * C + c
    edges = [(idx(r, c), idx(r, c + 1)) for r in range(R) for c in range(C - 1)] + \
            [(idx(r, c), idx(r + 1, c)) for r in range(R - 1) for c in range(C)]
    g = graphgen.from_edge_list(R * C, edges)
    depth, sigma, _ = bc.single_source(g, 0)
    for r, c in itertools.product(range(R), range(C)):
        assert depth[idx(r, c)] == r + c and sigma[idx(r, c)] == comb(r + c, r)
