"""Pins for min-label propagation: BFS closed form per iteration and connected
components (scipy) at the fixed point."""
from collections import deque

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components

import graphgen
import oracle


def bfs_dist(gs, s):
    dist = np.full(gs.V, -1)
    dist[s] = 0
    q = deque([s])
    while q:
        v = q.popleft()
        for u in gs.in_sources[gs.in_offsets[v]:gs.in_offsets[v + 1]]:
            if dist[u] < 0:
                dist[u] = dist[v] + 1
                q.append(u)
    return dist


@pytest.mark.parametrize("seed", range(5))
def test_labels_after_t_steps_bfs_closed_form(seed):
    g = graphgen.random_graph(30, 28, seed)
    gs = graphgen.symmetrize(g)
    dists = np.array([bfs_dist(gs, s) for s in range(gs.V)])  # dists[u, v]
    for t in range(0, 8):
        lab, it = oracle.labelprop(gs, max_iters=t)
        for v in range(gs.V):
            reach = [u for u in range(gs.V) if 0 <= dists[u, v] <= t]
            assert lab[v] == min(reach)


@pytest.mark.parametrize("scale,ef,seed", [(8, 4, 1), (12, 2, 7), (14, 8, 2)])
def test_fixed_point_is_component_minimum(scale, ef, seed):
    g = graphgen.rmat_graph(scale, ef, seed)
    gs = graphgen.symmetrize(g)
    lab, iters = oracle.labelprop(gs)
    A = sp.csr_matrix((np.ones(gs.E), gs.in_sources, gs.in_offsets), shape=(gs.V, gs.V))
    ncomp, comp = connected_components(A, directed=False)
    cmin = np.full(ncomp, gs.V)
    np.minimum.at(cmin, comp, np.arange(gs.V))
    assert np.array_equal(lab, cmin[comp])
    # iterations = max over v of BFS distance from its component minimum, plus the final unchanged pass
    if gs.V <= 4096:
        ecc = 0
        for m in np.unique(cmin):
            d = bfs_dist(gs, m)
            ecc = max(ecc, d.max())
        assert iters == ecc + 1


def test_symmetrize_is_symmetric_and_deduplicated():
    g = graphgen.rmat_graph(10, 8, 3)
    gs = graphgen.symmetrize(g)
    A = sp.csr_matrix((np.ones(gs.E), gs.in_sources, gs.in_offsets), shape=(gs.V, gs.V))
    assert (A != A.T).nnz == 0 and A.max() == 1 and A.diagonal().sum() == 0
