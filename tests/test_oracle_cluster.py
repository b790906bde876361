"""Pins for the clustering oracle (Section 5, frequency-based clustering).

The hand-worked example fixes the reading (strict threshold, descending order,
stable ties, untouched order of the other vertices, re-sorted rows); the
properties below check the same rules by brute force on generated graphs, and
PageRank's equivariance under relabelling ties the relabelled graph to the
original one."""
import json
import os

import numpy as np
import pytest

import graphgen
import oracle
from oracle import cluster as oc

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "clustering_example.json")


def test_hand_example():
    ex = json.load(open(GOLDEN))
    g = graphgen.from_edge_list(ex["V"], ex["edges"])
    perm, H, gc = oc.cluster(g)
    assert perm.tolist() == ex["perm"]
    assert H == ex["hot"]
    assert gc.in_offsets.tolist() == ex["in_offsets"]
    assert gc.in_sources.tolist() == ex["in_sources"]
    assert gc.out_degree.tolist() == ex["out_degree"]


def edge_set(g):
    dst = np.repeat(np.arange(g.V), np.diff(g.in_offsets))
    return set(zip(g.in_sources.tolist(), dst.tolist()))


def check_rules(g, perm, H, gc):
    V, E = g.V, g.E
    od = g.out_degree.astype(np.int64)
    assert sorted(perm.tolist()) == list(range(V))
    hot = [v for v in range(V) if od[v] * V > E]
    assert H == len(hot) and set(perm[:H].tolist()) == set(hot)
    for i in range(H - 1):  # descending, ties in original order
        a, b = perm[i], perm[i + 1]
        assert od[a] > od[b] or (od[a] == od[b] and a < b)
    assert perm[H:].tolist() == sorted(perm[H:].tolist())  # the rest keep their order
    inv = np.empty(V, dtype=np.int64)
    inv[perm] = np.arange(V)
    assert edge_set(gc) == {(int(inv[u]), int(inv[v])) for u, v in edge_set(g)}
    for v in range(V):  # rows ascending, no duplicates
        row = gc.in_sources[gc.in_offsets[v]:gc.in_offsets[v + 1]]
        assert np.all(np.diff(row) > 0)
    assert np.array_equal(gc.out_degree, np.bincount(gc.in_sources, minlength=V).astype(np.int32))
    assert np.array_equal(gc.out_degree, g.out_degree[perm])


@pytest.mark.parametrize("g", [graphgen.rmat_graph(10, 8, 5), graphgen.random_graph(500, 3000, 2),
                               graphgen.from_edge_list(5001, [(0, i) for i in range(1, 5001)])],
                         ids=["rmat10", "random500", "outstar"])
def test_rules_by_brute_force(g):
    perm, H, gc = oc.cluster(g)
    check_rules(g, perm, H, gc)


def test_no_vertex_above_average_is_identity():
    cyc = graphgen.from_edge_list(9, [(i, (i + 1) % 9) for i in range(9)])
    perm, H, gc = oc.cluster(cyc)
    assert H == 0 and perm.tolist() == list(range(9))
    assert np.array_equal(gc.in_offsets, cyc.in_offsets) and np.array_equal(gc.in_sources, cyc.in_sources)
    empty = graphgen.from_edge_list(4, [])
    perm, H, gc = oc.cluster(empty)
    assert H == 0 and perm.tolist() == [0, 1, 2, 3] and gc.E == 0


def test_pagerank_is_equivariant():
    g = graphgen.rmat_graph(12, 16, 9)
    perm, H, gc = oc.cluster(g)
    assert 0 < H < g.V
    r, _ = oracle.pagerank(g, iters=30)
    rc, _ = oracle.pagerank(gc, iters=30)
    assert np.max(np.abs(rc - r[perm])) <= 1e-15
