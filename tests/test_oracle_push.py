"""Pins for the push-direction oracle (oracle/push.py): the out-edge scatter must
give the same neighbour sums as the pull definition (Section 2: push and pull
differ only in which side of an edge a thread visits), checked against the C
pull oracle, a closed form and brute force on tiny graphs."""
import numpy as np
import pytest

import graphgen
import oracle
from oracle import push


@pytest.mark.parametrize("V,m,seed", [(1, 0, 0), (2, 1, 1), (9, 30, 2), (40, 200, 3)])
def test_out_edges_brute_force(V, m, seed):
    g = graphgen.random_graph(V, m, seed) if m else graphgen.from_edge_list(V, [])
    off, tgt = push.out_edges(g)
    edges = set()
    for v in range(g.V):
        for u in g.in_sources[g.in_offsets[v]:g.in_offsets[v + 1]]:
            edges.add((int(u), v))
    got = set()
    for u in range(g.V):
        row = tgt[off[u]:off[u + 1]]
        assert np.all(np.diff(row) > 0)  # ascending, no duplicates
        got |= {(u, int(v)) for v in row}
        assert off[u + 1] - off[u] == g.out_degree[u]
    assert got == edges


@pytest.mark.parametrize("N", [1, 3, 8, 64])
def test_push_segments_partition_edges(N):
    g = graphgen.rmat_graph(7, 6, 5)
    ps = push.push_segment(g, N)
    seen = []
    for s in range(ps.k):
        assert np.all(np.diff(ps.rows[s]) > 0)  # rows: distinct sources ascending
        assert np.all((ps.local_dst[s] >= 0) & (ps.local_dst[s] < N))
        for j, u in enumerate(ps.rows[s]):
            for d in ps.local_dst[s][ps.row_ptr[s][j]:ps.row_ptr[s][j + 1]]:
                seen.append((int(u), int(d) + s * N))
    assert len(seen) == g.E and len(set(seen)) == g.E
    off, tgt = push.out_edges(g)
    assert set(seen) == {(u, int(v)) for u in range(g.V) for v in tgt[off[u]:off[u + 1]]}
    # Q is the push layout's expansion: one row per (source, destination segment) pair
    pairs = {(u, v // N) for (u, v) in seen}
    assert ps.Q == len(pairs)


@pytest.mark.parametrize("scale,ef,seed,N", [(8, 8, 1, 16), (10, 4, 2, 100), (9, 16, 3, 512), (6, 3, 4, 1)])
def test_pagerank_push_step_equals_pull_oracle(scale, ef, seed, N):
    g = graphgen.rmat_graph(scale, ef, seed)
    rng = np.random.default_rng(seed)
    r = rng.random(g.V)
    r /= r.sum()
    ps = push.push_segment(g, N)
    got = push.pagerank_push_step(g, ps, r, 0.85)
    want = oracle.pagerank_step_at(g, r, np.arange(g.V, dtype=np.int32), 0.85)
    np.testing.assert_allclose(got, want, rtol=1e-13, atol=0)


def test_pagerank_push_closed_form_cycle_with_dangling():
    # 0 -> 1 -> 2 -> 0 plus 2 -> 3, vertex 3 dangling; start r = (a, b, c, e)
    g = graphgen.from_edge_list(4, [(0, 1), (1, 2), (2, 0), (2, 3)])
    r = np.array([0.1, 0.2, 0.3, 0.4])
    d = 0.85
    ps = push.push_segment(g, 2)
    got = push.pagerank_push_step(g, ps, r, d)
    D = 0.4
    tele = (1 - d) / 4 + d * D / 4
    want = np.array([tele + d * 0.3 / 2, tele + d * 0.1, tele + d * 0.2, tele + d * 0.3 / 2])
    np.testing.assert_allclose(got, want, rtol=1e-15)
    assert abs(got.sum() - 1.0) < 1e-15


@pytest.mark.parametrize("seed", range(4))
def test_labelprop_push_step_brute_force_and_fixed_point(seed):
    g = graphgen.random_graph(25, 40, seed)
    gs = graphgen.symmetrize(g)
    ps = push.push_segment(gs, 4)
    rng = np.random.default_rng(seed)
    lab = rng.permutation(gs.V).astype(np.int32)
    got = push.labelprop_push_step(ps, lab)
    for v in range(gs.V):
        nb = gs.in_sources[gs.in_offsets[v]:gs.in_offsets[v + 1]]
        assert got[v] == min([lab[v]] + [lab[u] for u in nb])
    cur = np.arange(gs.V, dtype=np.int32)
    for _ in range(gs.V + 1):
        nxt = push.labelprop_push_step(ps, cur)
        if np.array_equal(nxt, cur):
            break
        cur = nxt
    want, _ = oracle.labelprop(gs)
    np.testing.assert_array_equal(cur, want)


def test_planted_mistake_is_caught():
    # a scatter that uses the destination's own value instead of the source's
    # (the pull/push mix-up) must fail the pull-oracle comparison
    g = graphgen.rmat_graph(8, 8, 11)
    rng = np.random.default_rng(0)
    r = rng.random(g.V)
    r /= r.sum()
    ps = push.push_segment(g, 32)
    od = g.out_degree.astype(np.int64)
    contrib = np.where(od > 0, r / np.maximum(od, 1), 0.0)
    wrong = np.zeros(g.V)
    for s in range(ps.k):
        dst = ps.local_dst[s] + s * ps.N
        np.add.at(wrong, dst, contrib[dst])
    D = float(r[od == 0].sum())
    bad = 0.15 / g.V + 0.85 * (wrong + D / g.V)
    want = oracle.pagerank_step_at(g, r, np.arange(g.V, dtype=np.int32), 0.85)
    assert np.max(np.abs(bad - want)) > 1e-6
