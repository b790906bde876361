"""Pins for the segmenting part of the oracle (Sections 3.1-3.3).

The worked example of Section 3.1/3.3 is a golden fixture; everything else is
checked by brute force (sets of (segment, destination) pairs) and by the
requirement that segmented processing reproduces the unsegmented result.
"""
import json
import os

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

import graphgen
import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "segmenting_example.json")


def brute_force_layout(g, N, B):
    """Independent construction from the definition: rows of subgraph s are the
    distinct destinations v having an in-edge from [sN, sN+N)."""
    k = (g.V + N - 1) // N
    rows = {s: [] for s in range(k)}
    edges = {}
    for v in range(g.V):
        for u in g.in_sources[g.in_offsets[v]:g.in_offsets[v + 1]]:
            s = int(u) // N
            edges.setdefault((s, v), []).append(int(u) - s * N)
    for (s, v) in sorted(edges):
        rows[s].append(v)
    return k, rows, edges


def test_worked_example_from_paper():
    ex = json.load(open(GOLDEN))
    g = graphgen.from_edge_list(ex["V"], ex["edges"])
    seg = oracle.segment(g, ex["N"], B=2)
    assert seg.k == 2 and seg.Q == ex["expected_Q"]
    for s, want in enumerate(ex["expected_idxmap"]):
        got = seg.row_dst[seg.seg_row_begin[s]:seg.seg_row_begin[s + 1]].tolist()
        assert got == want
    assert abs(seg.q - 7 / 6) < 1e-15


def check_layout(g, N, B):
    seg = oracle.segment(g, N, B)
    k, rows, edges = brute_force_layout(g, N, B)
    assert seg.k == k and seg.nb == (g.V + B - 1) // B
    assert seg.Q == len(edges)
    r = 0
    for s in range(k):
        assert seg.seg_row_begin[s] == r
        for v in rows[s]:
            assert seg.row_dst[r] == v
            lo, hi = seg.row_ptr[r], seg.row_ptr[r + 1]
            assert seg.edge_src[lo:hi].tolist() == edges[(s, v)]
            r += 1
    assert seg.seg_row_begin[k] == r == seg.Q
    assert seg.row_ptr[seg.Q] == g.E
    # block index: first row of subgraph s with destination >= b*B
    for b in range(seg.nb + 1):
        for s in range(k):
            lo, hi = seg.seg_row_begin[s], seg.seg_row_begin[s + 1]
            want = lo + int(np.searchsorted(seg.row_dst[lo:hi], b * B, side="left"))
            assert seg.block_ptr[b * k + s] == want
    # q bounded by the number of segments and by the average degree (Section 3.4)
    if g.V:
        assert seg.Q <= k * g.V and seg.Q <= g.E
    return seg


@pytest.mark.parametrize("N,B", [(1, 1), (2, 3), (5, 4), (16, 16), (63, 7), (64, 1000), (1000, 5)])
def test_layout_bruteforce(N, B):
    g = graphgen.rmat_graph(6, 6, 21)
    check_layout(g, N, B)


def test_nested_segments_monotone_q():
    g = graphgen.rmat_graph(10, 8, 4)
    Qs = [oracle.segment(g, N, 64).Q for N in (8, 16, 32, 64, 128, 1024)]
    assert all(a >= b for a, b in zip(Qs, Qs[1:]))
    # one segment: Q = number of vertices with at least one in-edge
    assert oracle.segment(g, g.V, 64).Q == int((np.diff(g.in_offsets) > 0).sum())


@settings(max_examples=40, deadline=None)
@given(V=st.integers(1, 40), m=st.integers(0, 120), seed=st.integers(0, 10_000),
       N=st.integers(1, 43), B=st.integers(1, 43))
def test_segmented_equals_unsegmented(V, m, seed, N, B):
    g = graphgen.random_graph(V, m, seed)
    seg = check_layout(g, N, B)
    rng = np.random.default_rng(seed)
    r = rng.random(V)
    r /= r.sum()
    want, _ = oracle.pagerank(g, iters=1, r0=r)
    got = oracle.segmented_pagerank_step(g, seg, r)
    scale = 1 + np.diff(g.in_offsets)
    assert np.all(np.abs(got - want) <= 1e-14 * scale * np.maximum(want, 1e-300) + 1e-17)
    # label propagation is exact under segmenting
    lab = rng.permutation(V).astype(np.int32)
    gs = graphgen.symmetrize(g)
    segs = oracle.segment(gs, N, B)
    step = oracle.segmented_labelprop_step(segs, lab)
    want_l = lab.copy()
    for v in range(V):
        nb = gs.in_sources[gs.in_offsets[v]:gs.in_offsets[v + 1]]
        if nb.size:
            want_l[v] = min(lab[v], lab[nb].min())
    assert np.array_equal(step, want_l)


def test_merge_identity_for_untouched_vertices():
    g = graphgen.from_edge_list(5, [(0, 1), (3, 1)])
    seg = oracle.segment(g, 2, 2)
    out = oracle.merge(seg, np.array([1.0, 2.0]), oracle.SUM)
    assert out.tolist() == [0.0, 3.0, 0.0, 0.0, 0.0]
    out = oracle.merge(seg, np.array([4.0, 2.0]), oracle.MIN)
    assert out[1] == 2.0 and np.isinf(out[0]) and np.isinf(out[4])
