"""Input generator checks: determinism, CSC hygiene, R-MAT quadrant statistics."""
import numpy as np

import graphgen


def test_deterministic_and_thread_invariant():
    a = graphgen.rmat_graph(12, 8, 5, threads=1)
    b = graphgen.rmat_graph(12, 8, 5, threads=4)
    assert np.array_equal(a.in_offsets, b.in_offsets) and np.array_equal(a.in_sources, b.in_sources)
    c = graphgen.rmat_graph(12, 8, 6)
    assert not np.array_equal(a.in_sources[:100], c.in_sources[:100])


def test_csc_hygiene():
    g = graphgen.rmat_graph(13, 16, 1)
    off, src = g.in_offsets, g.in_sources
    assert off[0] == 0 and np.all(np.diff(off) >= 0) and off[-1] == g.E
    for v in range(0, g.V, 97):
        row = src[off[v]:off[v + 1]]
        assert np.all(np.diff(row) > 0) and not np.any(row == v)
    assert g.out_degree.sum() == g.E
    assert np.array_equal(np.bincount(src, minlength=g.V), g.out_degree)


def test_rmat_quadrant_statistics_unpermuted():
    scale = 14
    src, dst = graphgen.rmat_edges(scale, 16, 2, permute=False)
    top = 1 << (scale - 1)
    # top-level quadrant frequencies a, b, c, d of the recursion
    fa = np.mean((src < top) & (dst < top))
    fb = np.mean((src < top) & (dst >= top))
    fc = np.mean((src >= top) & (dst < top))
    assert abs(fa - 0.57) < 0.005 and abs(fb - 0.19) < 0.005 and abs(fc - 0.19) < 0.005


def test_permutation_is_bijection():
    p = graphgen.permutation(1000, 3)
    assert np.array_equal(np.sort(p), np.arange(1000))
