"""cagra_pagerank_iter_noalloc (static scratch, no workspace argument) against
cagra_pagerank_iter (caller workspace) through the C ABI: bit-identical ranks,
contributions and scalars on two graphs in a row, the second smaller, and the
capacity limit reported before any launch."""
import ctypes

import numpy as np
import pytest

import graphgen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cagra():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1608_01362_amd import cagra as c
    c.lib()
    return c


def run_both(cagra, g, N, B, T, contrib_type, restart=-1, iters=12):
    import torch
    dg = cagra.DeviceGraph.from_host(g)
    seg = cagra.build_segments(dg, N, B, T)
    a = cagra.PageRankState(dg, seg, contrib_type, restart)
    b = cagra.PageRankState(dg, seg, contrib_type, restart)
    a.start()
    b.start()
    for _ in range(iters):
        i, o = b.cur, 1 - b.cur
        a.step()
        cagra.pagerank_iter_noalloc(dg, seg, 0.85, contrib_type, b.rank[i], b.contrib[i], b.scalars[i], b.partial,
                                    b.rank[o], b.contrib[o], b.scalars[o], restart=restart)
        b.cur = o
        assert torch.equal(a.rank_now, b.rank_now)
        assert torch.equal(a.contrib[a.cur], b.contrib[b.cur])
        assert torch.equal(a.scalars_now, b.scalars_now)
    return a, b


def test_noalloc_matches_workspace_entry_point_twice(cagra):
    L = cagra.lib()
    assert L.cagra_noalloc_scratch_bytes() == 64 << 20
    # a larger graph, then a smaller one: the second call reuses the scratch
    run_both(cagra, graphgen.rmat_graph(16, 16, 1), 16384, 16384, 65536, cagra.F32)
    run_both(cagra, graphgen.rmat_graph(11, 8, 3), 300, 512, 1024, cagra.F32)
    # BF16 contributions, a personalized run and a graph with split merge blocks
    run_both(cagra, graphgen.rmat_graph(13, 16, 2), 2048, 1024, 4096, cagra.BF16)
    g = graphgen.rmat_graph(12, 16, 5)
    run_both(cagra, g, 1024, 512, 4096, cagra.F32, restart=int(np.argmax(g.out_degree)))
    instar = graphgen.from_edge_list(5001, [(i, 0) for i in range(1, 5001)])
    _, b = run_both(cagra, instar, 64, 256, 256, cagra.F32)
    assert b.seg.c.max_items > b.seg.c.nb  # the hub's block is split


def test_noalloc_rejects_beyond_the_static_scratch(cagra):
    """A segmentation whose iteration workspace exceeds the static scratch is
    rejected with CAGRA_E_CAPACITY before any launch (arguments never read)."""
    L = cagra.lib()
    s = cagra.CSegments()
    s.N, s.B, s.tile_edges = 4096, 8192, 65536
    V = 1 << 24
    s.V, s.E, s.Q, s.k, s.nb, s.ntiles = V, 1 << 26, 1 << 25, V // 4096, V // 8192, 1
    s.max_items = s.nb + 600  # 2 * 600 slots of 8192 int64 accumulators: 75 MiB
    for name in ("seg_row_begin", "row_ptr", "row_dst", "edge_src", "block_ptr", "tile_edge", "tile_seg",
                 "tile_span_row", "row_dst_lo", "block_items"):
        setattr(s, name, 4096)
    g = cagra.CGraph(V, 1 << 26, 4096, 4096, 4096)
    assert L.cagra_iter_workspace_bytes(ctypes.byref(s)) > L.cagra_noalloc_scratch_bytes()
    st = L.cagra_pagerank_iter_noalloc(ctypes.byref(g), ctypes.byref(s), 0.85, -1, cagra.F32, 1, 2, 3, 4, 5, 6, 7,
                                       None)
    assert st == cagra.E_CAPACITY
    assert b"static scratch" in L.cagra_last_error()
