"""Host logic of bench.py that needs no GPU: the in-edge sources of the
lower-bound control must form a valid CSC (the rules every entry point assumes)
and stay within a prefix of the vertex ids."""
import numpy as np

import graphgen


def test_lowest_id_sources_valid_csc():
    import torch
    import bench
    for g in (graphgen.rmat_graph(12, 8, 1), graphgen.from_edge_list(6, [(1, 0), (2, 0), (0, 5), (3, 5), (4, 5)]),
              graphgen.from_edge_list(3, [])):
        src = bench.lowest_id_sources(torch.from_numpy(np.ascontiguousarray(g.in_offsets))).numpy()
        assert src.dtype == np.int32 and src.size == g.E
        maxdeg = int(np.diff(g.in_offsets).max()) if g.V else 0
        for v in range(g.V):
            r = src[g.in_offsets[v]:g.in_offsets[v + 1]]
            d = r.size
            assert np.all(np.diff(r) > 0) and not np.any(r == v)
            # the first d ids, with v skipped when it falls among them
            want = np.arange(d + (1 if v < d else 0))
            want = want[want != v][:d]
            assert np.array_equal(r, want)
            assert d == 0 or r.max() <= maxdeg


def test_byte_models():
    """The method's algorithmic bytes per iteration (its per-subgraph CSR:
    sources, row pointers, 4-byte destinations, block index, vertex arrays)
    total E*we + 16Q + 4k(nb+1) + V(12 + 2wc) plus the last row pointer; the
    bytes this layout moves drop the row pointers and halve the destinations."""
    import bench
    V, E, Q, k, nb = 33554432, 1047207919, 575669056, 1024, 4096
    for wc, we in ((4, 2), (2, 2), (4, 4)):
        cg, cm = bench.csr_byte_model(V, E, Q, k, nb, wc, we)
        assert cg + cm == E * we + 16 * Q + 4 * k * (nb + 1) + V * (12 + 2 * wc) + 4
        g, m = bench.byte_model(V, E, Q, k, nb, wc, we)
        assert (cg - g, cm - m) == (4 * (Q + 1), 2 * Q)
