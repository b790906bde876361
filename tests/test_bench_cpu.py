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
