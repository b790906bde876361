"""The autotuner times real configurations and its choice passes PageRank parity."""
import numpy as np
import pytest

import graphgen
import oracle

pytestmark = pytest.mark.gpu


def test_autotune_choice_is_valid_and_correct(tmp_path):
    import torch
    assert torch.cuda.is_available()
    from paper_1608_01362_amd import autotune, cagra
    g = graphgen.rmat_graph(16, 16, 1)
    dg = cagra.DeviceGraph.from_host(g)
    cache = str(tmp_path / "tune.json")
    best, timed = autotune.tune(dg, cagra.F32, "pagerank", cache_path=cache, max_trials=4, log=print)
    assert timed and best.ms == min(c.ms for c in timed) and best.ms > 0
    again, timed2 = autotune.tune(dg, cagra.F32, "pagerank", cache_path=cache)
    assert timed2 == [] and again == best  # served from the cache
    seg = cagra.build_segments(dg, best.N, best.B, best.tile_edges)
    r, _, _ = cagra.pagerank(dg, seg, iters=20)
    want, _ = oracle.pagerank(g, iters=20)
    assert np.abs(r.double().cpu().numpy() - want).sum() <= 1e-6
