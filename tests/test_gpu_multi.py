"""Many uneven graphs in one persistent launch per kernel, captured into one HIP
graph: every graph's result equals its single-graph run bit for bit, replays of
the captured graph equal the eager run, and sampled graphs match the oracle."""
import numpy as np
import pytest

import graphgen
import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cagra():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1608_01362_amd import cagra as c
    c.lib()
    return c


@pytest.fixture(scope="module")
def batch(cagra):
    specs = graphgen.multigraph_specs(24, seed=4, scale_lo=6, scale_hi=14, ef_lo=2, ef_hi=16)
    gs = [graphgen.rmat_graph(s.scale, s.edge_factor, s.seed) for s in specs]
    gs.append(graphgen.from_edge_list(3, [(0, 1)]))  # tiny, mostly isolated
    dgs = [cagra.DeviceGraph.from_host(g) for g in gs]
    segs = [cagra.build_segments(d, min(2048, max(d.V, 1)), 1024, 4096) for d in dgs]
    return gs, dgs, segs


def test_multi_equals_single_and_oracle(cagra, batch):
    import torch
    gs, dgs, segs = batch
    mp = cagra.MultiPageRank(dgs, segs)
    mp.run_eager(20)
    torch.cuda.synchronize()
    for i, (g, d, s) in enumerate(zip(gs, dgs, segs)):
        single, _, _ = cagra.pagerank(d, s, iters=20)
        assert torch.equal(mp.rank_of(i), single), i
    for i in (0, 7, 15, len(gs) - 1):
        want, res = oracle.pagerank(gs[i], iters=20)
        assert np.abs(mp.rank_of(i).double().cpu().numpy() - want).sum() <= 1e-6
        sc = mp.scalars_of(i).cpu().numpy()
        assert abs(sc[1] - res[-1]) <= 1e-6 and abs(sc[2] - 1.0) <= 1e-5


def test_captured_graph_replays_match_eager(cagra, batch):
    import torch
    gs, dgs, segs = batch
    mp = cagra.MultiPageRank(dgs, segs)
    mp.run_eager(20)
    torch.cuda.synchronize()
    eager = mp.rank[mp.cur].clone()
    eager_sc = mp.scalars[mp.cur].clone()
    mp.capture(20)
    for rep in range(3):
        mp.rank[0].fill_(-1.0)  # eager work between replays
        mp.rank[1].fill_(-1.0)
        torch.cuda.synchronize()
        mp.replay()
        torch.cuda.synchronize()
        assert torch.equal(mp.rank[mp.cur], eager), rep
        assert torch.equal(mp.scalars[mp.cur], eager_sc), rep
