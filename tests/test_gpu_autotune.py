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


def test_tuned_ppr_choice_passes_column_parity():
    """The batched personalized PageRank configuration the autotuner picks on the
    64-seed R-MAT 22 / ef 16 / seed 4 workload: every eighth column within L1
    1e-6 of the oracle's single-seed personalized PageRank after 20 iterations."""
    import torch
    assert torch.cuda.is_available()
    from paper_1608_01362_amd import autotune, cagra
    g = graphgen.rmat_graph(22, 16, 4)
    rng = np.random.default_rng(4)
    ok = np.where((np.diff(g.in_offsets) > 0) | (g.out_degree > 0))[0]
    seeds = rng.choice(ok, size=64, replace=False).astype(np.int32)
    dg = cagra.DeviceGraph.from_host(g)
    best, timed = autotune.tune_ppr(dg, seeds, cache_path=None, log=print)
    assert timed and best.ms == min(c.ms for c in timed)
    seg = cagra.build_segments(dg, best.N, best.B, best.tile_edges)
    R, _ = cagra.ppr(dg, seg, seeds, iters=20)
    R = R.double().cpu().numpy()
    for j in range(0, 64, 8):
        want = oracle.ppr(g, int(seeds[j]), 20)
        assert np.abs(R[:, j] - want).sum() <= 1e-6, j


def test_tuned_multigraph_choice_equals_single_runs(tmp_path):
    """Per-size-class choices from tune_multi: every graph of the launch equals its
    single-graph run with the same segments bit for bit; the choice is cached."""
    import torch
    from paper_1608_01362_amd import autotune, cagra
    specs = graphgen.multigraph_specs(12, seed=7, scale_lo=8, scale_hi=15, ef_lo=4, ef_hi=16)
    gs = [graphgen.rmat_graph(s.scale, s.edge_factor, s.seed) for s in specs]
    dgs = [cagra.DeviceGraph.from_host(g) for g in gs]
    cache = str(tmp_path / "multi.json")
    choice, trials = autotune.tune_multi(dgs, cache_path=cache)
    assert trials and set(choice) == {0, 1, 2}
    again, trials2 = autotune.tune_multi(dgs, cache_path=cache)
    assert trials2 == [] and again == choice
    segs = autotune.multi_segments(dgs, choice)
    mp = cagra.MultiPageRank(dgs, segs)
    mp.run_eager(20)
    torch.cuda.synchronize()
    for i, (d, s) in enumerate(zip(dgs, segs)):
        single, _, _ = cagra.pagerank(d, s, iters=20)
        assert torch.equal(mp.rank_of(i), single), i
    want, _ = oracle.pagerank(gs[-1], iters=20)
    assert np.abs(mp.rank_of(len(gs) - 1).double().cpu().numpy() - want).sum() <= 1e-6
