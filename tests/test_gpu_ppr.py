"""Batched personalized PageRank (segmented SpMM over 64 seed columns) vs the
FP64 oracle's single-seed personalized PageRank, column by column."""
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


def seeds_for(g, n, seed):
    rng = np.random.default_rng(seed)
    ok = np.where((np.diff(g.in_offsets) > 0) | (g.out_degree > 0))[0]
    return rng.choice(ok, size=n, replace=False).astype(np.int32)


@pytest.mark.parametrize("N,B,T", [(1, 1, 64), (100, 64, 256), (4096, 512, 4096), (1 << 20, 512, 16384)])
def test_ppr_columns_match_oracle(cagra, N, B, T):
    g = graphgen.rmat_graph(12, 8, 7)
    dg = cagra.DeviceGraph.from_host(g)
    seg = cagra.build_segments(dg, N, B, T)
    seeds = seeds_for(g, 64, 1)
    R, st = cagra.ppr(dg, seg, seeds, iters=20)
    R = R.double().cpu().numpy()
    for j in range(0, 64, 7):
        want = oracle.ppr(g, int(seeds[j]), 20)
        assert np.abs(R[:, j] - want).sum() <= 1e-6, j
    sc = st.scalars_now.cpu().numpy()
    assert np.all(np.abs(sc[:, 2] - 1.0) <= 1e-5)
    assert np.allclose(sc[:, 2], R.sum(axis=0), atol=1e-9)


def test_ppr_partial_batch_and_single_column_identical(cagra):
    g = graphgen.rmat_graph(11, 16, 9)
    dg = cagra.DeviceGraph.from_host(g)
    seg = cagra.build_segments(dg, 512, 256, 1024)
    seeds = seeds_for(g, 5, 2)
    R5, _ = cagra.ppr(dg, seg, seeds, iters=20)
    for j in range(5):
        R1, _ = cagra.ppr(dg, seg, seeds[j:j + 1], iters=20)
        assert np.array_equal(R1[:, 0].cpu().numpy(), R5[:, j].cpu().numpy())  # lanes are independent
    # unused columns stay zero
    import torch
    st = cagra.PPRState(dg, seg, seeds)
    st.start()
    st.step()
    full = st.rank[st.cur].view(g.V, 64)
    assert torch.count_nonzero(full[:, 5:]) == 0


def test_ppr_rmat22_64_seeds(cagra):
    """R-MAT scale 22, edge factor 16, seed 4; 64 seed vertices; restart 0.15; 20 iterations."""
    g = graphgen.rmat_graph(22, 16, 4)
    dg = cagra.DeviceGraph.from_host(g)
    seg = cagra.build_segments(dg, 1 << 20, 512, 16384)
    seeds = seeds_for(g, 64, 4)
    R, st = cagra.ppr(dg, seg, seeds, iters=20)
    R = R.double().cpu().numpy()
    worst = 0.0
    for j in (0, 9, 18, 27, 36, 45, 54, 63):
        want = oracle.ppr(g, int(seeds[j]), 20)
        l1 = np.abs(R[:, j] - want).sum()
        worst = max(worst, l1)
        assert l1 <= 1e-6, (j, l1)
    print(f"worst column L1 {worst:.3e}")


@pytest.mark.parametrize("N,B", [(1, 1), (300, 128), (4096, 1024), (1 << 20, 4096)])
def test_single_seed_iteration_matches_oracle(cagra, N, B):
    """The single-vector iteration with a restart vertex (teleport and dangling
    mass returned to the seed) against the oracle's personalized PageRank, for
    seeds with and without out-edges; mass stays 1."""
    g = graphgen.rmat_graph(12, 8, 7)
    dg = cagra.DeviceGraph.from_host(g)
    seg = cagra.build_segments(dg, N, B, 4096)
    dangling = np.where((g.out_degree == 0) & (np.diff(g.in_offsets) > 0))[0]
    for s in [int(x) for x in seeds_for(g, 3, 5)] + [int(dangling[0])]:
        st = cagra.PageRankState(dg, seg, restart=s)
        st.start()
        for _ in range(20):
            st.step()
        want = oracle.ppr(g, s, 20)
        l1 = np.abs(st.rank_now.double().cpu().numpy() - want).sum()
        assert l1 <= 1e-6, (s, l1)
        sc = st.scalars_now.cpu().numpy()
        assert abs(sc[2] - 1.0) <= 1e-5 and sc[3] == 0.0


def test_single_seed_solve_to_residual(cagra):
    g = graphgen.rmat_graph(14, 16, 3)
    dg = cagra.DeviceGraph.from_host(g)
    seg = cagra.build_segments(dg, 4096, 2048, 16384)
    s = int(seeds_for(g, 1, 9)[0])
    res = cagra.pagerank_solve(dg, seg, tol=1e-6, restart=s)
    assert res.converged
    star = oracle.ppr(g, s, 300)
    assert np.abs(res.rank.double().cpu().numpy() - star).sum() <= 0.85 / 0.15 * 1e-6 + 1e-6


@pytest.mark.parametrize("tol,max_iters,every", [(1e-6, 100, 1), (1e-7, 100, 2), (1e-1, 100, 1), (1e-6, 6, 1),
                                                 (1e-6, 9, 4)])
def test_ppr_solve_equals_the_waiting_loop(cagra, tol, max_iters, every):
    """cagra_ppr_solve (the step after a check queued before the check is read
    back) stops where a loop that waits at every check stops, with the same
    vectors bit for bit; converged columns are within the contraction bound of
    the oracle's personalized PageRank."""
    import torch
    g = graphgen.rmat_graph(12, 8, 7)
    dg = cagra.DeviceGraph.from_host(g)
    seg = cagra.build_segments(dg, 1024, 512, 4096)
    seeds = seeds_for(g, 64, 3)
    st = cagra.PPRState(dg, seg, seeds)
    r = st.solve(tol=tol, max_iters=max_iters, check_every=every)
    got = st.ranks().clone()
    w = cagra.PPRState(dg, seg, seeds)
    w.start()
    it, worst, conv = 0, float("inf"), False
    while it < max_iters:
        w.step()
        it += 1
        if it % every and it < max_iters:
            continue
        worst = float(w.scalars_now[:, 1].max().item())
        if worst < tol:
            conv = True
            break
    print(f"ppr solve: {r.iters} iterations, residual {r.residual:.3e}, converged {r.converged}")
    assert (r.converged, r.iters) == (conv, it) and r.residual == worst
    assert torch.equal(got, w.ranks())
    if conv and tol <= 1e-6:
        R = got.double().cpu().numpy()
        for j in range(0, 64, 21):
            want = oracle.ppr(g, int(seeds[j]), 200)
            assert np.abs(R[:, j] - want).sum() <= 0.85 / 0.15 * tol + 1e-6, j


def test_ppr_solve_partial_batch_matches_full_batch_columns(cagra):
    """cagra_ppr_solve over 5 seeds: the columns stop where the 5-column
    waiting loop stops, columns past ncols stay zero, and each column equals
    the same column of a 64-seed solve stopped at the same iteration."""
    import torch
    g = graphgen.rmat_graph(11, 16, 9)
    dg = cagra.DeviceGraph.from_host(g)
    seg = cagra.build_segments(dg, 512, 256, 1024)
    seeds = seeds_for(g, 64, 5)
    st5 = cagra.PPRState(dg, seg, seeds[:5])
    r5 = st5.solve(tol=1e-6)
    full = st5.rank[st5.cur].view(g.V, 64)
    assert r5.converged and torch.count_nonzero(full[:, 5:]) == 0
    st64 = cagra.PPRState(dg, seg, seeds)
    st64.start()
    for _ in range(r5.iters):
        st64.step()
    assert torch.equal(st5.ranks(), st64.ranks()[:, :5])  # columns are independent lanes
    assert float(st64.scalars_now[:5, 1].max().item()) == r5.residual
