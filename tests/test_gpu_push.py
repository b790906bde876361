"""GPU parity for push-direction segmenting (expand, per-piece LDS scatter,
update) against the FP64 oracle.

Bars: label propagation bit-exact (per step and at the fixed point); one
PageRank step vertex by vertex within the FP32 bound (contributions rounded
once to FP32, sums exact up to 2^-56 per term, result rounded to FP32:
|err| <= 2^-22 * value + indeg * 2^-56); 20 iterations within L1 <= 1e-6 of the
FP64 oracle, as for the pull path. Sizes span many tiles, split subgraphs
(several pieces), ragged last segments, the largest segments the LDS holds
(16- and 32-bit edge words), k = 1 and N = 1, and graphs without edges."""
import numpy as np
import pytest

import graphgen
import oracle
from oracle import push as opush

pytestmark = pytest.mark.gpu

D = 0.85


@pytest.fixture(scope="module")
def cagra():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1608_01362_amd import cagra as c
    c.lib()
    return c


def push_segs(c, g, N, B, T):
    gt = graphgen.transpose(g)
    dg, dgt = c.DeviceGraph.from_host(g), c.DeviceGraph.from_host(gt)
    return dg, dgt, c.build_segments(dgt, N, B, T)


def one_step(c, g, N, B, T, seed=0):
    """One push step from a random (FP32) rank vector; returns (got, want)."""
    import torch
    dg, dgt, seg_t = push_segs(c, g, N, B, T)
    st = c.PushPageRankState(dg, seg_t)
    rng = np.random.default_rng(seed)
    r0 = rng.random(g.V).astype(np.float32)
    r0 /= r0.sum(dtype=np.float64)
    st.start(torch.from_numpy(r0.astype(np.float32)).cuda())
    st.step(D)
    got = st.rank_now.double().cpu().numpy()
    want = opush.pagerank_push_step(g, opush.push_segment(g, max(N, 1)), r0.astype(np.float64), D)
    return got, want, st, seg_t


def step_bound(g, want):
    indeg = np.diff(g.in_offsets).astype(np.float64)
    return 2.0 ** -22 * want + indeg * 2.0 ** -56 + 1e-30


@pytest.mark.parametrize("scale,ef,seed,N,B,T", [
    (10, 8, 1, 1, 64, 64),          # N = 1: every destination its own segment
    (12, 8, 2, 100, 256, 64),       # ragged last segment, many small tiles
    (13, 8, 3, 4096, 1024, 1024),   # few subgraphs, several pieces each
    (14, 16, 4, 20480, 8192, 65536),  # the largest PageRank segment, ragged last segment
    (13, 4, 5, 8192, 4096, 512),    # k = 1: one segment holds every vertex
])
def test_pagerank_push_step_vertexwise(cagra, scale, ef, seed, N, B, T):
    g = graphgen.rmat_graph(scale, ef, seed)
    got, want, st, seg_t = one_step(cagra, g, N, B, T, seed)
    err = np.abs(got - want)
    print(f"N={N} k={seg_t.k} Q={seg_t.Q} max rel {np.max(err / want):.3e}")
    assert np.all(err <= step_bound(g, want))


@pytest.mark.parametrize("N,B,T", [(64, 512, 256), (1000, 16384, 4096), (4096, 512, 1024), (8192, 8192, 65536)])
def test_pagerank_push_twenty_iterations(cagra, N, B, T):
    g = graphgen.rmat_graph(13, 8, 2)
    dg, dgt, seg_t = push_segs(cagra, g, N, B, T)
    r, _, _ = cagra.pagerank_push(dg, seg_t, iters=20)
    want, _ = oracle.pagerank(g, iters=20)
    l1 = float(np.abs(r.double().cpu().numpy() - want).sum())
    print(f"N={N} L1={l1:.3e}")
    assert l1 <= 1e-6


def test_pagerank_push_scalars_determinism_and_pull_agreement(cagra):
    import torch
    g = graphgen.rmat_graph(14, 16, 4)
    dg, dgt, seg_t = push_segs(cagra, g, 4096, 4096, 8192)
    st = cagra.PushPageRankState(dg, seg_t)
    st.start()
    r_prev = np.full(g.V, 1.0 / g.V)
    for _ in range(6):
        st.step()
        sc = st.scalars_now.cpu().numpy()
        r = st.rank_now.double().cpu().numpy()
        assert abs(sc[0] - r[g.out_degree == 0].sum()) <= 1e-12
        assert abs(sc[1] - np.abs(r - r_prev).sum()) <= 1e-12
        assert abs(sc[2] - r.sum()) <= 1e-12 and abs(sc[2] - 1.0) <= 1e-5
        r_prev = r
    r1, _, _ = cagra.pagerank_push(dg, seg_t, iters=20)
    r2, _, _ = cagra.pagerank_push(dg, seg_t, iters=20)
    assert torch.equal(r1, r2)
    seg = cagra.build_segments(dg, 4096, 4096, 8192)
    rp, _, _ = cagra.pagerank(dg, seg, iters=20)
    assert float((r1.double() - rp.double()).abs().sum()) <= 2e-6


@pytest.mark.parametrize("name", ["single_vertex", "no_edges", "instar", "outstar", "two_cycle"])
def test_pagerank_push_edge_cases(cagra, name):
    if name == "single_vertex":
        g = graphgen.from_edge_list(1, [])
    elif name == "no_edges":
        g = graphgen.from_edge_list(1000, [])
    elif name == "instar":
        g = graphgen.from_edge_list(9001, [(i, 0) for i in range(1, 9001)])
    elif name == "outstar":
        g = graphgen.from_edge_list(9001, [(0, i) for i in range(1, 9001)])
    else:
        g = graphgen.from_edge_list(7, [(0, 6), (6, 0)])
    for N, B, T in [(1, 1, 64), (64, 128, 64), (4096, 4096, 256)]:
        got, want, _, _ = one_step(cagra, g, N, B, T)
        assert np.all(np.abs(got - want) <= step_bound(g, want)), (name, N)


def test_capacity_and_argument_errors(cagra):
    import torch
    g = graphgen.rmat_graph(16, 4, 1)
    dg, dgt, seg_t = push_segs(cagra, g, 20481, 4096, 65536)  # N * 8 > LDS
    st_ws = cagra.push_workspace(seg_t)
    x = torch.zeros(g.V, dtype=torch.float32, device="cuda")
    sc = torch.zeros(4, dtype=torch.float64, device="cuda")
    vals = torch.empty(max(seg_t.Q, 1), dtype=torch.float32, device="cuda")
    with pytest.raises(cagra.CagraError) as e:
        cagra.pagerank_push_iter(dg, seg_t, D, x, x, sc, vals, x, x, sc.clone(), st_ws)
    assert e.value.status == -3  # CAGRA_E_CAPACITY: N * 8 bytes of accumulators exceed the LDS
    # a workspace one byte short is refused before anything is launched
    with pytest.raises(cagra.CagraError):
        cagra.labelprop_push_iter(seg_t, x.int(), vals.int(), x.int(), sc.int(), st_ws[:-1])


@pytest.mark.parametrize("scale,ef,seed,N,B,T", [
    (10, 4, 1, 1, 64, 64),
    (12, 8, 2, 100, 1024, 256),
    (14, 16, 3, 4096, 4096, 2048),
    (16, 4, 6, 40960, 8192, 65536),   # the largest label segment: 32-bit edge words, ragged
    (14, 4, 7, 1 << 20, 8192, 4096),  # one segment
])
def test_labelprop_push_bit_exact(cagra, scale, ef, seed, N, B, T):
    import torch
    gs = graphgen.symmetrize(graphgen.rmat_graph(scale, ef, seed))
    if N > gs.V:
        N = gs.V
    dg = cagra.DeviceGraph.from_host(gs)
    seg = cagra.build_segments(dg, N, B, T)  # undirected: the reverse graph is the graph
    # single steps from a random labelling, against the push oracle and the pull path
    rng = np.random.default_rng(seed)
    lab0 = rng.permutation(gs.V).astype(np.int32)
    ps = opush.push_segment(gs, N)
    want1 = opush.labelprop_push_step(ps, lab0)
    li = torch.from_numpy(lab0).cuda()
    lo = torch.empty_like(li)
    lp = torch.empty_like(li)
    vals = torch.empty(max(seg.Q, 1), dtype=torch.int32, device="cuda")
    ch = torch.zeros(1, dtype=torch.int32, device="cuda")
    ch2 = torch.zeros(1, dtype=torch.int32, device="cuda")
    cagra.labelprop_push_iter(seg, li, vals, lo, ch, cagra.push_workspace(seg))
    cagra.labelprop_iter(seg, li, vals, lp, ch2, cagra.iter_workspace(seg))
    assert np.array_equal(lo.cpu().numpy(), want1)
    assert torch.equal(lo, lp) and int(ch.item()) == int(ch2.item()) == int((want1 != lab0).sum())
    # the fixed point and its iteration count
    lab, it = cagra.labelprop_push(seg)
    want, it_ref = oracle.labelprop(gs)
    assert np.array_equal(lab.cpu().numpy(), want)
    assert it == it_ref


@pytest.mark.parametrize("tol,max_iters,every", [(1e-6, 100, 1), (1e-7, 100, 3), (1e-6, 4, 1), (1e-1, 100, 1)])
def test_push_solve_equals_the_waiting_loop(cagra, tol, max_iters, every):
    """cagra_pagerank_push_solve stops where a loop of push steps that reads the
    residual at every check stops, with the same ranks bit for bit; converged,
    it is within the contraction bound of the oracle's fixed point."""
    g = graphgen.rmat_graph(12, 8, 5)
    dg, dgt, seg_t = push_segs(cagra, g, 1024, 512, 4096)
    r, res, it = cagra.pagerank_push(dg, seg_t, iters=max_iters, tol=tol, check_every=every)
    st = cagra.PushPageRankState(dg, seg_t)
    st.start()
    n, resid = 0, float("inf")
    while n < max_iters:
        st.step(D)
        n += 1
        if n % every and n < max_iters:
            continue
        resid = float(st.scalars_now[1].item())
        if resid < tol:
            break
    print(f"push solve: {it} iterations (waiting loop {n}), residual {res[0]:.3e}")
    assert it == n and res[0] == resid
    assert np.array_equal(r.cpu().numpy(), st.rank_now.cpu().numpy())
    if resid < tol and tol <= 1e-6:
        star, _ = oracle.pagerank(g, iters=400, tol=1e-14)
        assert np.abs(r.double().cpu().numpy() - star).sum() <= D / (1 - D) * tol + 1e-6


def test_labelprop_push_solve_equals_the_waiting_loop(cagra):
    """cagra_labelprop_push_solve: the labels and count of a loop of push
    steps that reads the change count after every step."""
    import torch
    gs = graphgen.symmetrize(graphgen.rmat_graph(12, 4, 6))
    dg = cagra.DeviceGraph.from_host(gs)
    seg = cagra.build_segments(dg, 1024, 512, 4096)
    lab, it = cagra.labelprop_push(seg)
    cur = torch.arange(gs.V, dtype=torch.int32, device="cuda")
    nxt = torch.empty_like(cur)
    vals = torch.empty(max(seg.Q, 1), dtype=torch.int32, device="cuda")
    ch = torch.zeros(1, dtype=torch.int32, device="cuda")
    ws = cagra.push_workspace(seg)
    n = 0
    while True:
        cagra.labelprop_push_iter(seg, cur, vals, nxt, ch, ws)
        cur, nxt = nxt, cur
        n += 1
        if int(ch.item()) == 0:
            break
    assert it == n and torch.equal(lab, cur)
