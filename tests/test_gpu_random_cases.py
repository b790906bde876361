"""Seeded random cases through the C ABI: graph shapes (uniform, R-MAT, stars,
chains, isolated vertices) and segment / merge-block / tile sizes drawn with
their boundaries (1, powers of two and their neighbours, the 16-bit edge-word
limit, N >= V). Each case checks, against the FP64 oracle:

- the segment layout (Section 3.1 preprocessing), byte for byte;
- one PageRank step (Sections 3.2-3.3 and the Section 4 update) from a random
  start vector, vertex by vertex: the GPU rounds each contribution once, sums
  each subgraph row in FP32 (at most indeg(v) - 1 roundings, the merge is
  exact) and rounds the result once, so |err(v)| <= (indeg(v) + 2) * 2^-24 * r(v);
  with BF16 contributions (every fourth case) each contribution's rounding
  adds at most its BF16 unit roundoff 2^-8, relative, to the gathered sum;
- every third case, one personalized step (restart vertex s) from e_s against
  the oracle's personalized PageRank, within the same bound where the answer
  is non-zero and exactly zero elsewhere;
- one label-propagation step from a random labelling, exactly;
- the standalone paper-order merge of random buffer values: the FP32 sum
  bit-identical to an FP32 evaluation in the paper's order (per destination,
  subgraphs ascending), the compensated sum within one rounding of the exact
  sum, and the integer minimum exactly.
"""
import numpy as np
import pytest

import graphgen
import oracle
from layout_check import check_layout_vectorized

pytestmark = pytest.mark.gpu

NCASES = 160
EDGE16 = 32768


def fp32_paper_order_merge(ref, partial32):
    """Section 3.3 merge in FP32, subgraphs ascending; a subgraph holds each
    destination at most once, so one subgraph is one vector update."""
    out = np.zeros(ref.V, dtype=np.float32)
    for s in range(ref.k):
        lo, hi = ref.seg_row_begin[s], ref.seg_row_begin[s + 1]
        d = ref.row_dst[lo:hi]
        out[d] = (out[d] + partial32[lo:hi]).astype(np.float32)
    return out


@pytest.fixture(scope="module")
def cagra():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1608_01362_amd import cagra as c
    c.lib()
    return c


def make_graph(rng, i):
    kind = i % 6
    if kind == 0:
        V = int(rng.integers(1, 3000))
        return graphgen.random_graph(V, int(rng.integers(0, 8 * V + 1)), int(rng.integers(1 << 30)))
    if kind == 1:
        return graphgen.rmat_graph(int(rng.integers(4, 13)), int(rng.integers(1, 17)), int(rng.integers(1 << 30)))
    if kind == 2:  # in-star with a few extra edges: one long row
        V = int(rng.integers(2, 6000))
        e = [(u, 0) for u in range(1, V)] + [(0, int(x)) for x in rng.integers(1, V, size=min(V - 1, 20))]
        return graphgen.from_edge_list(V, e)
    if kind == 3:  # out-star: many rows of length one
        V = int(rng.integers(2, 6000))
        return graphgen.from_edge_list(V, [(0, u) for u in range(1, V)])
    if kind == 4:  # chain plus back edges
        V = int(rng.integers(2, 5000))
        e = [(u, u + 1) for u in range(V - 1)] + [(u + 1, u) for u in range(0, V - 1, 3)]
        return graphgen.from_edge_list(V, e)
    # mostly isolated vertices with a dense core
    V = int(rng.integers(50, 40000))
    core = int(rng.integers(2, 50))
    e = [(u, v) for u in range(core) for v in range(core) if u != v]
    return graphgen.from_edge_list(V, e)


def draw_sizes(rng, V):
    Ns = [1, 2, 3, 63, 64, 65, 4095, 4096, EDGE16 - 1, EDGE16, EDGE16 + 1, V, V + 3,
          int(rng.integers(1, V + 4))]
    Bs = [1, 2, 7, 64, 100, 512, 4096, 8192, int(rng.integers(1, 8193))]
    Ts = [64, 100, 1000, 4096, 65536]
    for _ in range(100):
        N = int(Ns[rng.integers(len(Ns))])
        if (V + N - 1) // N <= 4096:  # keep the segment count (and the oracle's block index) small
            break
    return N, int(Bs[rng.integers(len(Bs))]), int(Ts[rng.integers(len(Ts))])


@pytest.mark.parametrize("case", range(NCASES))
def test_random_case(cagra, case):
    import torch
    rng = np.random.default_rng(1000 + case)
    g = make_graph(rng, case)
    N, B, T = draw_sizes(rng, g.V)
    print(f"case {case}: V={g.V} E={g.E} N={N} B={B} T={T}", flush=True)
    dg = cagra.DeviceGraph.from_host(g)
    seg = cagra.build_segments(dg, N, B, T)
    ref = oracle.segment(g, N, B)
    check_layout_vectorized(cagra, g, seg, ref)

    # one PageRank step from a random start vector (positive, sums to 1)
    ct = cagra.BF16 if case % 4 == 3 else cagra.F32
    bound = (2.0 ** -8 if ct == cagra.BF16 else 0.0) + (np.diff(g.in_offsets).astype(np.float64) + 2) * 2.0 ** -24
    r0 = rng.random(g.V) + 0.01
    r0 = (r0 / r0.sum()).astype(np.float32)
    st = cagra.PageRankState(dg, seg, ct)
    st.start(torch.from_numpy(r0).cuda())
    st.step()
    got = st.rank_now.double().cpu().numpy()
    want = oracle.pagerank_step_at(g, r0.astype(np.float64), np.arange(g.V, dtype=np.int32))
    rel = np.abs(got - want) / want
    assert np.all(rel <= bound), f"max rel {rel.max():.3e}"

    # one personalized step from e_s
    if case % 3 == 1:
        s = int(rng.integers(g.V))
        sp = cagra.PageRankState(dg, seg, ct, restart=s)
        sp.start()
        sp.step()
        got = sp.rank_now.double().cpu().numpy()
        want = oracle.ppr(g, s, iters=1)
        nz = want > 0
        assert np.all(got[~nz] == 0.0)
        rel = np.abs(got[nz] - want[nz]) / want[nz]
        assert np.all(rel <= bound[nz]), f"personalized: max rel {rel.max():.3e}"

    # one label-propagation step from a random labelling
    lab = rng.permutation(g.V).astype(np.int32)
    lab_in = torch.from_numpy(lab).cuda()
    lab_out = torch.empty_like(lab_in)
    partial = torch.empty(max(seg.Q, 1), dtype=torch.int32, device="cuda")
    changed = torch.zeros(1, dtype=torch.int32, device="cuda")
    cagra.labelprop_iter(seg, lab_in, partial, lab_out, changed, cagra.iter_workspace(seg))
    want_lab = oracle.segmented_labelprop_step(ref, lab)
    assert np.array_equal(lab_out.cpu().numpy(), want_lab)
    assert int(changed.item()) == int(np.count_nonzero(want_lab != lab))

    # the standalone paper-order merge of random buffer values
    if seg.Q > 0:
        p = (rng.random(seg.Q) * np.exp(rng.normal(0, 3, seg.Q))).astype(np.float32)
        pd = torch.from_numpy(p).cuda()
        out = torch.empty(g.V, dtype=torch.float32, device="cuda")
        cagra.merge(seg, cagra.SUM_F32, pd, out)
        assert np.array_equal(out.cpu().numpy(), fp32_paper_order_merge(ref, p))
        cagra.merge(seg, cagra.SUM_F32_COMP, pd, out)
        exact = oracle.merge(ref, p.astype(np.float64), oracle.SUM)
        assert np.all(np.abs(out.cpu().numpy().astype(np.float64) - exact) <= 2.0 ** -23 * exact * 1.01 + 1e-38)
        li = rng.integers(-2 ** 31, 2 ** 31 - 1, seg.Q).astype(np.int32)
        oi = torch.empty(g.V, dtype=torch.int32, device="cuda")
        cagra.merge(seg, cagra.MIN_I32, torch.from_numpy(li).cuda(), oi)
        want = oracle.merge(ref, li.astype(np.float64), oracle.MIN)
        want = np.where(np.isinf(want), 2 ** 31 - 1, want).astype(np.int64)
        assert np.array_equal(oi.cpu().numpy().astype(np.int64), want)
