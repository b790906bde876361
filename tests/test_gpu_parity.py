"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle.

Bars: segment layout and label propagation bit-exact; FP32 PageRank within
L1 <= 1e-6 of the FP64 oracle after 20 iterations; float gathers/merges within
FP32 summation bounds; BF16 within the bound d*u/(1-d) (u = 2^-8, the BF16
unit roundoff) that follows from rounding every contribution once per step.
"""
import json
import os

import numpy as np
import pytest

import graphgen
import oracle

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "segmenting_example.json")


@pytest.fixture(scope="module")
def cagra():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1608_01362_amd import cagra as c
    c.lib()
    return c


def _host(t):
    return t.cpu().numpy()


def tiny_graphs():
    ex = json.load(open(GOLDEN))
    gs = [graphgen.from_edge_list(ex["V"], ex["edges"], name="paper_example"),
          graphgen.from_edge_list(1, [], name="single_vertex"),
          graphgen.from_edge_list(7, [(0, 6), (6, 0)], name="mostly_isolated"),
          graphgen.from_edge_list(5001, [(i, 0) for i in range(1, 5001)], name="instar5000"),
          graphgen.rmat_graph(8, 4, 3),
          graphgen.random_graph(300, 2000, 9)]
    return gs


def check_layout(c, g, N, B, T):
    dg = c.DeviceGraph.from_host(g)
    seg = c.build_segments(dg, N, B, T)
    ref = oracle.segment(g, N, B)
    h = seg.host()
    assert seg.c.k == ref.k and seg.c.nb == ref.nb and seg.Q == ref.Q
    assert np.array_equal(h["seg_row_begin"], ref.seg_row_begin)
    assert np.array_equal(h["row_ptr"], ref.row_ptr)
    assert np.array_equal(h["row_dst"], ref.row_dst)
    assert np.array_equal(h["row_dst_lo"].view(np.uint16).astype(np.int64), ref.row_dst.astype(np.int64) % B)
    assert np.array_equal(h["block_ptr"], ref.block_ptr)
    # edge words: 16-bit (flag bit 15) for N <= 32768, else 32-bit (flag bit 31)
    if N <= c.EDGE16_MAX_N:
        assert h["edge_src"].dtype == np.int16
        es, top = h["edge_src"].view(np.uint16).astype(np.uint32), 15
    else:
        assert h["edge_src"].dtype == np.int32
        es, top = h["edge_src"].view(np.uint32), 31
    assert np.array_equal((es & ((1 << top) - 1)).astype(np.int32), ref.edge_src)
    flags = np.zeros(g.E, dtype=bool)
    flags[ref.row_ptr[:-1]] = True
    assert np.array_equal((es >> top).astype(bool), flags)
    # gather tiles: row-aligned, inside one subgraph, covering every edge once
    te, ts, sr = h["tile_edge"], h["tile_seg"], h["tile_span_row"].reshape(-1, c.TILE_WAVES)
    nt = seg.c.ntiles
    assert te[0] == 0 and te[nt] == g.E and np.all(np.diff(te) >= 0)
    seg_e = ref.row_ptr[ref.seg_row_begin]
    rowstarts = set(ref.row_ptr.tolist())
    for t in range(nt):
        s = ts[t]
        assert seg_e[s] <= te[t] <= te[t + 1] <= seg_e[s + 1]
        assert te[t] in rowstarts
        ln = te[t + 1] - te[t]
        sl = -(-ln // c.TILE_WAVES)
        for w in range(c.TILE_WAVES):
            b = min(te[t] + w * sl, te[t + 1])
            lo, hi = ref.seg_row_begin[s], ref.seg_row_begin[s + 1]
            assert sr[t, w] == lo + np.searchsorted(ref.row_ptr[lo:hi], b, side="left")
    return dg, seg, ref


@pytest.mark.parametrize("gi", range(6))
@pytest.mark.parametrize("N,B,T", [(1, 1, 64), (3, 2, 64), (64, 100, 128), (1000, 16384, 65536), (10 ** 6, 7, 64)])
def test_builder_bit_exact(cagra, gi, N, B, T):
    g = tiny_graphs()[gi]
    if (g.V + N - 1) // N > 32768:
        pytest.skip("more than 32768 segments")
    check_layout(cagra, g, N, B, T)


@pytest.mark.parametrize("N,B,T", [(4096, 2048, 4096), (16384, 16384, 65536), (32768, 8192, 65536),
                                   (32769, 8192, 65536), (40960, 16384, 65536)])
def test_builder_bit_exact_rmat16(cagra, N, B, T):
    check_layout(cagra, graphgen.rmat_graph(16, 16, 1), N, B, T)


@pytest.mark.parametrize("N", [32767, 32768, 32769])
def test_gather_edge_word_width_boundary(cagra, N):
    """Around the 16/32-bit edge word switch: local indices use all 15 bits
    (R-MAT 16 has 65,536 vertices, so the segments are full), ragged shares."""
    import torch
    g = graphgen.rmat_graph(16, 16, 1)
    dg = cagra.DeviceGraph.from_host(g)
    seg = cagra.build_segments(dg, N, 8192, 1000)
    ref = oracle.segment(g, N, 8192)
    rng = np.random.default_rng(N)
    x = rng.random(g.V).astype(np.float32)
    part = torch.full((seg.Q,), float("nan"), dtype=torch.float32, device="cuda")
    cagra.segment_gather(seg, cagra.SUM_F32, cagra.F32, torch.from_numpy(x).cuda(), part)
    want = oracle.segment_gather(ref, x.astype(np.float64), oracle.SUM)
    got = _host(part).astype(np.float64)
    assert np.all(np.abs(got - want) <= _rows_len(ref) * 2.0 ** -23 * want + 1e-30)
    lab = rng.permutation(g.V).astype(np.int32)
    pl = torch.full((seg.Q,), -7, dtype=torch.int32, device="cuda")
    cagra.segment_gather(seg, cagra.MIN_I32, cagra.I32, torch.from_numpy(lab).cuda(), pl)
    want_l = oracle.segment_gather(ref, lab.astype(np.float64), oracle.MIN)
    assert np.array_equal(_host(pl), want_l.astype(np.int32))


def _rows_len(ref):
    return np.diff(ref.row_ptr)


@pytest.mark.parametrize("gi", [0, 3, 4, 5])
@pytest.mark.parametrize("N,T", [(1, 64), (5, 64), (128, 64), (1000, 256), (40960, 65536), (50000, 64)])
def test_gather_sum_min(cagra, gi, N, T):
    import torch
    g = tiny_graphs()[gi]
    dg, seg, ref = check_layout(cagra, g, N, 16, T) if g.V < 600 else (None, None, None)
    if dg is None:
        dg = cagra.DeviceGraph.from_host(g)
        seg = cagra.build_segments(dg, N, 16, T)
        ref = oracle.segment(g, N, 16)
    rng = np.random.default_rng(gi * 100 + N)
    x = rng.random(g.V).astype(np.float32)
    xd = torch.from_numpy(x).cuda()
    part = torch.full((max(seg.Q, 1),), float("nan"), dtype=torch.float32, device="cuda")
    cagra.segment_gather(seg, cagra.SUM_F32, cagra.F32, xd, part)
    want = oracle.segment_gather(ref, x.astype(np.float64), oracle.SUM)
    got = _host(part)[:seg.Q].astype(np.float64)
    ln = _rows_len(ref)
    assert np.all(np.abs(got - want) <= ln * 2.0 ** -23 * want + 1e-30)
    # bf16 values: the oracle runs on the same bf16-rounded values
    xb = torch.from_numpy(x).to(torch.bfloat16)
    cagra.segment_gather(seg, cagra.SUM_F32, cagra.BF16, xb.cuda().view(torch.int16), part)
    want_b = oracle.segment_gather(ref, xb.to(torch.float64).numpy(), oracle.SUM)
    got_b = _host(part)[:seg.Q].astype(np.float64)
    assert np.all(np.abs(got_b - want_b) <= ln * 2.0 ** -23 * want_b + 1e-30)
    # integer minimum: exact
    lab = rng.permutation(g.V).astype(np.int32)
    pl = torch.full((max(seg.Q, 1),), -7, dtype=torch.int32, device="cuda")
    cagra.segment_gather(seg, cagra.MIN_I32, cagra.I32, torch.from_numpy(lab).cuda(), pl)
    want_l = oracle.segment_gather(ref, lab.astype(np.float64), oracle.MIN)
    assert np.array_equal(_host(pl)[:seg.Q], want_l.astype(np.int32))


def fp32_sequential_merge(ref, partial32):
    """Section 3.3 merge evaluated in FP32 in the paper's order (subgraphs ascending)."""
    out = np.zeros(ref.V, dtype=np.float32)
    for b in range(ref.nb):
        for s in range(ref.k):
            lo, hi = ref.block_ptr[b * ref.k + s], ref.block_ptr[(b + 1) * ref.k + s]
            d = ref.row_dst[lo:hi]
            out[d] = (out[d] + partial32[lo:hi]).astype(np.float32)
    return out


@pytest.mark.parametrize("N,B", [(1, 1), (7, 5), (64, 64), (500, 3000), (4096, 16384)])
def test_merge_ordered(cagra, N, B):
    import math
    import torch
    g = graphgen.rmat_graph(12, 8, 17)
    dg = cagra.DeviceGraph.from_host(g)
    if (g.V + N - 1) // N > 32768:
        pytest.skip("too many segments")
    seg = cagra.build_segments(dg, N, B, 256)
    ref = oracle.segment(g, N, B)
    rng = np.random.default_rng(N + B)
    p = (rng.random(seg.Q) * np.exp(rng.normal(0, 3, seg.Q))).astype(np.float32)
    pd = torch.from_numpy(p).cuda()
    out = torch.empty(g.V, dtype=torch.float32, device="cuda")
    cagra.merge(seg, cagra.SUM_F32, pd, out)
    assert np.array_equal(_host(out), fp32_sequential_merge(ref, p))  # same order, same rounding
    cagra.merge(seg, cagra.SUM_F32_COMP, pd, out)
    exact = oracle.merge(ref, p.astype(np.float64), oracle.SUM)
    assert np.all(np.abs(_host(out).astype(np.float64) - exact) <= 2.0 ** -23 * np.abs(exact) * 1.01 + 1e-38)
    li = rng.integers(-2 ** 31, 2 ** 31 - 1, seg.Q).astype(np.int32)
    oi = torch.empty(g.V, dtype=torch.int32, device="cuda")
    cagra.merge(seg, cagra.MIN_I32, torch.from_numpy(li).cuda(), oi)
    want = oracle.merge(ref, li.astype(np.float64), oracle.MIN)
    want = np.where(np.isinf(want), 2 ** 31 - 1, want).astype(np.int64)
    assert np.array_equal(_host(oi).astype(np.int64), want)
    del math


def run_pagerank(cagra, g, N, B, T, iters=20, contrib=None):
    dg = cagra.DeviceGraph.from_host(g)
    seg = cagra.build_segments(dg, N, B, T)
    r, _, _ = cagra.pagerank(dg, seg, iters=iters, contrib_type=contrib if contrib is not None else cagra.F32)
    return r, dg, seg


def test_pagerank_rmat16_n16384(cagra):
    """R-MAT scale 16, edge factor 16, seed 1; 4 segments of 16,384 vertices; 20 iterations."""
    g = graphgen.rmat_graph(16, 16, 1)
    r, dg, seg = run_pagerank(cagra, g, 16384, 16384, 65536)
    assert seg.k == 4
    want, res = oracle.pagerank(g, iters=20)
    l1 = np.abs(_host(r).astype(np.float64) - want).sum()
    print(f"L1={l1:.3e} q={seg.q:.3f}")
    assert l1 <= 1e-6


@pytest.mark.parametrize("N,B,T", [(1, 1, 64), (7, 33, 64), (64, 1024, 256), (1000, 16384, 4096),
                                   (4096, 512, 65536), (1 << 20, 16384, 64)])
def test_pagerank_segment_sweep(cagra, N, B, T):
    g = graphgen.rmat_graph(13, 8, 2)
    if (g.V + N - 1) // N > 32768:
        pytest.skip("too many segments")
    r, dg, seg = run_pagerank(cagra, g, N, B, T)
    want, _ = oracle.pagerank(g, iters=20)
    assert np.abs(_host(r).astype(np.float64) - want).sum() <= 1e-6


def test_pagerank_scalars_and_determinism(cagra):
    import torch
    g = graphgen.rmat_graph(14, 16, 4)
    dg = cagra.DeviceGraph.from_host(g)
    seg = cagra.build_segments(dg, 4096, 4096, 8192)
    st = cagra.PageRankState(dg, seg)
    st.start()
    r_prev = np.full(g.V, 1.0 / g.V)
    for t in range(6):
        st.step()
        sc = _host(st.scalars_now)
        r = _host(st.rank_now).astype(np.float64)
        assert abs(sc[0] - r[g.out_degree == 0].sum()) <= 1e-12
        assert abs(sc[1] - np.abs(r - r_prev).sum()) <= 1e-12
        assert abs(sc[2] - r.sum()) <= 1e-12 and abs(sc[2] - 1.0) <= 1e-5
        r_prev = r
    r1, _, _ = cagra.pagerank(dg, seg, iters=20)
    r2, _, _ = cagra.pagerank(dg, seg, iters=20)
    assert torch.equal(r1, r2)


def test_pagerank_bf16_bound(cagra):
    g = graphgen.rmat_graph(14, 16, 5)
    r, dg, seg = run_pagerank(cagra, g, 8192, 8192, 65536, contrib=1)
    want, _ = oracle.pagerank(g, iters=20)
    l1 = np.abs(_host(r).astype(np.float64) - want).sum()
    print(f"bf16 L1={l1:.3e}")
    assert l1 <= 0.85 * 2.0 ** -8 / 0.15


@pytest.mark.parametrize("scale,ef,seed,N", [(10, 4, 1, 1), (12, 8, 2, 100), (14, 16, 3, 4096), (14, 4, 6, 1 << 20)])
def test_labelprop_exact(cagra, scale, ef, seed, N):
    g = graphgen.symmetrize(graphgen.rmat_graph(scale, ef, seed))
    if (g.V + N - 1) // N > 32768:
        pytest.skip("too many segments")
    dg = cagra.DeviceGraph.from_host(g)
    seg = cagra.build_segments(dg, N, 4096, 4096)
    lab, it = cagra.labelprop(seg)
    want, it_ref = oracle.labelprop(g)
    assert np.array_equal(_host(lab), want)
    assert it == it_ref


def test_abi_errors_on_device(cagra):
    import ctypes
    import torch
    g = graphgen.rmat_graph(10, 8, 1)
    dg = cagra.DeviceGraph.from_host(g)
    seg = cagra.build_segments(dg, 256, 256, 1024)
    ws = cagra.iter_workspace(seg)
    small = torch.empty(8, dtype=torch.uint8, device="cuda")
    x = torch.zeros(g.V, dtype=torch.float32, device="cuda")
    sc = torch.zeros(4, dtype=torch.float64, device="cuda")
    with pytest.raises(cagra.CagraError) as e:
        cagra.pagerank_iter(dg, seg, 0.85, cagra.F32, x, x, sc, x, x, x, sc, small)
    assert e.value.status == cagra.E_BUFFER
    with pytest.raises(cagra.CagraError) as e:
        cagra.pagerank_iter(dg, seg, 1.5, cagra.F32, x, x, sc, x, x, x, sc, ws)
    assert e.value.status == cagra.E_INVALID
    with pytest.raises(cagra.CagraError) as e:
        cagra.segment_gather(seg, cagra.MIN_I32, cagra.F32, x, x)
    assert e.value.status == cagra.E_INVALID
    del ctypes


def test_merge_item_bound_below_count(cagra):
    """max_items equal to nb makes the merge take every block whole (one work
    item, no slots): the same ranks bit for bit as the split merge. A bound
    between nb and the built item count is invalid: the workspace sized from it
    has no room for the slots of split blocks, so the merge touches no slot,
    merges nothing and turns the scalars into NaN."""
    g = graphgen.from_edge_list(5001, [(i, 0) for i in range(1, 5001)] + [(0, 1), (2, 3)])
    dg = cagra.DeviceGraph.from_host(g)
    seg = cagra.build_segments(dg, 64, 256, 4096)
    total, nb = int(_host(seg.arrays["block_items"])[-1]), int(seg.c.nb)
    assert total >= nb + 2 and seg.c.max_items == total  # split blocks; bound lowered to the count
    st = cagra.PageRankState(dg, seg)
    st.start()
    st.step()
    want = _host(st.rank_now).copy()
    assert np.isfinite(_host(st.scalars_now)).all()
    try:
        seg.c.max_items = nb
        whole = cagra.PageRankState(dg, seg)  # no slots in its workspace
        whole.start()
        whole.step()
        assert np.array_equal(_host(whole.rank_now), want)
        seg.c.max_items = nb + 1
        bad = cagra.PageRankState(dg, seg)  # room for two slots only
        bad.start()
        bad.step()
        assert np.isnan(_host(bad.scalars_now)).all()
    finally:
        seg.c.max_items = total


@pytest.mark.parametrize("name", ["instar", "clustered_rmat14"])
def test_fused_merge_split_blocks(cagra, name):
    """Merge blocks with far more entries than the mean are split into several
    work items whose exact fixed-point sums are combined with atomics. The
    result must equal the vertex update applied to the exact sum of the buffer
    entries (within one FP32 rounding), and repeat bit for bit."""
    import torch
    from fractions import Fraction
    if name == "instar":
        g = graphgen.from_edge_list(5001, [(i, 0) for i in range(1, 5001)] + [(0, 1), (2, 3)])
        N, B = 64, 256
    else:
        from oracle import cluster as oc
        _, _, g = oc.cluster(graphgen.rmat_graph(14, 16, 4))
        N, B = 1024, 512
    dg = cagra.DeviceGraph.from_host(g)
    seg = cagra.build_segments(dg, N, B, 4096)
    items = _host(seg.arrays["block_items"])
    assert items[-1] > seg.c.nb and items[-1] <= seg.c.max_items  # some block is split
    ranks = []
    for rep in range(2):
        st = cagra.PageRankState(dg, seg)
        st.start()
        st.step()
        st.step_split()  # gather, then the split merge
        ranks.append(_host(st.rank_now).copy())
        part = _host(st.partial)[:seg.Q].astype(np.float64)
        # after start, step, step_split: scalars[1] holds the first step's output,
        # whose dangling mass is the second step's input
        s0 = float(_host(st.scalars[1])[0])
    assert np.array_equal(ranks[0], ranks[1])
    # against the oracle's step from the same FP32 input vector, vertex by vertex:
    # contributions rounded once, FP32 row sums (at most indeg - 1 roundings), an
    # exact merge and one final rounding give (indeg + 2) * 2^-24 relative
    r1 = _host(st.rank[1 - st.cur]).astype(np.float64)
    step = oracle.pagerank_step_at(g, r1, np.arange(g.V, dtype=np.int32))
    indeg = np.diff(g.in_offsets)
    assert np.all(np.abs(ranks[0].astype(np.float64) - step) <= (indeg + 2) * 2.0 ** -24 * step)
    ref = oracle.segment(g, N, B)
    exact = [Fraction(0)] * g.V
    scale = 2 ** 56
    for r in range(seg.Q):
        x = Fraction(part[r]) * scale
        m = (abs(x) + Fraction(1, 2)).__floor__()
        exact[ref.row_dst[r]] += (m if x >= 0 else -m)
    d = 0.85
    base = (1.0 - d) / g.V + d * s0 / g.V
    want = np.array([base + d * float(Fraction(int(e)) / scale) for e in exact], dtype=np.float64)
    got = ranks[0].astype(np.float64)
    assert np.all(np.abs(got - want) <= np.spacing(np.float32(want)).astype(np.float64) * 1.01)


@pytest.mark.parametrize("N", [1, 3, 7])
def test_builder_bit_exact_many_segments(cagra, N):
    """Up to the 32,768-segment limit (keys of 15 bits: three stable digit passes
    in the segment-major reorder), ragged last segment."""
    from layout_check import check_layout_vectorized
    g = graphgen.rmat_graph(15, 8, 6)
    assert -(-g.V // N) <= 32768
    dg = cagra.DeviceGraph.from_host(g)
    seg = cagra.build_segments(dg, N, 512, 4096)
    check_layout_vectorized(cagra, g, seg, oracle.segment(g, N, 512))
