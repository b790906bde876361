"""GPU numerics beyond the per-algorithm parity tests: the BF16 conversion of
contributions against torch's round-to-nearest-even on every tie class and a
large random sample of bit patterns, and resuming an iteration from a saved
vector (checkpoint/resume) against an uninterrupted run."""
from types import SimpleNamespace

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


def test_bf16_contributions_round_to_nearest_even(cagra):
    """contrib = rank / 1 stored as BF16 must equal torch's RNE conversion for
    every finite value class: random bit patterns, exact ties (both parities),
    values just below and above ties, zeros, infinities, the largest finite
    value and normal values near the bottom of the range."""
    import torch
    rng = np.random.default_rng(0)
    hi = np.arange(1 << 16, dtype=np.uint32) << 16
    bits = np.concatenate([
        rng.integers(0, 1 << 32, size=1 << 22, dtype=np.uint64).astype(np.uint32),
        hi | 0x8000, hi | 0x7FFF, hi | 0x8001,
        np.array([0, 0x80000000, 0x7F800000, 0xFF800000, 0x7F7FFFFF, 0xFF7FFFFF, 0x00800000, 0x80800000],
                 dtype=np.uint32)])
    x = bits.view(np.float32)
    exp = (bits >> 23) & 0xFF
    x = x[(exp != 0xFF) | ((bits & 0x7FFFFF) == 0)]   # no NaN
    x = x[((x.view(np.uint32) >> 23) & 0xFF) != 0]    # normal values and infinities (no zeros/denormals)
    x = np.concatenate([x, np.array([0.0, -0.0], dtype=np.float32)])
    V = int(x.size)
    rank = torch.from_numpy(x.copy()).cuda()
    od = torch.ones(V, dtype=torch.int32, device="cuda")
    off = torch.zeros(V + 1, dtype=torch.int32, device="cuda")
    g = SimpleNamespace(c=cagra.CGraph(V, 0, off.data_ptr(), off.data_ptr(), od.data_ptr()))
    contrib = torch.empty(V, dtype=torch.int16, device="cuda")
    scal = torch.zeros(4, dtype=torch.float64, device="cuda")
    ws = torch.empty(32 * ((V + 16383) // 16384) + 256, dtype=torch.uint8, device="cuda")
    cagra.pagerank_init(g, cagra.BF16, rank, contrib, scal, ws)
    want = torch.from_numpy(x).to(torch.bfloat16).view(torch.int16)
    got = contrib.cpu()
    bad = (got != want).nonzero()
    assert bad.numel() == 0, [(hex(int(x.view(np.uint32)[i])), hex(int(got[i]) & 0xFFFF), hex(int(want[i]) & 0xFFFF))
                              for i in bad[:8, 0].tolist()]


def test_bf16_conversion_exhaustive(cagra):
    """Every one of the 2^32 FP32 bit patterns through the BF16 contribution
    path (rank / 1), in chunks, against torch's round-to-nearest-even: equal
    bits for every non-NaN pattern (denormals and both zeros included), and a
    NaN for every NaN pattern (payloads are not compared)."""
    import torch
    chunk = 1 << 26
    V = chunk
    od = torch.ones(V, dtype=torch.int32, device="cuda")
    off = torch.zeros(V + 1, dtype=torch.int32, device="cuda")
    g = SimpleNamespace(c=cagra.CGraph(V, 0, off.data_ptr(), off.data_ptr(), od.data_ptr()))
    contrib = torch.empty(V, dtype=torch.int16, device="cuda")
    scal = torch.zeros(4, dtype=torch.float64, device="cuda")
    ws = torch.empty(32 * ((V + 16383) // 16384) + 256, dtype=torch.uint8, device="cuda")
    for c0 in range(0, 1 << 32, chunk):
        bits = torch.arange(c0, c0 + chunk, dtype=torch.int64, device="cuda")
        bits = torch.where(bits >= (1 << 31), bits - (1 << 32), bits).to(torch.int32)
        x = bits.view(torch.float32)
        cagra.pagerank_init(g, cagra.BF16, x, contrib, scal, ws)
        want = x.to(torch.bfloat16).view(torch.int16)
        nan_in = torch.isnan(x)
        got_nan = ((contrib & 0x7F80) == 0x7F80) & ((contrib & 0x7F) != 0)
        bad = ((contrib != want) & ~nan_in) | (nan_in & ~got_nan)
        n_bad = int(bad.sum().item())
        if n_bad:
            i = int(bad.nonzero()[0, 0].item())
            raise AssertionError(f"{n_bad} mismatches in chunk {c0:#x}; first pattern {(c0 + i) & 0xFFFFFFFF:#010x}: "
                                 f"got {int(contrib[i].item()) & 0xFFFF:#06x} want {int(want[i].item()) & 0xFFFF:#06x}")


def test_pagerank_resume_from_saved_vector(cagra):
    """Ten iterations, a host copy of the rank vector, a fresh state started
    from it and ten more iterations give the uninterrupted twenty-iteration
    result (the restart recomputes contributions and the dangling mass from the
    saved ranks; the FP64 dangling sum may differ in its last bits, so ranks
    may differ by one FP32 rounding)."""
    import torch
    g = graphgen.rmat_graph(16, 16, 7)
    dg = cagra.DeviceGraph.from_host(g)
    seg = cagra.build_segments(dg, 16384, 8192, 65536)
    full = cagra.PageRankState(dg, seg)
    full.start()
    for _ in range(20):
        full.step()
    r20 = full.rank_now.double().cpu().numpy()
    part = cagra.PageRankState(dg, seg)
    part.start()
    for _ in range(10):
        part.step()
    saved = part.rank_now.cpu().clone()   # checkpoint through host memory
    del part
    res = cagra.PageRankState(dg, seg)
    res.start(saved.cuda())
    for _ in range(10):
        res.step()
    r = res.rank_now.double().cpu().numpy()
    assert np.all(np.abs(r - r20) <= 2.0 ** -23 * r20)
    want, _ = oracle.pagerank(g, iters=20)
    assert np.abs(r - want).sum() <= 1e-6


def test_labelprop_resume_from_saved_labels(cagra):
    """Three steps, saved labels, then steps to the fixed point from them: the
    same labels and the same total step count as one uninterrupted run."""
    import torch
    gs = graphgen.symmetrize(graphgen.rmat_graph(14, 8, 3))
    dg = cagra.DeviceGraph.from_host(gs)
    seg = cagra.build_segments(dg, 4096, 4096, 8192)
    want, it_ref = oracle.labelprop(gs)
    ws = cagra.iter_workspace(seg)
    part = torch.empty(max(seg.Q, 1), dtype=torch.int32, device="cuda")
    ch = torch.zeros(1, dtype=torch.int32, device="cuda")
    a = torch.arange(gs.V, dtype=torch.int32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        cagra.labelprop_iter(seg, a, part, b, ch, ws)
        a, b = b, a
    saved = a.cpu().clone()
    cur = saved.cuda()
    nxt = torch.empty_like(cur)
    steps = 3
    while True:
        cagra.labelprop_iter(seg, cur, part, nxt, ch, ws)
        cur, nxt = nxt, cur
        steps += 1
        if int(ch.item()) == 0:
            break
    assert np.array_equal(cur.cpu().numpy(), want)
    assert steps == it_ref
