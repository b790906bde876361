"""GPU parity for betweenness centrality (Brandes) as level-synchronous
segmented pulls with an active frontier: depths bit-exact, path counts and
centralities against the FP64 oracle within FP32 rounding, across segment sizes
(skipped inactive segments included)."""
import numpy as np
import pytest

import graphgen
from oracle import bc as obc

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cagra():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1608_01362_amd import cagra as c
    c.lib()
    return c


def segs(c, g, N, B=64, T=None):
    gt = graphgen.transpose(g)
    dg, dgt = c.DeviceGraph.from_host(g), c.DeviceGraph.from_host(gt)
    return dg, dgt, c.build_segments(dg, N, B, T), c.build_segments(dgt, N, B, T)


def starts(g, n, seed):
    cand = np.flatnonzero(g.out_degree > 0)
    return np.random.default_rng(seed).choice(cand, size=min(n, cand.size), replace=False)


def check(c, g, N, sources, B=64):
    dg, dgt, seg, seg_t = segs(c, g, N, B)
    got, levels = c.betweenness(seg, seg_t, sources)
    want = obc.betweenness(g, sources)
    got = got.cpu().numpy().astype(np.float64)
    assert np.allclose(got, want, rtol=2e-5, atol=1e-5 * max(1.0, want.max())), \
        float(np.max(np.abs(got - want) / (np.abs(want) + 1)))
    return levels


@pytest.mark.parametrize("name", ["random", "star", "path", "grid"])
def test_small_graphs(cagra, name):
    if name == "random":
        g = graphgen.random_graph(300, 1500, 4)
    elif name == "star":
        g = graphgen.from_edge_list(50, [(i, 0) for i in range(1, 50)] + [(0, i) for i in range(1, 50)])
    elif name == "path":
        g = graphgen.from_edge_list(40, [(i, i + 1) for i in range(39)])
    else:
        R, C = 12, 13
        g = graphgen.from_edge_list(R * C, [(r * C + c, r * C + c + 1) for r in range(R) for c in range(C - 1)] +
                                    [(r * C + c, (r + 1) * C + c) for r in range(R - 1) for c in range(C)])
    for N in (1, 7, 64, 1 << 20):
        check(cagra, g, N, starts(g, 6, 1))


@pytest.mark.parametrize("N", [64, 1000, 4096, 1 << 20])
def test_rmat14(cagra, N):
    g = graphgen.rmat_graph(14, 16, 3)
    levels = check(cagra, g, N, starts(g, 6, 2))
    print(f"N={N}: BFS levels per start {levels}")


def test_depths_and_path_counts(cagra):
    import torch
    g = graphgen.rmat_graph(16, 16, 5)
    s = int(starts(g, 1, 3)[0])
    dg, dgt, seg, seg_t = segs(cagra, g, 4096)
    st = cagra.BCState(seg, seg_t)
    st.add_source(s)
    depth, sigma, _ = obc.single_source(g, s)
    assert np.array_equal(st.depth.cpu().numpy(), depth.astype(np.int32))
    got = st.sigma.cpu().numpy().astype(np.float64)
    reached = depth >= 0
    assert np.allclose(got[reached], sigma[reached], rtol=1e-6)
    assert np.all(got[~reached] == 0)


def test_rmat20_two_starts(cagra):
    g = graphgen.rmat_graph(20, 16, 7)
    levels = check(cagra, g, 32768, starts(g, 2, 4), B=8192)
    print(f"R-MAT 20: BFS levels per start {levels}")
