"""GPU parity for collaborative filtering on the rating graph: the edge values
in the segmented order are bit-exact, and gradient steps match the FP64 oracle
within FP32 summation bounds across segment and block sizes."""
import numpy as np
import pytest

import graphgen
import oracle
from oracle import cf

pytestmark = pytest.mark.gpu
K = 64


@pytest.fixture(scope="module")
def cagra():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1608_01362_amd import cagra as c
    c.lib()
    return c


@pytest.fixture(scope="module")
def ratings():
    return graphgen.bipartite_ratings(11, 7, 12, 1)


def expected_seg_values(g, vals, ref, N):
    out = np.empty(g.E, dtype=np.float32)
    for s in range(ref.k):
        for r in range(ref.seg_row_begin[s], ref.seg_row_begin[s + 1]):
            v = ref.row_dst[r]
            lo, hi = g.in_offsets[v], g.in_offsets[v + 1]
            for p in range(ref.row_ptr[r], ref.row_ptr[r + 1]):
                u = s * N + ref.edge_src[p]
                out[p] = vals[lo + np.searchsorted(g.in_sources[lo:hi], u)]
    return out


@pytest.mark.parametrize("N", [1, 37, 512, 4096])
def test_edge_values_bit_exact(cagra, ratings, N):
    import torch
    g, vals, U, I = ratings
    if N == 1:
        g, vals, U, I = graphgen.bipartite_ratings(7, 4, 4, 2)
    dg = cagra.DeviceGraph.from_host(g)
    seg = cagra.build_segments(dg, N, 64)
    sv = cagra.segment_edge_values(dg, seg, torch.from_numpy(vals).cuda())
    want = expected_seg_values(g, vals, oracle.segment(g, N, 64), N)
    assert np.array_equal(sv.cpu().numpy()[:g.E], want)


def step_bound(g, vals, X, gamma):
    """Per entry: gamma * (FP32 summation bound of the gradient) + rounding of the update."""
    dst = np.repeat(np.arange(g.V), np.diff(g.in_offsets))
    xu, xv = np.abs(X[g.in_sources]), np.abs(X[dst])
    mag = np.abs(vals)[:, None] + (xu * xv).sum(axis=1, keepdims=True)
    S = np.zeros_like(X)
    np.add.at(S, dst, mag * xu)
    deg = np.diff(g.in_offsets)[:, None]
    return gamma * (deg + 2 * K) * 2.0 ** -23 * S


@pytest.mark.parametrize("N,B", [(1 << 30, 512), (512, 64), (4096, 512), (97, 1)])
def test_one_step_matches_oracle(cagra, ratings, N, B):
    import torch
    g, vals, U, I = ratings
    dg = cagra.DeviceGraph.from_host(g)
    seg = cagra.build_segments(dg, N, B)
    sv = cagra.segment_edge_values(dg, seg, torch.from_numpy(vals).cuda())
    X0 = cf.init_factors(g.V, K, 3, scale=0.3)
    st = cagra.CFState(dg, seg, sv, torch.from_numpy(X0).cuda())
    gamma, lam = 0.01, 0.05
    st.step(gamma, lam)
    got = st.x_now.cpu().numpy().astype(np.float64)
    X64 = X0.astype(np.float64)
    want, sq = cf.step(g, vals, X64, gamma, lam)
    tol = step_bound(g, vals, X64, gamma) + 2.0 ** -23 * np.abs(want) + 1e-12
    assert np.all(np.abs(got - want) <= tol), float(np.max(np.abs(got - want) / tol))
    assert float(st.sq.item()) == pytest.approx(sq, rel=1e-5)


def test_ten_steps_descend_and_track_oracle(cagra, ratings):
    import torch
    g, vals, U, I = ratings
    dg = cagra.DeviceGraph.from_host(g)
    seg = cagra.build_segments(dg, 1024, 256)
    sv = cagra.segment_edge_values(dg, seg, torch.from_numpy(vals).cuda())
    X0 = cf.init_factors(g.V, K, 5, scale=0.3)
    st = cagra.CFState(dg, seg, sv, torch.from_numpy(X0).cuda())
    X = X0.astype(np.float64)
    # plain gradient descent is stable for gamma below 2 / (largest Hessian eigenvalue),
    # about 2 / (max degree * K * mean(x)^2) here
    gamma, lam = 2e-4, 0.05
    sqs = []
    for _ in range(10):
        st.step(gamma, lam)
        sqs.append(float(st.sq.item()))
        X, _ = cf.step(g, vals, X, gamma, lam)
    got = st.x_now.cpu().numpy().astype(np.float64)
    assert np.max(np.abs(got - X)) <= 1e-4 * np.max(np.abs(X))
    assert all(b < a for a, b in zip(sqs, sqs[1:]))  # the squared error falls at this step size
    print(f"RMSE {np.sqrt(sqs[0] / g.E):.4f} -> {np.sqrt(sqs[-1] / g.E):.4f}")


def test_graph_without_ratings(cagra):
    import torch
    g = graphgen.from_edge_list(5, [])
    dg = cagra.DeviceGraph.from_host(g)
    seg = cagra.build_segments(dg, 2, 2)
    X0 = cf.init_factors(5, K, 1)
    st = cagra.CFState(dg, seg, torch.zeros(1, device="cuda"), torch.from_numpy(X0).cuda())
    st.step(0.1, 0.5)
    assert np.allclose(st.x_now.cpu().numpy(), X0 * (1 - 0.1 * 0.5), rtol=1e-6)
    assert float(st.sq.item()) == 0.0


@pytest.mark.parametrize("N,B,T", [(1, 4, 64), (2, 64, 64), (37, 7, 100), (4096, 512, 64)])
def test_one_step_short_rows_and_parts(cagra, N, B, T):
    """Segments of one or two sources (rows of one or two edges: nearly every
    edge starts a row) and 64-edge tiles (a wave's share splits into parts of
    zero to a few edges): the gather's per-part open rows and the completion of
    rows across parts, within the same FP32 bound."""
    import torch
    g, vals, U, I = graphgen.bipartite_ratings(7, 4, 4, 2)
    dg = cagra.DeviceGraph.from_host(g)
    seg = cagra.build_segments(dg, N, B, T)
    sv = cagra.segment_edge_values(dg, seg, torch.from_numpy(vals).cuda())
    X0 = cf.init_factors(g.V, K, 9, scale=0.3)
    st = cagra.CFState(dg, seg, sv, torch.from_numpy(X0).cuda())
    gamma, lam = 0.01, 0.05
    st.step(gamma, lam)
    got = st.x_now.cpu().numpy().astype(np.float64)
    X64 = X0.astype(np.float64)
    want, sq = cf.step(g, vals, X64, gamma, lam)
    tol = step_bound(g, vals, X64, gamma) + 2.0 ** -23 * np.abs(want) + 1e-12
    assert np.all(np.abs(got - want) <= tol), float(np.max(np.abs(got - want) / tol))
    assert float(st.sq.item()) == pytest.approx(sq, rel=1e-5)
