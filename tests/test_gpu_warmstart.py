"""Learned warm start on the GPU vs the FP64 reference (oracle/mlp.py)."""
import numpy as np
import pytest

import graphgen
import oracle
from oracle import mlp

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mods():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1608_01362_amd import cagra, warmstart
    cagra.lib()
    return cagra, warmstart


def bf16_params(net):
    import torch
    return net.weights.view(torch.bfloat16).double().cpu().numpy()


def host_norm(net):
    n = net.norm.double().cpu().numpy()
    return n[:3], 1.0 / n[3:]


def forward_error_bound(p, inter):
    """Per-row bound on |y_gpu - y| for the kernel's arithmetic against the FP64
    definition (same BF16 weights): FP32 rounding (u = 2^-24) of the
    standardization and of every dot product (at most n + 2 roundings for n
    terms), the GELU error of the erf approximation (Abramowitz & Stegun 7.1.26,
    1.5e-7, plus FP32 evaluation: 5e-7 |x| in all), the split of each hidden
    activation into two BF16 operands (|h - hi - lo| <= 2^-17 |h|), and errors
    carried through GELU (|GELU'| <= 1.13) and the next layer's weights."""
    W1, b1, W2, b2, w3, b3 = mlp.unpack(p)
    Z, z1, h1, z2, h2 = inter
    u = 2.0 ** -24
    gp = 1.13
    eg = lambda x: 5e-7 * np.abs(x)  # noqa: E731
    dz1 = 7 * u * (np.abs(Z) @ np.abs(W1).T + np.abs(b1))
    dh1 = gp * dz1 + eg(z1)
    dz2 = (dh1 + 2.0 ** -17 * np.abs(h1)) @ np.abs(W2).T + 130 * u * (np.abs(h1) @ np.abs(W2).T + np.abs(b2))
    dh2 = gp * dz2 + eg(z2)
    return dh2 @ np.abs(w3) + 66 * u * (np.abs(h2) @ np.abs(w3) + abs(b3)) + 1e-30


def test_features_match_reference(mods):
    cagra, ws = mods
    g = graphgen.rmat_graph(14, 16, 3)
    dg = cagra.DeviceGraph.from_host(g)
    for N in (1000, 1 << 20):
        seg = cagra.build_segments(dg, N, 4096, 4096)
        F = ws.features(dg, seg).double().cpu().numpy()
        want = mlp.degree_features_fast(g)
        assert np.allclose(F, want, rtol=4e-6, atol=1e-6)


def test_forward_and_gradient_match_reference(mods):
    import torch
    cagra, ws = mods
    rng = np.random.default_rng(0)
    n = 5000
    X = np.stack([rng.exponential(2, n), rng.exponential(1.5, n), rng.normal(2, 0.7, n)], axis=1)
    t = rng.normal(0, 1, n)
    net = ws.Network.create(3, X.mean(axis=0), X.std(axis=0))
    Fd = torch.from_numpy(X.astype(np.float32)).cuda()
    Td = torch.from_numpy(t.astype(np.float32)).cuda()
    p = bf16_params(net)
    mean, std = host_norm(net)
    y_ref, inter = mlp.forward(p, X.astype(np.float32).astype(np.float64), mean, std)
    y = net.forward(Fd).double().cpu().numpy()
    err = np.abs(y - y_ref)
    bound = forward_error_bound(p, inter)
    print(f"forward: max abs err {err.max():.3e}, max err/bound {np.max(err / bound):.3f}, "
          f"bound median {np.median(bound):.3e}")
    assert np.all(err <= bound)
    loss_ref, g_ref = mlp.loss_and_grad(p, X.astype(np.float32).astype(np.float64), t.astype(np.float32), mean, std)
    g, loss = net.grad(Fd, Td)
    g = g.double().cpu().numpy()
    assert abs(float(loss.item()) - loss_ref) <= 1e-4 * loss_ref
    assert np.max(np.abs(g - g_ref)) <= 1e-3 * np.max(np.abs(g_ref))
    # deterministic
    g2, _ = net.grad(Fd, Td)
    assert np.array_equal(g, g2.double().cpu().numpy())


def _splitmix64(z):
    m = (1 << 64) - 1
    z &= m
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & m
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & m
    return z ^ (z >> 31)


def test_training_inputs_match_definitions(mods):
    """Targets log(V r), the feature standardization (mean, 1/sample std) and
    the counter-based minibatch draws against their definitions on the host."""
    import torch
    cagra, ws = mods
    rng = np.random.default_rng(11)
    n = 200003
    X = np.stack([rng.exponential(2, n), rng.exponential(1.5, n), rng.normal(2, 0.7, n)], axis=1).astype(np.float32)
    F = torch.from_numpy(X).cuda()
    norm = ws.feature_norm(F).double().cpu().numpy()
    Xd = X.astype(np.float64)
    assert np.allclose(norm[:3], Xd.mean(axis=0), rtol=1e-6, atol=0)
    assert np.allclose(norm[3:], 1.0 / Xd.std(axis=0, ddof=1), rtol=1e-6, atol=0)
    const = torch.ones(10, 3, device="cuda")
    assert np.allclose(ws.feature_norm(const).cpu().numpy(), [1, 1, 1, 1e6, 1e6, 1e6])
    r = rng.dirichlet(np.ones(5000)).astype(np.float32)
    r[7] = 0.0
    t = torch.empty(5000, dtype=torch.float32, device="cuda")
    cagra._check(cagra.lib().cagra_mlp_targets(ws._p(torch.from_numpy(r).cuda()), 5000, ws._p(t), cagra._stream()),
                 "cagra_mlp_targets")
    want = np.log(5000 * np.maximum(r.astype(np.float64), 1e-30))
    assert np.allclose(t.double().cpu().numpy(), want, rtol=1e-6, atol=1e-6)
    T = torch.arange(n, dtype=torch.float32, device="cuda")
    seed, batch = 0xDEADBEEF12345, 1000
    for draw in (0, 3):
        Fb, Tb = ws.sample_rows(F, T, seed, draw, batch)
        idx = [(_splitmix64(seed + (draw * batch + i + 1) * 0x9E3779B97F4A7C15) * n) >> 64 for i in range(batch)]
        assert np.array_equal(Tb.cpu().numpy().astype(np.int64), np.array(idx))
        assert np.array_equal(Fb.cpu().numpy(), X[idx])
    # the draws cover the rows evenly (64 bins of a large draw within 6 sigma)
    _, Tb = ws.sample_rows(F, T, seed, 9, 1 << 20)
    h = np.bincount((Tb.cpu().numpy().astype(np.int64) * 64) // n, minlength=64)
    assert np.all(np.abs(h - (1 << 20) / 64) < 6 * np.sqrt((1 << 20) / 64))


def test_fused_learned_start_is_bit_identical(mods):
    """cagra_learned_start (network once per out-degree for vertices without
    in-edges) equals features -> network on every row -> softmax, bit for bit."""
    cagra, ws = mods
    g = graphgen.rmat_graph(16, 16, 8)
    dg = cagra.DeviceGraph.from_host(g)
    seg = cagra.build_segments(dg, 8192, 4096, 65536)
    F = ws.features(dg, seg)
    net = ws.Network.create(4, norm=ws.feature_norm(F))
    r_ref, ok_ref = ws.start_vector(net, F)
    r_fused, ok = ws.learned_start(net, dg, seg)
    indeg0 = float((np.diff(g.in_offsets) == 0).mean())
    print(f"vertices without in-edges: {indeg0:.3f}")
    assert ok and ok_ref and indeg0 > 0.2
    assert np.array_equal(r_ref.cpu().numpy().view(np.uint32), r_fused.cpu().numpy().view(np.uint32))


def test_adam_matches_definition(mods):
    import torch
    cagra, ws = mods
    net = ws.Network.create(1, np.zeros(3), np.ones(3))
    p = net.master.double().cpu().numpy()
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    rng = np.random.default_rng(5)
    for step in range(1, 4):
        g = rng.normal(0, 1, p.shape).astype(np.float32)
        net.adam(torch.from_numpy(g).cuda(), lr=1e-2)
        p, m, v = mlp.adam(p, g.astype(np.float64), m, v, step, lr=1e-2)
        got = net.master.double().cpu().numpy()
        assert np.max(np.abs(got - p)) <= 1e-6 * max(1.0, np.max(np.abs(p)))
    rne = net.master.to(torch.bfloat16).view(torch.int16)
    assert torch.equal(rne, net.weights)


def test_start_vector_and_fallback(mods):
    import torch
    cagra, ws = mods
    rng = np.random.default_rng(2)
    y = rng.normal(0, 3, 100000).astype(np.float32)

    class Fixed:
        def forward(self, F):
            return torch.from_numpy(y).cuda()
    r0, ok = ws.start_vector(Fixed(), torch.zeros(len(y), 3, device="cuda"))
    assert ok
    assert np.allclose(r0.double().cpu().numpy(), mlp.start_vector(y.astype(np.float64)), rtol=1e-6, atol=1e-12)
    y[17] = np.nan
    _, ok = ws.start_vector(Fixed(), torch.zeros(len(y), 3, device="cuda"))
    assert not ok


def test_learned_start_on_held_out_graph(mods):
    """Train on small R-MAT graphs, evaluate on a larger held-out one: both starts
    reach residual < 1e-6 and agree with the oracle's fixed point within the
    contraction bound; the learned start needs no more iterations."""
    import torch
    cagra, ws = mods
    Fs, Ts = [], []
    for i, sc in enumerate([10, 11, 12, 13, 12, 11, 13, 12]):
        g = graphgen.rmat_graph(sc, 16, 1000 + i)
        dg = cagra.DeviceGraph.from_host(g)
        seg = cagra.build_segments(dg, 4096, 4096, 16384)
        Fs.append(ws.features(dg, seg))
        Ts.append(ws.pagerank_target(dg, seg))
    F = torch.cat(Fs)
    T = torch.cat(Ts)
    net = ws.train(F, T, seed=0, steps=300, batch=16384, lr=3e-3, log=print)
    assert net.losses[-1] < net.losses[0]
    gt = graphgen.rmat_graph(15, 16, 5)
    dg = cagra.DeviceGraph.from_host(gt)
    seg = cagra.build_segments(dg, 32768, 8192, 65536)
    r_u, it_u, ms_u, used_u = ws.solve(dg, seg, tol=1e-6)
    r_w, it_w, ms_w, used_w = ws.solve(dg, seg, tol=1e-6, net=net)
    print(f"uniform: {it_u} iterations {ms_u:.2f} ms; learned ({used_w}): {it_w} iterations {ms_w:.2f} ms")
    assert used_w == "learned"
    ref, _ = oracle.pagerank(gt, iters=300, tol=1e-13)
    for r in (r_u, r_w):
        assert np.abs(r.double().cpu().numpy() - ref).sum() <= 0.85 / 0.15 * 1e-6 + 1e-6
    assert it_w < it_u
