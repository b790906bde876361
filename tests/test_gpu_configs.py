"""The GPU path at the full sizes of the workload configurations:

- the segment layout byte-identical to the oracle's on directed R-MAT 22 / ef 16
  / seed 2 for every segment size of the sweep (8,192 ... 40,960 and 2^20);
- 256 uneven R-MAT graphs (scale U{10..20}, edge factor U{8..32}, seed 4) in one
  captured launch: every graph bit-identical to its single-graph run, the eight
  largest within L1 1e-6 of the oracle after 20 iterations;
- the learned warm start trained on 200 R-MAT graphs (scale U{16..20}, ef 16)
  and run on the held-out R-MAT 24 / ef 24 / seed 5: both starts reach an L1
  residual below 1e-6 within the contraction bound of the oracle's fixed point,
  and the learned start needs fewer iterations.
"""
import time

import numpy as np
import pytest

import graphgen
import oracle
from layout_check import check_layout_vectorized

pytestmark = pytest.mark.gpu
D = 0.85


@pytest.fixture(scope="module")
def cagra():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1608_01362_amd import cagra as c
    c.lib()
    return c


@pytest.fixture(scope="module")
def rmat22():
    return graphgen.rmat_graph(22, 16, 2)


@pytest.mark.parametrize("N", [8192, 16384, 24576, 32768, 40960, 1 << 20])
def test_builder_bit_exact_rmat22(cagra, rmat22, N):
    import torch
    g = rmat22
    dg = cagra.DeviceGraph.from_host(g)
    seg = cagra.build_segments(dg, N, 8192, 262144)
    ref = oracle.segment(g, N, 8192)
    print(f"N={N}: k={seg.k} Q={seg.Q} q={seg.q:.3f} tiles={seg.c.ntiles}")
    check_layout_vectorized(cagra, g, seg, ref)
    del seg, dg
    torch.cuda.empty_cache()


def test_multigraph256_full_spec(cagra):
    import torch
    specs = graphgen.multigraph_specs(256, seed=4)
    t0 = time.perf_counter()
    gs = [graphgen.rmat_graph(s.scale, s.edge_factor, s.seed) for s in specs]
    print(f"256 graphs, {sum(g.E for g in gs)} edges, generated in {time.perf_counter() - t0:.1f} s", flush=True)
    dgs = [cagra.DeviceGraph.from_host(g) for g in gs]
    segs = [cagra.build_segments(d, min(32768, d.V), 8192, 65536) for d in dgs]
    mp = cagra.MultiPageRank(dgs, segs)
    mp.capture(20)
    mp.replay()
    torch.cuda.synchronize()
    for i, (d, s) in enumerate(zip(dgs, segs)):
        single, _, _ = cagra.pagerank(d, s, iters=20)
        assert torch.equal(mp.rank_of(i), single), i
        assert float(mp.scalars_of(i)[3].item()) == 0.0
    largest = sorted(range(len(gs)), key=lambda i: -gs[i].E)[:8]
    for i in largest:
        want, res = oracle.pagerank(gs[i], iters=20)
        l1 = float(np.abs(mp.rank_of(i).double().cpu().numpy() - want).sum())
        print(f"graph {i}: scale {specs[i].scale} ef {specs[i].edge_factor} E {gs[i].E}: L1 {l1:.3e}")
        assert l1 <= 1e-6
        assert abs(float(mp.scalars_of(i)[1].item()) - res[-1]) <= 1e-6


def test_learned_start_full_spec(cagra):
    import torch
    from paper_1608_01362_amd import warmstart as ws
    t0 = time.perf_counter()
    Fs, Ts = [], []
    for sp in graphgen.warmstart_training_specs():
        g = graphgen.rmat_graph(sp.scale, sp.edge_factor, sp.seed)
        dg = cagra.DeviceGraph.from_host(g)
        seg = cagra.build_segments(dg, 32768, 8192, 65536)
        Fs.append(ws.features(dg, seg))
        Ts.append(ws.pagerank_target(dg, seg))
        del dg, seg
    F, T = torch.cat(Fs), torch.cat(Ts)
    del Fs, Ts
    print(f"training rows {F.shape[0]} in {time.perf_counter() - t0:.1f} s", flush=True)
    net = ws.train(F, T, seed=0, steps=600, batch=65536, lr=3e-3)
    del F, T
    gt = graphgen.rmat_graph(24, 24, 5)
    dg = cagra.DeviceGraph.from_host(gt)
    seg = cagra.build_segments(dg, 32768, 8192, 262144)
    r_u, it_u, ms_u, _ = ws.solve(dg, seg, tol=1e-6)
    r_w, it_w, ms_w, used = ws.solve(dg, seg, tol=1e-6, net=net)
    print(f"held-out R-MAT 24: uniform {it_u} iterations {ms_u:.2f} ms; learned ({used}) {it_w} iterations "
          f"{ms_w:.2f} ms", flush=True)
    assert used == "learned"
    ref, res = oracle.pagerank(gt, iters=300, tol=1e-12)
    for r in (r_u, r_w):
        l1 = float(np.abs(r.double().cpu().numpy() - ref).sum())
        assert l1 <= D / (1 - D) * 1e-6 + 1e-6, l1
    assert it_w < it_u
