"""GPU parity for frequency-based clustering (Section 5): the relabelled graph
is bit-exact against the oracle, the segmentation of the clustered graph is
byte-identical to the oracle's, and PageRank on the clustered, segmented graph
matches the FP64 oracle on the original graph (read through perm)."""
import json
import os

import numpy as np
import pytest

import graphgen
import oracle
from layout_check import check_layout_vectorized
from oracle import cluster as oc

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "clustering_example.json")


@pytest.fixture(scope="module")
def cagra():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1608_01362_amd import cagra as c
    c.lib()
    return c


def check_bit_exact(c, g):
    dg = c.DeviceGraph.from_host(g)
    out, perm, H = c.cluster(dg)
    rperm, rH, rg = oc.cluster(g)
    assert H == rH
    assert np.array_equal(perm.cpu().numpy(), rperm)
    assert np.array_equal(out.in_offsets.cpu().numpy(), rg.in_offsets)
    assert np.array_equal(out.in_sources.cpu().numpy()[:g.E], rg.in_sources)
    assert np.array_equal(out.out_degree.cpu().numpy(), rg.out_degree)
    return dg, out, perm, rg


def small_graphs():
    ex = json.load(open(GOLDEN))
    return [graphgen.from_edge_list(ex["V"], ex["edges"], name="hand_example"),
            graphgen.from_edge_list(1, [], name="single_vertex"),
            graphgen.from_edge_list(9, [(i, (i + 1) % 9) for i in range(9)], name="cycle"),
            graphgen.from_edge_list(5001, [(0, i) for i in range(1, 5001)], name="outstar"),
            graphgen.from_edge_list(5001, [(i, 0) for i in range(1, 5001)], name="instar"),
            graphgen.random_graph(700, 5000, 3),
            graphgen.rmat_graph(10, 8, 5),
            graphgen.rmat_graph(16, 16, 1)]


@pytest.mark.parametrize("gi", range(8))
def test_cluster_bit_exact(cagra, gi):
    g = small_graphs()[gi]
    print(g.name, g.V, g.E, flush=True)
    check_bit_exact(cagra, g)


def test_cluster_bit_exact_rmat22(cagra):
    g = graphgen.rmat_graph(22, 16, 2)
    check_bit_exact(cagra, g)


@pytest.fixture(scope="module")
def clustered20(cagra):
    g = graphgen.rmat_graph(20, 16, 7)
    dg, out, perm, rg = check_bit_exact(cagra, g)
    return out, rg


@pytest.mark.parametrize("N", [4096, 32768])
def test_builder_on_clustered_graph_bit_exact(cagra, clustered20, N):
    """Segmenting the clustered graph: its sources crowd into the first
    segments, so most steps of the builder's reorder by segment id see one or a
    few distinct ids. The layout is byte-identical to the oracle's segmentation
    of the oracle's clustered graph."""
    out, rg = clustered20
    seg = cagra.build_segments(out, N, 8192, 262144)
    ref = oracle.segment(rg, N, 8192)
    print(f"N={N}: k={seg.k} Q={seg.Q} q={seg.q:.3f}", flush=True)
    check_layout_vectorized(cagra, rg, seg, ref)


@pytest.mark.parametrize("scale,N", [(16, 4096), (20, 32768)])
def test_pagerank_on_clustered_graph(cagra, scale, N):
    """Clustering then segmenting: 20 FP32 iterations within L1 1e-6 of the FP64
    oracle on the original graph, and a smaller expansion factor q."""
    g = graphgen.rmat_graph(scale, 16, 7)
    dg = cagra.DeviceGraph.from_host(g)
    out, perm, H = cagra.cluster(dg)
    seg = cagra.build_segments(out, N, 8192)
    seg0 = cagra.build_segments(dg, N, 8192)
    rank, _, _ = cagra.pagerank(out, seg, iters=20)
    r = rank.cpu().numpy().astype(np.float64)
    ref, _ = oracle.pagerank(g, iters=20)
    p = perm.cpu().numpy()
    l1 = float(np.abs(r - ref[p]).sum())
    print(f"scale {scale}: H={H} q {seg0.q:.3f} -> {seg.q:.3f}, L1 {l1:.3e}", flush=True)
    assert l1 <= 1e-6
    assert seg.Q < seg0.Q
