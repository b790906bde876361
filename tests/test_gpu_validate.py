"""The device CSC check accepts well-formed graphs and names the first
violation of each rule in corrupted copies (every read stays in bounds: the
offsets are checked before any edge is looked at)."""
from types import SimpleNamespace

import numpy as np
import pytest

import graphgen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cagra():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1608_01362_amd import cagra as c
    c.lib()
    return c


def host(V, off, src):
    off = np.asarray(off, dtype=np.int32)
    src = np.asarray(src, dtype=np.int32)
    od = np.zeros(V, dtype=np.int32)
    return SimpleNamespace(V=V, E=int(src.size), in_offsets=off, in_sources=src, out_degree=od)


@pytest.mark.parametrize("g", [graphgen.rmat_graph(12, 8, 1), graphgen.random_graph(300, 2000, 4),
                               graphgen.from_edge_list(1, []), graphgen.from_edge_list(50, [])])
def test_well_formed_graphs_pass(cagra, g):
    cagra.validate_graph(cagra.DeviceGraph.from_host(g))


def test_rmat_full_size_passes(cagra):
    cagra.validate_graph(cagra.DeviceGraph.from_host(graphgen.rmat_graph(20, 16, 2)))


@pytest.mark.parametrize("case,text", [
    ("first", "in_offsets[0] is not 0"),
    ("last", "in_offsets[V] is not E"),
    ("decreasing", "decreases at vertex 1"),
    ("range", "out of range at edge 3"),
    ("negative", "out of range at edge 0"),
    ("order", "not strictly ascending (or duplicated) at edge 1"),
    ("duplicate", "not strictly ascending (or duplicated) at edge 5"),
    ("self", "self-loop at edge 0"),
])
def test_corrupted_graphs_are_named(cagra, case, text):
    # base graph, V = 4: rows 0: [1, 2], 1: [0, 3], 2: [0, 1, 3], 3: []
    off, src = [0, 2, 4, 7, 7], [1, 2, 0, 3, 0, 1, 3]
    if case == "first":
        off = [1, 2, 4, 7, 7]
    elif case == "last":
        off = [0, 2, 4, 6, 6]
    elif case == "decreasing":
        off = [0, 3, 2, 7, 7]
    elif case == "range":
        src = [1, 2, 0, 4, 0, 1, 3]
    elif case == "negative":
        src = [-1, 2, 0, 3, 0, 1, 3]
    elif case == "order":
        src = [2, 1, 0, 3, 0, 1, 3]  # row 0 descending
    elif case == "duplicate":
        src = [1, 2, 0, 3, 1, 1, 3]  # row 2 lists 1 twice
    elif case == "self":
        src = [0, 2, 0, 3, 0, 1, 3]  # row 0 lists itself
    dg = cagra.DeviceGraph.from_host(host(4, off, src))
    with pytest.raises(cagra.CagraError) as e:
        cagra.validate_graph(dg)
    assert e.value.status == -1
    assert text in str(e.value), str(e.value)
