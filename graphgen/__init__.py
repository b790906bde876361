"""Seeded synthetic graph inputs (R-MAT) shared by the CPU checker and the GPU path.

Nothing here computes any part of the graph method: it only produces the input
arrays (an in-edge CSR, "CSC", plus out-degrees) that both sides consume.

The C source ``rmat.c`` is compiled with gcc into ``libgraphgen.so`` next to it
(``build()``); the functions below marshal numpy arrays through ctypes.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rmat.c")
_LIB = os.path.join(_HERE, "libgraphgen.so")
_lib = None

RMAT_A, RMAT_B, RMAT_C = 0.57, 0.19, 0.19


def build(force: bool = True) -> str:
    """Compile rmat.c with gcc/OpenMP into libgraphgen.so."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        p32 = ctypes.POINTER(ctypes.c_int32)
        lib.gg_rmat_edges.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                                      ctypes.c_double, ctypes.c_uint64, p32, p32, p32, ctypes.c_int]
        lib.gg_permutation.argtypes = [ctypes.c_int32, ctypes.c_uint64, p32]
        lib.gg_edges_to_csc.argtypes = [ctypes.c_int32, ctypes.c_int64, p32, p32, ctypes.c_int, p32, p32,
                                        ctypes.c_int]
        lib.gg_edges_to_csc.restype = ctypes.c_int64
        lib.gg_out_degree.argtypes = [ctypes.c_int32, ctypes.c_int64, p32, p32, ctypes.c_int]
        lib.gg_csc_both_directions.argtypes = [ctypes.c_int32, p32, p32, p32, p32, ctypes.c_int]
        lib.gg_splitmix_at.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
        lib.gg_splitmix_at.restype = ctypes.c_uint64
        lib.gg_pair_values.argtypes = [ctypes.c_int32, p32, p32, ctypes.c_uint64, ctypes.c_void_p, ctypes.c_int]
        _lib = lib
    return _lib


def _p(a):
    if a is None:
        return None
    assert a.dtype == np.int32 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def default_threads() -> int:
    return max(1, min(len(os.sched_getaffinity(0)), 16))


@dataclass
class Graph:
    """Directed graph as an in-edge CSR: sources of edges u->v are
    in_sources[in_offsets[v]:in_offsets[v+1]], ascending, no self-loops, no duplicates."""
    V: int
    in_offsets: np.ndarray
    in_sources: np.ndarray
    out_degree: np.ndarray
    name: str = ""

    @property
    def E(self) -> int:
        return int(self.in_offsets[-1])


def splitmix_at(seed: int, i: int) -> int:
    return int(_load().gg_splitmix_at(seed & (2**64 - 1), i))


def permutation(V: int, seed: int) -> np.ndarray:
    perm = np.empty(V, dtype=np.int32)
    _load().gg_permutation(V, seed, _p(perm))
    return perm


def rmat_edges(scale: int, edge_factor: int, seed: int, permute: bool = True,
               a=RMAT_A, b=RMAT_B, c=RMAT_C, threads: int | None = None):
    V = 1 << scale
    m = edge_factor * V
    perm = permutation(V, seed) if permute else None
    src = np.empty(m, dtype=np.int32)
    dst = np.empty(m, dtype=np.int32)
    _load().gg_rmat_edges(scale, m, a, b, c, seed, _p(perm), _p(src), _p(dst), threads or default_threads())
    return src, dst


def edges_to_graph(V: int, src: np.ndarray, dst: np.ndarray, drop_self: bool = True,
                   threads: int | None = None, name: str = "") -> Graph:
    src = np.ascontiguousarray(src, dtype=np.int32)
    dst = np.ascontiguousarray(dst, dtype=np.int32)
    m = src.shape[0]
    if m:
        assert src.min() >= 0 and src.max() < V and dst.min() >= 0 and dst.max() < V
    off = np.empty(V + 1, dtype=np.int32)
    buf = np.empty(max(m, 1), dtype=np.int32)
    th = threads or default_threads()
    E = int(_load().gg_edges_to_csc(V, m, _p(src), _p(dst), 1 if drop_self else 0, _p(off), _p(buf), th))
    ins = buf[:E].copy() if E < buf.shape[0] // 2 else buf[:E]
    outdeg = np.empty(V, dtype=np.int32)
    _load().gg_out_degree(V, E, _p(ins), _p(outdeg), th)
    return Graph(V, off, ins, outdeg, name)


def rmat_graph(scale: int, edge_factor: int, seed: int, permute: bool = True,
               threads: int | None = None) -> Graph:
    """Directed R-MAT (a,b,c,d = .57,.19,.19,.05), seeded vertex permutation,
    self-loops and duplicate edges removed."""
    src, dst = rmat_edges(scale, edge_factor, seed, permute, threads=threads)
    g = edges_to_graph(1 << scale, src, dst, True, threads, name=f"rmat{scale}_ef{edge_factor}_s{seed}")
    del src, dst
    return g


def symmetrize(g: Graph, threads: int | None = None) -> Graph:
    """Undirected version: every edge in both directions, duplicates removed."""
    E = g.E
    src = np.empty(2 * E, dtype=np.int32)
    dst = np.empty(2 * E, dtype=np.int32)
    th = threads or default_threads()
    _load().gg_csc_both_directions(g.V, _p(g.in_offsets), _p(g.in_sources), _p(src), _p(dst), th)
    return edges_to_graph(g.V, src, dst, True, th, name=g.name + "_sym")


def transpose(g: Graph, threads: int | None = None) -> Graph:
    """The graph with every edge reversed (its in-edges are g's out-edges)."""
    dst = np.repeat(np.arange(g.V, dtype=np.int32), np.diff(g.in_offsets))
    return edges_to_graph(g.V, dst, g.in_sources, True, threads, name=g.name + "_T")


def from_edge_list(V: int, edges, name: str = "") -> Graph:
    """Small graphs for tests: edges is an iterable of (u, v) meaning u -> v."""
    e = np.asarray(list(edges), dtype=np.int64).reshape(-1, 2)
    return edges_to_graph(V, e[:, 0].astype(np.int32), e[:, 1].astype(np.int32), True, 1, name)


def random_graph(V: int, m: int, seed: int) -> Graph:
    """Small uniform random digraph (for property tests): m sampled edges."""
    rng = np.random.default_rng(seed)
    src = rng.integers(0, V, size=m).astype(np.int32)
    dst = rng.integers(0, V, size=m).astype(np.int32)
    return edges_to_graph(V, src, dst, True, 1, name=f"rand{V}_{m}_{seed}")


@dataclass
class MultiGraphSpec:
    scale: int
    edge_factor: int
    seed: int


def bipartite_ratings(user_scale: int, item_scale: int, edge_factor: int, seed: int,
                      threads: int | None = None):
    """Synthetic rating graph: 2^user_scale users and 2^item_scale items; R-MAT
    draws (user, item) pairs (the item is the R-MAT column shifted down to
    item_scale bits), duplicates removed; every rating is an edge in both
    directions (users 0..U-1, items U..U+I-1) with value 1..5 from a hash of the
    pair. Returns (Graph, values[E] in the graph's in-edge order, U, I)."""
    assert item_scale <= user_scale
    U, I = 1 << user_scale, 1 << item_scale
    u, d = rmat_edges(user_scale, edge_factor, seed, threads=threads)
    it = (d >> (user_scale - item_scale)).astype(np.int32)
    src = np.concatenate([u, U + it]).astype(np.int32)
    dst = np.concatenate([U + it, u]).astype(np.int32)
    del u, d, it
    g = edges_to_graph(U + I, src, dst, True, threads, name=f"ratings_u{user_scale}_i{item_scale}_ef{edge_factor}_s{seed}")
    vals = np.empty(max(g.E, 1), dtype=np.float32)
    _load().gg_pair_values(g.V, _p(g.in_offsets), _p(g.in_sources), (seed * 7919 + 11) & (2**64 - 1),
                           vals.ctypes.data, threads or default_threads())
    return g, vals[:g.E], U, I


def multigraph_specs(count: int, seed: int, scale_lo: int = 10, scale_hi: int = 20,
                     ef_lo: int = 8, ef_hi: int = 32):
    """Per-graph (scale, edge factor, seed) for a batch of independent R-MAT graphs,
    drawn uniformly (inclusive ranges) from a seeded stream."""
    specs = []
    for i in range(count):
        r = splitmix_at(seed * 1000003 + 17, i)
        sc = scale_lo + (r & 0xFFFF) % (scale_hi - scale_lo + 1)
        ef = ef_lo + ((r >> 16) & 0xFFFF) % (ef_hi - ef_lo + 1)
        specs.append(MultiGraphSpec(int(sc), int(ef), int((r >> 32) & 0x7FFFFFFF)))
    return specs


def warmstart_training_specs(count: int = 200, seed: int = 1000, scale_lo: int = 16, scale_hi: int = 20,
                             edge_factor: int = 16):
    """(scale, edge factor, seed) of the warm-start training graphs: scale drawn
    uniformly (inclusive) from a numpy generator seeded with `seed`, graph i
    seeded seed + i."""
    import numpy as np
    rng = np.random.default_rng(seed)
    return [MultiGraphSpec(int(rng.integers(scale_lo, scale_hi + 1)), edge_factor, seed + i) for i in range(count)]
