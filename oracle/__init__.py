"""Plain FP64 CPU oracle for CSR-segmented pull traversal (arXiv 1608.01362).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, the smoke check and the
benchmark's CPU-baseline leg, never by the product package. It shares no code
with the GPU path; the only common module is ``graphgen`` (seeded inputs).

What each function follows:
  pagerank            Section 2 pull PageRank, normalized, dangling mass spread uniformly
  pagerank_paper_mode Section 4 PageRank listing taken literally (0.15 + 0.85*sum)
  ppr                 personalized PageRank, one restart vertex
  labelprop           synchronous min-label propagation (Section 6 application)
  segment             Section 3.1 preprocessing (subgraphs, idxMap, block index)
  segment_gather      Section 3.2 parallel segment processing (per-row buffer values)
  merge               Section 3.3 cache-aware merge
  segmented_pagerank_step  the three above composed with the PageRank update of Section 4
  cluster.cluster     Section 5 frequency-based clustering and relabelling (numpy, oracle/cluster.py)
  cf.step / gradient  collaborative filtering as gradient-descent matrix factorization (numpy, oracle/cf.py)
  bc.betweenness      Brandes' betweenness centrality from sampled starts (numpy, oracle/bc.py)

Parity pins for every function live in tests/test_oracle_*.py.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

SUM, MIN = 0, 1


def build(force: bool = True) -> str:
    """Compile oracle.c (gcc -O2, no fast-math, OpenMP) into liboracle.so."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        i32p = ctypes.POINTER(ctypes.c_int32)
        f64p = ctypes.POINTER(ctypes.c_double)
        I32, I64, F64, INT = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_int
        lib.oracle_pagerank.argtypes = [I32, i32p, i32p, i32p, F64, INT, F64, f64p, f64p, f64p, INT]
        lib.oracle_pagerank.restype = INT
        lib.oracle_pagerank_step_at.argtypes = [I32, i32p, i32p, i32p, F64, f64p, I64, i32p, f64p, INT]
        lib.oracle_dangling_mass.argtypes = [I32, i32p, f64p, INT]
        lib.oracle_dangling_mass.restype = F64
        lib.oracle_pagerank_paper_mode.argtypes = [I32, i32p, i32p, i32p, INT, f64p]
        lib.oracle_ppr.argtypes = [I32, i32p, i32p, i32p, F64, I32, INT, f64p, INT]
        lib.oracle_labelprop.argtypes = [I32, i32p, i32p, INT, i32p, INT]
        lib.oracle_labelprop.restype = INT
        lib.oracle_segment.argtypes = [I32, i32p, i32p, I32, I32, i32p, i32p, i32p, i32p, i32p]
        lib.oracle_segment.restype = I64
        lib.oracle_segment_gather.argtypes = [I64, I32, i32p, i32p, i32p, f64p, INT, f64p]
        lib.oracle_merge.argtypes = [I32, I64, I32, i32p, i32p, f64p, INT, f64p]
        _lib = lib
    return _lib


def _i32(a):
    if a is None:
        return None
    assert a.dtype == np.int32 and a.flags.c_contiguous, (a.dtype, a.flags)
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def _f64(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _threads(n):
    if n is not None:
        return n
    return max(1, min(len(os.sched_getaffinity(0)), 16))


# --------------------------------------------------------------------------- PageRank

def pagerank(g, iters: int = 20, d: float = 0.85, r0=None, tol: float = 0.0, threads=None):
    """Returns (r, residuals) with residuals[t] = ||r_{t+1}-r_t||_1. With tol > 0 stops at
    the first residual < tol (residuals then has the iterations actually run)."""
    r = np.empty(g.V, dtype=np.float64)
    res = np.zeros(max(iters, 1), dtype=np.float64)
    r0a = None if r0 is None else np.ascontiguousarray(r0, dtype=np.float64)
    t = _load().oracle_pagerank(g.V, _i32(g.in_offsets), _i32(g.in_sources), _i32(g.out_degree), d, iters,
                                tol, _f64(r0a), _f64(r), _f64(res), _threads(threads))
    return r, res[:t]


def pagerank_step_at(g, r, vertices, d: float = 0.85, threads=None):
    """One PageRank step from the full vector r, evaluated at the given vertices."""
    r = np.ascontiguousarray(r, dtype=np.float64)
    vs = np.ascontiguousarray(vertices, dtype=np.int32)
    out = np.empty(vs.shape[0], dtype=np.float64)
    _load().oracle_pagerank_step_at(g.V, _i32(g.in_offsets), _i32(g.in_sources), _i32(g.out_degree), d,
                                    _f64(r), vs.shape[0], _i32(vs), _f64(out), _threads(threads))
    return out


def dangling_mass(g, r, threads=None) -> float:
    r = np.ascontiguousarray(r, dtype=np.float64)
    return float(_load().oracle_dangling_mass(g.V, _i32(g.out_degree), _f64(r), _threads(threads)))


def pagerank_paper_mode(g, iters: int):
    R = np.empty(g.V, dtype=np.float64)
    _load().oracle_pagerank_paper_mode(g.V, _i32(g.in_offsets), _i32(g.in_sources), _i32(g.out_degree),
                                       iters, _f64(R))
    return R


def ppr(g, seed_vertex: int, iters: int = 20, d: float = 0.85, threads=None):
    r = np.empty(g.V, dtype=np.float64)
    _load().oracle_ppr(g.V, _i32(g.in_offsets), _i32(g.in_sources), _i32(g.out_degree), d, int(seed_vertex),
                       iters, _f64(r), _threads(threads))
    return r


# --------------------------------------------------------------------------- label propagation

def labelprop(gsym, max_iters: int = 1 << 20, threads=None):
    """Min-label propagation to the fixed point on an undirected graph (both directions stored).
    Returns (labels int32, iterations including the last, unchanged, one)."""
    lab = np.empty(gsym.V, dtype=np.int32)
    t = _load().oracle_labelprop(gsym.V, _i32(gsym.in_offsets), _i32(gsym.in_sources), max_iters, _i32(lab),
                                 _threads(threads))
    return lab, t


# --------------------------------------------------------------------------- segmenting

@dataclass
class Segments:
    V: int
    N: int
    B: int
    k: int
    nb: int
    Q: int
    seg_row_begin: np.ndarray  # [k+1]
    row_ptr: np.ndarray        # [Q+1]
    row_dst: np.ndarray        # [Q]  (idxMap)
    edge_src: np.ndarray       # [E]  source - s*N
    block_ptr: np.ndarray      # [(nb+1)*k], block_ptr[b*k+s]

    @property
    def q(self) -> float:
        return self.Q / self.V


def segment(g, N: int, B: int) -> Segments:
    """Section 3.1 preprocessing with segment id = src // N."""
    lib = _load()
    V = g.V
    k = (V + N - 1) // N
    nb = (V + B - 1) // B
    Q = int(lib.oracle_segment(V, _i32(g.in_offsets), _i32(g.in_sources), N, B, None, None, None, None, None))
    srb = np.empty(k + 1, dtype=np.int32)
    rp = np.empty(Q + 1, dtype=np.int32)
    rd = np.empty(max(Q, 1), dtype=np.int32)
    es = np.empty(max(g.E, 1), dtype=np.int32)
    bp = np.empty((nb + 1) * k, dtype=np.int32)
    lib.oracle_segment(V, _i32(g.in_offsets), _i32(g.in_sources), N, B, _i32(srb), _i32(rp), _i32(rd), _i32(es),
                       _i32(bp))
    return Segments(V, N, B, k, nb, Q, srb, rp, rd[:Q], es[:g.E], bp)


def segment_gather(seg: Segments, x, op: int = SUM):
    """Section 3.2: per-row buffer values (FP64) from vertex values x."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    part = np.empty(max(seg.Q, 1), dtype=np.float64)
    _load().oracle_segment_gather(seg.k, seg.N, _i32(seg.seg_row_begin), _i32(seg.row_ptr), _i32(seg.edge_src),
                                  _f64(x), op, _f64(part))
    return part[:seg.Q]


def merge(seg: Segments, partial, op: int = SUM):
    """Section 3.3: combine per-subgraph buffers into a dense vector (identity where no entry)."""
    p = np.ascontiguousarray(partial, dtype=np.float64)
    if p.shape[0] == 0:
        p = np.zeros(1, dtype=np.float64)
    out = np.empty(seg.V, dtype=np.float64)
    _load().oracle_merge(seg.V, seg.k, seg.B, _i32(seg.row_dst), _i32(seg.block_ptr), _f64(p), op, _f64(out))
    return out


def segmented_pagerank_step(g, seg: Segments, r, d: float = 0.85):
    """One PageRank step computed through segmenting: contributions r/outdeg
    (0 for dangling vertices), per-subgraph buffers, merge, then the vertex
    update with teleport and dangling mass."""
    r = np.ascontiguousarray(r, dtype=np.float64)
    outdeg = g.out_degree
    contrib = np.zeros(g.V, dtype=np.float64)
    nz = outdeg > 0
    contrib[nz] = r[nz] / outdeg[nz]
    D = dangling_mass(g, r)
    acc = merge(seg, segment_gather(seg, contrib, SUM), SUM)
    return (1.0 - d) / g.V + d * (acc + D / g.V)


def segmented_labelprop_step(seg: Segments, labels):
    lab = np.asarray(labels)
    part = segment_gather(seg, lab.astype(np.float64), MIN)
    m = merge(seg, part, MIN)
    out = np.minimum(lab.astype(np.float64), m)
    return out.astype(np.int32)
