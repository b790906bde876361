"""Push-direction segmenting, plain FP64 numpy (TEST INFRASTRUCTURE ONLY).

Imported by tests/ only; shares no code with the GPU path.

The paper builds the pull (in-edge) traversal and notes that segmenting applies
to the push (out-edge) version as well (Section 3, and Section 2's description
of push: each vertex updates the destinations of its outgoing edges). Here the
push version is written out directly:

  out_edges         out-edge CSR of a graph given as in-edge CSC (plain counting sort)
  push_segment      Section 3.1 applied to out-edges: subgraph s holds the edges
                    u -> v with v in [s*N, (s+1)*N), in rows of ascending source u
  push_sums         per-subgraph scatter: each edge adds x[u] to its destination's
                    accumulator; a segment's accumulators are complete after its
                    own subgraph (no merge across subgraphs is needed)
  pagerank_push_step / labelprop_push_step   the Section 4 vertex updates on top

Pins: tests/test_oracle_push.py (against the pull oracle, a closed form and
brute force on a tiny graph).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


def out_edges(g):
    """(out_offsets[V+1], out_targets[E]) with each row's targets ascending."""
    V = g.V
    dst = np.repeat(np.arange(V, dtype=np.int64), np.diff(g.in_offsets.astype(np.int64)))
    src = g.in_sources.astype(np.int64)
    order = np.lexsort((dst, src))  # by source, then destination
    off = np.zeros(V + 1, dtype=np.int64)
    np.add.at(off, src + 1, 1)
    off = np.cumsum(off)
    return off, dst[order]


@dataclass
class PushSegments:
    V: int
    N: int
    k: int
    rows: list        # per subgraph: sources u with at least one edge into segment s (ascending)
    row_ptr: list     # per subgraph: [len(rows)+1] edge offsets
    local_dst: list   # per subgraph: destination - s*N of each edge, grouped by row

    @property
    def Q(self) -> int:
        return int(sum(len(r) for r in self.rows))


def push_segment(g, N: int) -> PushSegments:
    """Cut the out-edges by destination segment (Section 3.1 with the roles of
    source and destination exchanged)."""
    off, tgt = out_edges(g)
    V = g.V
    k = (V + N - 1) // N
    src = np.repeat(np.arange(V, dtype=np.int64), np.diff(off))
    seg = tgt // N
    rows, row_ptr, local = [], [], []
    for s in range(k):
        m = seg == s
        u, v = src[m], tgt[m]  # already ordered by (u, v)
        ru, cnt = np.unique(u, return_counts=True)
        rows.append(ru.astype(np.int64))
        row_ptr.append(np.concatenate([[0], np.cumsum(cnt)]).astype(np.int64))
        local.append((v - s * N).astype(np.int64))
    return PushSegments(V, N, k, rows, row_ptr, local)


def push_sums(ps: PushSegments, x, op: str = "sum"):
    """acc[v] = sum (or min) over edges u -> v of x[u]; identity where v has no in-edge."""
    x = np.asarray(x)
    if op == "sum":
        acc = np.zeros(ps.V, dtype=np.float64)
    else:
        acc = np.full(ps.V, np.iinfo(np.int64).max, dtype=np.int64)
    for s in range(ps.k):
        vals = x[ps.rows[s]]                                   # expand: one value per row
        per_edge = np.repeat(vals, np.diff(ps.row_ptr[s]))     # the row's value on each of its edges
        dst = ps.local_dst[s] + s * ps.N
        if op == "sum":
            np.add.at(acc, dst, per_edge.astype(np.float64))
        else:
            np.minimum.at(acc, dst, per_edge.astype(np.int64))
    return acc


def pagerank_push_step(g, ps: PushSegments, r, d: float = 0.85):
    """One normalized PageRank step (teleport, dangling mass spread uniformly)
    with the neighbour sums taken in the push direction."""
    r = np.asarray(r, dtype=np.float64)
    od = g.out_degree.astype(np.int64)
    contrib = np.zeros(g.V, dtype=np.float64)
    nz = od > 0
    contrib[nz] = r[nz] / od[nz]
    D = float(r[~nz].sum())
    acc = push_sums(ps, contrib, "sum")
    return (1.0 - d) / g.V + d * (acc + D / g.V)


def labelprop_push_step(ps: PushSegments, labels):
    lab = np.asarray(labels).astype(np.int64)
    return np.minimum(lab, push_sums(ps, lab, "min")).astype(np.int32)
