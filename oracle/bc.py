"""Betweenness centrality from sampled start points (Brandes), FP64, numpy.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Reading of the paper (Section 4 EdgeMap with an active frontier; Section 6
evaluates BC from 12 start points; no algorithm is printed): Brandes'
dependency accumulation on the directed, unweighted graph. For each start s:
a level-synchronous BFS along edge directions gives depth d_s(v) and the number
of shortest paths sigma_s(v) (sigma_s(v) = sum of sigma_s(u) over in-edges
u -> v with d_s(u) = d_s(v) - 1); then, level by level from the deepest,
delta_s(u) = sum over out-edges u -> w with d_s(w) = d_s(u) + 1 of
sigma_s(u) / sigma_s(w) * (1 + delta_s(w)). BC(v) = sum over starts s != v of
delta_s(v). Unreached vertices have depth -1.
"""
from __future__ import annotations

import numpy as np


def _csr(g):
    """Out-edges (CSR) from the in-edge CSC."""
    dst = np.repeat(np.arange(g.V, dtype=np.int64), np.diff(g.in_offsets.astype(np.int64)))
    src = g.in_sources.astype(np.int64)
    order = np.lexsort((dst, src))
    off = np.zeros(g.V + 1, dtype=np.int64)
    np.add.at(off, src + 1, 1)
    return np.cumsum(off), dst[order], src[order]


def single_source(g, s: int, csr=None):
    """(depth, sigma, delta) for start s."""
    off, tgt, srt = csr if csr is not None else _csr(g)
    V = g.V
    depth = np.full(V, -1, dtype=np.int64)
    sigma = np.zeros(V)
    depth[s], sigma[s] = 0, 1.0
    levels = [np.array([s], dtype=np.int64)]
    while True:
        f = levels[-1]
        lens = off[f + 1] - off[f]
        if lens.sum() == 0:
            break
        starts = np.repeat(off[f], lens) + (np.arange(lens.sum()) - np.repeat(np.cumsum(lens) - lens, lens))
        u, w = srt[starts], tgt[starts]
        new = depth[w] < 0
        cand = np.unique(w[new])
        if cand.size == 0:
            break
        depth[cand] = len(levels)
        keep = depth[w] == len(levels)
        np.add.at(sigma, w[keep], sigma[u[keep]])
        levels.append(cand)
    delta = np.zeros(V)
    for d in range(len(levels) - 2, -1, -1):
        f = levels[d]
        lens = off[f + 1] - off[f]
        if lens.sum() == 0:
            continue
        starts = np.repeat(off[f], lens) + (np.arange(lens.sum()) - np.repeat(np.cumsum(lens) - lens, lens))
        u, w = srt[starts], tgt[starts]
        keep = depth[w] == d + 1
        np.add.at(delta, u[keep], sigma[u[keep]] / sigma[w[keep]] * (1.0 + delta[w[keep]]))
    return depth, sigma, delta


def betweenness(g, sources):
    """BC summed over the given start vertices (a start does not count for itself)."""
    csr = _csr(g)
    bc = np.zeros(g.V)
    for s in sources:
        _, _, delta = single_source(g, int(s), csr)
        delta[int(s)] = 0.0
        bc += delta
    return bc
