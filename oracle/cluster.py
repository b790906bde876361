"""Frequency-based clustering (Section 5) followed by relabelling: plain numpy.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Reading of the paper (Section 5, design and implementation of clustering):
  * a vertex is clustered when its out-degree is strictly above the average
    degree E / V;
  * clustered vertices come first, ordered by out-degree from high to low;
    the sort is stable, so equal out-degrees keep the original order;
  * every other vertex follows, in its original order;
  * the new id of a vertex is its position in that order, and the edge array
    is relabelled with the old -> new map. Each in-edge row then lists its
    sources ascending again (the layout every other step expects).

A library sort serves as the stable sort and as the row re-sort; there is no
other arithmetic.
"""
from __future__ import annotations

import numpy as np

import graphgen


def cluster_order(g):
    """Returns (perm, H): perm[i] = old id of new vertex i; H = clustered vertices."""
    od = g.out_degree.astype(np.int64)
    hot = od * g.V > g.E  # out-degree > E / V, in integers
    key = np.where(hot, od, 0)
    perm = np.argsort(-key, kind="stable")
    return perm.astype(np.int32), int(hot.sum())


def relabel(g, perm):
    """The graph with vertex perm[i] renamed i (rows ascending by new source id)."""
    V = g.V
    perm = np.asarray(perm, dtype=np.int64)
    inv = np.empty(V, dtype=np.int64)
    inv[perm] = np.arange(V)
    indeg = np.diff(g.in_offsets.astype(np.int64))
    dst = np.repeat(np.arange(V, dtype=np.int64), indeg)
    nd, ns = inv[dst], inv[g.in_sources.astype(np.int64)]
    order = np.lexsort((ns, nd))  # by new destination, then new source
    off = np.zeros(V + 1, dtype=np.int64)
    np.cumsum(indeg[perm], out=off[1:])
    return graphgen.Graph(V, off.astype(np.int32), ns[order].astype(np.int32),
                          g.out_degree[perm].astype(np.int32), name=g.name + "_clustered")


def cluster(g):
    """Returns (perm, H, relabelled graph)."""
    perm, H = cluster_order(g)
    return perm, H, relabel(g, perm)
