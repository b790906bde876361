"""Segment-layout comparison shared by the GPU builder tests (not a test module)."""
import numpy as np


def check_layout_vectorized(c, g, seg, ref):
    """Every segment array against the oracle's, with the tile checks in numpy."""
    h = seg.host()
    assert seg.c.k == ref.k and seg.c.nb == ref.nb and seg.Q == ref.Q
    for name in ("seg_row_begin", "row_ptr", "row_dst", "block_ptr"):
        assert np.array_equal(h[name], getattr(ref, name)), name
    B = seg.c.B
    assert np.array_equal(h["row_dst_lo"].view(np.uint16).astype(np.int64), ref.row_dst.astype(np.int64) % B)
    if seg.c.N <= c.EDGE16_MAX_N:
        es, top = h["edge_src"].view(np.uint16).astype(np.uint32), 15
    else:
        es, top = h["edge_src"].view(np.uint32), 31
    assert np.array_equal((es & ((1 << top) - 1)).astype(np.int32), ref.edge_src)
    flags = np.zeros(g.E, dtype=bool)
    flags[ref.row_ptr[:-1]] = True
    assert np.array_equal((es >> top).astype(bool), flags)
    te, ts = h["tile_edge"].astype(np.int64), h["tile_seg"].astype(np.int64)
    nt = seg.c.ntiles
    sr = h["tile_span_row"].reshape(-1, c.TILE_WAVES)[:nt]
    assert te[0] == 0 and te[nt] == g.E and np.all(np.diff(te) >= 0)
    seg_e = ref.row_ptr[ref.seg_row_begin].astype(np.int64)
    assert np.all(seg_e[ts] <= te[:nt]) and np.all(te[1:] <= seg_e[ts + 1])
    # tiles start on row starts; an empty tile (an empty last segment) may sit at the end, E = row_ptr[Q]
    rpe = ref.row_ptr.astype(np.int64)
    pos = np.searchsorted(rpe, te[:nt])
    assert np.all(rpe[np.minimum(pos, len(rpe) - 1)] == te[:nt])
    rp = ref.row_ptr[:-1].astype(np.int64)
    ln = te[1:] - te[:nt]
    sl = -(-ln // c.TILE_WAVES)
    b = np.minimum(te[:nt, None] + np.arange(c.TILE_WAVES)[None, :] * sl[:, None], te[1:, None])
    assert np.array_equal(sr, np.searchsorted(rp, b, side="left"))
