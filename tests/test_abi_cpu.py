"""The C ABI library loads without a GPU, exports every function the header
declares, and rejects bad arguments before any HIP call."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cagra.h")


@pytest.fixture(scope="module")
def cagra():
    from paper_1608_01362_amd import cagra as c
    if not os.path.exists(c.LIB_PATH):
        from paper_1608_01362_amd import _build
        _build.build()
    c.lib()
    return c


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cagra_[a-z0-9_]+)\s*\(", text)))


def test_exports_match_header(cagra):
    decl = declared_functions()
    assert decl == sorted(cagra.EXPORTS)
    out = subprocess.run(["nm", "-D", "--defined-only", cagra.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (cagra_\w+)", out))
    assert set(decl) <= exported
    L = cagra.lib()
    for name in decl:
        assert hasattr(L, name)
    assert L.cagra_abi_version() == cagra.ABI_VERSION == 2


def test_status_strings(cagra):
    L = cagra.lib()
    assert L.cagra_status_string(0) == b"CAGRA_OK"
    assert L.cagra_status_string(-4) == b"CAGRA_E_BUFFER"
    assert L.cagra_status_string(-6) == b"CAGRA_E_NOT_CONVERGED"
    assert L.cagra_status_string(-7) == b"CAGRA_E_RANGE"
    assert L.cagra_status_string(99) == b"CAGRA_E_UNKNOWN"


def _graph(c, V=10, E=5, off=1, src=1, od=1):
    return c.CGraph(V, E, off, src, od)


def _seg(c, N=4, B=4, T=64):
    s = c.CSegments()
    s.N, s.B, s.tile_edges = N, B, T
    return s


@pytest.mark.parametrize("mut,status", [
    (dict(V=0), -1), (dict(E=-1), -1), (dict(E=2 ** 31), -2), (dict(off=None), -1), (dict(src=None), -1),
])
def test_build_rejects_bad_graph(cagra, mut, status):
    L = cagra.lib()
    g = _graph(cagra, **mut)
    s = _seg(cagra)
    assert L.cagra_build_segments(ctypes.byref(g), ctypes.byref(s), None, 0, None) == status
    assert L.cagra_last_error()


@pytest.mark.parametrize("mut,status", [
    (dict(N=0), -1), (dict(B=0), -1), (dict(B=16385), -1), (dict(T=63), -1), (dict(N=1, V=40000), -3),
])
def test_build_rejects_bad_params(cagra, mut, status):
    L = cagra.lib()
    V = mut.pop("V", 10)
    g = _graph(cagra, V=V)
    s = _seg(cagra, **mut)
    assert L.cagra_build_segments(ctypes.byref(g), ctypes.byref(s), None, 0, None) == status


def test_query_needs_workspace(cagra):
    L = cagra.lib()
    g = _graph(cagra, V=100, E=50)
    s = _seg(cagra)
    need = L.cagra_query_workspace_bytes(100, 50, 4)
    assert need >= 50 * 4
    assert L.cagra_build_segments(ctypes.byref(g), ctypes.byref(s), None, 0, None) == -4
    assert L.cagra_build_segments(ctypes.byref(g), ctypes.byref(s), 1, need - 1, None) == -4


def test_calls_reject_unbuilt_segments(cagra):
    L = cagra.lib()
    s = _seg(cagra)
    assert L.cagra_segment_gather(ctypes.byref(s), 0, 0, 1, 1, None) == -1
    assert L.cagra_merge(ctypes.byref(s), 0, 1, 1, None) == -1
    assert L.cagra_labelprop_iter(ctypes.byref(s), 1, 1, 1, 1, 1, 1 << 20, None) == -1
    g = _graph(cagra)
    assert L.cagra_pagerank_iter(ctypes.byref(g), ctypes.byref(s), 0.85, -1, 0, 1, 1, 1, 1, 1, 1, 1, 1, 1 << 20,
                                 None) == -1
    assert L.cagra_pagerank_init(ctypes.byref(g), 5, 1, 1, 1, 1, 1 << 20, None) == -1
    assert L.cagra_pagerank_init(ctypes.byref(g), 0, 1, 1, 1, 1, 0, None) == -4
    assert L.cagra_segment_gather(None, 0, 0, 1, 1, None) == -1


def _fake_built(c, V=100, N=10, B=10, E=50, Q=20, align=16):
    s = _seg(c, N=N, B=B)
    s.V, s.E, s.Q, s.k, s.nb, s.ntiles = V, E, Q, -(-V // N), -(-V // B), 1
    for name in ("seg_row_begin", "row_ptr", "row_dst", "block_ptr", "tile_edge", "tile_seg", "tile_span_row",
                 "row_dst_lo", "block_items"):
        setattr(s, name, 4096)
    s.max_items = s.nb
    s.edge_src = 4096 + (0 if align == 16 else 4)
    return s


def test_validation_of_built_segments(cagra):
    L = cagra.lib()
    s = _fake_built(cagra, align=4)
    assert L.cagra_segment_gather(ctypes.byref(s), 0, 0, 1, 1, None) == -1  # misaligned edge_src
    s = _fake_built(cagra)
    assert L.cagra_segment_gather(ctypes.byref(s), 1, 0, 1, 1, None) == -1  # min with float values
    assert L.cagra_merge(ctypes.byref(s), 7, 1, 1, None) == -1
    # fused merge LDS: 8*B + 8*(k+1) + 64 bytes; B = 16384 with k = 4096 does not fit
    s = _fake_built(cagra, B=16384, V=32768, N=8)
    g = _graph(cagra, V=32768, E=50)
    assert L.cagra_pagerank_iter(ctypes.byref(g), ctypes.byref(s), 0.85, -1, 0, 1, 1, 1, 1, 1, 1, 1, 1, 1 << 20,
                                 None) == -3
    assert L.cagra_iter_workspace_bytes(ctypes.byref(s)) > 0
    # workspace too small is reported before any launch
    s = _fake_built(cagra)
    g = _graph(cagra, V=100, E=50)
    assert L.cagra_pagerank_iter(ctypes.byref(g), ctypes.byref(s), 0.85, -1, 0, 1, 1, 1, 1, 1, 1, 1, 1, 8, None) == -4


def test_edge_word_bytes(cagra):
    """16-bit edge words exactly when a local index fits 15 bits (N <= 32768)."""
    L = cagra.lib()
    assert L.cagra_edge_word_bytes(0) == 0
    assert L.cagra_edge_word_bytes(1) == 2
    assert L.cagra_edge_word_bytes(cagra.EDGE16_MAX_N) == 2
    assert L.cagra_edge_word_bytes(cagra.EDGE16_MAX_N + 1) == 4
    assert L.cagra_edge_word_bytes(1 << 24) == 4
    text = open(HEADER).read()
    assert re.search(r"#define CAGRA_EDGE16_MAX_N (\d+)", text).group(1) == str(cagra.EDGE16_MAX_N)


def test_cluster_validation(cagra):
    """cagra_cluster rejects bad arguments before any HIP call."""
    L = cagra.lib()
    assert L.cagra_cluster_workspace_bytes(0, 10) == 0
    assert L.cagra_cluster_workspace_bytes(10, -1) == 0
    assert L.cagra_cluster_workspace_bytes(10, 2 ** 31) == 0
    g = _graph(cagra, V=10, E=5, off=4096, src=8192, od=12288)
    assert L.cagra_cluster(None, 1, 1, 1, 1, None, 1, 1 << 20, None) == -1
    assert L.cagra_cluster(ctypes.byref(_graph(cagra, od=None)), 1, 1, 1, 1, None, 1, 1 << 20, None) == -1
    assert L.cagra_cluster(ctypes.byref(g), None, 1, 1, 1, None, 1, 1 << 20, None) == -1
    assert L.cagra_cluster(ctypes.byref(g), 1, 1, None, 1, None, 1, 1 << 20, None) == -1
    assert L.cagra_cluster(ctypes.byref(g), 1, 4096, 1, 1, None, 1, 1 << 20, None) == -1  # aliases in_offsets
    assert L.cagra_cluster(ctypes.byref(g), 1, 1, 8192, 1, None, 1, 1 << 20, None) == -1  # aliases in_sources
    assert L.cagra_cluster(ctypes.byref(g), 1, 1, 1, 1, None, None, 1 << 20, None) == -4  # no workspace
    assert L.cagra_cluster(ctypes.byref(g), 1, 1, 1, 1, None, 1, 0, None) == -4


def test_cf_validation(cagra):
    """cagra_segment_edge_values and cagra_cf_iter reject bad arguments before any HIP call."""
    L = cagra.lib()
    g = _graph(cagra, V=100, E=50)
    s = _fake_built(cagra)
    assert L.cagra_segment_edge_values(None, ctypes.byref(s), 1, 2, None) == -1
    assert L.cagra_segment_edge_values(ctypes.byref(g), ctypes.byref(s), None, 2, None) == -1
    assert L.cagra_segment_edge_values(ctypes.byref(g), ctypes.byref(s), 8, 8, None) == -1  # aliased
    assert L.cagra_cf_workspace_bytes(ctypes.byref(s)) >= 8
    ws = L.cagra_cf_workspace_bytes(ctypes.byref(s))
    args = lambda **kw: [kw.get(n, d) for n, d in (("vals", 1), ("gamma", 0.01), ("lam", 0.1), ("xi", 2), ("part", 3),
                                                    ("xo", 4), ("sq", 5), ("ws", 6), ("wsb", ws))]
    assert L.cagra_cf_iter(ctypes.byref(g), ctypes.byref(s), *args(xo=2), None) == -1  # x_in aliases x_out
    assert L.cagra_cf_iter(ctypes.byref(g), ctypes.byref(s), *args(gamma=-1.0), None) == -1
    assert L.cagra_cf_iter(ctypes.byref(g), ctypes.byref(s), *args(sq=None), None) == -1
    assert L.cagra_cf_iter(ctypes.byref(g), ctypes.byref(s), *args(wsb=4), None) == -4
    big = _fake_built(cagra, B=1024)
    assert L.cagra_cf_iter(ctypes.byref(g), ctypes.byref(big), *args(), None) == -3  # merge LDS


def test_push_validation(cagra):
    """The push-direction calls reject bad arguments before any HIP call."""
    L = cagra.lib()
    assert L.cagra_push_workspace_bytes(None) == 0
    s = _fake_built(cagra)
    ws = L.cagra_push_workspace_bytes(ctypes.byref(s))
    # plan (k+1, pieces+1, pieces ints), 4 FP64 sums per 4096 vertices, one 8-byte slot of N per piece
    assert ws >= (s.k + 1 + 2 * s.k) * 4 + 32 + s.k * s.N * 8
    g = _graph(cagra, V=100, E=50)
    pr = lambda **kw: [kw.get(n, d) for n, d in (("d", 0.85), ("ri", 1), ("ci", 2), ("si", 3), ("vals", 4),
                                                  ("ro", 5), ("co", 6), ("so", 7), ("ws", 8), ("wsb", ws))]
    assert L.cagra_pagerank_push_iter(ctypes.byref(g), ctypes.byref(_seg(cagra)), *pr(), None) == -1  # unbuilt
    assert L.cagra_pagerank_push_iter(ctypes.byref(g), ctypes.byref(s), *pr(d=1.5), None) == -1
    assert L.cagra_pagerank_push_iter(ctypes.byref(g), ctypes.byref(s), *pr(vals=None), None) == -1
    assert L.cagra_pagerank_push_iter(ctypes.byref(g), ctypes.byref(s), *pr(so=None), None) == -1
    assert L.cagra_pagerank_push_iter(ctypes.byref(g), ctypes.byref(s), *pr(wsb=ws - 1), None) == -4
    other = _graph(cagra, V=100, E=49)
    assert L.cagra_pagerank_push_iter(ctypes.byref(other), ctypes.byref(s), *pr(), None) == -1
    # LDS capacity (accumulators in 160 KiB): 8-byte accumulators fit up to
    # N = 20480, 4-byte ones up to N = 40960
    for N, ok in ((20480, True), (20481, False)):
        seg = _fake_built(cagra, V=2 * N, N=N, B=4096)
        wsb = L.cagra_push_workspace_bytes(ctypes.byref(seg))
        gb = _graph(cagra, V=2 * N, E=50)
        assert L.cagra_pagerank_push_iter(ctypes.byref(gb), ctypes.byref(seg), *pr(wsb=wsb - 1), None) == \
            (-4 if ok else -3)
    for N, ok in ((40960, True), (40961, False)):
        seg = _fake_built(cagra, V=2 * N, N=N, B=4096)
        wsb = L.cagra_push_workspace_bytes(ctypes.byref(seg))
        assert L.cagra_labelprop_push_iter(ctypes.byref(seg), 1, 2, 3, 4, 5, wsb - 1, None) == (-4 if ok else -3)
    assert L.cagra_labelprop_push_iter(ctypes.byref(s), None, 2, 3, 4, 5, ws, None) == -1


def test_validate_graph_arguments(cagra):
    """cagra_validate_graph rejects bad arguments before any HIP call."""
    L = cagra.lib()
    n = L.cagra_validate_workspace_bytes()
    assert n >= 56
    assert L.cagra_validate_graph(None, 1, n, None) == -1
    assert L.cagra_validate_graph(ctypes.byref(_graph(cagra, V=0)), 1, n, None) == -1
    assert L.cagra_validate_graph(ctypes.byref(_graph(cagra, E=2 ** 31)), 1, n, None) == -2
    assert L.cagra_validate_graph(ctypes.byref(_graph(cagra, src=None)), 1, n, None) == -1
    assert L.cagra_validate_graph(ctypes.byref(_graph(cagra)), None, n, None) == -4
    assert L.cagra_validate_graph(ctypes.byref(_graph(cagra)), 1, n - 1, None) == -4


def test_pagerank_solve_validation(cagra):
    """cagra_pagerank_solve rejects bad arguments before any HIP call."""
    L = cagra.lib()
    s = _fake_built(cagra)
    g = _graph(cagra, V=100, E=50)
    ws = L.cagra_iter_workspace_bytes(ctypes.byref(s))
    res = cagra.CPrResult()

    def call(p, r0=1, r1=2, c0=3, c1=4, sc=5, part=6, wsp=7, wsb=ws, result=res):
        return L.cagra_pagerank_solve(ctypes.byref(g), ctypes.byref(s), None if p is None else ctypes.byref(p),
                                      r0, r1, c0, c1, sc, part, wsp, wsb,
                                      None if result is None else ctypes.byref(result), None)

    ok = dict(damping=0.85, tol=1e-6, switch_tol=0.0, max_iters=100, check_every=1, contrib_type=cagra.F32)

    def P(**kw):
        d = dict(ok, **kw)
        return cagra.CPrParams(d["damping"], d["tol"], d["switch_tol"], d.get("restart", -1), d["max_iters"],
                               d["check_every"], d["contrib_type"])
    assert call(None) == cagra.E_INVALID
    assert call(P(), result=None) == cagra.E_INVALID
    assert call(P(tol=0.0)) == cagra.E_INVALID
    assert call(P(tol=float("nan"))) == cagra.E_INVALID
    assert call(P(max_iters=0)) == cagra.E_INVALID
    assert call(P(check_every=0)) == cagra.E_INVALID
    assert call(P(switch_tol=1e-4)) == cagra.E_INVALID          # finishing switch needs BF16 contributions
    assert call(P(switch_tol=-1.0, contrib_type=cagra.BF16)) == cagra.E_INVALID
    assert call(P(damping=2.0)) == cagra.E_INVALID
    assert call(P(contrib_type=7)) == cagra.E_INVALID
    assert call(P(restart=-2)) == cagra.E_INVALID
    assert call(P(restart=100)) == cagra.E_INVALID                # outside [-1, V)
    assert call(P(), r1=1) == cagra.E_INVALID                   # rank pair aliased
    assert call(P(), c1=3) == cagra.E_INVALID                   # contribution pair aliased
    assert call(P(), sc=None) == cagra.E_INVALID
    assert call(P(), wsb=ws - 1) == cagra.E_BUFFER
    assert L.cagra_last_error()


def test_ppr_solve_validation(cagra):
    """cagra_ppr_solve rejects bad arguments before any HIP call."""
    L = cagra.lib()
    s = _fake_built(cagra)
    g = _graph(cagra, V=100, E=50)
    ws = L.cagra_ppr_workspace_bytes(ctypes.byref(s))
    res = cagra.CPprResult()

    def call(p, ncols=4, seeds=9, r0=1, r1=2, c0=3, c1=4, sc=5, part=6, wsp=7, wsb=ws, result=res, seg=s, gr=g):
        return L.cagra_ppr_solve(ctypes.byref(gr), ctypes.byref(seg), None if p is None else ctypes.byref(p), ncols,
                                 seeds, r0, r1, c0, c1, sc, part, wsp, wsb,
                                 None if result is None else ctypes.byref(result), None)

    def P(damping=0.85, tol=1e-6, max_iters=100, check_every=1):
        return cagra.CPprParams(damping, tol, max_iters, check_every)
    assert call(None) == cagra.E_INVALID
    assert call(P(), result=None) == cagra.E_INVALID
    assert call(P(tol=0.0)) == cagra.E_INVALID
    assert call(P(tol=float("nan"))) == cagra.E_INVALID
    assert call(P(max_iters=0)) == cagra.E_INVALID
    assert call(P(check_every=0)) == cagra.E_INVALID
    assert call(P(damping=-0.1)) == cagra.E_INVALID
    assert call(P(), ncols=0) == cagra.E_INVALID
    assert call(P(), ncols=cagra.PPR_COLS + 1) == cagra.E_INVALID
    assert call(P(), seeds=None) == cagra.E_INVALID
    assert call(P(), r1=1) == cagra.E_INVALID                   # rank pair aliased
    assert call(P(), c1=3) == cagra.E_INVALID                   # contribution pair aliased
    assert call(P(), sc=None) == cagra.E_INVALID
    assert call(P(), wsb=ws - 1) == cagra.E_BUFFER
    assert call(P(), seg=_fake_built(cagra, B=1024, V=2048, N=1024)) == cagra.E_INVALID  # another graph's
    assert call(P(), seg=_fake_built(cagra, B=1024, V=2048, N=1024),
                gr=_graph(cagra, V=2048, E=50)) == cagra.E_CAPACITY  # B above 512
    assert L.cagra_last_error()


def test_labelprop_solve_validation(cagra):
    """cagra_labelprop_solve rejects bad arguments before any HIP call."""
    L = cagra.lib()
    s = _fake_built(cagra)
    ws = L.cagra_iter_workspace_bytes(ctypes.byref(s))
    res = cagra.CLpResult()

    def call(mi=100, every=1, l0=1, l1=2, part=3, ch=4, wsp=5, wsb=ws, result=res):
        return L.cagra_labelprop_solve(ctypes.byref(s), mi, every, l0, l1, part, ch, wsp, wsb,
                                       None if result is None else ctypes.byref(result), None)
    assert call(result=None) == cagra.E_INVALID
    assert call(mi=0) == cagra.E_INVALID
    assert call(every=0) == cagra.E_INVALID
    assert call(l0=None) == cagra.E_INVALID
    assert call(ch=None) == cagra.E_INVALID
    assert call(l1=1) == cagra.E_INVALID                        # label pair aliased
    assert call(wsb=ws - 1) == cagra.E_BUFFER
    assert call(wsp=None) == cagra.E_BUFFER
    assert L.cagra_last_error()


def test_push_solve_validation(cagra):
    """The push-direction solves reject bad arguments before any HIP call."""
    L = cagra.lib()
    s = _fake_built(cagra)
    g = _graph(cagra, V=100, E=50)
    ws = L.cagra_push_workspace_bytes(ctypes.byref(s))
    res = cagra.CPrResult()

    def P(**kw):
        d = dict(damping=0.85, tol=1e-6, switch_tol=0.0, restart=-1, max_iters=100, check_every=1,
                 contrib_type=cagra.F32)
        d.update(kw)
        return cagra.CPrParams(d["damping"], d["tol"], d["switch_tol"], d["restart"], d["max_iters"],
                               d["check_every"], d["contrib_type"])

    def call(p, r0=1, r1=2, c0=3, c1=4, sc=5, vals=6, wsp=7, wsb=ws, result=res):
        return L.cagra_pagerank_push_solve(ctypes.byref(g), ctypes.byref(s), None if p is None else ctypes.byref(p),
                                           r0, r1, c0, c1, sc, vals, wsp, wsb,
                                           None if result is None else ctypes.byref(result), None)
    assert call(None) == cagra.E_INVALID
    assert call(P(), result=None) == cagra.E_INVALID
    assert call(P(tol=0.0)) == cagra.E_INVALID
    assert call(P(max_iters=0)) == cagra.E_INVALID
    assert call(P(contrib_type=cagra.BF16)) == cagra.E_INVALID    # push gathers FP32 contributions
    assert call(P(switch_tol=1e-3)) == cagra.E_INVALID
    assert call(P(restart=3)) == cagra.E_INVALID                  # uniform teleport only
    assert call(P(), r1=1) == cagra.E_INVALID
    assert call(P(), sc=None) == cagra.E_INVALID
    assert call(P(), vals=None) == cagra.E_INVALID
    assert call(P(), wsb=ws - 1) == cagra.E_BUFFER
    lres = cagra.CLpResult()

    def lcall(mi=100, every=1, l0=1, l1=2, vals=3, ch=4, wsp=5, wsb=ws, result=lres):
        return L.cagra_labelprop_push_solve(ctypes.byref(s), mi, every, l0, l1, vals, ch, wsp, wsb,
                                            None if result is None else ctypes.byref(result), None)
    assert lcall(result=None) == cagra.E_INVALID
    assert lcall(mi=0) == cagra.E_INVALID
    assert lcall(l1=1) == cagra.E_INVALID
    assert lcall(ch=None) == cagra.E_INVALID
    assert lcall(vals=None) == cagra.E_INVALID
    assert lcall(wsb=ws - 1) == cagra.E_BUFFER
    assert L.cagra_last_error()
