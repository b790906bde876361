"""Project-written autotuner for the segment size N, merge block B and gather tile.

Section 3.4 of the paper frames segment size as a trade-off: smaller segments
fit a faster memory level but raise the expansion factor q (more merge work).
On gfx950 the levels are LDS (staged segments), L2 and the Infinity Cache.

1. Candidates: LDS-sized N (the largest segments a workgroup can stage for the
   value type, and a few smaller), an L2-sized and an Infinity-Cache-sized N,
   and one segment (N >= V); B values the merge kernel's LDS allows for k.
2. Pruning: the builder's query call gives the exact row count Q for each N
   cheaply; the byte model ranks candidates and drops those predicted worse
   than `prune_factor` times the best of their class. The classes are LDS-
   staged and cache-gathered segments: the byte model counts HBM bytes only,
   and a gather through the cache hierarchy pays for its random reads in
   requests, not bytes, so the two are never pruned against each other; the
   best staged candidates and the best cache-gathered one are always timed.
3. Timing: the survivors are built and timed (gather + merge, HIP events);
   the fastest wins. Results are cached in a JSON file keyed by the graph's
   size, value type and operation.
"""
from __future__ import annotations

import ctypes
import json
import os
from dataclasses import asdict, dataclass

from . import cagra

CACHE_DEFAULT = os.path.join(os.path.expanduser("~"), ".cache", "cagra_autotune.json")


@dataclass
class Choice:
    N: int
    B: int
    tile_edges: int
    staged: bool
    Q: int = 0
    predicted_bytes: int = 0
    ms: float = 0.0


def value_bytes(value_type: int) -> int:
    return 2 if value_type == cagra.BF16 else 4


def lds_staged_max(value_type: int) -> int:
    return cagra.STAGE_BYTES // value_bytes(value_type)


def candidate_segment_sizes(V: int, value_type: int):
    m = lds_staged_max(value_type)
    lds = {m, m // 2, (3 * m) // 4, m // 4}
    others = {1 << 20, 1 << 24}
    out = [n for n in lds | others if 1 <= n < V] + [max(V, 1)]  # N >= V is one segment
    return sorted(set(out))


def fused_merge_fits(B: int, k: int, acc_bytes: int = 8) -> bool:
    # 8*B + 8*(k+1) + 320 bytes of LDS (see include/cagra.h)
    return acc_bytes * B + 8 * (k + 1) + 320 <= cagra.LDS_BYTES


def edge_word_bytes(N: int) -> int:
    return 2 if N <= cagra.EDGE16_MAX_N else 4


def byte_model(V: int, E: int, Q: int, k: int, B: int, wc: int, we: int = 4) -> int:
    nb = -(-V // B)
    return we * E + wc * V + 4 * Q + 6 * Q + 4 * k * (nb + 1) + 12 * V + wc * V


def query_Q(dg, N: int, B: int, tile_edges: int) -> int:
    """Row count of the segmented graph from the builder's query call only."""
    import torch
    L = cagra.lib()
    c = cagra.CSegments()
    c.N, c.B, c.tile_edges = N, B, tile_edges
    qb = L.cagra_query_workspace_bytes(dg.V, dg.E, N)
    ws = torch.empty(max(qb, 1), dtype=torch.uint8, device="cuda")
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    cagra._check(L.cagra_build_segments(ctypes.byref(dg.c), ctypes.byref(c), ctypes.c_void_p(ws.data_ptr()), qb, st),
                 "cagra_build_segments(query)")
    return int(c.Q)


def select_pool(cands, prune_factor: float, max_trials: int):
    """Candidates to time: per class (LDS-staged / cache-gathered), those within
    prune_factor of the class's best predicted bytes, fewest bytes first; up to
    max_trials - 1 staged ones plus the best cache-gathered one."""
    def pruned(cls):
        if not cls:
            return []
        best_bytes = min(c.predicted_bytes for c in cls)
        return sorted([c for c in cls if c.predicted_bytes <= prune_factor * best_bytes],
                      key=lambda c: c.predicted_bytes)
    staged = pruned([c for c in cands if c.staged])
    unstaged = pruned([c for c in cands if not c.staged])
    if not staged:
        return unstaged[:max_trials]
    return staged[:max(1, max_trials - 1)] + unstaged[:1]


def _time_pagerank(dg, seg, value_type: int, reps: int = 3) -> float:
    import torch
    st = cagra.PageRankState(dg, seg, value_type)
    st.start()
    st.step()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        st.step()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def cache_key(dg, value_type: int, op: str, tag: str = "") -> str:
    return f"V{dg.V}:E{dg.E}:vt{value_type}:{op}:{tag}"


def load_cache(path: str) -> dict:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def save_cache(path: str, cache: dict) -> None:
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + ".tmp%d" % os.getpid()
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1)
    os.replace(tmp, path)


def tune(dg, value_type: int = cagra.F32, op: str = "pagerank", cache_path: str | None = CACHE_DEFAULT,
         tag: str = "", prune_factor: float = 1.6, max_trials: int = 6, B_list=(4096, 8192, 16384),
         tiles=(65536, 262144), log=None):
    """Returns (best Choice, list of timed Choices). Uses the cache when present."""
    key = cache_key(dg, value_type, op, tag)
    if cache_path:
        cache = load_cache(cache_path)
        if key in cache:
            return Choice(**cache[key]), []
    wc = value_bytes(value_type)
    cands = []
    for N in candidate_segment_sizes(dg.V, value_type):
        k = -(-dg.V // N)
        if k > 32768:
            continue
        Q = query_Q(dg, N, 8192, tiles[0])
        for B in B_list:
            if not fused_merge_fits(B, k):
                continue
            for T in tiles:
                cands.append(Choice(N, B, T, N <= lds_staged_max(value_type), Q,
                                    byte_model(dg.V, dg.E, Q, k, B, wc, edge_word_bytes(N))))
    pool = select_pool(cands, prune_factor, max_trials)
    timed = []
    for c in pool:
        seg = cagra.build_segments(dg, c.N, c.B, c.tile_edges)
        c.ms = _time_pagerank(dg, seg, value_type) if op == "pagerank" else _time_labelprop(seg)
        timed.append(c)
        if log:
            log(f"autotune N={c.N} B={c.B} T={c.tile_edges} Q={c.Q} bytes={c.predicted_bytes} -> {c.ms:.3f} ms")
        del seg
    best = min(timed, key=lambda c: c.ms)
    if cache_path:
        cache = load_cache(cache_path)
        cache[key] = asdict(best)
        save_cache(cache_path, cache)
    return best, timed


def _time_labelprop(seg, reps: int = 3) -> float:
    import torch
    V = seg.c.V
    lab = [torch.arange(V, dtype=torch.int32, device="cuda"), torch.empty(V, dtype=torch.int32, device="cuda")]
    partial = torch.empty(max(seg.Q, 1), dtype=torch.int32, device="cuda")
    changed = torch.zeros(1, dtype=torch.int32, device="cuda")
    ws = cagra.iter_workspace(seg)
    cagra.labelprop_iter(seg, lab[0], partial, lab[1], changed, ws)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for i in range(reps):
        cagra.labelprop_iter(seg, lab[i % 2], partial, lab[1 - i % 2], changed, ws)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


# ---------------------------------------------------------------- batched personalized PageRank

def ppr_candidates(V: int):
    """Segment sizes for 256-byte vertex records (64 FP32 columns): an LDS
    segment would hold 512 such rows, so the candidates are L2- to
    Infinity-Cache-sized (2^16 ... 2^22 vertices, 16 MB ... 1 GB of rows) and
    one segment; merge blocks of 256 and 512 rows (B x 256 bytes of LDS
    accumulators); gather tiles of 16 K and 64 K edges."""
    Ns = sorted({n for n in (1 << 16, 1 << 18, 1 << 20, 1 << 21, 1 << 22) if n < V} | {max(V, 1)})
    return [(N, B, T) for N in Ns for B in (256, 512) for T in (16384, 65536)]


def _time_ppr(dg, seg, seeds, reps: int = 3) -> float:
    import torch
    st = cagra.PPRState(dg, seg, seeds)
    st.start()
    st.step()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        st.step()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def tune_ppr(dg, seeds, cache_path: str | None = CACHE_DEFAULT, tag: str = "", log=None, prune_factor: float = 2.0):
    """Segment size N, merge block B and gather tile T for the batched
    personalized PageRank of `seeds` (up to 64 columns). Candidates whose
    buffer rows (Q x 256 bytes, read and written once per iteration) exceed
    prune_factor times the smallest candidate's are dropped before timing:
    with record-sized gathers served from the cache hierarchy, those buffer
    bytes are what differs between segment sizes. Returns (best Choice, timed)."""
    import torch
    key = cache_key(dg, cagra.F32, "ppr", f"{tag}:c{len(seeds)}")
    if cache_path:
        cache = load_cache(cache_path)
        if key in cache:
            return Choice(**cache[key]), []
    Qs = {}
    for N, _, _ in ppr_candidates(dg.V):
        if N not in Qs:
            Qs[N] = query_Q(dg, N, 512, 16384)
    qmin = min(Qs.values())
    timed = []
    for N, B, T in ppr_candidates(dg.V):
        k = -(-dg.V // N)
        if k > 32768 or Qs[N] > prune_factor * max(qmin, 1) + dg.V:
            continue
        seg = cagra.build_segments(dg, N, B, T)
        c = Choice(N, B, T, False, Qs[N], Qs[N] * 512, _time_ppr(dg, seg, seeds))
        timed.append(c)
        if log:
            log(f"autotune ppr N={N} B={B} T={T} q={Qs[N] / dg.V:.3f} -> {c.ms:.3f} ms")
        del seg
        torch.cuda.empty_cache()
    best = min(timed, key=lambda c: c.ms)
    if cache_path:
        cache = load_cache(cache_path)
        cache[key] = asdict(best)
        save_cache(cache_path, cache)
    return best, timed


# ---------------------------------------------------------------- many graphs in one launch

def size_class(V: int) -> int:
    """0: up to 2^13 vertices, 1: up to 2^17, 2: larger."""
    return 0 if V <= 1 << 13 else (1 if V <= 1 << 17 else 2)


MULTI_DEFAULT = (32768, 8192, 65536)


def multi_candidates():
    """(N, B, T) per size class: LDS-staged segments (the persistent kernels use
    16-bit edge words, N <= 32,768), merge blocks of 4 K and 8 K vertices, tiles
    of 16 K and 64 K edges. N is capped at the graph's V when used."""
    return [(N, B, T) for N in (8192, 16384, 32768) for B in (4096, 8192) for T in (16384, 65536)]


def _multi_segments(dgs, choice_by_class):
    out = []
    for d in dgs:
        N, B, T = choice_by_class[size_class(d.V)]
        out.append(cagra.build_segments(d, min(N, max(d.V, 1)), B, T))
    return out


def _time_multi(dgs, segs, iters: int = 20, reps: int = 2) -> float:
    import torch
    mp = cagra.MultiPageRank(dgs, segs)
    mp.run_eager(2)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        mp.run_eager(iters)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def tune_multi(dgs, cache_path: str | None = CACHE_DEFAULT, tag: str = "", log=None):
    """Per size class (size_class), the (N, B, T) of the graphs of that class in
    the persistent multi-graph launch: one pass of coordinate descent over the
    classes present (largest first), each class's candidates timed on the whole
    launch (start + 20 iterations of every graph) with the other classes held
    at their current choice. Returns ({class: (N, B, T)}, [(class, N, B, T, ms)])."""
    import torch
    classes = sorted({size_class(d.V) for d in dgs}, reverse=True)
    key = f"multi:{len(dgs)}:V{sum(d.V for d in dgs)}:E{sum(d.E for d in dgs)}:{tag}"
    if cache_path:
        cache = load_cache(cache_path)
        if key in cache:
            return {int(c): tuple(v) for c, v in cache[key].items()}, []
    choice = {c: MULTI_DEFAULT for c in (0, 1, 2)}
    trials = []
    for cl in classes:
        best = None
        for cand in multi_candidates():
            trial = dict(choice)
            trial[cl] = cand
            segs = _multi_segments(dgs, trial)
            ms = _time_multi(dgs, segs)
            del segs
            torch.cuda.empty_cache()
            trials.append((cl, *cand, round(ms, 4)))
            if log:
                log(f"autotune multi class {cl} N={cand[0]} B={cand[1]} T={cand[2]} -> {ms:.3f} ms")
            if best is None or ms < best[0]:
                best = (ms, cand)
        choice[cl] = best[1]
    if cache_path:
        cache = load_cache(cache_path)
        cache[key] = {str(c): list(v) for c, v in choice.items()}
        save_cache(cache_path, cache)
    return choice, trials


def multi_segments(dgs, choice):
    """Segments of every graph with its size class's (N, B, T)."""
    return _multi_segments(dgs, choice)
