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
