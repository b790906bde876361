"""ctypes binding of libcagra.so (include/cagra.h), plus the iteration driver.

Argument marshalling only: every step of the segmented traversal runs in the
library's HIP kernels. PyTorch provides device memory and the stream. The
library is required: importing works without it, but every call raises if
libcagra.so is missing (there is no fallback path).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libcagra.so")

# enums of include/cagra.h
OK, E_INVALID, E_OVERFLOW, E_CAPACITY, E_BUFFER, E_HIP, E_NOT_CONVERGED, E_RANGE = 0, -1, -2, -3, -4, -5, -6, -7
ABI_VERSION = 2
F32, BF16, I32 = 0, 1, 2
SUM_F32, MIN_I32, SUM_F32_COMP = 0, 1, 2
LDS_BYTES = 163840
STAGE_BYTES = 131072
TILE_WAVES = 16
EDGE16_MAX_N = 32768
CF_FACTORS = 64
PPR_COLS = 64

_c_i32, _c_i64, _c_size, _c_vp, _c_dbl = ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_double


class CGraph(ctypes.Structure):
    _fields_ = [("V", _c_i32), ("E", _c_i64), ("in_offsets", _c_vp), ("in_sources", _c_vp), ("out_degree", _c_vp)]


class CSegments(ctypes.Structure):
    _fields_ = [("N", _c_i32), ("B", _c_i32), ("tile_edges", _c_i32),
                ("V", _c_i32), ("k", _c_i32), ("nb", _c_i32), ("ntiles", _c_i32),
                ("E", _c_i64), ("Q", _c_i64), ("build_workspace_bytes", _c_size), ("max_items", _c_i32),
                ("seg_row_begin", _c_vp), ("row_ptr", _c_vp), ("row_dst", _c_vp), ("edge_src", _c_vp),
                ("block_ptr", _c_vp), ("tile_edge", _c_vp), ("tile_seg", _c_vp), ("tile_span_row", _c_vp),
                ("row_dst_lo", _c_vp), ("block_items", _c_vp)]


EXPORTS = [
    "cagra_abi_version", "cagra_status_string", "cagra_last_error", "cagra_max_merge_block",
    "cagra_edge_word_bytes", "cagra_cluster_workspace_bytes", "cagra_cluster", "cagra_segment_edge_values",
    "cagra_cf_workspace_bytes", "cagra_cf_iter", "cagra_bc_workspace_bytes", "cagra_bc_start",
    "cagra_bc_forward_level", "cagra_bc_backward_level", "cagra_query_workspace_bytes", "cagra_build_segments", "cagra_iter_workspace_bytes",
    "cagra_segment_gather", "cagra_merge", "cagra_pagerank_init", "cagra_pagerank_iter",
    "cagra_push_workspace_bytes", "cagra_pagerank_push_iter", "cagra_labelprop_push_iter",
    "cagra_pagerank_push_solve", "cagra_labelprop_push_solve",
    "cagra_validate_workspace_bytes", "cagra_validate_graph",
    "cagra_pagerank_merge", "cagra_pagerank_solve", "cagra_noalloc_scratch_bytes", "cagra_pagerank_iter_noalloc",
    "cagra_labelprop_iter", "cagra_labelprop_solve", "cagra_ppr_workspace_bytes", "cagra_ppr_init",
    "cagra_ppr_iter", "cagra_ppr_solve", "cagra_multi_query", "cagra_multi_setup", "cagra_multi_pagerank_start",
    "cagra_multi_pagerank_step", "cagra_features_workspace_bytes", "cagra_degree_features", "cagra_mlp_forward",
    "cagra_mlp_grad_workspace_bytes", "cagra_mlp_grad", "cagra_adam_step", "cagra_warm_start_workspace_bytes",
    "cagra_warm_start_vector", "cagra_mlp_targets", "cagra_feature_norm_workspace_bytes", "cagra_feature_norm",
    "cagra_sample_rows", "cagra_learned_start_workspace_bytes", "cagra_learned_start",
]


class CPrParams(ctypes.Structure):
    _fields_ = [("damping", _c_dbl), ("tol", _c_dbl), ("switch_tol", _c_dbl), ("restart_vertex", _c_i32),
                ("max_iters", _c_i32), ("check_every", _c_i32), ("contrib_type", _c_i32)]


class CPrResult(ctypes.Structure):
    _fields_ = [("iters", _c_i32), ("iters_bf16", _c_i32), ("final_buf", _c_i32), ("residual", _c_dbl),
                ("scalars", _c_dbl * 4)]


class CLpResult(ctypes.Structure):
    _fields_ = [("iters", _c_i32), ("final_buf", _c_i32), ("changed", _c_i32)]


class CPprParams(ctypes.Structure):
    _fields_ = [("damping", _c_dbl), ("tol", _c_dbl), ("max_iters", _c_i32), ("check_every", _c_i32)]


class CPprResult(ctypes.Structure):
    _fields_ = [("iters", _c_i32), ("final_buf", _c_i32), ("residual", _c_dbl)]


class CMulti(ctypes.Structure):
    _fields_ = [("ngraphs", _c_i32), ("max_k", _c_i32), ("max_B", _c_i32),
                ("total_V", _c_i64), ("total_Q", _c_i64), ("total_tiles", _c_i64), ("total_blocks", _c_i64),
                ("desc_bytes", _c_size), ("desc", _c_vp), ("rank", _c_vp * 2), ("contrib", _c_vp * 2),
                ("scalars", _c_vp * 2), ("partial", _c_vp), ("blk", _c_vp),
                ("grid_gather", _c_i32), ("grid_merge", _c_i32)]


class CagraError(RuntimeError):
    def __init__(self, status: int, fn: str, detail: str):
        super().__init__(f"{fn} -> {status} ({detail})")
        self.status = status


class NotConverged(CagraError):
    """An iteration cap was reached before the residual fell below tol; `result`
    holds what the run produced (for pagerank: (rank, residuals, steps))."""

    def __init__(self, fn: str, detail: str, result=None):
        super().__init__(E_NOT_CONVERGED, fn, detail)
        self.result = result


def check_range(scalars, fn: str = "pagerank"):
    """Raise CagraError(E_RANGE) when an iteration's range count (scalars[3],
    carried over from iteration to iteration) is non-zero: some merge block held
    non-finite buffer values or more absolute mass than the exact fixed-point
    sums allow, so the ranks are not exact. Reads the device scalars (syncs)."""
    c = float(scalars[3].item())
    if c != 0.0:
        raise CagraError(E_RANGE, fn, f"range count {c:g}: buffer values non-finite or beyond the exact "
                                      "fixed-point range in some iteration")


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"libcagra.so not built at {LIB_PATH}; run __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        GP, SP, st = ctypes.POINTER(CGraph), ctypes.POINTER(CSegments), _c_vp
        sig = {
            "cagra_abi_version": ([], ctypes.c_int),
            "cagra_status_string": ([ctypes.c_int], ctypes.c_char_p),
            "cagra_last_error": ([], ctypes.c_char_p),
            "cagra_max_merge_block": ([], _c_i32),
            "cagra_edge_word_bytes": ([_c_i32], _c_i32),
            "cagra_cluster_workspace_bytes": ([_c_i32, _c_i64], _c_size),
            "cagra_cluster": ([GP, _c_vp, _c_vp, _c_vp, _c_vp, _c_vp, _c_vp, _c_size, st], ctypes.c_int),
            "cagra_segment_edge_values": ([GP, SP, _c_vp, _c_vp, st], ctypes.c_int),
            "cagra_cf_workspace_bytes": ([SP], _c_size),
            "cagra_bc_workspace_bytes": ([SP], _c_size),
            "cagra_bc_start": ([_c_i32, _c_i32, _c_vp, _c_vp, _c_vp, st], ctypes.c_int),
            "cagra_bc_forward_level": ([SP, _c_i32, _c_vp, _c_vp, _c_vp, _c_vp, _c_vp, _c_vp, _c_vp, _c_size, st],
                                       ctypes.c_int),
            "cagra_bc_backward_level": ([SP, _c_i32, _c_i32, _c_vp, _c_vp, _c_vp, _c_vp, _c_vp, _c_vp, _c_vp, _c_vp,
                                         _c_size, st], ctypes.c_int),
            "cagra_cf_iter": ([GP, SP, _c_vp, _c_dbl, _c_dbl, _c_vp, _c_vp, _c_vp, _c_vp, _c_vp, _c_size, st],
                              ctypes.c_int),
            "cagra_query_workspace_bytes": ([_c_i32, _c_i64, _c_i32], _c_size),
            "cagra_build_segments": ([GP, SP, _c_vp, _c_size, st], ctypes.c_int),
            "cagra_iter_workspace_bytes": ([SP], _c_size),
            "cagra_segment_gather": ([SP, _c_i32, _c_i32, _c_vp, _c_vp, st], ctypes.c_int),
            "cagra_merge": ([SP, _c_i32, _c_vp, _c_vp, st], ctypes.c_int),
            "cagra_pagerank_init": ([GP, _c_i32, _c_vp, _c_vp, _c_vp, _c_vp, _c_size, st], ctypes.c_int),
            "cagra_pagerank_iter": ([GP, SP, _c_dbl, _c_i32, _c_i32, _c_vp, _c_vp, _c_vp, _c_vp, _c_vp, _c_vp,
                                     _c_vp, _c_vp, _c_size, st], ctypes.c_int),
            "cagra_pagerank_merge": ([GP, SP, _c_dbl, _c_i32, _c_i32, _c_vp, _c_vp, _c_vp, _c_vp, _c_vp, _c_vp,
                                      _c_vp, _c_size, st], ctypes.c_int),
            "cagra_labelprop_iter": ([SP, _c_vp, _c_vp, _c_vp, _c_vp, _c_vp, _c_size, st], ctypes.c_int),
            "cagra_labelprop_solve": ([SP, _c_i32, _c_i32, _c_vp, _c_vp, _c_vp, _c_vp, _c_vp, _c_size,
                                       ctypes.POINTER(CLpResult), st], ctypes.c_int),
            "cagra_noalloc_scratch_bytes": ([], _c_size),
            "cagra_pagerank_iter_noalloc": ([GP, SP, _c_dbl, _c_i32, _c_i32, _c_vp, _c_vp, _c_vp, _c_vp, _c_vp,
                                             _c_vp, _c_vp, st], ctypes.c_int),
            "cagra_pagerank_solve": ([GP, SP, ctypes.POINTER(CPrParams), _c_vp, _c_vp, _c_vp, _c_vp, _c_vp, _c_vp,
                                      _c_vp, _c_size, ctypes.POINTER(CPrResult), st], ctypes.c_int),
            "cagra_push_workspace_bytes": ([SP], _c_size),
            "cagra_validate_workspace_bytes": ([], _c_size),
            "cagra_validate_graph": ([GP, _c_vp, _c_size, st], ctypes.c_int),
            "cagra_pagerank_push_iter": ([GP, SP, _c_dbl, _c_vp, _c_vp, _c_vp, _c_vp, _c_vp, _c_vp, _c_vp, _c_vp,
                                          _c_size, st], ctypes.c_int),
            "cagra_labelprop_push_iter": ([SP, _c_vp, _c_vp, _c_vp, _c_vp, _c_vp, _c_size, st], ctypes.c_int),
            "cagra_pagerank_push_solve": ([GP, SP, ctypes.POINTER(CPrParams), _c_vp, _c_vp, _c_vp, _c_vp, _c_vp,
                                           _c_vp, _c_vp, _c_size, ctypes.POINTER(CPrResult), st], ctypes.c_int),
            "cagra_labelprop_push_solve": ([SP, _c_i32, _c_i32, _c_vp, _c_vp, _c_vp, _c_vp, _c_vp, _c_size,
                                            ctypes.POINTER(CLpResult), st], ctypes.c_int),
            "cagra_ppr_workspace_bytes": ([SP], _c_size),
            "cagra_features_workspace_bytes": ([SP], _c_size),
            "cagra_degree_features": ([GP, SP, _c_vp, _c_vp, _c_size, st], ctypes.c_int),
            "cagra_mlp_forward": ([_c_vp, _c_i64, _c_vp, _c_vp, _c_vp, st], ctypes.c_int),
            "cagra_mlp_grad_workspace_bytes": ([], _c_size),
            "cagra_mlp_grad": ([_c_vp, _c_vp, _c_i64, _c_vp, _c_vp, _c_vp, _c_vp, _c_vp, _c_size, st], ctypes.c_int),
            "cagra_adam_step": ([_c_vp, _c_vp, _c_vp, _c_vp, _c_vp, _c_i32, ctypes.c_float, ctypes.c_float,
                                 ctypes.c_float, ctypes.c_float, st], ctypes.c_int),
            "cagra_warm_start_workspace_bytes": ([_c_i32], _c_size),
            "cagra_warm_start_vector": ([_c_vp, _c_i32, _c_vp, _c_vp, _c_vp, _c_size, st], ctypes.c_int),
            "cagra_mlp_targets": ([_c_vp, _c_i32, _c_vp, st], ctypes.c_int),
            "cagra_feature_norm_workspace_bytes": ([_c_i64], _c_size),
            "cagra_feature_norm": ([_c_vp, _c_i64, _c_vp, _c_vp, _c_size, st], ctypes.c_int),
            "cagra_sample_rows": ([_c_vp, _c_vp, _c_i64, ctypes.c_uint64, _c_i64, _c_i32, _c_vp, _c_vp, st],
                                  ctypes.c_int),
            "cagra_learned_start_workspace_bytes": ([SP], _c_size),
            "cagra_learned_start": ([GP, SP, _c_vp, _c_vp, _c_vp, _c_vp, _c_vp, _c_size, st], ctypes.c_int),
            "cagra_multi_query": ([_c_i32, GP, SP, ctypes.POINTER(CMulti)], ctypes.c_int),
            "cagra_multi_setup": ([ctypes.POINTER(CMulti), GP, SP, st], ctypes.c_int),
            "cagra_multi_pagerank_start": ([ctypes.POINTER(CMulti), st], ctypes.c_int),
            "cagra_multi_pagerank_step": ([ctypes.POINTER(CMulti), _c_i32, _c_dbl, st], ctypes.c_int),
            "cagra_ppr_init": ([GP, _c_i32, _c_vp, _c_vp, _c_vp, _c_vp, _c_vp, _c_size, st], ctypes.c_int),
            "cagra_ppr_iter": ([GP, SP, _c_dbl, _c_i32, _c_vp, _c_vp, _c_vp, _c_vp, _c_vp, _c_vp, _c_vp, _c_vp,
                                _c_vp, _c_size, st], ctypes.c_int),
            "cagra_ppr_solve": ([GP, SP, ctypes.POINTER(CPprParams), _c_i32, _c_vp, _c_vp, _c_vp, _c_vp, _c_vp,
                                 _c_vp, _c_vp, _c_vp, _c_size, ctypes.POINTER(CPprResult), st], ctypes.c_int),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        if L.cagra_abi_version() != ABI_VERSION:
            raise RuntimeError(f"libcagra.so ABI {L.cagra_abi_version()} != binding ABI {ABI_VERSION}; rebuild")
        _lib = L
    return _lib


def _check(status: int, fn: str):
    if status != OK:
        raise CagraError(status, fn, lib().cagra_last_error().decode(errors="replace"))


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dev():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("no GPU visible: the segmented traversal runs only on the GPU")
    return torch.device("cuda")


# --------------------------------------------------------------------------- graph and segments

@dataclass
class DeviceGraph:
    V: int
    E: int
    in_offsets: object
    in_sources: object
    out_degree: object
    c: CGraph = field(default=None)

    @staticmethod
    def from_host(g) -> "DeviceGraph":
        """Upload a graphgen.Graph (numpy int32 CSC) to device memory."""
        import torch
        dev = _dev()
        off = torch.from_numpy(np.ascontiguousarray(g.in_offsets)).to(dev)
        src = torch.from_numpy(np.ascontiguousarray(g.in_sources)).to(dev) if g.E else \
            torch.zeros(1, dtype=torch.int32, device=dev)
        od = torch.from_numpy(np.ascontiguousarray(g.out_degree)).to(dev)
        dg = DeviceGraph(g.V, g.E, off, src, od)
        dg.c = CGraph(g.V, g.E, off.data_ptr(), src.data_ptr(), od.data_ptr())
        return dg


def validate_graph(dg: "DeviceGraph", stream=None):
    """Check the device CSC (offsets, source range, strictly ascending rows, no
    self-loops); raises CagraError naming the first violation."""
    import torch
    L = lib()
    n = L.cagra_validate_workspace_bytes()
    ws = torch.empty(n, dtype=torch.uint8, device=_dev())
    _check(L.cagra_validate_graph(ctypes.byref(dg.c), _ptr(ws), n, _stream(stream)), "cagra_validate_graph")


def cluster(dg: "DeviceGraph", stream=None):
    """Section 5 frequency-based clustering on the GPU. Returns (clustered
    DeviceGraph, perm, H): perm[i] (device int32) is the old id of new vertex i,
    H the number of clustered vertices."""
    import torch
    dev = _dev()
    L = lib()
    V, E = dg.V, dg.E
    wb = L.cagra_cluster_workspace_bytes(V, E)
    if wb == 0:
        _check(E_INVALID, "cagra_cluster_workspace_bytes")
    ws = torch.empty(wb, dtype=torch.uint8, device=dev)
    perm = torch.empty(V, dtype=torch.int32, device=dev)
    off = torch.empty(V + 1, dtype=torch.int32, device=dev)
    src = torch.empty(max(E, 1), dtype=torch.int32, device=dev)
    od = torch.empty(V, dtype=torch.int32, device=dev)
    hot = torch.empty(1, dtype=torch.int32, device=dev)
    _check(L.cagra_cluster(ctypes.byref(dg.c), _ptr(perm), _ptr(off), _ptr(src), _ptr(od), _ptr(hot), _ptr(ws), wb,
                           _stream(stream)), "cagra_cluster")
    H = int(hot.item())  # synchronizes the stream
    del ws
    out = DeviceGraph(V, E, off, src, od)
    out.c = CGraph(V, E, off.data_ptr(), src.data_ptr(), od.data_ptr())
    return out, perm, H


@dataclass
class Segments:
    c: CSegments
    arrays: dict

    @property
    def Q(self):
        return int(self.c.Q)

    @property
    def k(self):
        return int(self.c.k)

    @property
    def q(self):
        return self.c.Q / self.c.V

    def host(self) -> dict:
        return {k: v.cpu().numpy() for k, v in self.arrays.items()}


def default_tile_edges(N: int, value_bytes: int = 4) -> int:
    # enough edges per tile that staging a segment once costs well under its edge bytes
    return 65536


def build_segments(dg: DeviceGraph, N: int, B: int, tile_edges: int | None = None, stream=None) -> Segments:
    """Section 3.1 preprocessing on the GPU (query call, then build call)."""
    import torch
    dev = _dev()
    L = lib()
    c = CSegments()
    c.N, c.B, c.tile_edges = N, B, tile_edges or default_tile_edges(N)
    st = _stream(stream)
    qbytes = L.cagra_query_workspace_bytes(dg.V, dg.E, N)
    if qbytes == 0:
        _check(E_INVALID, "cagra_query_workspace_bytes")
    qws = torch.empty(qbytes, dtype=torch.uint8, device=dev)
    _check(L.cagra_build_segments(ctypes.byref(dg.c), ctypes.byref(c), _ptr(qws), qbytes, st),
           "cagra_build_segments(query)")
    del qws
    i32 = torch.int32
    k, nb, Q, E, nt = c.k, c.nb, c.Q, c.E, c.ntiles
    arrays = {
        "seg_row_begin": torch.empty(k + 1, dtype=i32, device=dev),
        "row_ptr": torch.empty(Q + 1, dtype=i32, device=dev),
        "row_dst": torch.empty(max(Q, 1), dtype=i32, device=dev),
        # 16-bit edge words for N <= EDGE16_MAX_N, 32-bit otherwise; the
        # allocation is rounded up to 16 bytes (the gather loads 16-byte chunks)
        "edge_src": (torch.empty(max(-(-E // 8) * 8, 8), dtype=torch.int16, device=dev) if N <= EDGE16_MAX_N
                     else torch.empty(max(-(-E // 4) * 4, 4), dtype=i32, device=dev)),
        "block_ptr": torch.empty((nb + 1) * k, dtype=i32, device=dev),
        "tile_edge": torch.empty(nt + 1, dtype=i32, device=dev),
        "tile_seg": torch.empty(max(nt, 1), dtype=i32, device=dev),
        "tile_span_row": torch.empty(max(nt, 1) * TILE_WAVES, dtype=i32, device=dev),
        "row_dst_lo": torch.empty(max(Q, 1), dtype=torch.int16, device=dev),
        "block_items": torch.empty(nb + 1, dtype=i32, device=dev),
    }
    for name, t in arrays.items():
        setattr(c, name, t.data_ptr())
    ws = torch.empty(c.build_workspace_bytes, dtype=torch.uint8, device=dev)
    _check(L.cagra_build_segments(ctypes.byref(dg.c), ctypes.byref(c), _ptr(ws), c.build_workspace_bytes, st),
           "cagra_build_segments(build)")
    torch.cuda.current_stream().synchronize() if stream is None else stream.synchronize()
    del ws
    # tighten the work-item bound to the actual count (lets the merge skip its
    # slot pass when no block is split)
    c.max_items = int(arrays["block_items"][nb].item())
    arrays["row_dst"] = arrays["row_dst"][:Q]
    arrays["edge_src"] = arrays["edge_src"][:E]
    arrays["tile_seg"] = arrays["tile_seg"][:nt]
    arrays["tile_span_row"] = arrays["tile_span_row"][:nt * TILE_WAVES]
    arrays["row_dst_lo"] = arrays["row_dst_lo"][:Q]
    return Segments(c, arrays)


# --------------------------------------------------------------------------- single calls

def iter_workspace(seg: Segments):
    import torch
    n = lib().cagra_iter_workspace_bytes(ctypes.byref(seg.c))
    return torch.empty(n, dtype=torch.uint8, device=_dev())


def segment_gather(seg: Segments, op: int, value_type: int, values, partial, stream=None):
    _check(lib().cagra_segment_gather(ctypes.byref(seg.c), op, value_type, _ptr(values), _ptr(partial),
                                      _stream(stream)), "cagra_segment_gather")


def merge(seg: Segments, op: int, partial, out, stream=None):
    _check(lib().cagra_merge(ctypes.byref(seg.c), op, _ptr(partial), _ptr(out), _stream(stream)), "cagra_merge")


def pagerank_init(dg: DeviceGraph, contrib_type: int, rank, contrib_out, scalars_out, workspace, stream=None):
    _check(lib().cagra_pagerank_init(ctypes.byref(dg.c), contrib_type, _ptr(rank), _ptr(contrib_out),
                                     _ptr(scalars_out), _ptr(workspace), workspace.numel(), _stream(stream)),
           "cagra_pagerank_init")


def pagerank_iter(dg: DeviceGraph, seg: Segments, damping: float, contrib_type: int, rank_in, contrib_in,
                  scalars_in, partial, rank_out, contrib_out, scalars_out, workspace, stream=None, restart: int = -1):
    _check(lib().cagra_pagerank_iter(ctypes.byref(dg.c), ctypes.byref(seg.c), damping, restart, contrib_type,
                                     _ptr(rank_in), _ptr(contrib_in), _ptr(scalars_in), _ptr(partial),
                                     _ptr(rank_out), _ptr(contrib_out), _ptr(scalars_out), _ptr(workspace),
                                     workspace.numel(), _stream(stream)), "cagra_pagerank_iter")


def pagerank_iter_noalloc(dg: DeviceGraph, seg: Segments, damping: float, contrib_type: int, rank_in, contrib_in,
                          scalars_in, partial, rank_out, contrib_out, scalars_out, stream=None, restart: int = -1):
    """cagra_pagerank_iter with the library's static scratch instead of a workspace."""
    _check(lib().cagra_pagerank_iter_noalloc(ctypes.byref(dg.c), ctypes.byref(seg.c), damping, restart, contrib_type,
                                             _ptr(rank_in), _ptr(contrib_in), _ptr(scalars_in), _ptr(partial),
                                             _ptr(rank_out), _ptr(contrib_out), _ptr(scalars_out), _stream(stream)),
           "cagra_pagerank_iter_noalloc")


def pagerank_merge(dg: DeviceGraph, seg: Segments, damping: float, contrib_type: int, rank_in, scalars_in,
                   partial, rank_out, contrib_out, scalars_out, workspace, stream=None, restart: int = -1):
    _check(lib().cagra_pagerank_merge(ctypes.byref(dg.c), ctypes.byref(seg.c), damping, restart, contrib_type,
                                      _ptr(rank_in), _ptr(scalars_in), _ptr(partial), _ptr(rank_out),
                                      _ptr(contrib_out), _ptr(scalars_out), _ptr(workspace), workspace.numel(),
                                      _stream(stream)), "cagra_pagerank_merge")


def labelprop_iter(seg: Segments, labels_in, partial, labels_out, changed_out, workspace, stream=None):
    _check(lib().cagra_labelprop_iter(ctypes.byref(seg.c), _ptr(labels_in), _ptr(partial), _ptr(labels_out),
                                      _ptr(changed_out), _ptr(workspace), workspace.numel(), _stream(stream)),
           "cagra_labelprop_iter")


# --------------------------------------------------------------------------- iteration driver

class PageRankState:
    """Device buffers for the PageRank power iteration (double-buffered)."""

    def __init__(self, dg: DeviceGraph, seg: Segments, contrib_type: int = F32, restart: int = -1):
        """restart: -1 for the uniform teleport, else the restart vertex of a
        personalized PageRank (start vector e_restart by default)."""
        import torch
        dev = _dev()
        V = dg.V
        self.dg, self.seg, self.contrib_type, self.restart = dg, seg, contrib_type, restart
        cdt = torch.float32 if contrib_type == F32 else torch.int16
        self.rank = [torch.empty(V, dtype=torch.float32, device=dev) for _ in range(2)]
        self.contrib = [torch.empty(V, dtype=cdt, device=dev) for _ in range(2)]
        self.scalars = [torch.zeros(4, dtype=torch.float64, device=dev) for _ in range(2)]
        self.partial = torch.empty(max(seg.Q, 1), dtype=torch.float32, device=dev)
        self.ws = iter_workspace(seg)
        self.cur = 0

    def start(self, rank0=None, stream=None):
        """rank0: device float32 [V] start vector (None: uniform 1/V, or e_restart
        for a personalized state)."""
        if rank0 is not None:
            self.rank[0].copy_(rank0)
        elif self.restart >= 0:
            self.rank[0].zero_()
            self.rank[0][self.restart] = 1.0
        else:
            self.rank[0].fill_(1.0 / self.dg.V)
        self.cur = 0
        pagerank_init(self.dg, self.contrib_type, self.rank[0], self.contrib[0], self.scalars[0], self.ws, stream)

    def step(self, damping: float = 0.85, stream=None):
        a, b = self.cur, 1 - self.cur
        pagerank_iter(self.dg, self.seg, damping, self.contrib_type, self.rank[a], self.contrib[a],
                      self.scalars[a], self.partial, self.rank[b], self.contrib[b], self.scalars[b], self.ws,
                      stream, self.restart)
        self.cur = b

    def step_split(self, damping: float = 0.85, stream=None, events=None):
        """Same step as step(), issued as the gather call then the merge call;
        events (3 torch.cuda.Event) are recorded before, between and after."""
        a, b = self.cur, 1 - self.cur
        if events:
            events[0].record()
        segment_gather(self.seg, SUM_F32, self.contrib_type, self.contrib[a], self.partial, stream)
        if events:
            events[1].record()
        pagerank_merge(self.dg, self.seg, damping, self.contrib_type, self.rank[a], self.scalars[a], self.partial,
                       self.rank[b], self.contrib[b], self.scalars[b], self.ws, stream, self.restart)
        if events:
            events[2].record()
        self.cur = b

    @property
    def rank_now(self):
        return self.rank[self.cur]

    @property
    def scalars_now(self):
        return self.scalars[self.cur]


@dataclass
class SolveResult:
    rank: object          # device float32 [V]
    iters: int
    iters_bf16: int
    residual: float
    scalars: list
    converged: bool


@dataclass
class PprSolveResult:
    iters: int
    residual: float       # largest column residual of the last check
    converged: bool


def pagerank_solve(dg: DeviceGraph, seg: Segments, tol: float = 1e-6, max_iters: int = 100, damping: float = 0.85,
                   contrib_type: int = F32, switch_tol: float = 0.0, rank0=None, check_every: int = 1,
                   stream=None, state: "SolveBuffers | None" = None, restart: int = -1) -> SolveResult:
    """cagra_pagerank_solve: power iteration to the first L1 residual < tol (the
    library's host-driven loop). BF16 contributions with switch_tol > 0 finish
    in FP32 once the residual is below switch_tol. Returns a SolveResult with
    converged False when max_iters ran out (CAGRA_E_NOT_CONVERGED); raises
    CagraError for any other failure, E_RANGE included."""
    buf = state or SolveBuffers(dg, seg, contrib_type, switch_tol)
    if rank0 is not None:
        buf.rank[0].copy_(rank0)
    elif restart >= 0:
        buf.rank[0].zero_()
        buf.rank[0][restart] = 1.0
    else:
        buf.rank[0].fill_(1.0 / dg.V)
    p = CPrParams(damping, tol, switch_tol, restart, max_iters, check_every, contrib_type)
    r = CPrResult()
    st = lib().cagra_pagerank_solve(ctypes.byref(dg.c), ctypes.byref(seg.c), ctypes.byref(p), _ptr(buf.rank[0]),
                                    _ptr(buf.rank[1]), _ptr(buf.contrib[0]), _ptr(buf.contrib[1]), _ptr(buf.scalars),
                                    _ptr(buf.partial), _ptr(buf.ws), buf.ws.numel(), ctypes.byref(r),
                                    _stream(stream))
    if st not in (OK, E_NOT_CONVERGED):
        _check(st, "cagra_pagerank_solve")
    return SolveResult(buf.rank[r.final_buf], int(r.iters), int(r.iters_bf16), float(r.residual),
                       list(r.scalars), st == OK)


class SolveBuffers:
    """Device buffers of cagra_pagerank_solve (reusable across calls)."""

    def __init__(self, dg: DeviceGraph, seg: Segments, contrib_type: int = F32, switch_tol: float = 0.0):
        import torch
        dev = _dev()
        V = dg.V
        wide = contrib_type == F32 or switch_tol > 0
        cdt = torch.float32 if wide else torch.int16
        self.rank = [torch.empty(V, dtype=torch.float32, device=dev) for _ in range(2)]
        self.contrib = [torch.empty(V, dtype=cdt, device=dev) for _ in range(2)]
        self.scalars = torch.zeros(8, dtype=torch.float64, device=dev)
        self.partial = torch.empty(max(seg.Q, 1), dtype=torch.float32, device=dev)
        self.ws = iter_workspace(seg)


def pagerank(dg: DeviceGraph, seg: Segments, iters: int = 20, damping: float = 0.85, contrib_type: int = F32,
             tol: float = 0.0, rank0=None, check_every: int = 1, switch_tol: float = 0.0,
             allow_not_converged: bool = False):
    """Power iteration; fixed `iters` steps (tol 0), or stop at the first L1
    residual < tol read back every `check_every` steps (through
    cagra_pagerank_solve, at most `iters` steps). Returns (rank tensor, residual
    list, steps): the list is None in fixed mode, else [last residual read].
    Raises NotConverged when tol > 0 and the cap is reached (unless
    allow_not_converged), and CagraError(E_RANGE) when an iteration's buffer
    values left the exact fixed-point range."""
    if tol > 0:
        r = pagerank_solve(dg, seg, tol=tol, max_iters=iters, damping=damping, contrib_type=contrib_type,
                           switch_tol=switch_tol, rank0=rank0, check_every=check_every)
        out = (r.rank.clone(), [r.residual], r.iters)
        if not r.converged and not allow_not_converged:
            raise NotConverged("cagra_pagerank_solve", f"no L1 residual < {tol:g} in {iters} iterations "
                                                       f"(last {r.residual:g})", out)
        return out
    stt = PageRankState(dg, seg, contrib_type)
    stt.start(rank0)
    for _ in range(iters):
        stt.step(damping)
    check_range(stt.scalars_now)
    return stt.rank_now.clone(), None, iters


def labelprop(seg: Segments, max_iters: int = 1 << 20, check_every: int = 1, labels0=None, stream=None):
    """cagra_labelprop_solve: min-label propagation from the vertex ids (or
    labels0) to the fixed point; returns (labels tensor, iterations including the
    final one without changes). At the cap (CAGRA_E_NOT_CONVERGED) the labels so
    far and max_iters are returned."""
    import torch
    dev = _dev()
    V = seg.c.V
    lab = [torch.arange(V, dtype=torch.int32, device=dev) if labels0 is None else labels0.to(torch.int32).clone(),
           torch.empty(V, dtype=torch.int32, device=dev)]
    partial = torch.empty(max(seg.Q, 1), dtype=torch.int32, device=dev)
    changed = torch.zeros(1, dtype=torch.int32, device=dev)
    ws = iter_workspace(seg)
    r = CLpResult()
    st = lib().cagra_labelprop_solve(ctypes.byref(seg.c), max_iters, check_every, _ptr(lab[0]), _ptr(lab[1]),
                                     _ptr(partial), _ptr(changed), _ptr(ws), ws.numel(), ctypes.byref(r),
                                     _stream(stream))
    if st not in (OK, E_NOT_CONVERGED):
        _check(st, "cagra_labelprop_solve")
    return lab[r.final_buf], int(r.iters)


# --------------------------------------------------------------------------- push direction

def push_workspace(seg_t: Segments):
    import torch
    n = lib().cagra_push_workspace_bytes(ctypes.byref(seg_t.c))
    return torch.empty(n, dtype=torch.uint8, device=_dev())


def pagerank_push_iter(dg: DeviceGraph, seg_t: Segments, damping: float, rank_in, contrib_in, scalars_in, vals,
                       rank_out, contrib_out, scalars_out, workspace, stream=None):
    _check(lib().cagra_pagerank_push_iter(ctypes.byref(dg.c), ctypes.byref(seg_t.c), damping, _ptr(rank_in),
                                          _ptr(contrib_in), _ptr(scalars_in), _ptr(vals), _ptr(rank_out),
                                          _ptr(contrib_out), _ptr(scalars_out), _ptr(workspace), workspace.numel(),
                                          _stream(stream)), "cagra_pagerank_push_iter")


def labelprop_push_iter(seg_t: Segments, labels_in, vals, labels_out, changed_out, workspace, stream=None):
    _check(lib().cagra_labelprop_push_iter(ctypes.byref(seg_t.c), _ptr(labels_in), _ptr(vals), _ptr(labels_out),
                                           _ptr(changed_out), _ptr(workspace), workspace.numel(), _stream(stream)),
           "cagra_labelprop_push_iter")


class PushPageRankState:
    """PageRank power iteration in the push direction: dg is the graph, seg_t
    the segmentation of its reverse (FP32 contributions)."""

    def __init__(self, dg: DeviceGraph, seg_t: Segments):
        import torch
        dev = _dev()
        V = dg.V
        self.dg, self.seg_t = dg, seg_t
        self.rank = [torch.empty(V, dtype=torch.float32, device=dev) for _ in range(2)]
        self.contrib = [torch.empty(V, dtype=torch.float32, device=dev) for _ in range(2)]
        self._sc = torch.zeros(8, dtype=torch.float64, device=dev)  # the pair, back to back
        self.scalars = [self._sc[:4], self._sc[4:]]
        self.vals = torch.empty(max(seg_t.Q, 1), dtype=torch.float32, device=dev)
        self.ws = push_workspace(seg_t)
        self.cur = 0

    def start(self, rank0=None, stream=None):
        if rank0 is None:
            self.rank[0].fill_(1.0 / self.dg.V)
        else:
            self.rank[0].copy_(rank0)
        self.cur = 0
        pagerank_init(self.dg, F32, self.rank[0], self.contrib[0], self.scalars[0], self.ws, stream)

    def step(self, damping: float = 0.85, stream=None):
        a, b = self.cur, 1 - self.cur
        pagerank_push_iter(self.dg, self.seg_t, damping, self.rank[a], self.contrib[a], self.scalars[a], self.vals,
                           self.rank[b], self.contrib[b], self.scalars[b], self.ws, stream)
        self.cur = b

    @property
    def rank_now(self):
        return self.rank[self.cur]

    @property
    def scalars_now(self):
        return self.scalars[self.cur]


def pagerank_push(dg: DeviceGraph, seg_t: Segments, iters: int = 20, damping: float = 0.85, tol: float = 0.0,
                  check_every: int = 1):
    """Push-direction power iteration; fixed `iters` steps (tol 0), or through
    cagra_pagerank_push_solve to the first L1 residual < tol read back every
    `check_every` steps (at most `iters`). Returns (rank tensor, residual list or
    None, steps): the list is None in fixed mode, else [last residual read]."""
    stt = PushPageRankState(dg, seg_t)
    if tol > 0:
        p = CPrParams(damping, tol, 0.0, -1, iters, check_every, F32)
        r = CPrResult()
        stt.rank[0].fill_(1.0 / dg.V)
        st = lib().cagra_pagerank_push_solve(ctypes.byref(dg.c), ctypes.byref(seg_t.c), ctypes.byref(p),
                                             _ptr(stt.rank[0]), _ptr(stt.rank[1]), _ptr(stt.contrib[0]),
                                             _ptr(stt.contrib[1]), _ptr(stt._sc), _ptr(stt.vals), _ptr(stt.ws),
                                             stt.ws.numel(), ctypes.byref(r), None)
        if st not in (OK, E_NOT_CONVERGED):
            _check(st, "cagra_pagerank_push_solve")
        return stt.rank[r.final_buf].clone(), [float(r.residual)], int(r.iters)
    stt.start()
    for _ in range(iters):
        stt.step(damping)
    return stt.rank_now.clone(), None, iters


def labelprop_push(seg_t: Segments, max_iters: int = 1 << 20):
    """Min-label propagation to the fixed point in the push direction (seg_t: the
    segmentation of the reverse graph, the graph itself when undirected)."""
    import torch
    dev = _dev()
    V = seg_t.c.V
    lab = [torch.arange(V, dtype=torch.int32, device=dev), torch.empty(V, dtype=torch.int32, device=dev)]
    vals = torch.empty(max(seg_t.Q, 1), dtype=torch.int32, device=dev)
    changed = torch.zeros(1, dtype=torch.int32, device=dev)
    ws = push_workspace(seg_t)
    r = CLpResult()
    st = lib().cagra_labelprop_push_solve(ctypes.byref(seg_t.c), max_iters, 1, _ptr(lab[0]), _ptr(lab[1]),
                                          _ptr(vals), _ptr(changed), _ptr(ws), ws.numel(), ctypes.byref(r), None)
    if st not in (OK, E_NOT_CONVERGED):
        _check(st, "cagra_labelprop_push_solve")
    return lab[r.final_buf], int(r.iters)


# --------------------------------------------------------------------------- batched personalized PageRank

class PPRState:
    """Device buffers for personalized PageRank over up to 64 restart vertices at once
    ([V][64] row-major vertex values)."""

    def __init__(self, dg: DeviceGraph, seg: Segments, seeds):
        import torch
        dev = _dev()
        self.dg, self.seg = dg, seg
        self.ncols = len(seeds)
        assert 1 <= self.ncols <= PPR_COLS
        self.seeds = torch.as_tensor(np.asarray(seeds, dtype=np.int32)).to(dev)
        V = dg.V
        self.rank = [torch.empty(V * PPR_COLS, dtype=torch.float32, device=dev) for _ in range(2)]
        self.contrib = [torch.empty(V * PPR_COLS, dtype=torch.float32, device=dev) for _ in range(2)]
        self._sc = torch.zeros(2 * PPR_COLS * 4, dtype=torch.float64, device=dev)  # the pair, back to back
        self.scalars = [self._sc[:PPR_COLS * 4], self._sc[PPR_COLS * 4:]]
        self.partial = torch.empty(max(seg.Q, 1) * PPR_COLS, dtype=torch.float32, device=dev)
        n = lib().cagra_ppr_workspace_bytes(ctypes.byref(seg.c))
        self.ws = torch.empty(n, dtype=torch.uint8, device=dev)
        self.cur = 0

    def start(self, stream=None):
        self.cur = 0
        _check(lib().cagra_ppr_init(ctypes.byref(self.dg.c), self.ncols, _ptr(self.seeds), _ptr(self.rank[0]),
                                    _ptr(self.contrib[0]), _ptr(self.scalars[0]), _ptr(self.ws), self.ws.numel(),
                                    _stream(stream)), "cagra_ppr_init")

    def step(self, damping: float = 0.85, stream=None):
        a, b = self.cur, 1 - self.cur
        _check(lib().cagra_ppr_iter(ctypes.byref(self.dg.c), ctypes.byref(self.seg.c), damping, self.ncols,
                                    _ptr(self.seeds), _ptr(self.rank[a]), _ptr(self.contrib[a]),
                                    _ptr(self.scalars[a]), _ptr(self.partial), _ptr(self.rank[b]),
                                    _ptr(self.contrib[b]), _ptr(self.scalars[b]), _ptr(self.ws), self.ws.numel(),
                                    _stream(stream)), "cagra_ppr_iter")
        self.cur = b

    def solve(self, tol: float = 1e-6, max_iters: int = 100, damping: float = 0.85, check_every: int = 1,
              stream=None) -> "PprSolveResult":
        """cagra_ppr_solve: from the seed vectors until every column's L1 residual
        is below tol; the current vectors are then the result. converged is
        False when max_iters ran out (CAGRA_E_NOT_CONVERGED)."""
        p = CPprParams(damping, tol, max_iters, check_every)
        r = CPprResult()
        st = lib().cagra_ppr_solve(ctypes.byref(self.dg.c), ctypes.byref(self.seg.c), ctypes.byref(p), self.ncols,
                                   _ptr(self.seeds), _ptr(self.rank[0]), _ptr(self.rank[1]), _ptr(self.contrib[0]),
                                   _ptr(self.contrib[1]), _ptr(self._sc), _ptr(self.partial), _ptr(self.ws),
                                   self.ws.numel(), ctypes.byref(r), _stream(stream))
        if st not in (OK, E_NOT_CONVERGED):
            _check(st, "cagra_ppr_solve")
        self.cur = int(r.final_buf)
        return PprSolveResult(int(r.iters), float(r.residual), st == OK)

    def ranks(self):
        """[V, ncols] view of the current vectors."""
        return self.rank[self.cur].view(self.dg.V, PPR_COLS)[:, :self.ncols]

    @property
    def scalars_now(self):
        return self.scalars[self.cur].view(PPR_COLS, 4)[:self.ncols]


def ppr(dg: DeviceGraph, seg: Segments, seeds, iters: int = 20, damping: float = 0.85):
    st = PPRState(dg, seg, seeds)
    st.start()
    for _ in range(iters):
        st.step(damping)
    return st.ranks().clone(), st


# --------------------------------------------------------------------------- many graphs at once

class MultiPageRank:
    """PageRank on many independent graphs with persistent kernels over a global
    tile / merge-block list; `run` captures the whole run into one HIP graph."""

    def __init__(self, dgs, segs):
        import torch
        dev = _dev()
        n = len(dgs)
        assert n == len(segs) and n >= 1
        self.dgs, self.segs = dgs, segs
        self.garr = (CGraph * n)(*[d.c for d in dgs])
        self.sarr = (CSegments * n)(*[s.c for s in segs])
        m = CMulti()
        _check(lib().cagra_multi_query(n, self.garr, self.sarr, ctypes.byref(m)), "cagra_multi_query")
        TV, TQ, TB = m.total_V, m.total_Q, m.total_blocks
        self.desc = torch.empty(m.desc_bytes, dtype=torch.uint8, device=dev)
        self.rank = [torch.empty(TV, dtype=torch.float32, device=dev) for _ in range(2)]
        self.contrib = [torch.empty(TV, dtype=torch.float32, device=dev) for _ in range(2)]
        self.scalars = [torch.zeros(4 * n, dtype=torch.float64, device=dev) for _ in range(2)]
        self.partial = torch.empty(max(TQ, 1), dtype=torch.float32, device=dev)
        self.blk = torch.empty(4 * max(TB, 1), dtype=torch.float64, device=dev)
        m.desc = self.desc.data_ptr()
        for p in range(2):
            m.rank[p] = self.rank[p].data_ptr()
            m.contrib[p] = self.contrib[p].data_ptr()
            m.scalars[p] = self.scalars[p].data_ptr()
        m.partial = self.partial.data_ptr()
        m.blk = self.blk.data_ptr()
        _check(lib().cagra_multi_setup(ctypes.byref(m), self.garr, self.sarr, _stream()), "cagra_multi_setup")
        self.m = m
        self.offsets = np.concatenate([[0], np.cumsum([d.V for d in dgs])]).astype(np.int64)
        self.cur = 0
        self.graph = None

    def start(self, stream=None):
        _check(lib().cagra_multi_pagerank_start(ctypes.byref(self.m), _stream(stream)), "cagra_multi_pagerank_start")
        self.cur = 0

    def step(self, damping: float = 0.85, stream=None):
        _check(lib().cagra_multi_pagerank_step(ctypes.byref(self.m), self.cur, damping, _stream(stream)),
               "cagra_multi_pagerank_step")
        self.cur = 1 - self.cur

    def run_eager(self, iters: int = 20, damping: float = 0.85):
        self.start()
        for _ in range(iters):
            self.step(damping)

    def capture(self, iters: int = 20, damping: float = 0.85):
        """Records start + `iters` iterations of every graph into one HIP graph."""
        import torch
        self.run_eager(1, damping)  # first launches set kernel attributes outside the capture
        torch.cuda.synchronize()
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        g = torch.cuda.CUDAGraph()
        with torch.cuda.stream(s):
            with torch.cuda.graph(g, stream=s):
                self.run_eager(iters, damping)
        torch.cuda.current_stream().wait_stream(s)
        self.graph = g
        self.graph_final = self.cur
        return g

    def replay(self):
        self.graph.replay()
        self.cur = self.graph_final

    def rank_of(self, i: int):
        return self.rank[self.cur][self.offsets[i]:self.offsets[i + 1]]

    def scalars_of(self, i: int):
        return self.scalars[self.cur][4 * i:4 * i + 4]


# --------------------------------------------------------------------------- collaborative filtering

def segment_edge_values(dg: DeviceGraph, seg: Segments, in_values, stream=None):
    """Edge values (float32, CSC order) permuted into the segmented edge order."""
    import torch
    out = torch.empty(max(dg.E, 1), dtype=torch.float32, device=_dev())
    _check(lib().cagra_segment_edge_values(ctypes.byref(dg.c), ctypes.byref(seg.c), _ptr(in_values), _ptr(out),
                                           _stream(stream)), "cagra_segment_edge_values")
    return out


class CFState:
    """Latent vectors [V][64] (double-buffered) and scratch for gradient-descent
    collaborative filtering on a rating graph through segmenting."""

    def __init__(self, dg: DeviceGraph, seg: Segments, seg_values, x0):
        import torch
        dev = _dev()
        self.dg, self.seg, self.vals = dg, seg, seg_values
        self.x = [x0.clone(), torch.empty_like(x0)]
        self.partial = torch.empty(max(seg.Q, 1) * CF_FACTORS, dtype=torch.float32, device=dev)
        n = lib().cagra_cf_workspace_bytes(ctypes.byref(seg.c))
        self.ws = torch.empty(n, dtype=torch.uint8, device=dev)
        self.sq = torch.zeros(1, dtype=torch.float64, device=dev)
        self.cur = 0

    def step(self, gamma: float, lam: float, stream=None):
        a, b = self.cur, 1 - self.cur
        _check(lib().cagra_cf_iter(ctypes.byref(self.dg.c), ctypes.byref(self.seg.c), _ptr(self.vals), gamma, lam,
                                   _ptr(self.x[a]), _ptr(self.partial), _ptr(self.x[b]), _ptr(self.sq),
                                   _ptr(self.ws), self.ws.numel(), _stream(stream)), "cagra_cf_iter")
        self.cur = b

    @property
    def x_now(self):
        return self.x[self.cur]


# --------------------------------------------------------------------------- betweenness centrality

class BCState:
    """Buffers for Brandes' betweenness centrality from sampled starts, with the
    segmentation of the graph (forward levels) and of its reverse (backward)."""

    def __init__(self, seg: Segments, seg_t: Segments):
        import torch
        dev = _dev()
        V = seg.c.V
        assert seg_t.c.V == V
        self.seg, self.seg_t = seg, seg_t
        self.depth = torch.empty(V, dtype=torch.int32, device=dev)
        self.sigma = torch.empty(V, dtype=torch.float32, device=dev)
        self.delta = torch.empty(V, dtype=torch.float32, device=dev)
        self.bc = torch.zeros(V, dtype=torch.float32, device=dev)
        self.vals = torch.empty(V, dtype=torch.float32, device=dev)
        self.sums = torch.empty(V, dtype=torch.float32, device=dev)
        self.partial = torch.empty(max(seg.Q, seg_t.Q, 1), dtype=torch.float32, device=dev)
        self.count = torch.zeros(1, dtype=torch.int32, device=dev)
        L = lib()
        self.ws = torch.empty(max(L.cagra_bc_workspace_bytes(ctypes.byref(seg.c)),
                                  L.cagra_bc_workspace_bytes(ctypes.byref(seg_t.c))), dtype=torch.uint8, device=dev)
        self.levels = []

    def add_source(self, source: int, stream=None):
        """Forward levels until the frontier is empty (one count read-back per
        level), then the backward levels; adds the start's dependencies to bc."""
        L, st = lib(), _stream(stream)
        V = self.seg.c.V
        _check(L.cagra_bc_start(V, source, _ptr(self.depth), _ptr(self.sigma), _ptr(self.delta), st), "cagra_bc_start")
        d = 0
        while True:
            _check(L.cagra_bc_forward_level(ctypes.byref(self.seg.c), d, _ptr(self.depth), _ptr(self.sigma),
                                            _ptr(self.vals), _ptr(self.partial), _ptr(self.sums), _ptr(self.count),
                                            _ptr(self.ws), self.ws.numel(), st), "cagra_bc_forward_level")
            if int(self.count.item()) == 0:
                break
            d += 1
        for dd in range(d - 1, -1, -1):
            _check(L.cagra_bc_backward_level(ctypes.byref(self.seg_t.c), dd, source, _ptr(self.depth),
                                             _ptr(self.sigma), _ptr(self.delta), _ptr(self.bc), _ptr(self.vals),
                                             _ptr(self.partial), _ptr(self.sums), _ptr(self.ws), self.ws.numel(), st),
                   "cagra_bc_backward_level")
        self.levels.append(d + 1)


def betweenness(seg: Segments, seg_t: Segments, sources):
    """BC summed over the given starts (FP32 tensor [V])."""
    st = BCState(seg, seg_t)
    for s in sources:
        st.add_source(int(s))
    return st.bc, st.levels
