"""Learned warm start of the PageRank power iteration (driver over the C ABI).

Features (log in-degree, log out-degree, mean log out-degree of in-neighbours)
come from the library's segmented pull; a 3 -> 64 -> 64 -> 1 GELU network with
BF16 weights (FP32 master copy, Adam) is trained on the GPU to predict
log(V * r*) from PageRank vectors r* that the method itself computes; its
output becomes the start vector softmax(y). The plain iteration from that
vector decides convergence, and the uniform start is the fallback whenever the
predicted vector is not usable.
"""
from __future__ import annotations

import ctypes
import time
from dataclasses import dataclass, field

import numpy as np

from . import cagra

NPARAM = 4481
OFF_W1, OFF_B1, OFF_W2, OFF_B2, OFF_W3, OFF_B3 = 0, 192, 256, 4352, 4416, 4480


def _p(t):
    return ctypes.c_void_p(t.data_ptr())


def features(dg, seg):
    """[V, 3] float32 device tensor."""
    import torch
    L = cagra.lib()
    F = torch.empty(dg.V * 3, dtype=torch.float32, device="cuda")
    n = L.cagra_features_workspace_bytes(ctypes.byref(seg.c))
    ws = torch.empty(n, dtype=torch.uint8, device="cuda")
    cagra._check(L.cagra_degree_features(ctypes.byref(dg.c), ctypes.byref(seg.c), _p(F), _p(ws), n,
                                         cagra._stream()), "cagra_degree_features")
    return F.view(dg.V, 3)


def init_params(seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    p = np.zeros(NPARAM, dtype=np.float32)
    p[OFF_W1:OFF_B1] = rng.normal(0, 1 / np.sqrt(3), 192)
    p[OFF_W2:OFF_B2] = rng.normal(0, 1 / np.sqrt(64), 64 * 64)
    p[OFF_W3:OFF_B3] = rng.normal(0, 1 / np.sqrt(64), 64)
    return p


@dataclass
class Network:
    master: object = None   # float32 [NPARAM]
    weights: object = None  # bf16 bits (int16) [NPARAM]
    m: object = None
    v: object = None
    norm: object = None     # float32 [6]: mean[3], 1/std[3]
    step: int = 0
    losses: list = field(default_factory=list)

    @staticmethod
    def create(seed: int, mean=None, std=None, norm=None):
        """Parameters from init_params(seed) (FP32 master, BF16 copy by round to
        nearest even in the library's Adam kernel convention), zero Adam state,
        and the feature standardization: either `norm` (device float32 [6], as
        cagra_feature_norm writes it) or host `mean`/`std` arrays."""
        import torch
        p = torch.from_numpy(init_params(seed)).cuda()
        net = Network()
        net.master = p
        net.weights = p.to(torch.bfloat16).view(torch.int16).contiguous()
        net.m = torch.zeros_like(p)
        net.v = torch.zeros_like(p)
        if norm is None:
            norm = torch.from_numpy(np.concatenate([np.asarray(mean, np.float32),
                                                    1.0 / np.asarray(std, np.float32)]).astype(np.float32)).cuda()
        net.norm = norm
        return net

    def forward(self, F):
        import torch
        n = F.shape[0]
        y = torch.empty(n, dtype=torch.float32, device="cuda")
        cagra._check(cagra.lib().cagra_mlp_forward(_p(F), n, _p(self.weights), _p(self.norm), _p(y),
                                                   cagra._stream()), "cagra_mlp_forward")
        return y

    def grad(self, F, t):
        import torch
        L = cagra.lib()
        g = torch.empty(NPARAM, dtype=torch.float32, device="cuda")
        loss = torch.empty(1, dtype=torch.float64, device="cuda")
        nws = L.cagra_mlp_grad_workspace_bytes()
        ws = torch.empty(nws, dtype=torch.uint8, device="cuda")
        cagra._check(L.cagra_mlp_grad(_p(F), _p(t), F.shape[0], _p(self.weights), _p(self.norm), _p(g), _p(loss),
                                      _p(ws), nws, cagra._stream()), "cagra_mlp_grad")
        return g, loss

    def adam(self, g, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.step += 1
        cagra._check(cagra.lib().cagra_adam_step(_p(self.master), _p(self.weights), _p(self.m), _p(self.v), _p(g),
                                                 self.step, lr, b1, b2, eps, cagra._stream()), "cagra_adam_step")


def pagerank_target(dg, seg, tol=1e-8, max_iters=100):
    """log(V * r*) (cagra_mlp_targets) with r* the method's own FP32 PageRank at
    residual < tol (or after max_iters iterations)."""
    import torch
    r, _, _ = cagra.pagerank(dg, seg, iters=max_iters, tol=tol, check_every=4, allow_not_converged=True)
    t = torch.empty(dg.V, dtype=torch.float32, device="cuda")
    cagra._check(cagra.lib().cagra_mlp_targets(_p(r), dg.V, _p(t), cagra._stream()), "cagra_mlp_targets")
    return t


def feature_norm(F):
    """Device float32 [6]: column means and 1/std of F [n, 3] (cagra_feature_norm)."""
    import torch
    L = cagra.lib()
    n = F.shape[0]
    norm = torch.empty(6, dtype=torch.float32, device="cuda")
    nws = L.cagra_feature_norm_workspace_bytes(n)
    ws = torch.empty(nws, dtype=torch.uint8, device="cuda")
    cagra._check(L.cagra_feature_norm(_p(F), n, _p(norm), _p(ws), nws, cagra._stream()), "cagra_feature_norm")
    return norm


def sample_rows(F, T, seed: int, draw: int, batch: int, out=None):
    """Minibatch `draw` of `batch` rows (cagra_sample_rows); returns (Fb, Tb)."""
    import torch
    if out is None:
        out = (torch.empty(batch, 3, dtype=torch.float32, device="cuda"),
               torch.empty(batch, dtype=torch.float32, device="cuda"))
    Fb, Tb = out
    cagra._check(cagra.lib().cagra_sample_rows(_p(F), _p(T), F.shape[0], seed & (2 ** 64 - 1), draw, batch, _p(Fb),
                                               _p(Tb), cagra._stream()), "cagra_sample_rows")
    return Fb, Tb


def train(F, T, seed: int = 0, steps: int = 400, batch: int = 65536, lr: float = 3e-3, log=None):
    """Minibatch Adam on rows (F [n,3], T [n]) held on the GPU; deterministic row sampling."""
    net = Network.create(seed, norm=feature_norm(F))
    n = F.shape[0]
    bufs = None
    for s in range(steps):
        Fb, Tb = bufs = sample_rows(F, T, seed, s, min(batch, n), bufs)
        g, loss = net.grad(Fb, Tb)
        net.adam(g, lr=lr)
        if log and (s % 100 == 0 or s == steps - 1):
            lv = float(loss.item())
            net.losses.append(lv)
            log(f"train step {s} loss {lv:.4f}")
    return net


def start_vector(net: Network, F):
    """(rank0 device float32 [V], usable) -- softmax of the network output."""
    import torch
    L = cagra.lib()
    V = F.shape[0]
    y = net.forward(F)
    r0 = torch.empty(V, dtype=torch.float32, device="cuda")
    sc = torch.zeros(4, dtype=torch.float64, device="cuda")
    n = L.cagra_warm_start_workspace_bytes(V)
    ws = torch.empty(n, dtype=torch.uint8, device="cuda")
    cagra._check(L.cagra_warm_start_vector(_p(y), V, _p(r0), _p(sc), _p(ws), n, cagra._stream()),
                 "cagra_warm_start_vector")
    s = sc.cpu().numpy()
    usable = s[1] == 0 and np.isfinite(s[2]) and s[2] > 0
    return r0, bool(usable)


def learned_start(net: Network, dg, seg, ws=None):
    """(rank0, usable): the start vector in one library call (cagra_learned_start:
    features, the network, softmax), bit-identical to start_vector(net,
    features(dg, seg))."""
    import torch
    L = cagra.lib()
    r0 = torch.empty(dg.V, dtype=torch.float32, device="cuda")
    sc = torch.zeros(4, dtype=torch.float64, device="cuda")
    n = L.cagra_learned_start_workspace_bytes(ctypes.byref(seg.c))
    if ws is None or ws.numel() < n:
        ws = torch.empty(n, dtype=torch.uint8, device="cuda")
    cagra._check(L.cagra_learned_start(ctypes.byref(dg.c), ctypes.byref(seg.c), _p(net.weights), _p(net.norm),
                                       _p(r0), _p(sc), _p(ws), n, cagra._stream()), "cagra_learned_start")
    s = sc.cpu().numpy()
    usable = s[1] == 0 and np.isfinite(s[2]) and s[2] > 0
    return r0, bool(usable)


def solve(dg, seg, tol=1e-6, max_iters=100, net: Network | None = None, ws=None, buffers=None):
    """PageRank to residual < tol from the uniform start (net None) or the learned one.
    Returns (rank, iterations, ms including features and network time, start used).
    ws / buffers: optional preallocated start workspace and solve buffers (so
    that the timing covers no allocation)."""
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rank0, used = None, "uniform"
    if net is not None:
        rank0, ok = learned_start(net, dg, seg, ws)
        if ok:
            used = "learned"
        else:
            rank0 = None
            used = "uniform (fallback)"
    res = cagra.pagerank_solve(dg, seg, tol=tol, max_iters=max_iters, rank0=rank0, state=buffers)
    torch.cuda.synchronize()
    return res.rank.clone(), res.iters, (time.perf_counter() - t0) * 1e3, used
