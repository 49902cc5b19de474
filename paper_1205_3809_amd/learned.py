"""Learned vertex ordering: an MLP that predicts smallest-last ranks.

Every numeric step runs in libgcolor.so kernels (features, forward, gradient,
Adam, score-to-key map, colouring); this module only schedules them:

* targets: exact smallest-last positions from the library's host routine,
  mapped on the device to log(1 + rank) / log(n) (0 = coloured first);
* training: minibatches of vertices drawn (seeded) across the training
  graphs, mean squared error, Adam on FP32 master weights, BF16 copies for
  the forward pass;
* inference: features -> scores -> keys -> color_graph(priority=keys); with
  the fallback on, the natural-order colouring is also computed and the one
  with fewer colours is returned.
"""
from __future__ import annotations

import ctypes
import os
import time
from typing import List, NamedTuple, Optional, Sequence

import numpy as np
import torch

from . import _binding as B

NF = 8
NH = 64
NPARAM = 4801
W1, B1, W2, B2, W3, B3 = 0, 512, 576, 4672, 4736, 4800


def _vp(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _check(rc: int, where: str):
    if rc != 0:
        raise B.GColorError(rc, where)


def _stream():
    return B._stream_handle(None)


def features(row_ptr: torch.Tensor, col_idx: torch.Tensor, seed: int = 0x5EED) -> torch.Tensor:
    n = row_ptr.numel() - 1
    out = torch.empty((max(n, 0), NF), dtype=torch.float32, device=row_ptr.device)
    nb = int(B._lib.gcolor_features_workspace_bytes(max(n, 0)))
    ws = torch.empty(max(nb, 1), dtype=torch.uint8, device=row_ptr.device)
    _check(B._lib.gcolor_features(n, _vp(row_ptr), _vp(col_idx), seed, _vp(out), _vp(ws), nb, _stream()),
           "gcolor_features")
    return out


def smallest_last_rank(row_ptr: np.ndarray, col_idx: np.ndarray):
    """Exact smallest-last positions (host routine of the library)."""
    row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int32)
    col_idx = np.ascontiguousarray(col_idx, dtype=np.int32)
    n = row_ptr.shape[0] - 1
    rank = np.zeros(max(n, 1), dtype=np.int32)
    deg = ctypes.c_int32()
    _check(B._lib.gcolor_smallest_last_host(n, row_ptr.ctypes.data_as(ctypes.c_void_p),
                                            col_idx.ctypes.data_as(ctypes.c_void_p),
                                            rank.ctypes.data_as(ctypes.c_void_p), ctypes.byref(deg)),
           "gcolor_smallest_last_host")
    return rank[:n], int(deg.value)


class MLP:
    """Parameters on one device: FP32 master, BF16 copy, normalisation, Adam state."""

    def __init__(self, device="cuda", seed: int = 0):
        rng = np.random.default_rng(seed)
        p = np.zeros(NPARAM, dtype=np.float32)
        # He-uniform initialisation
        p[W1:B1] = rng.uniform(-1, 1, NH * NF) * np.sqrt(6.0 / NF)
        p[W2:B2] = rng.uniform(-1, 1, NH * NH) * np.sqrt(6.0 / NH)
        p[W3:B3] = rng.uniform(-1, 1, NH) * np.sqrt(6.0 / NH)
        p[B3] = 0.5
        self.device = torch.device(device)
        self.master = torch.from_numpy(p).to(self.device)
        self.wbf = torch.zeros(NPARAM, dtype=torch.int16, device=self.device)
        self.norm = torch.from_numpy(np.r_[np.zeros(NF), np.ones(NF)].astype(np.float32)).to(self.device)
        self.mom = torch.zeros(NPARAM, dtype=torch.float32, device=self.device)
        self.vel = torch.zeros(NPARAM, dtype=torch.float32, device=self.device)
        self.step = 0
        self.refresh()

    def refresh(self):
        _check(B._lib.gcolor_mlp_refresh_bf16(_vp(self.master), _vp(self.wbf), _stream()), "refresh_bf16")

    def fit_norm(self, feats: Sequence[torch.Tensor]):
        """Per-feature mean and standard deviation of log1p(feature) over the
        vertices of every tensor in feats (library kernels)."""
        acc = torch.zeros(2 * NF, dtype=torch.float64, device=self.device)
        total = 0
        for f in feats:
            _check(B._lib.gcolor_feature_stats(f.shape[0], _vp(f), _vp(acc), _stream()), "feature_stats")
            total += f.shape[0]
        norm = torch.empty(2 * NF, dtype=torch.float32, device=self.device)
        _check(B._lib.gcolor_feature_norm(total, _vp(acc), _vp(norm), _stream()), "feature_norm")
        self.norm = norm

    def scores(self, feat: torch.Tensor) -> torch.Tensor:
        out = torch.empty(feat.shape[0], dtype=torch.float32, device=self.device)
        _check(B._lib.gcolor_mlp_forward(feat.shape[0], _vp(feat), _vp(self.master), _vp(self.wbf),
                                         _vp(self.norm), _vp(out), _stream()), "mlp_forward")
        return out

    def grad(self, idx: torch.Tensor, feat: torch.Tensor, target: torch.Tensor) -> torch.Tensor:
        """Gradient of the mean squared error over the vertices idx (last entry: loss)."""
        nb = idx.numel()
        partial = torch.empty(B._lib.gcolor_mlp_partial_floats(nb), dtype=torch.float32, device=self.device)
        g = torch.empty(NPARAM + 1, dtype=torch.float32, device=self.device)
        _check(B._lib.gcolor_mlp_grad(nb, _vp(idx), _vp(feat), _vp(target), _vp(self.master), _vp(self.wbf),
                                      _vp(self.norm), _vp(partial), _vp(g), _stream()), "mlp_grad")
        return g

    def adam(self, g: torch.Tensor, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.step += 1
        _check(B._lib.gcolor_mlp_adam(_vp(self.master), _vp(self.wbf), _vp(self.mom), _vp(self.vel), _vp(g),
                                      lr, beta1, beta2, eps, self.step, _stream()), "mlp_adam")

    def state(self) -> dict:
        return {"master": self.master.cpu().numpy(), "wbf": self.wbf.cpu().numpy(), "norm": self.norm.cpu().numpy(),
                "step": np.array([self.step])}

    def save(self, path: str):
        np.savez(path, **self.state())

    @classmethod
    def load(cls, path: str, device="cuda"):
        d = np.load(path)  # plain arrays, no pickles
        m = cls(device)
        m.master = torch.from_numpy(d["master"].astype(np.float32)).to(m.device)
        m.norm = torch.from_numpy(d["norm"].astype(np.float32)).to(m.device)
        m.step = int(d["step"][0])
        m.refresh()
        return m


class TrainReport(NamedTuple):
    losses: List[float]
    seconds: float
    vertices: int


def rank_targets(rank: torch.Tensor) -> torch.Tensor:
    """Training targets of smallest-last positions r of n (device int32):
    log(1 + r) / log(n), in [0, 1] and monotone in r (library kernel).  The
    log scale spreads out the head of the order (the dense core, coloured
    first), where the colour count is decided; a plain r / (n - 1) target
    lets the many low-degree vertices dominate the squared error."""
    out = torch.empty(rank.numel(), dtype=torch.float32, device=rank.device)
    _check(B._lib.gcolor_rank_targets(rank.numel(), _vp(rank), _vp(out), _stream()), "rank_targets")
    return out


def train(model: MLP, graphs, epochs: int = 3, batch: int = 65536, lr: float = 2e-3, seed: int = 7,
          feat_seed: int = 0x5EED, log=None) -> TrainReport:
    """graphs: list of (row_ptr, col_idx) numpy CSR.  Targets from the exact
    smallest-last order; every numeric step on the device."""
    dev = model.device
    feats, targs = [], []
    for rp, ci in graphs:
        rpd = torch.from_numpy(np.ascontiguousarray(rp)).to(dev)
        cid = torch.from_numpy(np.ascontiguousarray(ci)).to(dev)
        feats.append(features(rpd, cid, feat_seed))
        rank, _ = smallest_last_rank(rp, ci)
        targs.append(rank_targets(torch.from_numpy(rank).to(dev)))
    model.fit_norm(feats)
    F = torch.cat(feats, 0)
    T = torch.cat(targs, 0)
    N = F.shape[0]
    rng = np.random.default_rng(seed)
    losses = []
    t0 = time.perf_counter()
    for ep in range(epochs):
        perm = torch.from_numpy(rng.permutation(N).astype(np.int32)).to(dev)
        tot, nb = 0.0, 0
        for s in range(0, N, batch):
            idx = perm[s:s + batch]
            g = model.grad(idx, F, T)
            model.adam(g, lr=lr)
            tot += float(g[NPARAM].item()) if (nb % 16 == 0) else 0.0
            nb += 1
        torch.cuda.synchronize()
        g = model.grad(perm[:batch], F, T)
        losses.append(float(g[NPARAM].item()))
        if log:
            log("epoch %d: minibatch loss %.5f" % (ep, losses[-1]))
    torch.cuda.synchronize()
    return TrainReport(losses, time.perf_counter() - t0, N)


def keys_from_scores(scores: torch.Tensor) -> torch.Tensor:
    keys = torch.empty(scores.numel(), dtype=torch.int32, device=scores.device)
    bad = torch.zeros(1, dtype=torch.int32, device=scores.device)
    _check(B._lib.gcolor_scores_to_keys(scores.numel(), _vp(scores), _vp(keys), _vp(bad), _stream()),
           "scores_to_keys")
    return keys, bad


def order_learned(model: MLP, row_ptr: torch.Tensor, col_idx: torch.Tensor, feat_seed: int = 0x5EED):
    """Priority keys (int32 bit patterns of uint32) for color_graph, from one
    library call (features, MLP forward, key map); also the NaN flag."""
    n = row_ptr.numel() - 1
    keys = torch.empty(max(n, 0), dtype=torch.int32, device=row_ptr.device)
    bad = torch.zeros(1, dtype=torch.int32, device=row_ptr.device)
    nb = int(B._lib.gcolor_order_learned_workspace_bytes(max(n, 0)))
    ws = torch.empty(max(nb, 1), dtype=torch.uint8, device=row_ptr.device)
    _check(B._lib.gcolor_order_learned(n, _vp(row_ptr), _vp(col_idx), feat_seed, _vp(model.master), _vp(model.wbf),
                                       _vp(model.norm), _vp(keys), _vp(bad), _vp(ws), nb, _stream()),
           "gcolor_order_learned")
    return keys, bad


def color_learned(model: MLP, row_ptr: torch.Tensor, col_idx: torch.Tensor, fallback: bool = True):
    """Colour with the learned order; with the fallback, also colour in
    natural order and keep whichever uses fewer colours.  Returns
    (colors, used_learned, learned_colours, natural_colours or None)."""
    keys, bad = order_learned(model, row_ptr, col_idx)
    if int(bad.item()):
        raise B.GColorError(-1, "order_learned: NaN score")
    col, st = B.color_graph_ex(row_ptr, col_idx, keys, stats=True)
    if not fallback:
        return col, True, st.num_colors, None
    nat, st2 = B.color_graph_ex(row_ptr, col_idx, None, stats=True)
    if st2.num_colors < st.num_colors:
        return nat, False, st.num_colors, st2.num_colors
    return col, True, st.num_colors, st2.num_colors
