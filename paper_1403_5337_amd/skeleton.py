"""Training and use of the learned skeleton proposer (HODLR_LEARNED).

Everything numerical runs in the library (hodlr_skel_features,
hodlr_skel_labels, hodlr_mlp_adam_step, hodlr_build); this module only
orders fronts, draws minibatches and keeps the parameters.

Training data: per front, the RCB-ordered front and its separator graph go
through hodlr_skel_features (8 features per block side vertex) and
hodlr_skel_labels (1 on the rows/columns the full-pivot LU of a wide BDLR
skeleton keeps, by default; or on ACA's pivots), so the scorer learns which
vertices a skeleton needs.
"""
from __future__ import annotations

import json
import os
from typing import Iterable, List, Tuple

import numpy as np
import torch

from . import hodlr as H

WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "skel_mlp.npy")
META = os.path.join(os.path.dirname(os.path.abspath(__file__)), "skel_mlp.json")


def order_front(front, leaf: int, device="cuda"):
    """(K, rowptr, col, coords) of the front in RCB order, on the device."""
    dev = torch.device(device)
    xyz = torch.from_numpy(np.ascontiguousarray(front.coords, dtype=np.float32)).to(dev)
    perm = H.hodlr_order_rcb(xyz, leaf)
    K = H.hodlr_permute(front.K.to(dev), perm)
    rp, ci = H.hodlr_permute_graph(torch.from_numpy(front.indptr).to(dev), torch.from_numpy(front.indices).to(dev),
                                   perm)
    coords = H.hodlr_permute_rows(xyz, perm)
    return K, rp, ci, coords


def front_samples(front, leaf: int, tol: float, source="lu", depth=4) -> Tuple[torch.Tensor, torch.Tensor]:
    """(features (2 n L, 8), labels (2 n L,)) of one front, on the device."""
    K, rp, ci, xyz = order_front(front, leaf)
    feats = H.hodlr_skel_features(rp, ci, xyz, K, leaf)
    labels = H.hodlr_skel_labels(K, leaf, tol, 32, graph=(rp, ci), source=source, depth=depth)
    return feats, labels


def init_params(seed: int, device="cuda") -> torch.Tensor:
    """He-scaled uniform weights, zero biases, in the library's layout."""
    g = torch.Generator(device="cpu").manual_seed(seed)
    parts = []
    for fan_in, fan_out in ((8, 64), (64, 64)):
        bound = (6.0 / fan_in) ** 0.5
        parts.append((torch.rand(fan_out * fan_in, generator=g) * 2 - 1) * bound)
        parts.append(torch.zeros(fan_out))
    parts.append((torch.rand(64, generator=g) * 2 - 1) * (3.0 / 64) ** 0.5)
    parts.append(torch.zeros(1))
    p = torch.cat(parts).to(torch.float32)
    assert p.numel() == H.MLP_PARAMS
    return p.to(device)


def train(feats: torch.Tensor, labels: torch.Tensor, steps: int, batch: int = 8192, lr: float = 3e-3,
          pos_weight: float | None = None, seed: int = 0, params: torch.Tensor | None = None,
          log_every: int = 0) -> Tuple[torch.Tensor, List[float]]:
    """Adam on minibatches drawn uniformly (seeded) from the samples."""
    dev = feats.device
    N = feats.shape[0]
    if pos_weight is None:
        pos = float(labels.sum().item())
        pos_weight = (N - pos) / max(pos, 1.0)
    p = init_params(seed, dev) if params is None else params.clone().to(torch.float32).contiguous()
    m = torch.zeros_like(p)
    v = torch.zeros_like(p)
    g = torch.Generator(device="cpu").manual_seed(seed + 1)
    losses = []
    for step in range(1, steps + 1):
        idx = torch.randint(0, N, (min(batch, N),), generator=g).to(dev)
        xb = feats.index_select(0, idx).contiguous()
        yb = labels.index_select(0, idx).contiguous()
        losses.append(H.hodlr_mlp_adam_step(xb, yb, p, m, v, step, lr, pos_weight))
        if log_every and step % log_every == 0:
            print(f"# step {step} loss {losses[-1]:.4f}", flush=True)
    return p, losses


def save(params: torch.Tensor, meta: dict, path: str = WEIGHTS, meta_path: str = META):
    np.save(path, params.detach().cpu().numpy().astype(np.float32), allow_pickle=False)
    with open(meta_path, "w") as f:
        json.dump(meta, f, indent=1, sort_keys=True)


def load(device="cuda", path: str = WEIGHTS) -> torch.Tensor:
    a = np.load(path, allow_pickle=False)
    if a.shape != (H.MLP_PARAMS,) or a.dtype != np.float32:
        raise ValueError(f"{path}: expected {H.MLP_PARAMS} float32 parameters")
    return torch.from_numpy(a).to(device)


def concat_samples(pairs: Iterable[Tuple[torch.Tensor, torch.Tensor]]):
    fs, ls = zip(*pairs)
    return torch.cat(fs).contiguous(), torch.cat(ls).contiguous()
