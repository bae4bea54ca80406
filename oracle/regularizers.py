"""Training regularisers and per-cell statistics (oracle; test infrastructure).

Supplementary material, "Loss functions", and Sec. 3.5 (densification and
pruning), restated in float64:

* contribution of cell i over a set of rays: ``sum_rays T a`` (the per-cell
  sparsity term L_sparse(i) and the statistic the pruning EMA tracks), where
  ``a`` is the cell's opacity on the ray and ``T`` the transmittance in
  front of it;
* normal loss ``L_normal = sum_i sum_rays T a max(n_i . d, 0)^2`` with
  ``n_i`` the unit normal of cell i and ``d`` the unit ray direction;
* connectivity loss ``L_connect = sum_i sum_{j in Cech(i)} max(r_i + r_j -
  d_ij, 0)^2`` over the pairs of overlapping spheres (the Cech graph),
  ``d_ij = |p_i - p_j|``.

Gradients come from torch autograd on the same float64 replay as
:mod:`oracle.adjoint`.
"""
from __future__ import annotations

import numpy as np
import torch

from .adjoint import PARAMS, _ends
from .camera import generate_rays
from .cell import scene_tensors, shade
from .walk import walk_records

F64 = torch.float64


def _replay_terms(S, o, d, rec, nray):
    """Per-record opacity, colour and transmittance in front, plus RGBA."""
    lo, hi = _ends(S, o, d, rec)
    ci = rec.cell
    alpha, colour, _ = shade(o, d[rec.ray], lo, hi, S["p"][ci], S["normal"][ci], S["occ_logit"][ci],
                             S["rgb"][ci], S["tex"][ci], S["sigma_scale"], S["tau"])
    C = ci.numel()
    counts = torch.bincount(rec.ray, minlength=nray)
    start = torch.cumsum(counts, 0) - counts
    slot = torch.arange(C) - start[rec.ray]
    kmax = int(counts.max()) if C else 1
    A = torch.zeros(nray, kmax, dtype=F64).index_put((rec.ray, slot), alpha)
    Col = torch.zeros(nray, kmax, 3, dtype=F64).index_put((rec.ray, slot), colour)
    trans = torch.cumprod(1.0 - A, dim=1)
    t_before = torch.cat([torch.ones(nray, 1, dtype=F64), trans[:, :-1]], dim=1)
    rgb = ((t_before * A).unsqueeze(-1) * Col).sum(1)
    rgba = torch.cat([rgb, (1.0 - trans[:, -1]).unsqueeze(-1)], dim=-1)
    weight = t_before[rec.ray, slot] * alpha        # T a per record
    return rgba, weight


def regularized_gradients(scene, cam, G, lambda_normal: float = 0.0, lambda_sparse: float = 0.0, pix=None):
    """Gradients of ``sum(G * RGBA) + lambda_normal L_normal + lambda_sparse
    L_sparse`` over the pixels ``pix`` of ``cam`` (L_sparse summed over all
    cells).  Returns (grads dict of float64 arrays, values dict with
    'normal', 'sparse', 'total', per-cell 'contribution' [n])."""
    S0 = scene_tensors(scene)
    _, rec = walk_records(scene, cam, pix, S=S0)
    S = scene_tensors(scene, requires_grad=True)
    o, d, _ = generate_rays(cam, pix)
    rgba, weight = _replay_terms(S, o, d, rec, d.shape[0])
    nh = S["normal"][rec.cell]
    nh = nh / torch.linalg.norm(nh, dim=-1, keepdim=True)
    cosd = (nh * d[rec.ray]).sum(-1)
    l_normal = (weight * torch.clamp(cosd, min=0.0) ** 2).sum()
    l_sparse = weight.sum()
    Gt = torch.as_tensor(np.asarray(G, dtype=np.float64))
    L = (rgba * Gt).sum() + lambda_normal * l_normal + lambda_sparse * l_sparse
    L.backward()
    grads = {k: S[k].grad.numpy().copy() if S[k].grad is not None else np.zeros(tuple(S[k].shape))
             for k in PARAMS}
    contrib = torch.zeros(int(scene.n), dtype=F64).index_add(0, rec.cell, weight.detach())
    values = {"normal": float(l_normal.detach()), "sparse": float(l_sparse.detach()), "total": float(L.detach()),
              "contribution": contrib.numpy()}
    return grads, values


def normal_loss_value(scene, cam, pix=None) -> float:
    """L_normal alone (no autograd), for difference quotients."""
    S = scene_tensors(scene)
    _, rec = walk_records(scene, cam, pix, S=S)
    o, d, _ = generate_rays(cam, pix)
    _, weight = _replay_terms(S, o, d, rec, d.shape[0])
    nh = S["normal"][rec.cell]
    nh = nh / torch.linalg.norm(nh, dim=-1, keepdim=True)
    cosd = (nh * d[rec.ray]).sum(-1)
    return float((weight * torch.clamp(cosd, min=0.0) ** 2).sum())


def connect_loss(scene, lam: float = 1.0):
    """``lam * L_connect`` by brute force over all ordered pairs i != j, and
    its gradients with respect to p and radius (float64 numpy)."""
    p = torch.tensor(np.asarray(scene.p, dtype=np.float64), requires_grad=True)
    r = torch.tensor(np.asarray(scene.radius, dtype=np.float64), requires_grad=True)
    n = p.shape[0]
    diff = p.unsqueeze(1) - p.unsqueeze(0)
    off = ~torch.eye(n, dtype=torch.bool)
    dist = torch.sqrt((diff * diff).sum(-1).masked_fill(~off, 1.0))
    ov = torch.clamp(r.unsqueeze(1) + r.unsqueeze(0) - dist, min=0.0) * off
    L = lam * (ov * ov).sum()
    L.backward()
    return float(L.detach()), {"p": p.grad.numpy().copy(), "radius": r.grad.numpy().copy()}
