"""Adjoint of the renderer by autograd replay, float64 (oracle; test infrastructure).

The walk fixes the discrete decisions of each ray: the cells it crosses in
order, and which constraint binds each end of each bounded interval (camera
start, the sphere of the cell, or the bisector plane against a named
neighbour).  Those ends are then re-evaluated from the parameters with the
same formulas (:mod:`oracle.cell`), the pieces are shaded and composited, and
torch autograd in float64 gives the gradient of ``L = sum <G, RGBA>`` with
respect to every cell parameter: site, power, radius, normal, density logit,
base colour and texture.  Gradients reach a neighbour ``j`` through the
bisector planes that bind an interval.

Where a decision changes under a perturbation the loss has a kink; the
gradient returned is that of the branch the forward took.
"""
from __future__ import annotations

import numpy as np
import torch

from .camera import generate_rays
from .cell import bisector, plane_hit, scene_tensors, shade, sphere_interval
from .walk import BIND_CAMERA, BIND_PLANE, BIND_SPHERE, Records, walk_records

F64 = torch.float64
PARAMS = ("p", "power", "radius", "normal", "occ_logit", "rgb", "tex")


def _ends(S, o, d, rec: Records):
    P, W, R = S["p"], S["power"], S["radius"]
    ci = rec.cell
    C = ci.numel()
    lo = torch.zeros(C, dtype=F64)
    hi = torch.zeros(C, dtype=F64)
    dr = d[rec.ray]

    def sphere(idx, which):
        t0, t1, _ = sphere_interval(o, dr[idx], P[ci[idx]], R[ci[idx]])
        return t0 if which == 0 else t1

    def plane(idx, jsel):
        j = jsel[idx]
        m, h = bisector(P[ci[idx]], W[ci[idx]], P[j], W[j])
        a, b = plane_hit(o, dr[idx], P[ci[idx]], m, h)
        return b / a

    for kind_t, j_t, out, which in ((rec.lo_kind, rec.lo_j, "lo", 0), (rec.hi_kind, rec.hi_j, "hi", 1)):
        vals = lo if out == "lo" else hi
        idx_s = torch.nonzero(kind_t == BIND_SPHERE).flatten()
        idx_p = torch.nonzero(kind_t == BIND_PLANE).flatten()
        if idx_s.numel():
            vals = vals.index_put((idx_s,), sphere(idx_s, which))
        if idx_p.numel():
            vals = vals.index_put((idx_p,), plane(idx_p, j_t))
        if out == "lo":
            lo = vals
        else:
            hi = vals
    return lo, hi


def replay_rgba(S, o, d, rec: Records, nray: int):
    """Differentiable RGBA [nray,4] from the recorded decisions."""
    lo, hi = _ends(S, o, d, rec)
    ci = rec.cell
    alpha, colour, _ = shade(o, d[rec.ray], lo, hi, S["p"][ci], S["normal"][ci], S["occ_logit"][ci],
                             S["rgb"][ci], S["tex"][ci], S["sigma_scale"], S["tau"])
    C = ci.numel()
    if C == 0:
        return torch.zeros(nray, 4, dtype=F64)
    counts = torch.bincount(rec.ray, minlength=nray)
    start = torch.cumsum(counts, 0) - counts
    slot = torch.arange(C) - start[rec.ray]
    kmax = int(counts.max())
    A = torch.zeros(nray, kmax, dtype=F64).index_put((rec.ray, slot), alpha)
    Col = torch.zeros(nray, kmax, 3, dtype=F64).index_put((rec.ray, slot), colour)
    trans = torch.cumprod(1.0 - A, dim=1)
    t_before = torch.cat([torch.ones(nray, 1, dtype=F64), trans[:, :-1]], dim=1)
    rgb = ((t_before * A).unsqueeze(-1) * Col).sum(1)
    return torch.cat([rgb, (1.0 - trans[:, -1]).unsqueeze(-1)], dim=-1)


def loss_from_rgba(rgba, G) -> float:
    return float((np.asarray(rgba, dtype=np.float64) * np.asarray(G, dtype=np.float64)).sum())


def adjoint_gradients(scene, cam, G, pix=None, return_records: bool = False):
    """Gradients of ``L = sum(G * RGBA)`` over pixels ``pix`` of ``cam``.

    ``G`` is [R,4] (R = number of pixels).  Returns a dict of float64 numpy
    arrays shaped like the scene fields, plus the loss value."""
    S0 = scene_tensors(scene)
    rgba0, rec = walk_records(scene, cam, pix, S=S0)
    S = scene_tensors(scene, requires_grad=True)
    o, d, _ = generate_rays(cam, pix)
    rgba = replay_rgba(S, o, d, rec, d.shape[0])
    Gt = torch.as_tensor(np.asarray(G, dtype=np.float64))
    L = (rgba * Gt).sum()
    L.backward()
    grads = {k: S[k].grad.numpy().copy() if S[k].grad is not None else np.zeros(tuple(S[k].shape))
             for k in PARAMS}
    out = (grads, float(L.detach()))
    if return_records:
        out = out + (rec, rgba.detach().numpy(), rgba0)
    return out
