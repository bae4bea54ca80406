"""Painter form of the renderer, float64 (oracle; test infrastructure).

For each ray, every cell whose sphere the ray meets gets its bounded interval
by brute force over all bisector planes:

    lo = max(t_sphere_in, 0, max_{j: a<0} b/a),  hi = min(t_sphere_out, min_{j: a>0} b/a)

(``a = d.m``, ``b = h - (o - p_i).m``; a plane with ``a = 0`` empties the
interval when ``b < 0``).  Non-empty pieces are composited in increasing
power distance from the camera centre, ``pow(o, p_i)`` (ties: lowest index),
which is a valid painter's order for every ray through ``o`` (appendix B,
theorem on power diagrams).  This is an independent route to the walk's
result and is compared with it in the tests.
"""
from __future__ import annotations

import numpy as np
import torch

from .camera import generate_rays
from .cell import scene_tensors, shade

F64 = torch.float64
INF = float("inf")


def render_painter(scene, cam, pix=None, chunk_elems: int = 1 << 21, S=None) -> np.ndarray:
    if S is None:
        S = scene_tensors(scene)
    P, W, R = S["p"], S["power"], S["radius"]
    N = P.shape[0]
    o, d, valid = generate_rays(cam, pix)
    nray = d.shape[0]
    rgba = np.zeros((nray, 4))
    key = ((o.unsqueeze(0) - P) ** 2).sum(-1) - W
    # order of all cells by (key, index)
    order = np.lexsort((np.arange(N), key.numpy()))
    rank = np.empty(N, dtype=np.int64)
    rank[order] = np.arange(N)
    jidx = torch.arange(N)
    with torch.no_grad():
        for r in range(nray):
            if not bool(valid[r]):
                continue
            dr = d[r]
            oc = o - P
            beta = (oc * dr).sum(-1)
            D = beta * beta - ((oc * oc).sum(-1) - R * R)
            hit = torch.nonzero(D > 0).flatten()
            if hit.numel() == 0:
                continue
            sq = torch.sqrt(D[hit])
            lo = torch.clamp(-beta[hit] - sq, min=0.0)
            hi = -beta[hit] + sq
            rows = max(1, chunk_elems // N)
            for s0 in range(0, hit.numel(), rows):
                ci = hit[s0:s0 + rows]
                m = P.unsqueeze(0) - P[ci].unsqueeze(1)
                h = 0.5 * ((m * m).sum(-1) + W[ci].unsqueeze(1) - W.unsqueeze(0))
                a = (m * dr).sum(-1)
                b = h - (m * (o - P[ci]).unsqueeze(1)).sum(-1)
                notself = jidx.unsqueeze(0) != ci.unsqueeze(1)
                safe_a = torch.where(a != 0, a, torch.ones_like(a))
                t = b / safe_a
                up = torch.where(notself & (a > 0), t, torch.full_like(t, INF)).min(dim=1).values
                dn = torch.where(notself & (a < 0), t, torch.full_like(t, -INF)).max(dim=1).values
                blocked = (notself & (a == 0) & (b < 0)).any(dim=1)
                lo[s0:s0 + rows] = torch.maximum(lo[s0:s0 + rows], dn)
                hi[s0:s0 + rows] = torch.where(blocked, torch.full_like(up, -INF),
                                               torch.minimum(hi[s0:s0 + rows], up))
            ok = lo < hi
            if not ok.any():
                continue
            cells = hit[ok]
            lo_k, hi_k = lo[ok], hi[ok]
            srt = torch.as_tensor(np.argsort(rank[cells.numpy()], kind="stable"))
            cells, lo_k, hi_k = cells[srt], lo_k[srt], hi_k[srt]
            n = cells.numel()
            alpha, colour, _ = shade(o, dr.expand(n, 3), lo_k, hi_k, P[cells], S["normal"][cells],
                                     S["occ_logit"][cells], S["rgb"][cells], S["tex"][cells],
                                     S["sigma_scale"], S["tau"])
            T = 1.0
            C = torch.zeros(3, dtype=F64)
            for k in range(n):
                C = C + T * alpha[k] * colour[k]
                T = T * (1.0 - float(alpha[k]))
            rgba[r, :3] = C.numpy()
            rgba[r, 3] = 1.0 - T
    return rgba
