"""Brute-force walk form of the renderer, float64 (oracle; test infrastructure).

For each ray ``x(t) = o + t d``, ``t >= 0``:

1. the start cell is ``argmin_j pow(o, j)`` over all sites (ties: lowest
   index);
2. in the current cell ``i`` the exit is the nearest crossing, at or after the
   current ``t``, of any bisector plane of ``i`` against every other site
   ``j`` that the ray leaves through (``d . m > 0``), found by brute force over
   all ``j`` (ties: lowest index); the next cell is that ``j``.  No exit means
   the ray stays in ``i`` forever;
3. the rendered piece of cell ``i`` is ``[t, t_exit]`` clipped by the sphere
   ``B(p_i, r_i)`` (Sec. 3.2: the power cell intersected with its sphere;
   ray tracing walks cell to cell and uses the sphere bounds in the lengths);
4. its opacity and radiance come from :func:`oracle.cell.shade`, composited
   front to back, ``C += T a c``, ``T *= 1 - a``, with no early termination
   (Sec. 3.1, exact segment sum).  Output RGBA with ``A = 1 - T``; the
   background is black.

The walk also records, per contribution, which constraint binds each end of
the bounded interval, so that the adjoint can replay it.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional

import numpy as np
import torch

from .camera import generate_rays
from .cell import scene_tensors, shade

F64 = torch.float64
INF = float("inf")

# binding kinds for the ends of a bounded interval
BIND_CAMERA = 0   # t = 0 (ray start)
BIND_PLANE = 1    # bisector plane against neighbour j
BIND_SPHERE = 2   # the cell's own sphere


@dataclasses.dataclass
class Records:
    """Contributions of a batch of rays, in walk order per ray."""
    ray: torch.Tensor       # [C] int64, index into the batch
    cell: torch.Tensor      # [C] int64
    lo: torch.Tensor        # [C] float64
    hi: torch.Tensor        # [C] float64
    lo_kind: torch.Tensor   # [C] int64
    lo_j: torch.Tensor      # [C] int64 (neighbour for BIND_PLANE, else -1)
    hi_kind: torch.Tensor   # [C] int64
    hi_j: torch.Tensor      # [C] int64
    steps: torch.Tensor     # [B] int64, cells walked per ray

    def cell_sequence(self, ray: int) -> List[int]:
        return self.cell[self.ray == ray].tolist()


def _first_argmin(vals: torch.Tensor) -> torch.Tensor:
    """Row-wise argmin with ties broken towards the lowest index."""
    vmin = vals.min(dim=1, keepdim=True).values
    idx = torch.arange(vals.shape[1]).expand_as(vals)
    big = torch.full_like(idx, vals.shape[1])
    return torch.where(vals == vmin, idx, big).min(dim=1).values


def start_cells(S, o: torch.Tensor) -> torch.Tensor:
    """argmin_j pow(o, j) for a single point o [3] (ties: lowest index)."""
    diff = o.unsqueeze(0) - S["p"]
    key = (diff * diff).sum(-1) - S["power"]
    return _first_argmin(key.unsqueeze(0))[0]


def _walk_batch(S, o, d, max_steps: int, chunk_elems: int):
    """Walk a batch of rays sharing origin ``o``; returns RGBA [B,4] and
    the contribution records."""
    P, W, R = S["p"], S["power"], S["radius"]
    N = P.shape[0]
    B = d.shape[0]
    i0 = start_cells(S, o)
    cell = torch.full((B,), int(i0), dtype=torch.int64)
    prev = torch.full((B,), -1, dtype=torch.int64)
    t_cur = torch.zeros(B, dtype=F64)
    active = torch.ones(B, dtype=torch.bool)
    T = torch.ones(B, dtype=F64)
    C = torch.zeros(B, 3, dtype=F64)
    steps = torch.zeros(B, dtype=torch.int64)
    recs = {k: [] for k in ("ray", "cell", "lo", "hi", "lo_kind", "lo_j", "hi_kind", "hi_j")}
    jidx = torch.arange(N)

    for _ in range(max_steps):
        act = torch.nonzero(active).flatten()
        if act.numel() == 0:
            break
        # exits by brute force over all bisector planes, in row chunks
        t_exit = torch.empty(act.numel(), dtype=F64)
        nxt = torch.empty(act.numel(), dtype=torch.int64)
        rows = max(1, chunk_elems // N)
        for s0 in range(0, act.numel(), rows):
            sl = act[s0:s0 + rows]
            ci = cell[sl]
            Pi, Wi = P[ci], W[ci]
            m = P.unsqueeze(0) - Pi.unsqueeze(1)                       # [b,N,3]
            h = 0.5 * ((m * m).sum(-1) + Wi.unsqueeze(1) - W.unsqueeze(0))
            a = (m * d[sl].unsqueeze(1)).sum(-1)
            b = h - (m * (o - Pi).unsqueeze(1)).sum(-1)
            cand = (a > 0) & (jidx.unsqueeze(0) != ci.unsqueeze(1))
            tj = torch.where(cand, b / torch.where(cand, a, torch.ones_like(a)),
                             torch.full_like(a, INF))
            tj = torch.where(tj >= t_cur[sl].unsqueeze(1), tj, torch.full_like(tj, INF))
            te = tj.min(dim=1).values
            t_exit[s0:s0 + rows] = te
            nxt[s0:s0 + rows] = torch.where(torch.isfinite(te), _first_argmin(tj),
                                            torch.full_like(te, -1, dtype=torch.int64))

        ci = cell[act]
        oc = o - P[ci]
        beta = (oc * d[act]).sum(-1)
        D = beta * beta - ((oc * oc).sum(-1) - R[ci] * R[ci])
        sq = torch.sqrt(torch.clamp(D, min=0.0))
        s_in, s_out = -beta - sq, -beta + sq
        tc = t_cur[act]
        lo = torch.maximum(tc, s_in)
        hi = torch.minimum(t_exit, s_out)
        ok = (D > 0) & (lo < hi)

        if ok.any():
            k = torch.nonzero(ok).flatten()
            rays = act[k]
            cells = ci[k]
            alpha, colour, _ = shade(o, d[rays], lo[k], hi[k], P[cells], S["normal"][cells],
                                     S["occ_logit"][cells], S["rgb"][cells], S["tex"][cells],
                                     S["sigma_scale"], S["tau"])
            C[rays] += (T[rays] * alpha).unsqueeze(-1) * colour
            T[rays] = T[rays] * (1.0 - alpha)
            lo_sphere = s_in[k] > tc[k]
            first = prev[rays] < 0
            recs["ray"].append(rays)
            recs["cell"].append(cells)
            recs["lo"].append(lo[k])
            recs["hi"].append(hi[k])
            recs["lo_kind"].append(torch.where(lo_sphere, torch.full_like(rays, BIND_SPHERE),
                                               torch.where(first, torch.full_like(rays, BIND_CAMERA),
                                                           torch.full_like(rays, BIND_PLANE))))
            recs["lo_j"].append(torch.where(lo_sphere | first, torch.full_like(rays, -1), prev[rays]))
            hi_sphere = s_out[k] < t_exit[k]
            recs["hi_kind"].append(torch.where(hi_sphere, torch.full_like(rays, BIND_SPHERE),
                                               torch.full_like(rays, BIND_PLANE)))
            recs["hi_j"].append(torch.where(hi_sphere, torch.full_like(rays, -1), nxt[k]))

        steps[act] += 1
        prev[act] = ci
        t_cur[act] = torch.maximum(tc, t_exit)
        cell[act] = torch.where(nxt >= 0, nxt, ci)
        active[act] = torch.isfinite(t_exit)
    else:
        if active.any():
            raise RuntimeError("oracle walk exceeded max_steps")

    cat = {k: (torch.cat(v) if v else torch.zeros(0, dtype=torch.int64 if k not in ("lo", "hi") else F64))
           for k, v in recs.items()}
    rgba = torch.cat([C, (1.0 - T).unsqueeze(-1)], dim=-1)
    return rgba, Records(steps=steps, **cat)


def _order_records(rec: Records) -> Records:
    """Stable sort of records by ray (walk order is kept within a ray)."""
    order = torch.sort(rec.ray, stable=True).indices
    return Records(ray=rec.ray[order], cell=rec.cell[order], lo=rec.lo[order], hi=rec.hi[order],
                   lo_kind=rec.lo_kind[order], lo_j=rec.lo_j[order], hi_kind=rec.hi_kind[order],
                   hi_j=rec.hi_j[order], steps=rec.steps)


def walk_records(scene, cam, pix=None, max_steps: int = 100000, chunk_elems: int = 1 << 21,
                 S=None):
    """RGBA [R,4] (numpy float64) and the ordered contribution records for
    the pixels ``pix`` (row-major indices; default all) of ``cam``."""
    if S is None:
        S = scene_tensors(scene)
    o, d, valid = generate_rays(cam, pix)
    rgba = torch.zeros(d.shape[0], 4, dtype=F64)
    vidx = torch.nonzero(valid).flatten()
    with torch.no_grad():
        sub_rgba, rec = _walk_batch(S, o, d[vidx], max_steps, chunk_elems)
    rgba[vidx] = sub_rgba
    rec.ray = vidx[rec.ray] if rec.ray.numel() else rec.ray
    steps = torch.zeros(d.shape[0], dtype=torch.int64)
    steps[vidx] = rec.steps
    rec.steps = steps
    return rgba.numpy(), _order_records(rec)


def render_walk(scene, cam, pix=None, max_steps: int = 100000, chunk_elems: int = 1 << 21,
                S=None) -> np.ndarray:
    """RGBA [R,4] float64 for pixels ``pix`` (default the whole image,
    row-major) by the brute-force walk."""
    return walk_records(scene, cam, pix, max_steps, chunk_elems, S)[0]
