"""Dense point sampling along one ray (oracle pin; test infrastructure).

Labels each sample point ``x(t_k)`` straight from the definitions -- the
owning cell is ``argmin_j pow(x, j)`` (appendix B, power cell), the point
counts for that cell only if it lies in the cell's sphere (Sec. 3.2), and is
dense only if ``(x - p_i).n < delta_i`` (Sec. 3.3) -- without any bisector
plane or interval formula.  Summing sample lengths per cell gives the lengths
the segment form must reproduce as the step goes to zero.
"""
from __future__ import annotations

import numpy as np
import torch

F64 = torch.float64


def dense_sample_ray(S, o, d, t_max: float, dt: float, delta=None, chunk: int = 200000):
    """Returns a list of (cell, inside_length, dense_length) in order of
    first appearance along the ray.

    ``delta`` maps cell index -> displacement of the dipole face for this
    ray (default 0 for every cell)."""
    P, W, R, Nrm = S["p"], S["power"], S["radius"], S["normal"]
    N = P.shape[0]
    nh = Nrm / torch.linalg.norm(Nrm, dim=-1, keepdim=True)
    dvec = torch.zeros(N, dtype=F64)
    if delta is not None:
        for c, v in delta.items():
            dvec[int(c)] = float(v)
    n_steps = int(np.ceil(t_max / dt))
    inside_len = torch.zeros(N, dtype=F64)
    dense_len = torch.zeros(N, dtype=F64)
    first_t = torch.full((N,), float("inf"), dtype=F64)
    for s0 in range(0, n_steps, chunk):
        t = (torch.arange(s0, min(n_steps, s0 + chunk), dtype=F64) + 0.5) * dt
        x = o.unsqueeze(0) + t.unsqueeze(1) * d.unsqueeze(0)
        diff = x.unsqueeze(1) - P.unsqueeze(0)
        pw = (diff * diff).sum(-1) - W.unsqueeze(0)
        lab = torch.argmin(pw, dim=1)
        rel = x - P[lab]
        inside = (rel * rel).sum(-1) <= R[lab] ** 2
        dense = inside & ((rel * nh[lab]).sum(-1) < dvec[lab])
        inside_len += torch.bincount(lab[inside], minlength=N).to(F64) * dt
        dense_len += torch.bincount(lab[dense], minlength=N).to(F64) * dt
        first_t = first_t.scatter_reduce(0, lab[inside], t[inside], reduce="amin")
    cells = torch.nonzero(inside_len > 0).flatten()
    cells = cells[torch.argsort(first_t[cells])]
    return [(int(c), float(inside_len[c]), float(dense_len[c])) for c in cells]
