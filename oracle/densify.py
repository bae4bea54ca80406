"""Densification and pruning (oracle; test infrastructure).

Sec. 3.5, "Densification and Pruning", restated in float64:

* per-cell photometric error of a training view: the pixels' errors
  distributed over the cells by their contribution,
  ``err_i = sum_rays T a e_ray`` (``T`` the transmittance in front of the
  cell, ``a`` its opacity on the ray, ``e_ray`` the pixel's error, given);
* exponential moving averages ``ema <- beta ema + (1 - beta) value`` of that
  error and of the per-cell contribution ``sum_rays T a``;
* pruning: cells whose contribution average is below a threshold are
  removed;
* densification: ``n_new`` cells are drawn from the multinomial distribution
  proportional to the error average of the remaining cells (inverse CDF of
  the caller's uniform draws ``u``); each draw adds a copy of the drawn cell
  moved by ``spread * r * delta`` (``delta`` a standard normal triple, given).

Readings (the paper gives no more detail): the pixel error is the caller's
(e.g. the L1 norm of the RGB residual); pruning comes before drawing; the
kept cells stay in their order, the new cells follow in draw order and carry
their parent's averages; a draw maps to the first cell whose cumulative
weight exceeds ``u * total`` (zero-weight cells are never drawn); with no
kept cell or a zero total no cell is added.
"""
from __future__ import annotations

import numpy as np
import torch

from .camera import generate_rays
from .cell import scene_tensors
from .regularizers import _replay_terms
from .walk import walk_records

F64 = np.float64
FIELDS = ("p", "power", "radius", "normal", "occ_logit", "rgb", "tex")


def cell_error(scene, cam, pixel_error, pix=None) -> np.ndarray:
    """``sum_rays T a e_ray`` per cell [n] for the pixels ``pix`` of
    ``cam`` (``pixel_error`` [rays], one value per pixel in ``pix`` order)."""
    S = scene_tensors(scene)
    _, rec = walk_records(scene, cam, pix, S=S)
    o, d, _ = generate_rays(cam, pix)
    _, weight = _replay_terms(S, o, d, rec, d.shape[0])
    e = torch.as_tensor(np.asarray(pixel_error, dtype=F64))
    return torch.zeros(int(scene.n), dtype=torch.float64).index_add(0, rec.cell, weight * e[rec.ray]).numpy()


def ema(prev, value, beta: float) -> np.ndarray:
    """float32 ``beta prev + (1 - beta) value``, formed in float64."""
    b = float(np.float32(beta))
    prev = np.asarray(prev, np.float32).astype(F64)
    value = np.asarray(value, np.float32).astype(F64)
    return (b * prev + (1.0 - b) * value).astype(np.float32)


def draw(weights, u) -> np.ndarray:
    """Indices into ``weights`` for uniform draws ``u`` in [0, 1): the first
    index whose cumulative weight exceeds ``u * total``."""
    cdf = np.cumsum(np.asarray(weights, dtype=F64))
    x = np.asarray(u, dtype=np.float32).astype(F64) * cdf[-1]
    return np.minimum(np.searchsorted(cdf, x, side="right"), cdf.size - 1)


def densify_prune(scene, err_ema, contrib_ema, u, delta, prune_below: float, spread: float):
    """One densify-and-prune update.  Returns (new scene as a dict of float32
    arrays, new error average, new contribution average, parent index per
    new cell in the input numbering)."""
    err_ema = np.asarray(err_ema, np.float32)
    contrib_ema = np.asarray(contrib_ema, np.float32)
    keep = contrib_ema >= np.float32(prune_below)
    kept = np.nonzero(keep)[0]
    u = np.asarray(u, np.float32)
    if kept.size == 0 or u.size == 0 or not err_ema[kept].astype(F64).sum() > 0.0:
        parents = np.zeros(0, dtype=np.int64)
    else:
        parents = kept[draw(err_ema[kept], u)]
    out = {f: np.asarray(getattr(scene, f), np.float32)[np.concatenate([kept, parents])].copy() for f in FIELDS}
    if parents.size:
        d = np.asarray(delta, np.float32)[: parents.size].astype(F64)
        p0 = np.asarray(scene.p, np.float32)[parents].astype(F64)
        r0 = np.asarray(scene.radius, np.float32)[parents].astype(F64)
        s = float(np.float32(spread))
        out["p"][kept.size:] = (p0 + (s * r0)[:, None] * d).astype(np.float32)
    idx = np.concatenate([kept, parents])
    return out, err_ema[idx].copy(), contrib_ema[idx].copy(), parents
