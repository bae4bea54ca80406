"""Steiner cells for the ray walk (oracle; test infrastructure).

Supplementary material, section "Steiner points for ray tracing", Alg. 1,
restated in float64.  The walk crosses the unbounded power cells, and in
empty space those are left unregularised and can be long and thin; Steiner
cells fill the empty space so that a ray crosses fewer cells.  Per round
(six in the paper):

1. draw candidate points from a normal distribution with the per-axis mean
   and standard deviation of the current sites (scene cells and the Steiner
   cells of earlier rounds);
2. a candidate ``x`` is valid when it lies outside every sphere,
   ``|x - p_i|^2 - r_i^2 > 0`` for all i;
3. its nearest cell is the one of least power ``|x - p_i|^2 - r_i^2``;
   the candidate's radius is its distance to that cell's sphere,
   ``r_hat = |x - p_near| - r_near``;
4. it is kept when ``2 r_near <= r_hat <= 6 r_near``.

Readings (the paper is silent on them):

* the random draws are inputs: ``z[round, j]`` is a standard normal triple
  and the candidate is ``mean + std * z`` per axis (population standard
  deviation), rounded to float32 because it becomes a float32 site; every
  test is made on that float32 point in float64 arithmetic;
* within a round every candidate is tested against the cells present when
  the round starts, and the kept candidates join together at the end of the
  round (the printed loop adds each one as it is kept; testing candidates of
  one random sample against each other would make the result depend on the
  sample's order, and the round-at-a-time reading keeps the rounds
  data-parallel);
* the power used by the test and the nearest-cell search is the sphere's,
  ``r^2``, as printed, also for scenes whose power weights differ from
  ``r^2``;
* the new cell's radius is ``float32(r_hat)``; its power weight is
  ``r_hat^2 - r_near^2 + w_near``, which places its bisector with the
  nearest cell on that cell's sphere (for ``w = r^2`` this is the paper's
  ``w_hat = r_hat^2``).  The new cells are empty (zero density).

Ties in the nearest-cell search go to the lower index in the order: scene
cells first, then Steiner cells in the order they were kept.
"""
from __future__ import annotations

import numpy as np

F64 = np.float64


def evaluate_candidates(P, R, W, x, lo: float = 2.0, hi: float = 6.0, chunk: int = 256):
    """One pass of the test over candidate points ``x`` [S,3] (float64
    values of float32 points) against cells ``P`` [M,3], radii ``R`` [M]
    and weights ``W`` [M] (float64).  Returns (keep [S] bool, r_hat [S],
    w_hat [S], near [S] int64); r_hat/w_hat/near are meaningful where the
    candidate is valid (outside every sphere), -1 / nan elsewhere."""
    S = x.shape[0]
    keep = np.zeros(S, dtype=bool)
    r_hat = np.full(S, np.nan)
    w_hat = np.full(S, np.nan)
    near = np.full(S, -1, dtype=np.int64)
    R2 = R * R
    for a in range(0, S, chunk):
        xs = x[a:a + chunk]
        diff = xs[:, None, :] - P[None, :, :]
        pw = (diff * diff).sum(-1) - R2[None, :]          # power of x w.r.t. each sphere
        j = np.argmin(pw, axis=1)                          # first index among ties
        best = pw[np.arange(xs.shape[0]), j]
        valid = best > 0.0                                 # outside every sphere
        d = np.sqrt(((xs - P[j]) ** 2).sum(-1))
        rh = d - R[j]
        ok = valid & (lo * R[j] <= rh) & (rh <= hi * R[j])
        sl = slice(a, a + xs.shape[0])
        keep[sl] = ok
        near[sl] = np.where(valid, j, -1)
        r_hat[sl] = np.where(valid, rh, np.nan)
        w_hat[sl] = np.where(valid, rh * rh - R2[j] + W[j], np.nan)
    return keep, r_hat, w_hat, near


def steiner_points(p, radius, power, z, lo: float = 2.0, hi: float = 6.0):
    """All rounds of the insertion.  ``p`` [N,3], ``radius`` [N], ``power``
    [N] (float32 scene values), ``z`` [rounds, S, 3] standard normal draws.

    Returns a dict of the kept cells in the order they were kept:
    ``p`` [A,3] float32, ``radius`` [A] float32, ``power`` [A] float32,
    ``near`` [A] int64 (index of the nearest cell in the combined order),
    ``round`` [A] int64, and ``candidate`` [A] int64 (index in its round)."""
    P = np.asarray(p, dtype=np.float32).astype(F64)
    R = np.asarray(radius, dtype=np.float32).astype(F64)
    W = np.asarray(power, dtype=np.float32).astype(F64)
    z = np.asarray(z, dtype=np.float32).astype(F64)
    out = {k: [] for k in ("p", "radius", "power", "near", "round", "candidate")}
    for it in range(z.shape[0]):
        mean = P.mean(axis=0)
        std = P.std(axis=0)
        x = (mean[None, :] + std[None, :] * z[it]).astype(np.float32).astype(F64)
        keep, r_hat, w_hat, near = evaluate_candidates(P, R, W, x, lo, hi)
        idx = np.nonzero(keep)[0]
        np_ = x[idx]
        nr = r_hat[idx].astype(np.float32).astype(F64)
        nw = w_hat[idx].astype(np.float32).astype(F64)
        out["p"].append(np_.astype(np.float32))
        out["radius"].append(nr.astype(np.float32))
        out["power"].append(nw.astype(np.float32))
        out["near"].append(near[idx])
        out["round"].append(np.full(idx.size, it, dtype=np.int64))
        out["candidate"].append(idx.astype(np.int64))
        P = np.concatenate([P, np_])
        R = np.concatenate([R, nr])
        W = np.concatenate([W, nw])
    res = {k: np.concatenate(v) if v else np.zeros(0) for k, v in out.items()}
    res["p"] = res["p"].reshape(-1, 3).astype(np.float32)
    return res
