"""Steiner cells for the ray walk (oracle; test infrastructure).

Supplementary material, section "Steiner points for ray tracing", Alg. 1,
restated in float64.  The walk crosses the unbounded power cells, and in
empty space those are left unregularised and can be long and thin; Steiner
cells fill the empty space so that a ray crosses fewer cells.  The
algorithm, in its own order:

    for each of the rounds (six in the paper):
        draw a sample S of points from a normal distribution with the
        per-axis mean and standard deviation of the cells' sites
        for each point x of S, in order:
            if |x - p_i|^2 - r_i^2 > 0 for every cell i of the set:
                near  = the cell of least |x - p_i|^2 - r_i^2
                r_hat = |x - p_near| - r_near
                if 2 r_near <= r_hat <= 6 r_near:
                    add the cell (x, r_hat) to the set

The set grows inside the loop over S: a point is tested against the scene's
cells, the cells kept in earlier rounds and the cells kept earlier in the
same round (``steiner_round``).

Readings (the paper is silent on them):

* the random draws are inputs: ``z[round, j]`` is a standard normal triple
  and the point is ``mean + std * z`` per axis (population standard
  deviation of the sites in the set when the round starts), rounded to
  float32 because it becomes a float32 site; every test is made on that
  float32 point in float64 arithmetic;
* the power used by the test and the nearest-cell search is the sphere's,
  ``r^2``, as printed, also for scenes whose power weights differ from
  ``r^2``;
* the new cell's radius is ``float32(r_hat)``; its power weight is
  ``r_hat^2 - r_near^2 + w_near``, rounded to float32, which places its
  bisector with the nearest cell on that cell's sphere (for ``w = r^2`` this
  is the paper's ``w_hat = r_hat^2``).  Later points are tested against the
  float32 radius.  The new cells are empty (zero density);
* ties in the nearest-cell search go to the lower index in the order: scene
  cells first, then Steiner cells in the order they were kept.
"""
from __future__ import annotations

import numpy as np

F64 = np.float64


def _sq_dist(x, P):
    """|x - P_i|^2 for one point x [3] and cells P [M,3], summed x, y, z in
    that order."""
    d = x[None, :] - P
    return (d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2]


def evaluate_candidates(P, R, W, x, lo: float = 2.0, hi: float = 6.0, chunk: int = 256):
    """The test of Alg. 1 for points ``x`` [S,3] (float64 values) against a
    FIXED set of cells ``P`` [M,3], radii ``R`` [M], weights ``W`` [M]: each
    point is judged on its own, nothing is added to the set.  Returns (keep
    [S] bool, r_hat [S], w_hat [S], near [S] int64); r_hat / w_hat / near are
    meaningful where the point is outside every sphere, nan / -1 elsewhere.
    (A building block of the tests; the insertion itself is
    ``steiner_round``.)"""
    S = x.shape[0]
    keep = np.zeros(S, dtype=bool)
    r_hat = np.full(S, np.nan)
    w_hat = np.full(S, np.nan)
    near = np.full(S, -1, dtype=np.int64)
    R2 = R * R
    for a in range(0, S, chunk):
        xs = x[a:a + chunk]
        d = xs[:, None, :] - P[None, :, :]
        pw = ((d[..., 0] * d[..., 0] + d[..., 1] * d[..., 1]) + d[..., 2] * d[..., 2]) - R2[None, :]
        j = np.argmin(pw, axis=1)                          # first index among ties
        best = pw[np.arange(xs.shape[0]), j]
        valid = best > 0.0                                 # outside every sphere
        e = xs - P[j]
        dist = np.sqrt((e[:, 0] * e[:, 0] + e[:, 1] * e[:, 1]) + e[:, 2] * e[:, 2])
        rh = dist - R[j]
        ok = valid & (lo * R[j] <= rh) & (rh <= hi * R[j])
        sl = slice(a, a + xs.shape[0])
        keep[sl] = ok
        near[sl] = np.where(valid, j, -1)
        r_hat[sl] = np.where(valid, rh, np.nan)
        w_hat[sl] = np.where(valid, rh * rh - R2[j] + W[j], np.nan)
    return keep, r_hat, w_hat, near


def steiner_round(P, R, W, m: int, X, lo: float = 2.0, hi: float = 6.0):
    """The inner loop of Alg. 1 over the points ``X`` [S,3] (float64 values
    of float32 points), in order.  ``P`` [cap,3], ``R`` [cap], ``W`` [cap]
    hold the current set in their first ``m`` rows and receive the kept
    cells after them (float64 copies of the float32 values).  Returns (the
    new count, the indices in X of the kept points, the nearest cell of each
    kept point in the combined order)."""
    kept, nears = [], []
    for j in range(X.shape[0]):
        x = X[j]
        pw = _sq_dist(x, P[:m]) - R[:m] * R[:m]      # power of x w.r.t. every sphere of the set
        i = int(np.argmin(pw))                       # least power; ties: lowest index
        if not pw[i] > 0.0:
            continue                                 # x lies in (or on) a sphere
        dist = float(np.sqrt(_sq_dist(x, P[i:i + 1])[0]))
        rh = dist - R[i]
        if lo * R[i] <= rh <= hi * R[i]:
            P[m] = x
            R[m] = float(np.float32(rh))
            W[m] = float(np.float32(rh * rh - R[i] * R[i] + W[i]))
            m += 1
            kept.append(j)
            nears.append(i)
    return m, np.asarray(kept, dtype=np.int64), np.asarray(nears, dtype=np.int64)


def steiner_points(p, radius, power, z, lo: float = 2.0, hi: float = 6.0):
    """All rounds of the insertion.  ``p`` [N,3], ``radius`` [N], ``power``
    [N] (float32 scene values), ``z`` [rounds, S, 3] standard normal draws.

    Returns a dict of the kept cells in the order they were kept:
    ``p`` [A,3] float32, ``radius`` [A] float32, ``power`` [A] float32,
    ``near`` [A] int64 (index of the nearest cell in the combined order),
    ``round`` [A] int64, and ``candidate`` [A] int64 (index in its round)."""
    p = np.asarray(p, dtype=np.float32)
    z = np.asarray(z, dtype=np.float32).astype(F64)
    n = p.shape[0]
    rounds, S = z.shape[0], z.shape[1]
    cap = n + rounds * S
    P = np.zeros((cap, 3))
    R = np.zeros(cap)
    W = np.zeros(cap)
    P[:n] = p.astype(F64)
    R[:n] = np.asarray(radius, dtype=np.float32).astype(F64)
    W[:n] = np.asarray(power, dtype=np.float32).astype(F64)
    m = n
    rnd, cand, near = [], [], []
    for it in range(rounds):
        mean = P[:m].mean(axis=0)
        std = P[:m].std(axis=0)
        X = (mean[None, :] + std[None, :] * z[it]).astype(np.float32).astype(F64)
        m, kept, nr = steiner_round(P, R, W, m, X, lo, hi)
        rnd.append(np.full(kept.size, it, dtype=np.int64))
        cand.append(kept)
        near.append(nr)
    return {"p": P[n:m].astype(np.float32).reshape(-1, 3), "radius": R[n:m].astype(np.float32),
            "power": W[n:m].astype(np.float32), "near": np.concatenate(near),
            "round": np.concatenate(rnd), "candidate": np.concatenate(cand)}
