"""Face adjacency of the power diagram (oracle; test infrastructure).

Two routes, used to pin each other and then the GPU build:

* ``lifted_hull_edges``: the regular triangulation (dual of the unbounded
  power diagram, which the ray walk needs, appendix C) as the lower convex
  hull of the lifted points ``(p_i, |p_i|^2 - w_i)`` (the textbook lifting
  map; Qhull through scipy).  Sites off the lower hull have empty cells.
* ``lp_face_exists``: brute force from the power-cell definition (appendix
  B): cells i and j share a 2-D face iff some point of their bisector plane
  is strictly closer in power to i and j than to every other site, found by a
  linear program on that plane.
"""
from __future__ import annotations

import numpy as np


def lifted_hull_edges(p, w):
    """Sorted array of undirected edges (i < j) of the regular triangulation."""
    from scipy.spatial import ConvexHull
    p = np.asarray(p, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    lifted = np.c_[p, (p * p).sum(1) - w]
    hull = ConvexHull(lifted, qhull_options="Qt")
    lower = hull.equations[:, 3] < 0
    edges = set()
    for simplex in hull.simplices[lower]:
        s = sorted(int(v) for v in simplex)
        for a in range(4):
            for b in range(a + 1, 4):
                edges.add((s[a], s[b]))
    return np.array(sorted(edges), dtype=np.int64).reshape(-1, 2)


def lp_face_exists(p, w, i: int, j: int, box=1e3) -> bool:
    """True iff cells i and j share a face of positive area inside the box:
    ``box`` is a half-width (the cube ``|x_a| <= box``) or a pair
    ``(lo[3], hi[3])`` of corners."""
    from scipy.optimize import linprog
    p = np.asarray(p, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    n = p.shape[0]
    # variables (x0, x1, x2, s); maximise s
    # on the bisector:  2 x.(p_j - p_i) = |p_j|^2 - |p_i|^2 - w_j + w_i
    a_eq = np.r_[2.0 * (p[j] - p[i]), 0.0][None]
    b_eq = np.array([(p[j] @ p[j]) - (p[i] @ p[i]) - w[j] + w[i]])
    # for k != i, j:  pow(x,k) - pow(x,i) >= s, i.e.
    #   2 x.(p_k - p_i) + s <= |p_k|^2 - |p_i|^2 - w_k + w_i
    rows, rhs = [], []
    for k in range(n):
        if k in (i, j):
            continue
        rows.append(np.r_[2.0 * (p[k] - p[i]), 1.0])
        rhs.append((p[k] @ p[k]) - (p[i] @ p[i]) - w[k] + w[i])
    if np.ndim(box) == 0:
        lo, hi = -float(box) * np.ones(3), float(box) * np.ones(3)
    else:
        lo, hi = np.asarray(box[0], dtype=np.float64), np.asarray(box[1], dtype=np.float64)
    bounds = [(lo[a], hi[a]) for a in range(3)] + [(None, 1.0)]
    res = linprog(c=[0, 0, 0, -1.0], A_ub=np.array(rows) if rows else None,
                  b_ub=np.array(rhs) if rows else None, A_eq=a_eq, b_eq=b_eq,
                  bounds=bounds, method="highs")
    return bool(res.status == 0 and -res.fun > 1e-9)


def lp_edges(p, w, box: float = 1e3):
    n = len(p)
    out = [(i, j) for i in range(n) for j in range(i + 1, n) if lp_face_exists(p, w, i, j, box)]
    return np.array(out, dtype=np.int64).reshape(-1, 2)
