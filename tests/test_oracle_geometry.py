"""Pins of the oracle's geometry against definitions and closed forms.

* bisector offset sign: two cells on a line, boundary at the closed-form
  radical-plane position (appendix B, power bisector; the sign follows the
  power-cell definition);
* radical plane of overlapping spheres contains their intersection circle
  (Sec. 3.2, radical-plane figure);
* equal weights reduce the power cell to the Voronoi cell (appendix B), so the
  start cell is the nearest site (scipy k-d tree);
* interval lengths match dense point sampling labelled straight from the
  argmin-power definition, the sphere bound and the dipole half-space;
* the walk equals the painter form; cells met along every ray come in
  increasing power distance from the camera (appendix B, theorem);
* each walk transition point is equidistant in power to both cells and no
  other site is closer (it lies on a face of the power diagram).
"""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from oracle.cell import scene_tensors, shade
from conftest import make_scene


def _cam_line(o, d):
    """A 1-pixel pinhole camera whose only ray is o + t d."""
    d = np.asarray(d, dtype=np.float64)
    d = d / np.linalg.norm(d)
    c2w = W.look_at(np.asarray(o, dtype=np.float64), np.asarray(o) + d)
    return W.Camera(model=0, width=1, height=1, c2w=c2w, fx=1.0, fy=1.0, cx=0.5, cy=0.5)


def test_two_cell_bisector_closed_form():
    # cells at x=-0.5 and x=+0.5, weights 0.2 and 0: radical plane at x=(w1-w2)/2=0.1
    tex = np.zeros((2, 8, 51))
    sc = make_scene([[-0.5, 0, 0], [0.5, 0, 0]], power=[0.2, 0.0], radius=[1.0, 1.0],
                    normal=[[0, 0, 1], [0, 0, 1]], tex=tex)
    cam = _cam_line([-3.0, 0.0, -0.5], [1.0, 0.0, 0.0])
    rgba, rec = oracle.walk_records(sc, cam)
    assert rec.cell.tolist() == [0, 1]
    half = np.sqrt(1.0 - 0.25)
    # ray at z=-0.5: sphere chords x in [-0.5-half, -0.5+half] and [0.5-half, 0.5+half]
    np.testing.assert_allclose(rec.lo.numpy() - 3.0, [-0.5 - half, 0.1], atol=1e-12)
    np.testing.assert_allclose(rec.hi.numpy() - 3.0, [0.1, 0.5 + half], atol=1e-12)
    assert rec.hi_kind.tolist() == [oracle.walk.BIND_PLANE, oracle.walk.BIND_SPHERE]


def test_radical_plane_contains_sphere_intersection_circle():
    rng = np.random.default_rng(3)
    for _ in range(20):
        pi, pj = rng.normal(size=3), rng.normal(size=3)
        dist = np.linalg.norm(pj - pi)
        ri, rj = rng.uniform(0.6, 1.0) * dist, rng.uniform(0.6, 1.0) * dist
        if ri + rj <= dist:
            continue
        # a point on the intersection circle of the two spheres
        e = (pj - pi) / dist
        xa = (dist ** 2 + ri ** 2 - rj ** 2) / (2 * dist)
        perp = np.cross(e, rng.normal(size=3))
        perp /= np.linalg.norm(perp)
        x = pi + xa * e + np.sqrt(ri ** 2 - xa ** 2) * perp
        m, h = oracle.bisector(torch.tensor(pi), torch.tensor(ri ** 2), torch.tensor(pj), torch.tensor(rj ** 2))
        assert abs(float((torch.tensor(x - pi) * m).sum() - h)) < 1e-12
    # disjoint spheres: the plane misses both
    pi, pj = np.zeros(3), np.array([3.0, 0, 0])
    m, h = oracle.bisector(torch.tensor(pi), torch.tensor(1.0), torch.tensor(pj), torch.tensor(0.25))
    xplane = float(h / m[0])
    assert 1.0 < xplane < 3.0 - 0.5


def test_equal_weights_start_cell_is_nearest_site():
    from scipy.spatial import cKDTree
    rng = np.random.default_rng(5)
    p = rng.uniform(-1, 1, size=(500, 3))
    S = {"p": torch.tensor(p), "power": torch.full((500,), 0.37, dtype=torch.float64)}
    tree = cKDTree(p)
    for q in rng.uniform(-2, 2, size=(50, 3)):
        i0 = int(oracle.walk.start_cells(S, torch.tensor(q)))
        assert i0 == int(tree.query(q)[1])


def _tiny_scene(seed, n=10, disp_equal=False):
    rng = np.random.default_rng(seed)
    p = rng.uniform(-0.8, 0.8, size=(n, 3))
    tex = rng.normal(0, 0.1, size=(n, 8, 51))
    if disp_equal:
        tex[:, :, 0:2] = tex[:, :1, 0:2]   # all detail sites of a cell coincide
    else:
        tex[:, :, 2] = 0.0                 # no displacement
    return make_scene(p, power=rng.uniform(0.0, 0.3, n), radius=rng.uniform(0.4, 0.9, n), tex=tex, seed=seed)


@pytest.mark.parametrize("seed,disp_equal", [(0, False), (1, False), (2, True), (3, True)])
def test_walk_lengths_match_dense_sampling(seed, disp_equal):
    sc = _tiny_scene(seed, disp_equal=disp_equal)
    S = scene_tensors(sc)
    rng = np.random.default_rng(100 + seed)
    dt = 2e-5
    for _ in range(3):
        o = rng.normal(size=3)
        o = 2.5 * o / np.linalg.norm(o)
        d = -o / np.linalg.norm(o) + rng.normal(0, 0.15, size=3)
        cam = _cam_line(o, d)
        _, rec = oracle.walk_records(sc, cam)
        oo, dd, _ = oracle.generate_rays(cam)
        alpha, colour, ell = shade(oo, dd[rec.ray], rec.lo, rec.hi, S["p"][rec.cell], S["normal"][rec.cell],
                                   S["occ_logit"][rec.cell], S["rgb"][rec.cell], S["tex"][rec.cell],
                                   S["sigma_scale"], S["tau"])
        delta = None
        if disp_equal:   # equal detail sites: every soft-Voronoi weight is 1/K
            delta = {c: float(sc.tex[c, :, 2].astype(np.float64).mean()) for c in range(sc.n)}
        ref = oracle.dense_sample_ray(S, oo, dd[0], t_max=6.0, dt=dt, delta=delta)
        ref_in = {c: li for c, li, _ in ref}
        ref_dense = {c: ld for c, _, ld in ref}
        walk_in = {int(c): float(h - l) for c, l, h in zip(rec.cell, rec.lo, rec.hi)}
        walk_dense = {int(c): float(e) for c, e in zip(rec.cell, ell)}
        for c in set(ref_in) | set(walk_in):
            assert abs(ref_in.get(c, 0.0) - walk_in.get(c, 0.0)) < 3 * dt, (c, ref_in.get(c), walk_in.get(c))
            assert abs(ref_dense.get(c, 0.0) - walk_dense.get(c, 0.0)) < 3 * dt
        # order of first appearance = walk order (cells longer than the step)
        ref_order = [c for c, li, _ in ref if li > 3 * dt]
        walk_order = [int(c) for c in rec.cell if walk_in[int(c)] > 3 * dt]
        assert ref_order == walk_order


@pytest.mark.parametrize("seed", [0, 1])
def test_walk_equals_painter(seed):
    sc = W.scene_uniform(300, seed=seed)
    sc.radius *= 3.0          # heavier overlap so that planes bind often
    cam = W.pinhole(W.random_eyes(1, 3.0, seed + 7)[0], 24, 20, 60.0)
    a = oracle.render_walk(sc, cam)
    b = oracle.render_painter(sc, cam)
    assert np.abs(a - b).max() <= 1e-12
    assert a[:, 3].max() > 0.5


def test_walk_order_is_increasing_power_distance():
    sc = W.scene_uniform(400, seed=11)
    sc.radius *= 2.5
    cam = W.pinhole(W.random_eyes(1, 2.0, 12)[0], 16, 16, 90.0)
    _, rec = oracle.walk_records(sc, cam)
    S = scene_tensors(sc)
    o, _, _ = oracle.generate_rays(cam)
    key = oracle.power_distance(o.unsqueeze(0), S["p"], S["power"])
    for r in range(cam.n_rays):
        cells = rec.cell[rec.ray == r]
        if cells.numel() > 1:
            assert bool((key[cells][1:] > key[cells][:-1]).all())


def test_walk_transitions_lie_on_power_faces():
    sc = W.scene_uniform(200, seed=21)
    sc.radius *= 3.0
    cam = W.pinhole(W.random_eyes(1, 2.5, 22)[0], 10, 10, 60.0)
    S = scene_tensors(sc)
    o, d, _ = oracle.generate_rays(cam)
    _, rec = oracle.walk_records(sc, cam)
    checked = 0
    for c, hk, hj, hi, r in zip(rec.cell, rec.hi_kind, rec.hi_j, rec.hi, rec.ray):
        if int(hk) != oracle.walk.BIND_PLANE:
            continue
        x = o + float(hi) * d[int(r)]
        pw = oracle.power_distance(x.unsqueeze(0), S["p"], S["power"])
        assert abs(float(pw[int(c)] - pw[int(hj)])) < 1e-10
        assert float(pw.min()) >= float(pw[int(c)]) - 1e-10
        checked += 1
    assert checked > 20


@pytest.mark.parametrize("seed,equal", [(0, True), (1, False), (2, False)])
def test_lifted_hull_adjacency_matches_lp(seed, equal):
    from oracle.adjacency import lifted_hull_edges, lp_edges
    rng = np.random.default_rng(seed)
    p = rng.uniform(-1, 1, size=(24, 3))
    w = np.full(24, 0.1) if equal else rng.uniform(0, 0.2, size=24)
    a = {tuple(e) for e in lifted_hull_edges(p, w)}
    b = {tuple(e) for e in lp_edges(p, w)}
    assert a == b and len(a) > 30


def test_equal_weight_adjacency_is_delaunay():
    from scipy.spatial import Delaunay
    from oracle.adjacency import lifted_hull_edges
    rng = np.random.default_rng(9)
    p = rng.uniform(-1, 1, size=(200, 3))
    tri = Delaunay(p)
    edges = set()
    for s in tri.simplices:
        s = sorted(int(v) for v in s)
        edges |= {(s[a], s[b]) for a in range(4) for b in range(a + 1, 4)}
    assert {tuple(e) for e in lifted_hull_edges(p, np.zeros(200))} == edges
