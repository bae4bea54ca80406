"""Pins of the Steiner-cell oracle (supplementary material, Steiner points,
Alg. 1): closed forms on one and two spheres, the power-nearest choice, the
in-loop insertion (a later point of a round is tested against the cells kept
earlier in that round), the round structure, a pure-Python brute force, and
the invariance of the image when empty cells are added outside the spheres
of a scene with w = r^2."""
import math

import numpy as np
import pytest

import workloads as W
from oracle.cell import bisector
from oracle.steiner import evaluate_candidates, steiner_points, steiner_round
from oracle.walk import render_walk


def _evaluate(P, R, x, Wt=None):
    P = np.asarray(P, float)
    R = np.asarray(R, float)
    Wt = R * R if Wt is None else np.asarray(Wt, float)
    return evaluate_candidates(P, R, Wt, np.asarray(x, float))


def test_single_sphere_closed_form():
    # sphere at the origin, radius 1: r_hat = |x| - 1, kept for 2 <= r_hat <= 6
    xs = [[0.5, 0, 0], [1.0, 0, 0], [2.5, 0, 0], [3.0, 0, 0], [0, 4.0, 0], [0, 0, 7.0], [7.5, 0, 0]]
    keep, r_hat, w_hat, near = _evaluate([[0, 0, 0]], [1.0], xs)
    assert keep.tolist() == [False, False, False, True, True, True, False]
    # inside and on the sphere: not valid at all
    assert near[0] == -1 and near[1] == -1 and np.isnan(r_hat[0]) and np.isnan(r_hat[1])
    assert r_hat[2:].tolist() == [1.5, 2.0, 3.0, 6.0, 6.5]
    # w = r^2 scene: the new weight is r_hat^2 (the paper's parameterisation)
    assert np.allclose(w_hat[2:], np.array(r_hat[2:]) ** 2, rtol=0, atol=1e-15)


def test_nearest_is_by_power_not_by_surface_distance():
    # A: radius 0.25 at the origin; B: radius 2 whose surface is closer to x
    # (0.9 vs 1.0), but x has the smaller power w.r.t. A (1.5 vs 4.41)
    P = [[0, 0, 0], [1.25, 2.9, 0]]
    R = [0.25, 2.0]
    keep, r_hat, _, near = _evaluate(P, R, [[1.25, 0, 0]])
    assert near[0] == 0 and r_hat[0] == pytest.approx(1.0, abs=1e-15)
    assert keep[0]            # 2 * 0.25 <= 1.0 <= 6 * 0.25; by B's surface it would be 0.9 < 4


def test_new_weight_puts_the_bisector_on_the_nearest_sphere():
    rng = np.random.default_rng(11)
    P = rng.uniform(-1, 1, (30, 3))
    R = rng.uniform(0.05, 0.2, 30)
    Wt = (R / 1.5) ** 2                      # weights unlike r^2, as in the workloads
    x = rng.uniform(-2, 2, (400, 3))
    keep, r_hat, w_hat, near = _evaluate(P, R, x, Wt)
    assert keep.sum() > 5
    for j in np.nonzero(keep)[0]:
        i = near[j]
        m, h = bisector(np.asarray(P[i], float), float(Wt[i]), x[j], float(w_hat[j]))
        # plane (y - p_i).m <= h: its distance from p_i is h / |m| = r_i
        assert h / np.linalg.norm(m) == pytest.approx(R[i], rel=1e-12)


def _round(P, R, X, Wt=None, lo=2.0, hi=6.0):
    P = np.asarray(P, float)
    R = np.asarray(R, float)
    Wt = R * R if Wt is None else np.asarray(Wt, float)
    X = np.asarray(X, float)
    cap = len(P) + len(X)
    PP, RR, WW = np.zeros((cap, 3)), np.zeros(cap), np.zeros(cap)
    PP[:len(P)], RR[:len(P)], WW[:len(P)] = P, R, Wt
    m, kept, near = steiner_round(PP, RR, WW, len(P), X, lo, hi)
    return kept.tolist(), near.tolist(), PP[len(P):m], RR[len(P):m], WW[len(P):m]


def test_later_point_is_tested_against_cells_kept_earlier_in_the_round():
    # unit sphere at the origin; three points of one round, in this order:
    #   (3, 0, 0): r_hat = 3 - 1 = 2, ratio 2: kept as a cell of radius 2
    #   (3.5, 0, 0): outside the unit sphere (ratio 2.5 against it alone) but
    #       0.5 from the centre of the cell just kept, inside its radius 2:
    #       rejected
    #   (3, 7, 0): power 49 - 4 = 45 w.r.t. the kept cell vs 58 - 1 = 57
    #       w.r.t. the unit sphere, so the kept cell is its nearest:
    #       r_hat = 7 - 2 = 5, ratio 2.5: kept.  Against the unit sphere alone
    #       it would have r_hat = sqrt(58) - 1 = 6.62, ratio > 6: rejected.
    kept, near, P, R, Wt = _round([[0, 0, 0]], [1.0], [[3, 0, 0], [3.5, 0, 0], [3, 7, 0]])
    assert kept == [0, 2]
    assert near == [0, 1]
    assert P.tolist() == [[3, 0, 0], [3, 7, 0]]
    assert R.tolist() == [2.0, 5.0]
    # w = r^2 scene: the new weights are r_hat^2
    assert Wt.tolist() == [4.0, 25.0]
    # judged one by one against the unit sphere alone, the verdicts differ
    keep_fixed, _, _, _ = _evaluate([[0, 0, 0]], [1.0], [[3, 0, 0], [3.5, 0, 0], [3, 7, 0]])
    assert keep_fixed.tolist() == [True, True, False]


def test_order_within_a_round_decides():
    # the same two points in the other order: (3.5, 0, 0) first is kept with
    # r_hat 2.5; then (3, 0, 0) lies inside its sphere (0.5 < 2.5) and is
    # rejected
    kept, near, _, R, _ = _round([[0, 0, 0]], [1.0], [[3.5, 0, 0], [3, 0, 0]])
    assert kept == [0] and near == [0] and R.tolist() == [2.5]


def test_tie_between_scene_cell_and_kept_cell_goes_to_the_scene_cell():
    # after (3, 0, 0) is kept (radius 2), the points of equal power w.r.t.
    # the unit sphere and the kept cell satisfy |x|^2 - 1 = |x - (3,0,0)|^2 - 4,
    # i.e. x = 1; (1, 6, 0) has power 36 w.r.t. both
    kept, near, _, R, _ = _round([[0, 0, 0]], [1.0], [[3, 0, 0], [1, 6, 0]], lo=0.0, hi=100.0)
    assert kept == [0, 1]
    assert near == [0, 0]                  # the scene cell (lower index) wins the tie
    assert R[1] == float(np.float32(math.sqrt(37.0) - 1.0))   # stored as the float32 site radius


def test_rounds_see_earlier_rounds_and_use_their_statistics():
    p = np.array([[-1, 0, 0], [1, 0, 0]], np.float32)
    r = np.array([0.1, 0.1], np.float32)
    w = r * r
    # round 1: mean 0, std (1, 0, 0): candidate x = (0.5, 0, 0) -> nearest site 1, r_hat 0.4 (ratio 4)
    # round 2: sites -1, 1, 0.5 -> mean 1/6, std sqrt(13/18) along x
    m2, s2 = 1.0 / 6.0, math.sqrt(13.0 / 18.0)
    z = np.zeros((2, 2, 3), np.float32)
    z[0, 0, 0] = 0.5
    z[0, 1, 0] = 3.0          # x = 3: nearest site 1, r_hat 1.9 (ratio 19): rejected
    z[1, 0, 0] = (0.6 - m2) / s2     # inside the round-1 Steiner sphere (centre 0.5, radius 0.4)
    z[1, 1, 0] = (-0.5 - m2) / s2    # nearest site 0, r_hat 0.4: kept
    out = steiner_points(p, r, w, z)
    assert out["round"].tolist() == [0, 1] and out["candidate"].tolist() == [0, 1]
    assert out["near"].tolist() == [1, 0]
    assert np.allclose(out["p"], [[0.5, 0, 0], [-0.5, 0, 0]], atol=2e-7)
    assert np.allclose(out["radius"], [0.4, 0.4], atol=3e-7)


def _brute(P, R, Wt, x, lo=2.0, hi=6.0):
    res = []
    for xj in x:
        best, bi = math.inf, -1
        for i in range(len(P)):
            pw = sum((float(xj[a]) - float(P[i][a])) ** 2 for a in range(3)) - float(R[i]) ** 2
            if pw < best:
                best, bi = pw, i
        if not best > 0:
            res.append(None)
            continue
        d = math.sqrt(sum((float(xj[a]) - float(P[bi][a])) ** 2 for a in range(3)))
        rh = d - float(R[bi])
        res.append((bi, rh, lo * float(R[bi]) <= rh <= hi * float(R[bi])))
    return res


def test_vectorised_test_matches_pure_python_brute_force():
    rng = np.random.default_rng(5)
    P = rng.uniform(-1, 1, (40, 3))
    R = rng.uniform(0.05, 0.3, 40)
    Wt = R * R
    x = rng.normal(0, 1.2, (97, 3))
    keep, r_hat, _, near = evaluate_candidates(P, R, Wt, x, chunk=7)
    ref = _brute(P, R, Wt, x)
    assert any(v is None for v in ref) and any(v is not None and v[2] for v in ref)
    for j, v in enumerate(ref):
        if v is None:
            assert near[j] == -1 and not keep[j]
        else:
            assert near[j] == v[0] and keep[j] == v[2]
            assert r_hat[j] == pytest.approx(v[1], rel=1e-13, abs=1e-14)


def test_kept_cells_lie_outside_every_earlier_sphere():
    # every kept cell lies outside the spheres of the scene and of every cell
    # kept before it, in its own round too, and its radius is 2..6 times its
    # nearest cell's
    sc = W.scene_uniform(256, seed=3)
    z = W.steiner_draws(3, 512, seed=9)
    out = steiner_points(sc.p, sc.radius, sc.power, z)
    assert out["p"].shape[0] > 20
    P = np.concatenate([sc.p, out["p"]]).astype(float)
    R = np.concatenate([sc.radius, out["radius"]]).astype(float)
    n = sc.n
    for a in range(out["p"].shape[0]):
        q = out["p"][a].astype(float)
        pw = ((q[None, :] - P[:n + a]) ** 2).sum(-1) - R[:n + a] ** 2
        assert (pw > 0).all()
        assert int(np.argmin(pw)) == out["near"][a]
        ratio = out["radius"][a] / R[out["near"][a]]
        assert 2 - 1e-6 <= ratio <= 6 + 1e-6
    # within a round, some later point was rejected or re-targeted because of
    # an earlier one: the in-loop verdicts differ from judging the round's
    # points against the round-start set alone
    mean, std = sc.p.astype(float).mean(0), sc.p.astype(float).std(0)
    X = (mean + std * z[0].astype(float)).astype(np.float32).astype(float)
    keep0, _, _, _ = evaluate_candidates(sc.p.astype(float), sc.radius.astype(float), sc.power.astype(float), X)
    kept0 = out["candidate"][out["round"] == 0]
    assert set(kept0.tolist()) != set(np.nonzero(keep0)[0].tolist())


def test_empty_cells_outside_the_spheres_leave_the_image_unchanged():
    # w = r^2: an empty cell whose sphere meets no sphere of the scene (it
    # touches its nearest one) takes no point of any sphere, so the bounded
    # cells, and the image, stay (up to the float32 rounding of the new
    # radius and weight, which can move a bisector by ~1e-8)
    sc = W.scene_uniform(48, seed=21)
    sc.power = (sc.radius.astype(np.float64) ** 2).astype(np.float32)
    z = W.steiner_draws(6, 256, seed=22)
    out = steiner_points(sc.p, sc.radius, sc.power, z)
    P, R = sc.p.astype(float), sc.radius.astype(float)
    q, rq = out["p"].astype(float), out["radius"].astype(float)
    gap = np.sqrt(((q[:, None, :] - P[None]) ** 2).sum(-1)) - (rq[:, None] + R[None])
    sel = (gap > -1e-6).all(axis=1)
    assert sel.sum() >= 5
    a = sel.sum()
    aug = W.Scene(p=np.concatenate([sc.p, out["p"][sel]]),
                  power=np.concatenate([sc.power, out["power"][sel]]),
                  radius=np.concatenate([sc.radius, out["radius"][sel]]),
                  normal=np.concatenate([sc.normal, np.tile(np.float32([0, 0, 1]), (a, 1))]),
                  occ_logit=np.concatenate([sc.occ_logit, np.full(a, -np.inf, np.float32)]),
                  rgb=np.concatenate([sc.rgb, np.zeros((a, 3), np.float32)]),
                  tex=np.concatenate([sc.tex, np.zeros((a,) + sc.tex.shape[1:], np.float32)]))
    cam = W.pinhole(np.array([0.3, -2.6, 0.4]), 24, 24)
    img0 = render_walk(sc, cam)
    img1 = render_walk(aug, cam)
    assert np.abs(img0).max() > 0.05
    assert np.abs(img1 - img0).max() <= 1e-6
