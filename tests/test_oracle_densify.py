"""Pins of the densify/prune oracle (Sec. 3.5): the multinomial draw on a hand
case and in distribution, the moving average's closed form, the pruning
boundary, and the per-cell error against the telescoping of the segment sum
(sum over cells of T a e = sum over rays of A e)."""
import numpy as np
import pytest

import workloads as W
from oracle.densify import cell_error, densify_prune, draw, ema
from oracle.regularizers import regularized_gradients
from oracle.walk import render_walk


def test_draw_hand_case():
    w = [0.0, 1.0, 3.0, 0.0, 4.0]          # cumulative 0, 1, 4, 4, 8
    u = [0.0, 0.124, 0.125, 0.49, 0.5, 0.999]
    assert draw(w, u).tolist() == [1, 1, 2, 2, 4, 4]


def test_draw_frequencies_follow_the_weights():
    rng = np.random.default_rng(3)
    w = rng.uniform(0, 1, 40) ** 3
    w[[5, 17]] = 0.0
    u = rng.uniform(0, 1, 400000).astype(np.float32)
    f = np.bincount(draw(w, u), minlength=40) / u.size
    p = w / w.sum()
    assert f[5] == 0 and f[17] == 0
    sd = np.sqrt(p * (1 - p) / u.size)
    assert (np.abs(f - p) <= 5 * sd + 1e-7).all()


def test_moving_average_closed_form():
    beta, v = 0.9, 2.5
    e = np.zeros(3, np.float32)
    for k in range(1, 31):
        e = ema(e, np.full(3, v, np.float32), beta)
        assert e[0] == pytest.approx(v * (1 - np.float32(beta).astype(float) ** k), rel=2e-6)


def test_prune_boundary_is_inclusive_and_new_cells_follow_parents():
    sc = W.scene_uniform(10, seed=1)
    contrib = np.array([0.5, 0.1, 0.2, 0.0, 0.3, 0.2, 0.9, 0.05, 0.2, 0.4], np.float32)
    err = np.array([1, 0, 0, 5, 2, 0, 1, 0, 0, 0], np.float32)
    u = np.array([0.0, 0.3, 0.99], np.float32)
    delta = np.array([[1, 0, 0], [0, -1, 0], [0, 0, 2]], np.float32)
    out, e2, c2, par = densify_prune(sc, err, contrib, u, delta, prune_below=0.2, spread=0.5)
    kept = [0, 2, 4, 5, 6, 8, 9]                # contribution >= 0.2 (0.2 itself kept)
    # weights over kept cells: 1, 0, 2, 0, 1, 0, 0 -> cumulative 1, 1, 3, 3, 4, 4, 4 (total 4)
    assert par.tolist() == [0, 4, 6]            # u*4 = 0 -> cell 0; 1.2 -> cell 4; 3.96 -> cell 6
    assert out["p"].shape == (10, 3)
    assert np.array_equal(out["radius"][:7], sc.radius[kept])
    for k, i in enumerate(par):
        assert np.array_equal(out["tex"][7 + k], sc.tex[i]) and out["occ_logit"][7 + k] == sc.occ_logit[i]
        assert e2[7 + k] == err[i] and c2[7 + k] == contrib[i]
        expect = sc.p[i].astype(float) + 0.5 * float(sc.radius[i]) * delta[k].astype(float)
        assert np.allclose(out["p"][7 + k], expect, atol=1e-6)
    # nothing to draw from: no new cells
    out0, _, _, par0 = densify_prune(sc, np.zeros(10, np.float32), contrib, u, delta, 0.2, 0.5)
    assert par0.size == 0 and out0["p"].shape == (7, 3)


def test_cell_error_telescopes_and_reduces_to_the_contribution():
    sc = W.scene_uniform(150, seed=6)
    sc.radius = (sc.radius * 2.5).astype(np.float32)
    cam = W.pinhole(W.random_eyes(1, 2.6, 2)[0], 14, 12, 60.0)
    rng = np.random.default_rng(1)
    e = rng.uniform(0, 2, cam.n_rays)
    err = cell_error(sc, cam, e)
    A = render_walk(sc, cam)[:, 3]
    assert A.max() > 0.3
    # the cells' contributions along a ray sum to its opacity A
    assert err.sum() == pytest.approx(float((A * e).sum()), rel=1e-12)
    _, vals = regularized_gradients(sc, cam, np.zeros((cam.n_rays, 4)))
    assert np.allclose(cell_error(sc, cam, np.ones(cam.n_rays)), vals["contribution"], rtol=1e-13, atol=1e-15)
