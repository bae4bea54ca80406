"""Pins of the oracle's training regularisers (supplementary material, loss
functions) and of the per-cell contribution statistic:
  * the contributions summed over cells equal the rendered opacity A of the
    independent painter form (every ray: sum_k T_k a_k = 1 - T_end);
  * a single cell: L_normal = A max(n.d, 0)^2 with n.d computed here;
  * the normal-loss gradient against float64 central differences of the
    loss value (walk re-run at each point);
  * the connectivity loss and its gradient in closed form for two spheres,
    zero without overlap, and central differences on a random set."""
import numpy as np
import pytest

import oracle
import workloads as W
from oracle.adjoint import PARAMS


def _f64(sc):
    return W.Scene(*(getattr(sc, f).astype(np.float64) for f in PARAMS), sigma_scale=sc.sigma_scale, tau=sc.tau)


def test_contributions_sum_to_painter_opacity():
    sc = W.scene_uniform(120, seed=5)
    sc.radius = (sc.radius * 3.0).astype(np.float32)
    cam = W.pinhole(W.random_eyes(1, 2.8, 9)[0], 12, 10, 60.0)
    G = np.zeros((cam.n_rays, 4))
    _, vals = oracle.regularized_gradients(sc, cam, G)
    A = oracle.render_painter(sc, cam)[:, 3].sum()
    assert A > 1.0
    assert abs(vals["contribution"].sum() - A) <= 1e-9 * A
    assert abs(vals["sparse"] - A) <= 1e-9 * A


def test_single_cell_normal_loss_closed_form():
    sc = W.scene_uniform(1, seed=2)
    sc.p[:] = 0.0
    sc.radius[:] = 0.5
    sc.power[:] = 0.01
    sc.normal[:] = np.array([[0.3, -0.2, -0.9]], dtype=np.float32)   # faces away from the camera: n.d > 0
    cam = W.pinhole(np.array([0.0, 0.3, 2.0]), 6, 5, 40.0)
    G = np.zeros((cam.n_rays, 4))
    _, vals = oracle.regularized_gradients(sc, cam, G)
    A = oracle.render_walk(sc, cam)[:, 3]
    o, d, _ = oracle.generate_rays(cam)
    n = sc.normal[0].astype(np.float64)
    n /= np.linalg.norm(n)
    cosd = d.numpy() @ n
    ref = (A * np.maximum(cosd, 0.0) ** 2).sum()
    assert A.max() > 0.1 and ref > 0
    assert abs(vals["normal"] - ref) <= 1e-9 * ref


@pytest.mark.parametrize("field,idx", [("normal", (7, 0)), ("normal", (3, 2)), ("occ_logit", (7,)), ("p", (3, 1))])
def test_normal_loss_gradient_matches_central_differences(field, idx):
    sc = _f64(W.scene_uniform(40, seed=4))
    sc.radius *= 3.0
    cam = W.pinhole(W.random_eyes(1, 2.6, 12)[0], 8, 7, 60.0)
    G = np.zeros((cam.n_rays, 4))
    grads, _ = oracle.regularized_gradients(sc, cam, G, lambda_normal=1.0)
    g = grads[field][idx]
    h = 1e-6
    arr = getattr(sc, field)
    base = arr[idx]
    arr[idx] = base + h
    lp = oracle.normal_loss_value(sc, cam)
    arr[idx] = base - h
    lm = oracle.normal_loss_value(sc, cam)
    arr[idx] = base
    fd = (lp - lm) / (2 * h)
    assert abs(g - fd) <= 1e-5 * max(1.0, abs(fd)), (g, fd)


def test_connect_loss_two_spheres_closed_form():
    sc = W.scene_uniform(2, seed=0)
    sc.p[:] = np.array([[0.0, 0.0, 0.0], [0.3, 0.4, 0.0]], dtype=np.float32)
    sc.radius[:] = np.array([0.4, 0.35], dtype=np.float32)
    L, g = oracle.connect_loss(sc, lam=2.0)
    ov = 0.4 + 0.35 - 0.5
    assert abs(L - 2.0 * 2 * ov * ov) < 1e-6
    assert np.allclose(g["radius"], [2.0 * 4 * ov, 2.0 * 4 * ov], atol=1e-6)
    u = np.array([0.3, 0.4, 0.0]) / 0.5                   # unit vector from p0 to p1
    assert np.allclose(g["p"][0], 2.0 * 4 * ov * u, atol=1e-6)
    assert np.allclose(g["p"][1], -2.0 * 4 * ov * u, atol=1e-6)
    sc.radius[:] = np.array([0.2, 0.25], dtype=np.float32)
    L0, g0 = oracle.connect_loss(sc)
    assert L0 == 0.0 and not g0["p"].any() and not g0["radius"].any()


def test_connect_loss_central_differences():
    sc = _f64(W.scene_uniform(30, seed=6))
    sc.radius *= 4.0
    L, g = oracle.connect_loss(sc)
    assert L > 0
    h = 1e-6
    for field, idx in (("p", (4, 1)), ("radius", (9,)), ("p", (11, 2))):
        arr = getattr(sc, field)
        base = arr[idx]
        arr[idx] = base + h
        lp, _ = oracle.connect_loss(sc)
        arr[idx] = base - h
        lm, _ = oracle.connect_loss(sc)
        arr[idx] = base
        assert abs(g[field][idx] - (lp - lm) / (2 * h)) <= 1e-6 * max(1.0, abs(g[field][idx]))
