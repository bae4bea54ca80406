"""Pins of the oracle's shading and camera model against closed forms.

* one cell, ray along the normal: dense length ``r + delta`` with
  ``delta = mean_k d_k`` when all detail sites coincide (soft-Voronoi weights
  uniform, Sec. 3.4 Eq. svdisp), opacity ``1 - exp(-sigma (r + delta))`` and
  colour ``rgb + mean_k mean_m c_km`` when every SV axis is zero (Sec. 3.3,
  Sec. 3.4 Eq. svrad);
* soft-Voronoi limits: tau = 0 is uniform, large tau is the hard Voronoi
  assignment to the nearest detail site;
* Spherical-Voronoi limit: one dominant axis along the ray selects its colour;
* density limits: vanishing density is transparent, huge density opaque;
* the tangent frame is orthonormal and right-handed;
* pinhole: the image edge sits at half the vertical field of view;
* equidistant fisheye: the polar angle equals image radius / f, pixels past
  the image circle are masked;
* compositing invariants: alpha in [0,1], |C| <= max|c| * A;
* distinct detail sites: with a hard soft-Voronoi, the displacement is the
  site owning the undisplaced hit and the radiance the site owning the
  displaced hit (hand-computed closed form, Sec. 3.4 Eq. svdisp then
  Eq. svrad); with a moderate temperature, the displacement blended at the
  undisplaced hit (computed by hand) gives the dense length that dense point
  sampling measures.
"""
import math

import numpy as np
import torch

import oracle
import workloads as W
from conftest import make_scene
from oracle.cell import onb, scene_tensors, shade, soft_voronoi_weights

F64 = torch.float64


def _one_cell(delta_vals, lam=0.3, axes_zero=True, seed=0):
    rng = np.random.default_rng(seed)
    tex = rng.normal(0, 0.1, size=(1, 8, 51))
    tex[0, :, 0:2] = [0.03, -0.02]          # all detail sites coincide
    tex[0, :, 2] = delta_vals
    if axes_zero:
        tex[0, :, 3:27] = 0.0
    return make_scene([[0, 0, 0]], power=0.0, radius=1.0, normal=[[0, 0, 1]], occ_logit=lam,
                      rgb=[[0.2, 0.5, 0.7]], tex=tex)


def _cam_line(o, d):
    d = np.asarray(d, dtype=np.float64)
    c2w = W.look_at(np.asarray(o, dtype=np.float64), np.asarray(o) + d / np.linalg.norm(d))
    return W.Camera(model=0, width=1, height=1, c2w=c2w, fx=1.0, fy=1.0, cx=0.5, cy=0.5)


def test_single_cell_closed_form():
    dvals = np.linspace(-0.3, 0.4, 8)
    sc = _one_cell(dvals)
    delta = float(sc.tex[0, :, 2].astype(np.float64).mean())
    cam = _cam_line([0, 0, 5.0], [0, 0, -1.0])
    rgba = oracle.render_walk(sc, cam)[0]
    sigma = 10.0 * math.log1p(math.exp(float(sc.occ_logit[0])))
    alpha = 1.0 - math.exp(-sigma * (1.0 + delta))
    colour = sc.rgb[0].astype(np.float64) + sc.tex[0, :, 27:51].astype(np.float64).reshape(8, 8, 3).mean(axis=(0, 1))
    np.testing.assert_allclose(rgba[3], alpha, rtol=0, atol=1e-13)
    np.testing.assert_allclose(rgba[:3], alpha * colour, rtol=0, atol=1e-13)
    # from the other side the dense half is behind the face: length 1 - delta
    rgba2 = oracle.render_walk(sc, _cam_line([0, 0, -5.0], [0, 0, 1.0]))[0]
    np.testing.assert_allclose(rgba2[3], 1.0 - math.exp(-sigma * (1.0 + delta)), atol=1e-13)


def test_single_cell_oblique_ray_dense_length():
    # ray through the centre at angle phi to the face plane; no displacement
    sc = _one_cell(np.zeros(8))
    for phi in (0.3, 0.7, 1.2):
        d = np.array([math.cos(phi), 0.0, -math.sin(phi)])
        o = -3.0 * d
        rgba = oracle.render_walk(sc, _cam_line(o, d))[0]
        sigma = 10.0 * math.log1p(math.exp(float(sc.occ_logit[0])))
        # chord of length 2 through the centre; the dense half is z < 0: length 1
        np.testing.assert_allclose(rgba[3], 1.0 - math.exp(-sigma * 1.0), atol=1e-13)


def test_soft_voronoi_limits():
    rng = np.random.default_rng(2)
    s = torch.tensor(rng.normal(0, 0.1, size=(8, 2)))
    u = torch.tensor(rng.normal(0, 0.1, size=(5, 2)))
    w0 = soft_voronoi_weights(u, s.expand(5, 8, 2), 0.0)
    np.testing.assert_allclose(w0.numpy(), 1.0 / 8, atol=1e-15)
    wh = soft_voronoi_weights(u, s.expand(5, 8, 2), 1e6)
    nearest = torch.cdist(u, s).argmin(dim=1)
    np.testing.assert_allclose(wh.numpy(), np.eye(8)[nearest.numpy()], atol=1e-12)


def test_spherical_voronoi_dominant_axis():
    rng = np.random.default_rng(4)
    tex = rng.normal(0, 0.1, size=(1, 8, 51))
    tex[0, :, 0:2] = 0.0
    tex[0, :, 3:27] = 0.0
    d = np.array([0.0, 0.0, -1.0])
    tex[0, :, 3 + 3 * 5:3 + 3 * 5 + 3] = 200.0 * d    # axis 5 points along the ray
    sc = make_scene([[0, 0, 0]], power=0.0, radius=1.0, normal=[[0, 0, 1]], occ_logit=1.0,
                    rgb=[[0, 0, 0]], tex=tex)
    S = scene_tensors(sc)
    o = torch.tensor([0, 0, 5.0], dtype=F64)
    dd = torch.tensor(d, dtype=F64).unsqueeze(0)
    _, colour, _ = shade(o, dd, torch.tensor([4.0], dtype=F64), torch.tensor([6.0], dtype=F64), S["p"], S["normal"],
                         S["occ_logit"], S["rgb"], S["tex"], 10.0, 20.0)
    expect = sc.tex[0, :, 27:51].astype(np.float64).reshape(8, 8, 3)[:, 5, :].mean(axis=0)
    np.testing.assert_allclose(colour[0].numpy(), expect, atol=1e-12)


def test_density_limits():
    sc = _one_cell(np.zeros(8), lam=-80.0)
    cam = _cam_line([0, 0, 5.0], [0, 0, -1.0])
    assert oracle.render_walk(sc, cam)[0][3] < 1e-30
    sc = _one_cell(np.zeros(8), lam=80.0)
    assert oracle.render_walk(sc, cam)[0][3] == 1.0


def test_onb_orthonormal_right_handed():
    rng = np.random.default_rng(7)
    n = torch.tensor(rng.normal(size=(200, 3)))
    n = n / torch.linalg.norm(n, dim=1, keepdim=True)
    t1, t2 = onb(n)
    for a, b in ((t1, t2), (t1, n), (t2, n)):
        np.testing.assert_allclose((a * b).sum(-1).numpy(), 0.0, atol=1e-14)
    for a in (t1, t2):
        np.testing.assert_allclose(torch.linalg.norm(a, dim=1).numpy(), 1.0, atol=1e-14)
    np.testing.assert_allclose(torch.cross(t1, t2, dim=1).numpy(), n.numpy(), atol=1e-14)


def test_pinhole_edge_is_half_fov():
    cam = W.pinhole([0, -3.0, 0.0], 160, 120, 60.0)
    ang = oracle.camera.fov_check_angle(cam, cam.cx, 0.0)
    assert abs(ang - math.radians(30.0)) < 1e-6
    assert oracle.camera.fov_check_angle(cam, cam.cx, cam.cy) < 1e-12


def test_fisheye_equidistant():
    cam = W.fisheye([0, -3.0, 0.0], 101, 101, 180.0)
    f = float(np.float32(cam.f_fish))
    for rho in (0.0, 10.0, 30.0, 50.0):
        ang = oracle.camera.fov_check_angle(cam, float(np.float32(cam.cx)) + rho, float(np.float32(cam.cy)))
        assert abs(ang - rho / f) < 1e-9
    _, _, valid = oracle.generate_rays(cam)
    assert not bool(valid[0])                   # image corner lies past the circle
    assert bool(valid[50 * 101 + 50])


def test_composite_invariants():
    sc = W.scene_uniform(256, seed=3)
    sc.radius *= 2.0
    cam = W.pinhole(W.random_eyes(1, 3.0, 9)[0], 20, 20, 60.0)
    rgba, rec = oracle.walk_records(sc, cam)
    assert (rgba[:, 3] >= 0).all() and (rgba[:, 3] <= 1).all()
    cmax = np.abs(sc.rgb).max() + np.abs(sc.tex[:, :, 27:]).max()
    assert (np.abs(rgba[:, :3]).max(axis=1) <= cmax * rgba[:, 3] + 1e-12).all()


def _sites_scene(pos, disp, tau, radius=2.0, lam=0.3, seed=5):
    # one cell at the origin, normal +z (face frame t1 = x, t2 = y), detail
    # sites at the given face positions with the given displacements, all
    # Spherical-Voronoi axes zero (each site's colour is the mean of its M
    # colours) and distinct colours per site
    rng = np.random.default_rng(seed)
    tex = np.zeros((1, 8, 51))
    tex[0, :, 0:2] = pos
    tex[0, :, 2] = disp
    tex[0, :, 27:51] = rng.uniform(-1, 1, size=(8, 24))
    return make_scene([[0, 0, 0]], power=0.0, radius=radius, normal=[[0, 0, 1]], occ_logit=lam,
                      rgb=[[0.2, 0.5, 0.7]], tex=tex, tau=tau)


def test_texture_point_is_the_hit_with_the_displaced_face():
    # Hard soft-Voronoi (tau = 1e4): the ray o = (5.2, 0, 5), d = (-1, 0, -1)/sqrt(2)
    # meets the undisplaced face z = 0 at xbar = (0.2, 0, 0), on detail site 0
    # (d_0 = 0.3), so delta = 0.3 (Eq. svdisp at xbar); the displaced face
    # z = 0.3 is met at x = (0.5, 0, 0.3), on detail site 1, so the radiance is
    # site 1's (Eq. svrad at x): rgb + mean_m c_1m.  Evaluating the radiance at
    # xbar (site 0), or the displacement at x (d_1 = -0.1), changes the result.
    pos = [[0.2, 0.0], [0.5, 0.0]] + [[-3.0, -3.0]] * 6
    disp = [0.3, -0.1] + [0.05] * 6
    sc = _sites_scene(pos, disp, tau=1e4, lam=-3.0)
    rgba = oracle.render_walk(sc, _cam_line([5.2, 0.0, 5.0], [-1.0, 0.0, -1.0]))[0]
    # with s the distance along (-1, 0, -1) per unit of x: the sphere |x| <= 2
    # is crossed for s in [s0, s1], 2 s^2 - 20.4 s + 48.04 = 0; the dense side
    # z < delta is s > 5 - delta
    delta = float(np.float32(0.3))
    s1 = (20.4 + math.sqrt(20.4 ** 2 - 8 * 48.04)) / 4.0
    ell = math.sqrt(2.0) * (s1 - (5.0 - delta))
    sigma = 10.0 * math.log1p(math.exp(float(sc.occ_logit[0])))
    alpha = 1.0 - math.exp(-sigma * ell)
    cols = sc.tex[0, :, 27:51].astype(np.float64).reshape(8, 8, 3).mean(axis=1)   # per-site colour
    colour = sc.rgb[0].astype(np.float64) + cols[1]
    np.testing.assert_allclose(rgba[3], alpha, rtol=0, atol=2e-6)
    np.testing.assert_allclose(rgba[:3], alpha * colour, rtol=0, atol=2e-6)
    # the alternatives a plausible slip would give are far away
    assert np.abs(rgba[:3] - alpha * (sc.rgb[0] + cols[0])).max() > 0.05
    ell_wrong = math.sqrt(2.0) * (s1 - (5.0 + 0.1))
    assert abs(rgba[3] - (1.0 - math.exp(-sigma * ell_wrong))) > 0.05


def test_displacement_at_the_undisplaced_hit_by_dense_sampling():
    # Moderate tau = 20, three distinct detail-site positions (site 0, site 1,
    # and six coincident sites): delta is computed here by hand from the
    # soft-Voronoi weights at the undisplaced hit xbar (Eq. svdisp), the cell's
    # dense length is then measured by dense point sampling of
    # (x - p).n < delta along the ray (no interval formula), and compared with
    # the opacity the walk gives.
    pos = [[0.1, 0.0], [-0.1, 0.05]] + [[0.0, -0.2]] * 6
    disp = [0.25, -0.15] + [0.05] * 6
    tau = 20.0
    sc = _sites_scene(pos, disp, tau=tau, lam=-2.0)
    o = np.array([0.7, 0.3, 4.0])
    d = np.array([-0.1, 0.05, -1.0])
    cam = _cam_line(o, d)
    R0, D0, _ = oracle.generate_rays(cam)
    o64, d64 = R0.numpy(), D0.numpy()[0]
    # hand evaluation: xbar on z = 0, weights exp(-tau |ubar - s_k|) / sum
    tbar = -o64[2] / d64[2]
    ubar = (o64 + tbar * d64)[:2]
    s = sc.tex[0, :, 0:2].astype(np.float64)
    dk = sc.tex[0, :, 2].astype(np.float64)
    e = np.exp(-tau * np.linalg.norm(ubar[None, :] - s, axis=1))
    delta = float((e * dk).sum() / e.sum())
    assert min(abs(delta - v) for v in (0.25, -0.15, 0.05)) > 0.02   # a blend, not one site's value
    S = scene_tensors(sc)
    segs = oracle.dense_sample_ray(S, torch.tensor(o64), torch.tensor(d64), 8.0, 2e-5, delta={0: delta})
    (cell, inside, dense), = segs
    sigma = 10.0 * math.log1p(math.exp(float(sc.occ_logit[0])))
    alpha = oracle.render_walk(sc, cam)[0][3]
    ell_walk = -math.log1p(-alpha) / sigma
    assert cell == 0
    assert abs(ell_walk - dense) <= 1e-4
    # the displacement taken at the displaced hit instead, or none at all,
    # gives a dense length far outside the sampling error
    tx = (delta - o64[2]) / d64[2]
    ux = (o64 + tx * d64)[:2]
    ex = np.exp(-tau * np.linalg.norm(ux[None, :] - s, axis=1))
    delta_x = float((ex * dk).sum() / ex.sum())
    for wrong in (delta_x, 0.0):
        segw = oracle.dense_sample_ray(S, torch.tensor(o64), torch.tensor(d64), 8.0, 2e-5, delta={0: wrong})
        assert abs(segw[0][2] - dense) > 2e-3, wrong
