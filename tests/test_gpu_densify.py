"""GPU parity of densification and pruning (Sec. 3.5) against the FP64
oracle (pinned in test_oracle_densify.py): the per-cell error statistic of
the backward, the moving average, and the densify/prune update."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W

pytestmark = pytest.mark.gpu


def _flush(msg):
    print(msg, flush=True)


@pytest.mark.parametrize("walk", [False, True])
def test_error_statistic_matches_oracle(walk):
    import paper_2604_24994_amd as pf
    _flush(f"case error statistic walk={walk}: 200 sites, radius x3, 2 views")
    sc = W.scene_uniform(200, seed=2)
    sc.radius = (sc.radius * 3.0).astype(np.float32)
    eyes = W.random_eyes(2, 2.7, 40)
    cams = [W.pinhole(eyes[0], 20, 16, 60.0), W.pinhole(eyes[1], 18, 14, 70.0)]
    rng = np.random.default_rng(4)
    errs = [rng.uniform(0, 2, c.n_rays) for c in cams]
    params = {f: torch.tensor(getattr(sc, f), device="cuda", requires_grad=True)
              for f in ("p", "power", "radius", "normal", "occ_logit", "rgb", "tex")}
    box = (np.min([c.c2w[:, 3] for c in cams], 0), np.max([c.c2w[:, 3] for c in cams], 0))
    scene = pf.build_scene(params, sigma_scale=sc.sigma_scale, tau=sc.tau, box=box)
    stats = {"pixel_error": torch.tensor(np.concatenate(errs), dtype=torch.float32, device="cuda")}
    fn = pf.render_trace_diff if walk else pf.render_raster_diff
    imgs = fn(scene, cams, stats=stats)
    sum(im.sum() for im in imgs).backward()
    torch.cuda.synchronize()
    got = stats["error"].cpu().numpy().astype(np.float64)
    ref = sum(oracle.cell_error(sc, c, e.astype(np.float32)) for c, e in zip(cams, errs))
    err = np.abs(got - ref).max()
    _flush(f"  max err {err:.3e} (max {ref.max():.3f}, {int((ref > 0).sum())} cells)")
    assert (ref > 0).sum() > 20
    assert err <= 1e-5 * max(1.0, ref.max())


def test_moving_average_matches_oracle():
    import paper_2604_24994_amd as pf
    _flush("case ema")
    rng = np.random.default_rng(7)
    e = rng.uniform(0, 1, 10000).astype(np.float32)
    g = torch.tensor(e, device="cuda")
    for k in range(3):
        v = rng.uniform(0, 3, e.size).astype(np.float32)
        e = oracle.ema(e, v, 0.95)
        pf.ema_update(g, torch.tensor(v, device="cuda"), 0.95)
    assert np.array_equal(g.cpu().numpy(), e)


def _check_draws(parents_gpu, parents_ref, err, keep, u):
    """Parents agree, except where u * total lies within rounding of a
    cumulative-weight boundary (the two sides sum in different orders)."""
    diff = np.nonzero(parents_gpu != parents_ref)[0]
    if diff.size:
        cdf = np.cumsum(err[keep].astype(np.float64))
        x = u.astype(np.float64) * cdf[-1]
        gap = np.abs(cdf[None, :] - x[diff, None]).min(axis=1)
        assert (gap <= 1e-12 * cdf[-1]).all(), diff
    return diff.size


@pytest.mark.parametrize("n,n_new,q", [(5000, 777, 0.3), (1048576, 10486, 0.1)])
def test_densify_prune_matches_oracle(n, n_new, q):
    import paper_2604_24994_amd as pf
    _flush(f"case densify n={n} n_new={n_new} prune quantile {q}")
    sc = W.scene_uniform(n, seed=9) if n <= 5000 else W.c3_scene()
    rng = np.random.default_rng(10)
    err = (rng.uniform(0, 1, n) ** 4).astype(np.float32)
    err[rng.uniform(0, 1, n) < 0.2] = 0.0
    contrib = rng.exponential(1.0, n).astype(np.float32)
    below = float(np.quantile(contrib, q))
    u = rng.uniform(0, 1, n_new).astype(np.float32)
    delta = rng.standard_normal((n_new, 3)).astype(np.float32)
    ref, re, rc, rpar = oracle.densify_prune(sc, err, contrib, u, delta, below, 0.5)
    out, ge, gc, gpar = pf.densify_prune(pf.to_device_params(sc), torch.tensor(err), torch.tensor(contrib),
                                         torch.tensor(u), torch.tensor(delta), below, 0.5)
    torch.cuda.synchronize()
    keep = contrib >= np.float32(below)
    nk = int(keep.sum())
    assert out["p"].shape[0] == ref["p"].shape[0] == nk + n_new
    gpar = gpar.cpu().numpy().astype(np.int64)
    nd = _check_draws(gpar, rpar, err, keep, u)
    _flush(f"  kept {nk}, drawn {n_new}, parents differing at a boundary: {nd}")
    same = np.concatenate([np.arange(nk), nk + np.nonzero(gpar == rpar)[0]])
    for f in ("p", "power", "radius", "normal", "occ_logit", "rgb", "tex"):
        assert np.array_equal(out[f].cpu().numpy()[same], ref[f][same]), f
    assert np.array_equal(ge.cpu().numpy()[same], re[same]) and np.array_equal(gc.cpu().numpy()[same], rc[same])


def test_densify_edge_cases_and_rebuild():
    import paper_2604_24994_amd as pf
    _flush("case densify edges")
    sc = W.scene_uniform(300, seed=12)
    d = pf.to_device_params(sc)
    ones = torch.ones(300)
    u = torch.rand(5)
    delta = torch.randn(5, 3)
    # everything pruned: nothing kept, nothing drawn
    out, _, _, par = pf.densify_prune(d, ones, torch.zeros(300), u, delta, 0.5, 0.5)
    assert out["p"].shape[0] == 0 and par.numel() == 0
    # zero total error: kept cells only
    out, _, _, par = pf.densify_prune(d, torch.zeros(300), ones, u, delta, 0.5, 0.5)
    assert out["p"].shape[0] == 300 and par.numel() == 0
    # a normal update builds and renders
    out, _, _, par = pf.densify_prune(d, ones, ones, u, delta, 0.5, 0.5)
    assert out["p"].shape[0] == 305 and par.numel() == 5
    scene = pf.build_scene(out, sigma_scale=sc.sigma_scale, tau=sc.tau)
    img = pf.render_raster(scene, W.pinhole(W.random_eyes(1, 3.0, 5)[0], 32, 24, 60.0))[0]
    assert torch.isfinite(img).all() and float(img[..., 3].max()) > 0.1
