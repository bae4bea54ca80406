"""GPU parity of the training regularisers and statistics against the FP64
oracle (itself pinned in test_oracle_regularizers.py):
  * normal loss (weighted into the backward), sparsity through the A
    channel, per-cell contribution and the normal-loss value;
  * a store-mode state refuses a second backward;
  * connectivity loss over the sphere-overlap graph: value and gradients
    against brute force over all pairs."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from conftest import assert_grad_close

pytestmark = pytest.mark.gpu

PARAMS = ("p", "power", "radius", "normal", "occ_logit", "rgb", "tex")


def _flush(msg):
    print(msg, flush=True)


def _rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-30)


@pytest.mark.parametrize("lam_n,lam_s", [(0.7, 0.3), (2.0, 0.0)])
def test_normal_and_sparsity_losses_match_oracle(lam_n, lam_s):
    import paper_2604_24994_amd as pf
    _flush(f"case regularisers lambda_normal={lam_n} lambda_sparse={lam_s}: 200 sites, radius x3, 2 views")
    sc = W.scene_uniform(200, seed=0)
    sc.radius = (sc.radius * 3.0).astype(np.float32)
    eyes = W.random_eyes(2, 2.7, 30)
    cams = [W.pinhole(eyes[0], 20, 16, 60.0), W.pinhole(eyes[1], 18, 14, 70.0)]
    rng = np.random.default_rng(0)
    Gs = [rng.normal(size=(c.n_rays, 4)) for c in cams]
    params = {f: torch.tensor(getattr(sc, f), device="cuda", requires_grad=True) for f in PARAMS}
    scene = pf.build_scene(params, sigma_scale=sc.sigma_scale, tau=sc.tau)
    stats = {}
    imgs = pf.render_raster_diff(scene, cams, lambda_normal=lam_n, stats=stats)
    loss = sum((img.reshape(-1, 4) * torch.tensor(G, device="cuda", dtype=torch.float32)).sum() + lam_s * img[..., 3].sum()
               for img, G in zip(imgs, Gs))
    loss.backward()
    torch.cuda.synchronize()
    g_gpu = {f: params[f].grad.cpu().numpy().astype(np.float64) for f in PARAMS}
    g_ref = {f: np.zeros_like(g_gpu[f]) for f in PARAMS}
    contrib_ref = np.zeros(sc.n)
    normal_ref = 0.0
    for cam, G in zip(cams, Gs):
        gr, vals = oracle.regularized_gradients(sc, cam, G, lambda_normal=lam_n, lambda_sparse=lam_s)
        for f in PARAMS:
            g_ref[f] += gr[f].reshape(g_ref[f].shape)
        contrib_ref += vals["contribution"]
        normal_ref += vals["normal"]
    for f in PARAMS:
        assert_grad_close(g_gpu[f], g_ref[f], f, log=_flush)
    c = stats["contribution"].cpu().numpy().astype(np.float64)
    nl = float(stats["normal_loss"].cpu()[0])
    _flush(f"  contribution max err {np.abs(c - contrib_ref).max():.3e} (max {contrib_ref.max():.3f}); "
           f"normal loss {nl:.6f} vs {normal_ref:.6f}")
    assert np.abs(c - contrib_ref).max() <= 1e-5 * max(1.0, contrib_ref.max())
    assert abs(nl - normal_ref) <= 1e-5 * max(1.0, normal_ref)


def test_store_state_is_consumed_by_backward():
    import paper_2604_24994_amd as pf
    _flush("case consumed state")
    sc = W.scene_uniform(100, seed=1)
    scene = pf.build_scene(pf.to_device_params(sc), sigma_scale=sc.sigma_scale, tau=sc.tau)
    cam = W.pinhole(W.random_eyes(1, 3.0, 3)[0], 16, 12, 60.0)
    buf, state = pf.render_raster_state(scene, cam)
    grads = {f: torch.zeros_like(scene.params[f]) for f in PARAMS}
    d = torch.ones_like(buf)
    pf.backward(scene, state, d, grads)
    with pytest.raises(Exception, match="already used"):
        pf.backward(scene, state, d, grads)
    state.release()


@pytest.mark.parametrize("n,scale", [(400, 3.0), (1500, 2.0)])
def test_connect_loss_matches_brute_force(n, scale):
    import paper_2604_24994_amd as pf
    _flush(f"case connectivity loss: {n} sites, radius x{scale}")
    sc = W.scene_uniform(n, seed=2)
    sc.radius = (sc.radius * scale).astype(np.float32)
    scene = pf.build_scene(pf.to_device_params(sc), sigma_scale=sc.sigma_scale, tau=sc.tau)
    grads = {f: torch.zeros_like(scene.params[f]) for f in ("p", "radius")}
    val = pf.connect_loss(scene, 0.5, grads)
    torch.cuda.synchronize()
    L_ref, g_ref = oracle.connect_loss(sc, 0.5)
    L = float(val.cpu()[0])
    rp = _rel(grads["p"].cpu().numpy().astype(np.float64), g_ref["p"])
    rr = _rel(grads["radius"].cpu().numpy().astype(np.float64), g_ref["radius"])
    _flush(f"  loss {L:.6f} vs {L_ref:.6f}; grad p rel {rp:.3e}, radius rel {rr:.3e}")
    assert L_ref > 0 and abs(L - L_ref) <= 1e-5 * L_ref
    assert rp <= 1e-4 and rr <= 1e-4
