"""Parity at the 1,048,576-cell workload in the launch configuration of the
timed training step: 8 views of 1600x1066 rendered in one store-mode launch,
on a scene rebuilt in place after the sites moved by N(0, 1e-4), through the
autograd path.  Forward colours and backward gradients on 32 seeded pixels
per view (256 in all) are checked against the FP64 oracle, which walks every
sampled ray by brute force over all cells (one worker process per view)."""
import multiprocessing as mp
import time

import numpy as np
import pytest
import torch

import oracle
import workloads as W
from conftest import grad_errors, worst_component

pytestmark = pytest.mark.gpu
PARAMS = ("p", "power", "radius", "normal", "occ_logit", "rgb", "tex")
PER_VIEW = 32


def _flush(msg):
    print(msg, flush=True)


def _pixels(cam, n, seed):
    rng = np.random.default_rng(seed)
    xs = rng.integers(cam.width // 4, 3 * cam.width // 4, size=n)
    ys = rng.integers(cam.height // 4, 3 * cam.height // 4, size=n)
    return np.unique(ys * cam.width + xs)


def _moved_scene():
    sc = W.c3_scene()
    z = np.random.default_rng(13).standard_normal(sc.p.shape).astype(np.float32)
    sc.p = (sc.p + np.float32(1e-4) * z).astype(np.float32)
    return sc


def _oracle_view(args):
    """Oracle adjoint of one view's sampled pixels (runs in a worker
    process): gradients as (rows, values) of the cells they touch."""
    v, pix, G = args
    torch.set_num_threads(2)
    sc = _moved_scene()
    cam = W.c3_cameras(n_views=8)[v]
    t0 = time.time()
    gr, _, rec, _, rgba = oracle.adjoint_gradients(sc, cam, G, pix=pix, return_records=True)
    out = {}
    for f in PARAMS:
        g = gr[f].reshape(sc.n, -1)
        rows = np.nonzero(np.abs(g).max(axis=1))[0]
        out[f] = (rows, g[rows])
    return v, out, rgba, int(rec.cell.numel()), time.time() - t0


def test_c3_training_step_forward_and_gradients_on_sampled_pixels():
    import paper_2604_24994_amd as pf
    _flush(f"case C3 training step: 1,048,576 cells, 8 views 1600x1066, sites moved and rebuilt, "
           f"{PER_VIEW} seeded pixels per view")
    t0 = time.time()
    sc = W.c3_scene()
    cams = W.c3_cameras(n_views=8)
    params = {f: torch.tensor(getattr(sc, f), device="cuda", requires_grad=True) for f in PARAMS}
    scene = pf.build_scene(params, sigma_scale=sc.sigma_scale, tau=sc.tau)
    # the sites move as after an optimiser update; the adjacency is rebuilt
    # in place, seeded by the first build
    sc.p = _moved_scene().p
    with torch.no_grad():
        params["p"].copy_(torch.tensor(sc.p))
    pf.update_scene(scene, params)
    imgs = pf.render_raster_diff(scene, cams)
    rng = np.random.default_rng(4)
    picks, Gs, loss = [], [], 0.0
    for v, (c, im) in enumerate(zip(cams, imgs)):
        pix = _pixels(c, PER_VIEW, seed=100 + v)
        G = rng.normal(size=(len(pix), 4))
        sel = im.reshape(-1, 4)[torch.as_tensor(pix, device="cuda")]
        loss = loss + (sel * torch.tensor(G, dtype=torch.float32, device="cuda")).sum()
        picks.append(pix)
        Gs.append(G)
    loss.backward()
    torch.cuda.synchronize()
    _flush(f"  GPU done in {time.time() - t0:.1f}s")
    g_gpu = {f: params[f].grad.cpu().numpy().astype(np.float64) for f in PARAMS}
    got = [im.detach().reshape(-1, 4)[torch.as_tensor(p, device="cuda")].cpu().numpy().astype(np.float64)
           for im, p in zip(imgs, picks)]
    scene.destroy()
    g_ref = {f: np.zeros_like(g_gpu[f]).reshape(sc.n, -1) for f in PARAMS}
    t1 = time.time()
    with mp.get_context("spawn").Pool(8) as pool:
        for v, out, rgba, ncontrib, dt in pool.imap_unordered(_oracle_view, list(zip(range(8), picks, Gs))):
            err = np.abs(got[v] - rgba).max()
            _flush(f"  view {v}: oracle {dt:.1f}s, colour err {err:.3e}, contributions {ncontrib}")
            assert err <= 1e-4
            for f in PARAMS:
                rows, vals = out[f]
                g_ref[f][rows] += vals
    _flush(f"  oracle done in {time.time() - t1:.1f}s")
    # Per tensor: the 1e-3 bar.  Per component (an entry's error against
    # 1e-3 max(|ref entry|, 1e-2 |ref|_inf)): at this scale a few of the
    # millions of non-zero entries carry the FP32 rounding of derivatives far
    # larger than themselves (e.g. a cell behind 40 others whose opacity
    # derivative is scaled by 1/(d.n) of a nearly grazed dipole face); the
    # bar holds for all but 1e-5 of the non-zero entries (at least 10 may
    # exceed it), and every entry stays within 5e-3.
    failed = []
    for f in PARAMS:
        ref = g_ref[f].reshape(g_gpu[f].shape)
        t, c = grad_errors(g_gpu[f], ref)
        g1, r1 = g_gpu[f].reshape(-1), ref.reshape(-1)
        scale = np.abs(r1).max()
        nz = np.nonzero((r1 != 0) | (g1 != 0))[0]
        ratio = np.abs(g1[nz] - r1[nz]) / np.maximum(np.abs(r1[nz]), 1e-2 * scale)
        over = int((ratio > 1e-3).sum())
        i, gi, ri, _ = worst_component(g_gpu[f], ref)
        width = int(np.prod(g_gpu[f].shape[1:])) if g_gpu[f].ndim > 1 else 1
        _flush(f"  {f:10s} |ref|max {scale:.4e}  rel {t:.3e}  per-component {c:.3e}  entries over 1e-3: {over} of "
               f"{len(nz)}  (worst: cell {i // width} component {i % width}, GPU {gi:.6e} oracle {ri:.6e})")
        if not (scale > 0 and t <= 1e-3 and c <= 5e-3 and over <= max(10, 1e-5 * len(nz))):
            failed.append(f)
    assert not failed, failed
