"""The 4,194,304-cell workload: a training step (4 views 2048x1365, the
forward replayed inside the backward instead of stored) runs while a server
renders requests on four resident scenes of 0.5M, 1M, 2M and 4M cells.
Checks: the step's library memory stays a few GiB (no stored contribution
records), its colours equal the FP64 oracle on sampled pixels, the training
gradients equal those of the same step run alone, and every served image
equals a render of that camera alone; raster and walk agree on sampled
pixels of the training views.  Timings are printed."""
import multiprocessing as mp
import threading
import time

import numpy as np
import pytest
import torch

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

FIELDS = ("p", "power", "radius", "normal", "occ_logit", "rgb", "tex")


def _flush(msg):
    print(msg, flush=True)


def _train_step(pf, params, sc, cams, tgt):
    scene = pf.build_scene(params, sigma_scale=sc.sigma_scale, tau=sc.tau)
    for v in params.values():
        v.grad = None
    imgs = pf.render_raster_diff(scene, cams, state_mode=pf.RECOMPUTE)
    rgb = torch.cat([im.reshape(-1, 4)[:, :3] for im in imgs])
    ((rgb - tgt) ** 2).mean().backward()
    torch.cuda.synchronize()
    grads = {f: params[f].grad.clone() for f in FIELDS}
    return scene, imgs, grads


def _oracle_pixels(args):
    """FP64 oracle colours of sampled pixels of one training view (runs in
    a worker process)."""
    c, pix = args
    torch.set_num_threads(4)
    sc = W.c3_scene(n=4194304)
    cam = W.c3_cameras(n_views=4, width=2048, height=1365)[c]
    return c, oracle.render_walk(sc, cam, pix=pix)


def test_c5_training_while_serving():
    import paper_2604_24994_amd as pf
    from paper_2604_24994_amd import serve
    t0 = time.time()
    _flush("case C5: generating 4,194,304 training cells and serving scenes of 0.5M, 1M, 2M, 4M cells")
    sc = W.c3_scene(n=4194304)
    cams = W.c3_cameras(n_views=4, width=2048, height=1365)
    tgt = torch.cat([torch.as_tensor(t, device="cuda").reshape(-1, 3) for t in W.targets(cams)])
    params = {k: v.requires_grad_(True) for k, v in pf.to_device_params(sc).items()}
    sizes = (524288, 1048576, 2097152, 4194304)
    serve_scenes = {}
    for i, n in enumerate(sizes):
        s = W.c3_scene(seed=10 + i, n=n)
        serve_scenes[i] = pf.build_scene(s, sigma_scale=s.sigma_scale, tau=s.tau)
        del s
    torch.cuda.synchronize()
    _flush(f"  inputs ready in {time.time() - t0:.1f}s; "
           f"HBM in use {torch.cuda.memory_allocated() / 2**30:.1f} GiB (torch)")

    # the step alone; the recompute-mode backward keeps no records between
    # forward and backward and replays the forward in windows of at most
    # 2 GiB of records, so the library's own memory stays a few GiB
    t1 = time.time()
    pf.memory_stats(reset_peak=True)
    scene, imgs, g_alone = _train_step(pf, params, sc, cams, tgt)
    peak = pf.memory_stats()["peak"]
    _flush(f"  training step alone: {time.time() - t1:.2f}s; library memory peak {peak / 2**30:.2f} GiB")
    assert peak < 6 * 2**30
    # colours of the step's raster against the oracle on 2 seeded pixels per view
    picks = [W.pixel_sample(cam, 2, seed=40 + c) for c, cam in enumerate(cams)]
    with mp.get_context("spawn").Pool(4) as pool:
        for c, ref in pool.imap_unordered(_oracle_pixels, [(c, p) for c, p in enumerate(picks)]):
            got = imgs[c].detach().reshape(-1, 4)[torch.as_tensor(picks[c], device="cuda")].cpu().numpy()
            err = float(np.abs(got.astype(np.float64) - ref).max())
            _flush(f"  view {c}: colour err vs oracle {err:.2e} (A {ref[:, 3].round(3).tolist()})")
            assert err <= 1e-4
    # raster and walk agree on sampled pixels of the views
    for c, (cam, img) in enumerate(zip(cams, imgs)):
        trc = pf.render_trace(scene, cam, max_steps=8192)[0]
        pix = W.pixel_sample(cam, 4096, seed=c)
        a = img.detach().reshape(-1, 4)[pix]
        b = trc.reshape(-1, 4)[pix]
        assert float((a - b).abs().max()) <= 1e-4
    scene.destroy()

    # requests at 100 req/s over the four scenes, the mixed resolutions and
    # cameras, submitted at their arrival times while the step runs
    reqs = W.request_stream(100.0, 2.0, seed=5, n_scenes=4)
    srv = serve.Server(serve_scenes, hbm_budget_bytes=24 << 30, n_workers=2)
    futs = []

    def submit_all():
        start = time.perf_counter()
        for r in reqs:
            due = start + r.arrival_s
            now = time.perf_counter()
            if due > now:
                time.sleep(due - now)
            futs.append(srv.submit(r.scene_id, r.camera, arrival=due))

    th = threading.Thread(target=submit_all)
    try:
        th.start()
        time.sleep(0.2)
        t2 = time.time()
        scene, _, g_mix = _train_step(pf, params, sc, cams, tgt)
        t_mix = time.time() - t2
        th.join(timeout=120)
        assert not th.is_alive()
        served = [f.result(timeout=300) for f in futs]
    finally:
        srv.close()
    scene.destroy()
    lat = np.array(srv.latencies) * 1e3
    _flush(f"  training step beside serving: {t_mix:.2f}s; served {len(reqs)} requests: "
           f"p50 {np.percentile(lat, 50):.0f} ms, p99 {np.percentile(lat, 99):.0f} ms")

    # atomics add in a different order: equal up to float32 rounding
    for f in FIELDS:
        a, b = g_alone[f], g_mix[f]
        rel = float((a - b).abs().max()) / max(float(a.abs().max()), 1e-30)
        _flush(f"  grad {f:10s} alone vs beside serving: rel {rel:.2e}")
        assert rel <= 1e-5, f

    # every image served beside the training step equals the camera rendered alone
    for r, img in zip(reqs, served):
        alone = pf.render_raster(serve_scenes[r.scene_id], r.camera)[0]
        assert torch.equal(alone, img)
    _flush(f"  {len(reqs)} served images equal their renders alone; total {time.time() - t0:.1f}s")
