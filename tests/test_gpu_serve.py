"""Serving: continuous batching over a resident scene returns, for every
request, the image of that camera rendered alone (bitwise), admits work by
the HBM budget, and batches requests that arrive while others run."""
import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu


def _flush(msg):
    print(msg, flush=True)


def _mixed_requests(n, seed):
    rng = np.random.default_rng(seed)
    res = [(64, 64), (96, 54), (128, 128), (160, 90)]
    out = []
    for i in range(n):
        w, h = res[int(rng.integers(0, len(res)))]
        eye = W.unit_vectors(rng, 1)[0] * 3.0
        cam = W.fisheye(eye, w, h) if rng.uniform() < 0.3 else W.pinhole(eye, w, h)
        out.append(W.Request(arrival_s=0.002 * i, camera=cam, scene_id=0))
    return out


@pytest.mark.parametrize("budget_mb,expect_batching", [(2048, True), (1, False)])
def test_results_equal_alone_and_in_mix(budget_mb, expect_batching):
    """budget 1 MB is raised to the largest single request: then at most
    that many bytes are ever in flight, whatever the batching."""
    import paper_2604_24994_amd as pf
    from paper_2604_24994_amd import serve
    _flush(f"case serve budget={budget_mb}MB")
    sc = W.scene_uniform(3000, seed=2)
    scene = pf.build_scene(sc)
    reqs = _mixed_requests(40, seed=budget_mb)
    alone = [pf.render_raster(scene, r.camera)[0].clone() for r in reqs]
    torch.cuda.synchronize()
    budget = budget_mb << 20
    if budget < max(serve.request_bytes(scene, r.camera) for r in reqs):
        budget = max(serve.request_bytes(scene, r.camera) for r in reqs)   # one request at a time
    srv = serve.Server({0: scene}, hbm_budget_bytes=budget, n_workers=2)
    base = pf.memory_stats(reset_peak=True)
    try:
        futs = [srv.submit(0, r.camera) for r in reqs]
        imgs = [f.result(timeout=120) for f in futs]
    finally:
        srv.close()
    torch.cuda.synchronize()
    lib_peak = pf.memory_stats()["peak"] - base["live"]
    sizing = max(serve.request_bytes(scene, r.camera) for r in reqs)
    _flush(f"  library device memory in flight at most {lib_peak} B; budget {budget} B, "
           f"admitted at most {srv.peak_inflight} B")
    # the library's own device requests never exceeded the admitted bounds
    # (the images are the caller's tensors, also inside the bounds), plus the
    # sizing query of the one request being admitted (bounded like it)
    assert lib_peak <= srv.peak_inflight + sizing
    assert srv.peak_inflight <= budget
    for a, b in zip(alone, imgs):
        assert torch.equal(a, b)
    _flush(f"  batches {srv.batches}")
    assert sum(srv.batches) == len(reqs)
    assert srv.peak_inflight <= budget
    if expect_batching:
        assert max(srv.batches) > 1


def test_plain_server_matches():
    import paper_2604_24994_amd as pf
    from paper_2604_24994_amd import serve
    sc = W.scene_uniform(1500, seed=4)
    scene = pf.build_scene(sc)
    reqs = _mixed_requests(10, seed=9)
    srv = serve.PlainServer({0: scene})
    try:
        stats = serve.replay(srv, reqs)
    finally:
        srv.close()
    assert stats["requests"] == 10 and stats["p99_ms"] >= stats["p50_ms"] > 0
