"""Work counters of the composite and the walk (pf_render_opts.counters)
against the oracle's own walk on a 1,024-cell scene (full 64x64 image).

The scene has low density (no ray gets near T = 1e-6, where the GPU stops
and the oracle does not) and a large domain box (nearly every ray leaves the box
inside the last cell it enters, where the oracle's walk ends too), so that
the GPU walk and the oracle walk the same cells: cells walked, pieces
(bounded intervals) and contributions (alpha > 0) are counted from the
oracle's records and compared with the counters.  The composite evaluates
the same pieces, so its contribution count equals the walk's."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from oracle.cell import scene_tensors, shade

pytestmark = pytest.mark.gpu


def _flush(msg):
    print(msg, flush=True)


def _oracle_counts(sc, cam):
    rgba, rec = oracle.walk_records(sc, cam)
    o, d, _ = oracle.generate_rays(cam)
    S = scene_tensors(sc)
    c = rec.cell
    with torch.no_grad():
        alpha, _, _ = shade(o, d[rec.ray], rec.lo, rec.hi, S["p"][c], S["normal"][c], S["occ_logit"][c],
                            S["rgb"][c], S["tex"][c], S["sigma_scale"], S["tau"])
    return rec.steps.numpy(), int(rec.cell.numel()), int((alpha > 0).sum()), rgba


def test_counters_match_the_oracle_walk():
    import paper_2604_24994_amd as pf
    _flush("case counters: 1024 sites (low density), 64x64 pinhole, box 30, raster and walk counters vs the oracle")
    sc, cam = W.c1_scene(), W.pinhole(W.random_eyes(1, 3.0, 1)[0], 64, 64, 60.0)
    sc.occ_logit = (sc.occ_logit - 4.0).astype(np.float32)
    scene = pf.build_scene(sc, box=((-30.0,) * 3, (30.0,) * 3))
    rc = torch.zeros(6, dtype=torch.int64, device="cuda")
    tc = torch.zeros(6, dtype=torch.int64, device="cuda")
    ras = pf.render_raster(scene, cam, counters=rc)[0]
    trc, trunc = pf.render_trace(scene, cam, counters=tc, return_truncated=True)
    torch.cuda.synchronize()
    rc, tc = rc.cpu().numpy(), tc.cpu().numpy()
    o_steps, o_pieces, o_contrib, o_rgba = _oracle_counts(sc, cam)
    _flush(f"  raster: tests {rc[0]}, hits {rc[1]}, contributions {rc[2]}, wave steps {rc[3]} / {rc[4]} / {rc[5]}")
    _flush(f"  walk: rays {tc[0]}, cells {tc[1]}, pieces {tc[2]}, contributions {tc[3]}, faces {tc[4]}, "
           f"max cells {tc[5]}")
    _flush(f"  oracle: cells {o_steps.sum()}, pieces {o_pieces}, contributions {o_contrib}, "
           f"max cells {o_steps.max()}, min T {1 - o_rgba[:, 3].max():.3e}")
    assert trunc == 0
    assert 1 - o_rgba[:, 3].max() > 1e-3          # no early termination anywhere
    img = trc[0].detach().cpu().numpy().reshape(-1, 4).astype(np.float64)
    assert np.abs(img - o_rgba).max() <= 1e-4
    assert tc[0] == cam.n_rays
    # beyond the box the oracle may still cross faces of far unbounded cells
    # (0.8% of its steps on this scene); inside it the walks are the same
    assert o_steps.sum() * 0.98 <= tc[1] <= o_steps.sum() and tc[5] <= o_steps.max()
    # pieces: the GPU computes one wherever the ray meets the cell's cull
    # ball; the oracle records the non-empty bounded intervals
    assert tc[2] >= o_pieces
    assert abs(int(tc[3]) - o_contrib) <= 2
    assert rc[2] == tc[3]
    assert rc[0] >= rc[1] >= rc[2] > 0
    assert rc[3] >= rc[4] >= rc[5] > 0
    assert rc[2] <= 64 * rc[5] and rc[1] <= 64 * rc[4]
    assert tc[4] > tc[1]
    # counters accumulate over the views of a call
    tc2 = torch.zeros(6, dtype=torch.int64, device="cuda")
    pf.render_trace(scene, [cam, cam], counters=tc2)
    tc2 = tc2.cpu().numpy()
    assert (tc2[:5] == 2 * tc[:5]).all() and tc2[5] == tc[5]
    scene.destroy()
