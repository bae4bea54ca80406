"""Pin of the oracle adjoint: FP64 central differences of the full oracle
(walk re-run at each perturbed point, so every discrete decision is made
again from scratch) against the autograd replay.  Entries whose perturbation
changes any discrete decision of the walk are skipped (kinks)."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from oracle.adjoint import PARAMS


def _f64_scene(sc):
    return W.Scene(*(getattr(sc, f).astype(np.float64) for f in PARAMS),
                   sigma_scale=sc.sigma_scale, tau=sc.tau)


def _decisions(rec):
    return (rec.ray.tolist(), rec.cell.tolist(), rec.lo_kind.tolist(), rec.lo_j.tolist(),
            rec.hi_kind.tolist(), rec.hi_j.tolist())


@pytest.mark.parametrize("seed", [0, 1])
def test_adjoint_matches_central_differences(seed):
    sc = _f64_scene(W.scene_uniform(48, seed=seed))
    sc.radius *= 3.5
    cam = W.pinhole(W.random_eyes(1, 2.6, 40 + seed)[0], 7, 6, 60.0)
    rng = np.random.default_rng(seed)
    G = rng.normal(size=(cam.n_rays, 4))
    grads, L0, rec, _, _ = oracle.adjoint_gradients(sc, cam, G, return_records=True)
    base = _decisions(rec)
    used = np.unique(rec.cell.numpy())
    checked = {k: 0 for k in PARAMS}
    for name in PARAMS:
        arr = getattr(sc, name)
        flat_idx = []
        for c in used[:12]:
            per_cell = int(np.prod(arr.shape[1:])) if arr.ndim > 1 else 1
            offs = rng.choice(per_cell, size=min(per_cell, 3), replace=False)
            flat_idx += [c * per_cell + int(o) for o in offs]
        for fi in flat_idx:
            h = 1e-6 * max(1.0, abs(arr.flat[fi]))
            vals = []
            ok = True
            for sgn in (1, -1):
                sp = sc.copy()
                getattr(sp, name).flat[fi] += sgn * h
                rgba, r2 = oracle.walk_records(sp, cam)
                if _decisions(r2) != base:
                    ok = False
                    break
                vals.append(oracle.loss_from_rgba(rgba, G))
            if not ok:
                continue
            fd = (vals[0] - vals[1]) / (2 * h)
            g = grads[name].flat[fi]
            assert abs(fd - g) <= 1e-6 * max(1.0, abs(g)), (name, fi, fd, g)
            checked[name] += 1
    for name in PARAMS:
        assert checked[name] > 0, checked
    # gradients reach neighbours through binding planes
    assert np.abs(grads["power"]).max() > 0


def test_adjoint_replay_reproduces_forward():
    sc = W.scene_uniform(200, seed=4)
    sc.radius *= 3.0
    cam = W.pinhole(W.random_eyes(1, 2.8, 5)[0], 12, 12, 60.0)
    G = np.ones((cam.n_rays, 4))
    _, _, rec, replay, fwd = oracle.adjoint_gradients(sc, cam, G, return_records=True)
    assert np.abs(replay - fwd).max() < 1e-12
