"""Writes the stored expected colours of the sampled-pixel parity tests.

Every value here comes from the FP64 oracle (``oracle.render_walk``: start
cell by argmin power distance over all sites, each exit by brute force over
every bisector plane, Sec. 3.1 exact segment sum) on the seeded synthetic
scenes of ``workloads``; nothing comes from the GPU path.  A full frame at
these sizes is out of the oracle's reach (it is O(N) per walk step), so the
fixtures hold seeded pixels spread over the whole image:

* ``c2_pinhole.npz``: 4,096 pixels of the 1280x720 pinhole (60 degrees) on
  the 262,144-cell mixture scene;
* ``c2_fisheye.npz``: 4,096 pixels of the 1024x1024 180-degree equidistant
  fisheye at the same pose (Appendix D: the fisheye is rendered without
  approximation, so each of its rays is compared with the oracle's);
* ``c3_views.npz``: 32 pixels in each of the 8 views of 1600x1066 on the
  1,048,576-cell scene after its sites moved by ``1e-4 N(0, I)`` (seed 13),
  the scene of the timed training step's parity test.

Each file holds ``view`` (int32), ``pix`` (int64, row-major), ``rgba``
(float64 [n, 4]) and the recipe as a string.  Usage:

    python tests/golden/make_golden.py [c2_pinhole c2_fisheye c3_views] [--workers K]

The rays are split over worker processes (fork; one torch thread each).
"""
from __future__ import annotations

import argparse
import multiprocessing as mp
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads as W  # noqa: E402

C3_MOVE_SEED = 13
C3_MOVE_SCALE = 1e-4

# name -> (pixels per view, pixel seed base)
SETS = {
    "c2_pinhole": (4096, 41),
    "c2_fisheye": (4096, 42),
    "c3_views": (32, 43),
}

_G = {}   # scene tensors and cameras, shared with forked workers


def c3_moved_scene():
    """The 1,048,576-cell scene with its sites moved as after an optimiser
    update (float32 sum, as the GPU test forms it)."""
    sc = W.c3_scene()
    z = np.random.default_rng(C3_MOVE_SEED).standard_normal(sc.p.shape).astype(np.float32)
    sc.p = (sc.p + np.float32(C3_MOVE_SCALE) * z).astype(np.float32)
    return sc


def cases(name):
    """(scene, [(view, camera, pixels)]) of a fixture set."""
    per_view, seed = SETS[name]
    if name == "c3_views":
        cams = W.c3_cameras(n_views=8)
        return c3_moved_scene(), [(v, c, W.pixel_sample(c, per_view, seed + 100 * v)) for v, c in enumerate(cams)]
    cam, fish = W.c2_cameras()
    c = cam if name == "c2_pinhole" else fish
    return W.c2_scene(), [(0, c, W.pixel_sample(c, per_view, seed))]


def _work(item):
    view, pix = item
    import torch
    torch.set_num_threads(1)
    cam = _G["cams"][view]
    return view, pix, oracle.render_walk(_G["scene"], cam, pix=pix, chunk_elems=1 << 22, S=_G["S"])


def make(name, workers, chunk=16):
    t0 = time.time()
    scene, views = cases(name)
    _G["scene"] = scene
    _G["S"] = oracle.scene_tensors(scene)
    _G["cams"] = {v: c for v, c, _ in views}
    items = [(v, pix[i:i + chunk]) for v, _, pix in views for i in range(0, len(pix), chunk)]
    out = {}
    done = 0
    with mp.get_context("fork").Pool(workers) as pool:
        for view, pix, rgba in pool.imap_unordered(_work, items):
            for p, c in zip(pix, rgba):
                out[(view, int(p))] = c
            done += len(pix)
            print(f"{name}: {done}/{sum(len(p) for _, _, p in views)} rays, {time.time() - t0:.0f} s", flush=True)
    keys = sorted(out)
    view = np.array([k[0] for k in keys], dtype=np.int32)
    pix = np.array([k[1] for k in keys], dtype=np.int64)
    rgba = np.stack([out[k] for k in keys]).astype(np.float64)
    recipe = (f"{name}: oracle.render_walk (FP64 brute-force walk) on workloads "
              f"{'c3_scene() moved by 1e-4 N(0,I) seed 13, c3_cameras(8)' if name == 'c3_views' else 'c2_scene(), c2_cameras()'}"
              f"; pixels workloads.pixel_sample(cam, {SETS[name][0]}, seed {SETS[name][1]}"
              f"{' + 100 view' if name == 'c3_views' else ''})")
    path = os.path.join(HERE, name + ".npz")
    np.savez_compressed(path, view=view, pix=pix, rgba=rgba, recipe=np.array(recipe))
    print(f"wrote {path}: {len(pix)} pixels in {time.time() - t0:.0f} s", flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("names", nargs="*", default=list(SETS))
    ap.add_argument("--workers", type=int, default=os.cpu_count())
    a = ap.parse_args()
    for n in a.names:
        make(n, a.workers)


if __name__ == "__main__":
    main()
