#!/usr/bin/env python
"""Throughput benchmark on one MI355X.

Workload: 1,048,576 cells (80% on 64 flattened Gaussians, 20% in a background
shell), 8 pinhole views of 1600x1066 on random poses on a sphere of radius 4,
FP32, synthetic seeded inputs resident in HBM before timing starts.

One step = rebuild the scene's adjacency (pf_build_scene) and rasterise the 8
views (pf_render_raster); with ``--backward`` (once available) the step also
takes the L2 loss against seeded noise targets and runs pf_backward.
Prints ONE JSON line (see ``main``).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np
import torch

HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--cells", type=int, default=1048576)
    ap.add_argument("--views", type=int, default=8)
    ap.add_argument("--width", type=int, default=1600)
    ap.add_argument("--height", type=int, default=1066)
    ap.add_argument("--cpu-rays", type=int, default=4, help="oracle sample size for the CPU baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--verbose", action="store_true")
    return ap.parse_args()


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def cpu_baseline(sc, cam, n_rays: int):
    """The FP64 oracle (walk form) on ``n_rays`` seeded central pixels of one
    view, timed on this host's cores."""
    import oracle
    from oracle.cell import scene_tensors
    rng = np.random.default_rng(11)
    xs = rng.integers(cam.width // 4, 3 * cam.width // 4, size=n_rays)
    ys = rng.integers(cam.height // 4, 3 * cam.height // 4, size=n_rays)
    pix = np.unique(ys * cam.width + xs)
    S = scene_tensors(sc)
    t0 = time.perf_counter()
    oracle.render_walk(sc, cam, pix=pix, S=S, chunk_elems=1 << 24)
    dt = time.perf_counter() - t0
    return {"value": len(pix) / dt / 1e6, "unit": "Mrays/s", "cores": torch.get_num_threads(),
            "kind": "oracle",
            "sample": f"{len(pix)} seeded central pixels of view 0 at {sc.n} cells, FP64 brute-force walk, {dt:.1f} s"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the multi-GPU layout is described in DESIGN.md)", file=sys.stderr)
        sys.exit(2)
    import workloads as W
    import paper_2604_24994_amd as pf
    from paper_2604_24994_amd import _lib

    t0 = time.time()
    sc = W.c3_scene(n=args.cells)
    cams = W.c3_cameras(n_views=args.views, width=args.width, height=args.height)
    log(f"inputs generated in {time.time() - t0:.1f}s")
    params = pf.to_device_params(sc)
    rays = sum(c.n_rays for c in cams)
    out = torch.empty(4 * rays, dtype=torch.float32, device="cuda")
    stream = torch.cuda.current_stream()

    def step():
        scene = pf.build_scene(params, sigma_scale=sc.sigma_scale, tau=sc.tau, stream=stream)
        pf.render_raster(scene, cams, stream=stream, out=out)
        return scene

    for i in range(args.warmup):
        s = step()
        torch.cuda.synchronize()
        if i == 0:
            info = s.info()
            log(f"scene: {info}")
        s.destroy()
    log("warmup done")

    _lib.profile_enable(True)
    _lib.profile_read()
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(args.steps):
        s = step()
        s.destroy()
    ev1.record(stream)
    torch.cuda.synchronize()
    prof = _lib.profile_read()
    _lib.profile_enable(False)
    ms = ev0.elapsed_time(ev1) / args.steps
    value = rays / (ms * 1e-3) / 1e6
    log(f"step {ms:.2f} ms, kernels: " + ", ".join(f"{k}={v[1] / max(1, v[0]):.3f}ms x{v[0]}" for k, v in prof.items()))

    dom = max(prof.items(), key=lambda kv: kv[1][1]) if prof else ("none", (1, 0.0))
    roof = {"kernel": dom[0], "bound": "hbm", "achieved": None, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": None, "traffic": None,
            "avg_ms": dom[1][1] / max(1, dom[1][0])}
    res = {
        "metric": "Mrays/s fwd at 1M cells (raster, adjacency rebuilt every step)",
        "value": round(value, 3),
        "unit": "Mrays/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{args.cells} cells, {args.views} pinhole views {args.width}x{args.height}, "
                               "build + raster forward",
                   "cells": args.cells, "views": args.views, "width": args.width, "height": args.height},
        "kernels_ms": {k: round(v[1] / max(1, v[0]), 4) for k, v in prof.items()},
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        log("timing the oracle sample on the host CPU")
        res["cpu_baseline"] = cpu_baseline(sc, cams[0], args.cpu_rays)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
