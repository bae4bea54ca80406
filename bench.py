#!/usr/bin/env python
"""Throughput benchmark on one MI355X.

Workload: 1,048,576 cells (80% on 64 flattened Gaussians, 20% in a background
shell), 8 pinhole views of 1600x1066 on random poses on a sphere of radius 4,
FP32, synthetic seeded inputs resident in HBM before timing starts.

One step (default ``--mode train``) = one training iteration: rebuild the
scene's adjacency from the current parameters (pf_build_scene), rasterise the
8 views with a forward state (pf_render_raster), take the L2 loss against
seeded U(0,1) noise targets in torch, and run the backward (pf_backward via
torch.autograd) into zeroed gradient buffers.  ``--mode fwd`` times build +
forward only.  The JSON line also carries forward-only and ray-walk
throughput and, with ``--serve-seconds``, serving latency of a Poisson
request stream (batched server vs one call per request) on the same scene.
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
FP32_PEAK_TFLOPS = 157.3          # published MI355X FP32 vector peak (packed FMA)
# Algorithmic floating-point work per contribution (a pixel-cell pair with
# alpha > 0), counted from the model's formulas with FMA = 2 and exp, sqrt,
# reciprocal = 1: local frame 19 (FP64), sphere interval 3, 15 bisector
# faces x 14, camera clip 1, face frame 12, projections 30, soft-Voronoi set
# for the displacement 189 + split/opacity 33, radiance (a second soft-Voronoi
# set 189 + 8 detail sites x 128 for the Spherical-Voronoi blend) 1,027,
# compositing 9: about 1,700.  The backward recomputes the forward and runs
# its adjoint at twice the forward's work (reverse-mode ratio): 5,100.
FLOPS_FWD_PER_CONTRIB = 1700
FLOPS_BWD_PER_CONTRIB = 5100

# HBM bytes per launch on this workload (1,048,576 cells, 8 views 1600x1066)
# from rocprofv3 --pmc FETCH_SIZE and WRITE_SIZE (KiB per dispatch), scaled
# by what the same counters read for a 1 GiB device-to-device copy
# (FETCH_SIZE reads 0.5 GiB: x2.0; WRITE_SIZE reads 1 GiB: x1.0).  Valid only
# for the kernel sources with these hashes; otherwise the bench reports null.
FETCH_SCALE, WRITE_SCALE = 2.0, 1.0
_SRC_SHADE = {"pf_shade.hpp": "fafcd449bb434a34", "pf_internal.hpp": "cf1b6d1fee18a09d",
              "pf_record.hpp": "d8db4e8267ff8479"}
TRAFFIC = {
    "k_bwd_cell": {"fetch_kib": 7865870.9, "write_kib": 2407941.7,
                   "sources": {"pf_backward.hip": "fb3e4556d9e14fb8", **_SRC_SHADE}},
    "k_raster_store": {"fetch_kib": 17647219.1, "write_kib": 11375718.7,
                       "sources": {"pf_render.hip": "1e3097ce83ad03bf", **_SRC_SHADE}},
    "k_trace": {"fetch_kib": 8362805.2, "write_kib": 46637.5,
                "sources": {"pf_render.hip": "1e3097ce83ad03bf", **_SRC_SHADE}},
    "k_clip": {"fetch_kib": 409452.2, "write_kib": 180425.5,
               "sources": {"pf_build.hip": "60ddab952277c61e", "pf_internal.hpp": "cf1b6d1fee18a09d",
                           "pf_record.hpp": "d8db4e8267ff8479"}},
}


def traffic_bytes(kernel: str):
    """Measured HBM bytes per launch of ``kernel`` if its sources are the
    ones the counters were taken on, else None."""
    import hashlib
    t = TRAFFIC.get(kernel)
    if t is None:
        return None
    csrc = os.path.join(ROOT, "paper_2604_24994_amd", "csrc")
    for f, h in t["sources"].items():
        with open(os.path.join(csrc, f), "rb") as fh:
            if hashlib.sha256(fh.read()).hexdigest()[:16] != h:
                return None
    return int(1024 * (FETCH_SCALE * t["fetch_kib"] + WRITE_SCALE * t["write_kib"]))


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--cells", type=int, default=1048576)
    ap.add_argument("--views", type=int, default=8)
    ap.add_argument("--width", type=int, default=1600)
    ap.add_argument("--height", type=int, default=1066)
    ap.add_argument("--mode", choices=["train", "fwd"], default="train")
    ap.add_argument("--serve-seconds", type=float, default=30.0, help="measured serving window (after the warm-up)")
    ap.add_argument("--serve-warmup", type=float, default=2.0, help="serving warm-up excluded from the statistics")
    ap.add_argument("--serve-rate", type=float, default=200.0)
    ap.add_argument("--recompute-steps", type=int, default=2,
                    help="recompute-mode training steps timed beside the store-mode ones (0: skip)")
    ap.add_argument("--cpu-rays", type=int, default=32,
                    help="oracle sample size for the CPU baseline (about 16 s per ray and core)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-densify", action="store_true", help="skip the densify/prune side measurement")
    ap.add_argument("--steiner-cand", type=int, default=-1,
                    help="Steiner side measurement: candidates per round (-1: cells / 16, 0: skip)")
    ap.add_argument("--verbose", action="store_true")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only copy MIB MiB device to device once (reference for the HBM byte counters) and exit")
    return ap.parse_args()


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


_ORACLE = {}   # scene tensors and cameras shared with forked oracle workers


def _oracle_rays(item):
    import oracle
    torch.set_num_threads(1)
    v, pix = item
    oracle.render_walk(_ORACLE["scene"], _ORACLE["cams"][v], pix=pix, S=_ORACLE["S"], chunk_elems=1 << 22)
    return len(pix)


def _oracle_timed(sc, cams, items, procs: int) -> float:
    """Seconds for the oracle to walk the (view, pixels) items on ``procs``
    forked worker processes of one torch thread each."""
    import multiprocessing as mp
    from oracle.cell import scene_tensors
    _ORACLE.update(scene=sc, cams=cams, S=scene_tensors(sc))
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(procs) as pool:
        sum(pool.map(_oracle_rays, items, chunksize=1))
    return time.perf_counter() - t0


def cpu_baseline(sc, cams, n_rays: int, c1: bool = True):
    """The FP64 oracle (walk form, as written) on a bounded seeded sample of
    the bench workload, timed on all host cores (one worker process per core,
    rays split between them), plus the full 128x128 image of the 1,024-cell
    scene."""
    import workloads as W
    procs = min(os.cpu_count() or 1, 16)
    n_rays = max(n_rays, procs)
    per = max(1, n_rays // len(cams))
    items = []
    for v, c in enumerate(cams):
        pix = W.pixel_sample(c, per, 11 + v)
        items += [(v, pix[i:i + 1]) for i in range(len(pix))]
    items = items[:n_rays]
    dt = _oracle_timed(sc, cams, items, procs)
    res = {"value": len(items) / dt / 1e6, "unit": "Mrays/s", "cores": procs, "kind": "oracle",
           "cpu": cpu_model(), "host_cpus": os.cpu_count(),
           "sample": f"{len(items)} seeded pixels over the {len(cams)} views at {sc.n} cells, FP64 brute-force walk "
                     f"(O(cells) per step), {procs} worker processes, {dt:.1f} s"}
    if c1:
        sc1, cam1 = W.c1_scene(), W.c1_camera()
        rows = [(0, np.arange(y * cam1.width, (y + 1) * cam1.width)) for y in range(cam1.height)]
        dt1 = _oracle_timed(sc1, [cam1], rows, procs)
        res["c1_full_image"] = {"cells": sc1.n, "rays": cam1.n_rays, "seconds": round(dt1, 2),
                                "mrays_s": round(cam1.n_rays / dt1 / 1e6, 6)}
    return res


def _rate(fn, rays):
    fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(2):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return round(rays / (e0.elapsed_time(e1) / 2 * 1e-3) / 1e6, 2)


# VALU issue rate of the chip (unpacked FP32 lane-operations per second):
# 256 CUs x 64 lanes x 2.4 GHz.
VALU_LANE_OPS = 256 * 64 * 2.4e9
# Algorithmic bytes a walk step gathers (read once from HBM or cache), by the
# model's data: per cell entered its site and radius (16 B), cull radius (4),
# face range (8); per exit face scanned its neighbour (4) and plane (16); per
# piece (sphere hit) the face count and normal (20) and the detail sites'
# positions and displacements (96); per contribution the texture (1,632) and
# base colour (12).  Raster faces read for a piece are counted among the
# exit faces of that cell.
WALK_BYTES = {"cell": 28, "face": 20, "piece": 116, "contribution": 1644}


def work_counters(pf, scene, cams, out, rays, rates):
    """Work counters of one plain raster and one walk of the bench views:
    per-ray averages, the lane efficiency of the composite, its VALU fraction
    by the algorithmic op counts (115 per pixel-cell test, 1,300 per
    contribution), and the walk's gathered bytes per step and rate."""
    rc = torch.zeros(6, dtype=torch.int64, device="cuda")
    tc = torch.zeros(6, dtype=torch.int64, device="cuda")
    pf.render_raster(scene, cams, out=out, counters=rc)
    pf.render_trace(scene, cams, out=out, counters=tc)
    torch.cuda.synchronize()
    r, t = [int(x) for x in rc.cpu()], [int(x) for x in tc.cpu()]
    ras_s = rays / (rates["raster_fwd_mrays_s"] * 1e6)
    walk_s = rays / (rates["trace_fwd_mrays_s"] * 1e6)
    ops = 115 * r[0] + 1300 * r[2]
    raster = {"pixel_cell_tests": r[0], "sphere_hits": r[1], "contributions": r[2],
              "wave_steps": r[3], "wave_steps_with_piece": r[4], "wave_steps_shaded": r[5],
              "tests_per_ray": round(r[0] / rays, 2), "contributions_per_ray": round(r[2] / rays, 2),
              "lanes_per_piece_step": round(r[1] / max(1, r[4]), 2),
              "lanes_per_shaded_step": round(r[2] / max(1, r[5]), 2),
              "alg_ops": ops, "valu_frac_alg": round(ops / (ras_s * VALU_LANE_OPS), 4)}
    gathered = (WALK_BYTES["cell"] * t[1] + WALK_BYTES["face"] * t[4] + WALK_BYTES["piece"] * t[2] +
                WALK_BYTES["contribution"] * t[3])
    walk = {"rays": t[0], "cells_per_ray": round(t[1] / max(1, t[0]), 2),
            "pieces_per_ray": round(t[2] / max(1, t[0]), 2), "contributions_per_ray": round(t[3] / max(1, t[0]), 2),
            "faces_per_cell": round(t[4] / max(1, t[1]), 2), "max_cells_one_ray": t[5],
            "bytes_per_cell_walked": round(gathered / max(1, t[1]), 1),
            "gathered_gb_s": round(gathered / walk_s / 1e9, 1), "hbm_peak_gb_s": HBM_PEAK_GBS}
    return raster, walk


def walk_cells_per_ray(pf, scene, cams, out):
    tc = torch.zeros(6, dtype=torch.int64, device="cuda")
    pf.render_trace(scene, cams, out=out, counters=tc)
    t = [int(x) for x in tc.cpu()]
    return round(t[1] / max(1, t[0]), 3), round(t[3] / max(1, t[0]), 3)


def steiner_side(pf, W, sc, params, cams, out, rays, args):
    """Steiner cells (6 rounds) on the bench scene: insertion time, cells
    kept, and forward rates of the scene with them as empty cells."""
    n_cand = args.steiner_cand if args.steiner_cand > 0 else max(1, args.cells // 16)
    z = torch.as_tensor(W.steiner_draws(6, n_cand)).cuda()
    base = {k: v.detach() for k, v in params.items()}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    cells = pf.steiner(base, z)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3
    aug = pf.append_empty_cells(base, cells)
    t0 = time.perf_counter()
    scene = pf.build_scene(aug, sigma_scale=sc.sigma_scale, tau=sc.tau)
    torch.cuda.synchronize()
    build_ms = (time.perf_counter() - t0) * 1e3
    base_scene = pf.build_scene(base, sigma_scale=sc.sigma_scale, tau=sc.tau)
    ref = [im.clone() for im in pf.render_raster(base_scene, cams)]
    img = pf.render_raster(scene, cams)
    change = max(float((a - b).abs().max()) for a, b in zip(img, ref))
    cells_before, contrib_before = walk_cells_per_ray(pf, base_scene, cams, out)
    cells_after, contrib_after = walk_cells_per_ray(pf, scene, cams, out)
    base_scene.destroy()
    res = {"candidates_per_round": n_cand, "kept_per_round": cells["round_counts"],
           "cells_added": int(cells["p"].shape[0]), "insert_ms": round(ms, 1), "build_ms": round(build_ms, 1),
           "trace_fwd_mrays_s": _rate(lambda: pf.render_trace(scene, cams, out=out), rays),
           "raster_fwd_mrays_s": _rate(lambda: pf.render_raster(scene, cams, out=out), rays),
           "walk_cells_per_ray": [cells_before, cells_after],
           "walk_contributions_per_ray": [contrib_before, contrib_after],
           "max_image_change": float(f"{change:.3g}")}
    scene.destroy()
    # the paper's parameterisation, power = r^2: same sites and radii
    tied = dict(base)
    tied["power"] = (base["radius"] * base["radius"]).contiguous()
    cells_t = pf.steiner(tied, z)
    aug_t = pf.append_empty_cells(tied, cells_t)
    s_tied = pf.build_scene(tied, sigma_scale=sc.sigma_scale, tau=sc.tau)
    s_aug = pf.build_scene(aug_t, sigma_scale=sc.sigma_scale, tau=sc.tau)
    ref = [im.clone() for im in pf.render_raster(s_tied, cams)]
    img = pf.render_raster(s_aug, cams)
    change_t = max(float((a - b).abs().max()) for a, b in zip(img, ref))
    tb, _ = walk_cells_per_ray(pf, s_tied, cams, out)
    ta, _ = walk_cells_per_ray(pf, s_aug, cams, out)
    res["tied_power"] = {"cells_added": int(cells_t["p"].shape[0]), "walk_cells_per_ray": [tb, ta],
                         "trace_fwd_mrays_s": [_rate(lambda: pf.render_trace(s_tied, cams, out=out), rays),
                                               _rate(lambda: pf.render_trace(s_aug, cams, out=out), rays)],
                         "max_image_change": float(f"{change_t:.3g}")}
    s_tied.destroy()
    s_aug.destroy()
    return res


def densify_side(pf, sc, params, args):
    """One densify-and-prune update on the bench scene (moving averages of
    seeded per-cell statistics, prune the lowest 5% by contribution, draw 1%
    new cells) followed by the rebuild of the new cell set."""
    n = args.cells
    g = torch.Generator(device="cuda").manual_seed(7)
    stat = torch.rand(n, device="cuda", generator=g)
    ema_e = torch.zeros(n, device="cuda")
    ema_c = torch.zeros(n, device="cuda")
    n_new = max(1, n // 100)
    u = torch.rand(n_new, device="cuda", generator=g)
    delta = torch.randn(n_new, 3, device="cuda", generator=g)
    base = {k: v.detach() for k, v in params.items()}
    below = float(torch.quantile(stat[:65536], 0.05)) * 0.1
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pf.ema_update(ema_e, stat, 0.9)
    pf.ema_update(ema_c, stat, 0.9)
    out, _, _, par = pf.densify_prune(base, ema_e, ema_c, u, delta, below, 0.5)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    scene = pf.build_scene(out, sigma_scale=sc.sigma_scale, tau=sc.tau)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    res = {"cells_in": n, "cells_out": int(out["p"].shape[0]), "drawn": int(par.numel()),
           "update_ms": round((t1 - t0) * 1e3, 2), "rebuild_ms": round((t2 - t1) * 1e3, 2)}
    scene.destroy()
    return res


def main():
    args = parse()
    if args.copy_calibration:
        n = args.copy_calibration << 18          # float32 elements in MIB MiB
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(one process drives one GPU; the multi-GPU layout is not built)", file=sys.stderr)
        sys.exit(2)
    import workloads as W
    import paper_2604_24994_amd as pf
    from paper_2604_24994_amd import _lib

    t0 = time.time()
    sc = W.c3_scene(n=args.cells)
    cams = W.c3_cameras(n_views=args.views, width=args.width, height=args.height)
    log(f"inputs generated in {time.time() - t0:.1f}s")
    cpu = None
    if not args.no_cpu_baseline:
        # before the GPU is initialised: the oracle runs in forked worker processes
        log("timing the oracle sample on the host CPU")
        cpu = cpu_baseline(sc, cams, args.cpu_rays)
        log(f"cpu baseline: {cpu}")
    params = {k: v.requires_grad_(args.mode == "train") for k, v in pf.to_device_params(sc).items()}
    rays = sum(c.n_rays for c in cams)
    out = torch.empty(4 * rays, dtype=torch.float32, device="cuda")
    tgt = torch.cat([torch.as_tensor(t, device="cuda").reshape(-1, 3) for t in W.targets(cams)])
    stream = torch.cuda.current_stream()

    held = {"scene": None}
    gen = torch.Generator(device="cuda").manual_seed(11)

    def step(state_mode=pf.STORE):
        # the sites move a little between steps, as after an optimiser update,
        # and the adjacency is rebuilt (seeded by the previous step's)
        with torch.no_grad():
            params["p"].add_(torch.randn(params["p"].shape, device="cuda", generator=gen), alpha=1e-4)
        if held["scene"] is None:
            held["scene"] = pf.build_scene(params, sigma_scale=sc.sigma_scale, tau=sc.tau, stream=stream)
        else:
            pf.update_scene(held["scene"], params, stream=stream)
        scene = held["scene"]
        if args.mode == "fwd":
            pf.render_raster(scene, cams, stream=stream, out=out)
            return scene
        for v in params.values():
            v.grad = None
        imgs = pf.render_raster_diff(scene, cams, state_mode=state_mode)
        rgb = torch.cat([im.reshape(-1, 4)[:, :3] for im in imgs])
        loss = ((rgb - tgt) ** 2).mean()
        loss.backward()
        return scene

    for i in range(max(1, args.warmup)):
        s = step()
        torch.cuda.synchronize()
        if i == 0:
            log(f"scene: {s.info()}")
    log("warmup done")

    _lib.profile_enable(True)
    _lib.profile_read()
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(args.steps):
        s = step()
    ev1.record(stream)
    torch.cuda.synchronize()
    prof = _lib.profile_read()
    _lib.profile_enable(False)
    ms = ev0.elapsed_time(ev1) / args.steps
    value = rays / (ms * 1e-3) / 1e6
    kms = {k: v[1] / args.steps for k, v in prof.items()}
    from paper_2604_24994_amd.autograd import LAST_FORWARD
    nrec = LAST_FORWARD["records"]   # contributions of the timed step's forward
    log(f"step {ms:.2f} ms, kernel ms/step: " + ", ".join(f"{k}={v:.2f}" for k, v in sorted(kms.items(), key=lambda kv: -kv[1])))

    extra = {}
    if args.mode == "train" and args.recompute_steps > 0:
        # the same step with the traversal replayed inside the backward (no
        # records kept between forward and backward), beside a store step's
        # memory high-water mark
        mem = {}
        for name, mode in (("store", pf.STORE), ("recompute", pf.RECOMPUTE)):
            torch.cuda.synchronize()
            pf.memory_stats(reset_peak=True)
            step(mode)
            torch.cuda.synchronize()
            mem[name] = pf.memory_stats()["peak"]
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(args.recompute_steps):
            step(pf.RECOMPUTE)
        e1.record(stream)
        torch.cuda.synchronize()
        rms = e0.elapsed_time(e1) / args.recompute_steps
        extra["recompute"] = {"ms_per_step": round(rms, 3), "mrays_s": round(rays / (rms * 1e-3) / 1e6, 3),
                              "steps": args.recompute_steps,
                              "library_peak_bytes": mem["recompute"], "store_library_peak_bytes": mem["store"],
                              "window_bytes": 2 << 30}
        log(f"recompute: {extra['recompute']}")

    # side measurements on one built scene (not part of the timed step)
    scene = pf.build_scene({k: v.detach() for k, v in params.items()}, sigma_scale=sc.sigma_scale, tau=sc.tau)
    box = scene.info()
    for name, fn in (("raster_fwd", lambda: pf.render_raster(scene, cams, out=out)),
                     ("trace_fwd", lambda: pf.render_trace(scene, cams, out=out))):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(2):
            fn()
        e1.record()
        torch.cuda.synchronize()
        extra[name + "_mrays_s"] = round(rays / (e0.elapsed_time(e1) / 2 * 1e-3) / 1e6, 2)
    log(f"side: {extra}")
    extra["raster_work"], extra["walk_work"] = work_counters(pf, scene, cams, out, rays, extra)
    log(f"raster work: {extra['raster_work']}")
    log(f"walk work: {extra['walk_work']}")
    if not args.no_densify:
        extra["densify"] = densify_side(pf, sc, params, args)
        log(f"densify: {extra['densify']}")
    if args.steiner_cand != 0:
        extra["steiner"] = steiner_side(pf, W, sc, params, cams, out, rays, args)
        log(f"steiner: {extra['steiner']}")
    serving = None
    if args.serve_seconds > 0:
        from paper_2604_24994_amd import serve
        reqs = W.request_stream(args.serve_rate, args.serve_warmup + args.serve_seconds)
        serving = {"rate_req_s": args.serve_rate, "seconds": args.serve_seconds, "warmup_s": args.serve_warmup}
        for name, srv in (("batched", serve.Server({0: scene}, hbm_budget_bytes=16 << 30)),
                          ("plain", serve.PlainServer({0: scene}))):
            try:
                st = serve.replay(srv, reqs, warmup_s=args.serve_warmup)
            finally:
                srv.close()
            serving[name] = {k: round(v, 3) for k, v in st.items()}
            log(f"serving {name}: {serving[name]}")

    dom_name, dom_ms = max(kms.items(), key=lambda kv: kv[1]) if kms else ("none", 0.0)
    dom_launches = prof[dom_name][0] / args.steps if prof else 1
    avg_ms = dom_ms / max(1, dom_launches)
    per = {"k_bwd_cell": FLOPS_BWD_PER_CONTRIB, "k_raster_store": FLOPS_FWD_PER_CONTRIB,
           "k_raster": FLOPS_FWD_PER_CONTRIB}.get(dom_name)
    achieved = per * nrec / max(1, dom_launches) / (avg_ms * 1e-3) / 1e12 if (per and nrec) else None
    roof = {"kernel": dom_name, "bound": "alu",
            "achieved": round(achieved, 4) if achieved is not None else None,
            "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": round(achieved / FP32_PEAK_TFLOPS, 5) if achieved is not None else None,
            "traffic": traffic_bytes(dom_name), "avg_ms": round(avg_ms, 4),
            "units_per_launch": f"{nrec} contributions x {per} flops" if per else None}
    res = {
        "metric": ("Mrays/s fwd+bwd at 1M cells (raster training step incl. adjacency rebuild)"
                   if args.mode == "train" else "Mrays/s fwd at 1M cells (raster, adjacency rebuilt every step)"),
        "value": round(value, 3),
        "unit": "Mrays/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": max(1, args.warmup),
        "ms_per_step": round(ms, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{args.cells} cells, {args.views} pinhole views {args.width}x{args.height}, "
                               + ("site update + adjacency rebuild + raster fwd + L2 loss + bwd" if args.mode == "train"
                                  else "site update + adjacency rebuild + raster fwd"),
                   "cells": args.cells, "views": args.views, "width": args.width, "height": args.height},
        "kernels_ms_per_step": {k: round(v, 3) for k, v in kms.items()},
        "scene": {"hidden": box["n_hidden"], "faces": box["n_faces"]},
        **extra,
        "serving": serving,
        "roofline": roof,
    }
    if cpu is not None:
        res["cpu_baseline"] = cpu
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
