"""Continuous-batching render server over resident scenes.

Scenes stay built in HBM.  Requests (scene id, camera) queue on arrival; a
pool of worker threads, each with its own HIP stream, repeatedly takes the
oldest waiting requests of one scene that fit the free HBM budget and a ray
cap, and renders them as ONE batched pf_render_raster call (all of the
batch's tiles in one composite launch).  Requests arriving while batches run
join the next batch as soon as a worker and budget free up, so device work
of consecutive batches overlaps.  Each request's image is the same as a
render of that camera alone (views never interact).

``PlainServer`` is the per-request baseline: one pf_render_raster call per
request, in arrival order, one stream.
"""
from __future__ import annotations

import collections
import threading
import time
from concurrent.futures import Future
from typing import Dict, List, Optional

import numpy as np
import torch

from .api import Scene, render_raster


def request_bytes(scene: Scene, cam) -> int:
    """Device memory a request holds while in flight: its RGBA output, the
    per-(view, cell) key/count/offset arrays and the tile pair lists (an
    estimate of 24 B per cell)."""
    n = int(scene.params["p"].shape[0])
    return 16 * int(cam.width) * int(cam.height) + 24 * n


class _Req:
    __slots__ = ("scene_id", "cam", "arrival", "future", "nbytes", "rays")

    def __init__(self, scene_id, cam, arrival, nbytes):
        self.scene_id = scene_id
        self.cam = cam
        self.arrival = arrival
        self.future = Future()
        self.nbytes = nbytes
        self.rays = int(cam.width) * int(cam.height)


def take_batch(queue: "collections.deque", inflight: int, budget: int, max_batch_rays: int,
               max_batch: int) -> list:
    """Admission policy (host logic): the oldest waiting request picks the
    scene; requests of that scene are admitted in arrival order while the
    batch stays under ``max_batch`` requests and ``max_batch_rays`` rays (a
    single larger request is admitted alone) and the bytes in flight stay
    within ``budget``.  Admission stops at the first request of that scene
    that does not fit, so requests of a scene are never reordered; requests
    of other scenes keep their places.  Removes the batch from ``queue``."""
    if not queue:
        return []
    first = queue[0]
    if inflight + first.nbytes > budget:
        return []
    batch, rays, nbytes = [], 0, 0
    keep = collections.deque()
    while queue:
        r = queue.popleft()
        fits = (r.scene_id == first.scene_id and len(batch) < max_batch and
                (not batch or rays + r.rays <= max_batch_rays) and
                inflight + nbytes + r.nbytes <= budget)
        if fits:
            batch.append(r)
            rays += r.rays
            nbytes += r.nbytes
        else:
            keep.append(r)
            if r.scene_id == first.scene_id:
                break
    while keep:
        queue.appendleft(keep.pop())
    return batch


class Server:
    def __init__(self, scenes: Dict[int, Scene], hbm_budget_bytes: int = 8 << 30, max_batch_rays: int = 8 << 20,
                 max_batch: int = 64, n_workers: int = 2, t_min: float = 1e-6):
        self.scenes = scenes
        self.budget = int(hbm_budget_bytes)
        self.max_batch_rays = int(max_batch_rays)
        self.max_batch = int(max_batch)
        self.t_min = t_min
        self._queue: collections.deque = collections.deque()
        self._cv = threading.Condition()
        self._inflight = 0
        self.peak_inflight = 0
        self._stop = False
        self.latencies: List[float] = []
        self.batches: List[int] = []
        self.rays_done = 0
        self._workers = [threading.Thread(target=self._run, daemon=True, name=f"pf-serve-{i}")
                         for i in range(n_workers)]
        for w in self._workers:
            w.start()

    def submit(self, scene_id: int, cam, arrival: Optional[float] = None) -> Future:
        """Queues a request; the future resolves to its [H,W,4] image."""
        if scene_id not in self.scenes:
            raise KeyError(f"unknown scene {scene_id}")
        req = _Req(scene_id, cam, time.perf_counter() if arrival is None else arrival,
                   request_bytes(self.scenes[scene_id], cam))
        if req.nbytes > self.budget:
            raise ValueError("request needs more than the whole HBM budget")
        with self._cv:
            self._queue.append(req)
            self._cv.notify()
        return req.future

    def _take_batch(self) -> List[_Req]:
        batch = take_batch(self._queue, self._inflight, self.budget, self.max_batch_rays, self.max_batch)
        self._inflight += sum(r.nbytes for r in batch)
        self.peak_inflight = max(self.peak_inflight, self._inflight)
        return batch

    def _run(self):
        stream = torch.cuda.Stream()
        while True:
            with self._cv:
                batch: List[_Req] = []
                while not self._stop:
                    if self._queue:
                        batch = self._take_batch()
                        if batch:
                            break
                    self._cv.wait(timeout=0.05)
                if self._stop and not batch:
                    return
            nbytes = sum(r.nbytes for r in batch)
            try:
                with torch.cuda.stream(stream):
                    imgs = render_raster(self.scenes[batch[0].scene_id], [r.cam for r in batch],
                                         t_min=self.t_min, stream=stream)
                    ev = torch.cuda.Event()
                    ev.record(stream)
                ev.synchronize()
                done = time.perf_counter()
                with self._cv:
                    for r in batch:
                        self.latencies.append(done - r.arrival)
                        self.rays_done += r.rays
                    self.batches.append(len(batch))
                for r, img in zip(batch, imgs):
                    r.future.set_result(img)
            except Exception as e:   # noqa: BLE001 - forwarded to the callers
                for r in batch:
                    r.future.set_exception(e)
            finally:
                with self._cv:
                    self._inflight -= nbytes
                    self._cv.notify_all()

    def close(self):
        with self._cv:
            self._stop = True
            self._cv.notify_all()
        for w in self._workers:
            w.join()


class PlainServer:
    """Baseline: one render call per request, arrival order, one stream."""

    def __init__(self, scenes: Dict[int, Scene], t_min: float = 1e-6):
        self.scenes = scenes
        self.t_min = t_min
        self._queue: collections.deque = collections.deque()
        self._cv = threading.Condition()
        self._stop = False
        self.latencies: List[float] = []
        self.rays_done = 0
        self._worker = threading.Thread(target=self._run, daemon=True, name="pf-plain")
        self._worker.start()

    def submit(self, scene_id: int, cam, arrival: Optional[float] = None) -> Future:
        req = _Req(scene_id, cam, time.perf_counter() if arrival is None else arrival, 0)
        with self._cv:
            self._queue.append(req)
            self._cv.notify()
        return req.future

    def _run(self):
        stream = torch.cuda.Stream()
        while True:
            with self._cv:
                while not self._queue and not self._stop:
                    self._cv.wait(timeout=0.05)
                if self._stop and not self._queue:
                    return
                r = self._queue.popleft()
            try:
                with torch.cuda.stream(stream):
                    img = render_raster(self.scenes[r.scene_id], r.cam, t_min=self.t_min, stream=stream)[0]
                    ev = torch.cuda.Event()
                    ev.record(stream)
                ev.synchronize()
                self.latencies.append(time.perf_counter() - r.arrival)
                self.rays_done += r.rays
                r.future.set_result(img)
            except Exception as e:   # noqa: BLE001
                r.future.set_exception(e)

    def close(self):
        with self._cv:
            self._stop = True
            self._cv.notify_all()
        self._worker.join()


def replay(server, requests, time_scale: float = 1.0) -> dict:
    """Submits ``requests`` (objects with arrival_s, camera, scene_id) at
    their arrival times, waits for all, and returns latency statistics."""
    t0 = time.perf_counter()
    futs = []
    for req in requests:
        due = t0 + req.arrival_s * time_scale
        now = time.perf_counter()
        if due > now:
            time.sleep(due - now)
        futs.append(server.submit(req.scene_id, req.camera, arrival=max(due, t0)))
    for f in futs:
        f.result()
    wall = time.perf_counter() - t0
    lat = np.array(server.latencies[-len(futs):]) * 1e3
    rays = sum(int(r.camera.width) * int(r.camera.height) for r in requests)
    return {"requests": len(futs), "p50_ms": float(np.percentile(lat, 50)),
            "p99_ms": float(np.percentile(lat, 99)), "frames_per_s": len(futs) / wall,
            "mrays_per_s": rays / wall / 1e6, "wall_s": wall}
