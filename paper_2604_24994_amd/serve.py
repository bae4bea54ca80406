"""Continuous-batching render server over resident scenes.

Scenes stay built in HBM.  Requests (scene id, camera) queue on arrival,
each sized by the library's bound on the device memory its render requests
(pf_query_workspace, exact in the scene's tile-pair lists for that camera)
plus its RGBA output.  A pool of worker threads, each with its own HIP
stream, repeatedly takes the oldest waiting requests of one scene whose
bounds fit the free part of the HBM budget (and a ray cap), and renders
them as ONE batched pf_render_raster call: one composite launch over the
(request, tile) work items of the whole batch, one workgroup per item, which
the hardware dispatcher hands to whichever CU frees up.  Requests arriving
while batches run join the next batch as soon as a worker and budget free
up, so device work of consecutive batches overlaps; a request that does not
fit waits until enough in-flight work completes.  Each request's image is
the same as a render of that camera alone (views never interact).

``PlainServer`` is the per-request baseline: one pf_render_raster call per
request, in arrival order, one stream.
"""
from __future__ import annotations

import collections
import threading
import time
from concurrent.futures import Future
from typing import Callable, Dict, List, Optional

import numpy as np
import torch

from .api import Scene, query_workspace, render_raster


def request_bytes(scene: Scene, cam, stream=None) -> int:
    """Device memory a request holds while in flight: the library's upper
    bound for rendering it (pf_query_workspace, which runs the cull-and-count
    pass of this camera on ``stream``) plus its RGBA output (16 B/pixel)."""
    return query_workspace(scene, [cam], 0, stream=stream) + 16 * int(cam.width) * int(cam.height)


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
    """``hbm_budget_bytes``: device bytes the requests in flight may hold
    together (None: 80% of the free device memory when the server starts).
    ``render_fn(scene, cams, stream) -> images`` and ``sizer(scene, cam) ->
    bytes`` replace the library calls (host tests of the policy); ``streams``
    False runs the workers without device streams."""

    def __init__(self, scenes: Dict[int, Scene], hbm_budget_bytes: Optional[int] = None,
                 max_batch_rays: int = 8 << 20, max_batch: int = 64, n_workers: int = 2, t_min: float = 1e-6,
                 render_fn: Optional[Callable] = None, sizer: Optional[Callable] = None, streams: bool = True):
        self.scenes = scenes
        if hbm_budget_bytes is None:
            hbm_budget_bytes = int(0.8 * torch.cuda.mem_get_info()[0])
        self.budget = int(hbm_budget_bytes)
        self.max_batch_rays = int(max_batch_rays)
        self.max_batch = int(max_batch)
        self.t_min = t_min
        self._streams = streams
        self._render = render_fn or (lambda scene, cams, stream: render_raster(scene, cams, t_min=self.t_min,
                                                                               stream=stream))
        if sizer is None:
            self._qstream = torch.cuda.Stream()
            self._qlock = threading.Lock()

            def sizer(scene, cam):
                with self._qlock:
                    return request_bytes(scene, cam, stream=self._qstream)
        self._sizer = sizer
        self._queue: collections.deque = collections.deque()
        self._cv = threading.Condition()
        self._inflight = 0
        self.peak_inflight = 0
        self._stop = False
        self.latencies: List[float] = []
        self.batches: List[int] = []
        self.admitted: List[tuple] = []     # (time, in-flight bytes after admission)
        self.rays_done = 0
        self._workers = [threading.Thread(target=self._run, daemon=True, name=f"pf-serve-{i}")
                         for i in range(n_workers)]
        for w in self._workers:
            w.start()

    def submit(self, scene_id: int, cam, arrival: Optional[float] = None) -> Future:
        """Queues a request; the future resolves to its [H,W,4] image."""
        if scene_id not in self.scenes:
            raise KeyError(f"unknown scene {scene_id}")
        arrival = time.perf_counter() if arrival is None else arrival
        req = _Req(scene_id, cam, arrival, int(self._sizer(self.scenes[scene_id], cam)))
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
        if batch:
            self.admitted.append((time.perf_counter(), self._inflight))
        return batch

    def _run(self):
        stream = torch.cuda.Stream() if self._streams else None
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
                if stream is not None:
                    with torch.cuda.stream(stream):
                        imgs = self._render(self.scenes[batch[0].scene_id], [r.cam for r in batch], stream)
                        ev = torch.cuda.Event()
                        ev.record(stream)
                    ev.synchronize()
                else:
                    imgs = self._render(self.scenes[batch[0].scene_id], [r.cam for r in batch], None)
                done = time.perf_counter()
                with self._cv:
                    for r in batch:
                        self.latencies.append(done - r.arrival)
                        self.rays_done += r.rays
                    self.batches.append(len(batch))
                for r, img in zip(batch, imgs):
                    r.future.done_at = done
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
                done = time.perf_counter()
                self.latencies.append(done - r.arrival)
                self.rays_done += r.rays
                r.future.done_at = done
                r.future.set_result(img)
            except Exception as e:   # noqa: BLE001
                r.future.set_exception(e)

    def close(self):
        with self._cv:
            self._stop = True
            self._cv.notify_all()
        self._worker.join()


def replay(server, requests, time_scale: float = 1.0, warmup_s: float = 0.0) -> dict:
    """Submits ``requests`` (objects with arrival_s, camera, scene_id) at
    their arrival times, waits for all, and returns latency statistics of the
    requests that arrive at or after ``warmup_s`` (arrival to completion) and
    their throughput over the window from ``warmup_s`` to the last one's
    completion."""
    t0 = time.perf_counter()
    futs, arrivals = [], []
    for req in requests:
        due = t0 + req.arrival_s * time_scale
        now = time.perf_counter()
        if due > now:
            time.sleep(due - now)
        arrival = max(due, t0)
        futs.append(server.submit(req.scene_id, req.camera, arrival=arrival))
        arrivals.append(arrival)
    for f in futs:
        f.result()
    meas = [i for i, req in enumerate(requests) if req.arrival_s >= warmup_s]
    if not meas:
        raise ValueError("no request arrives after the warm-up")
    lat = np.array([futs[i].done_at - arrivals[i] for i in meas]) * 1e3
    start = t0 + warmup_s * time_scale
    wall = max(futs[i].done_at for i in meas) - start
    rays = sum(int(requests[i].camera.width) * int(requests[i].camera.height) for i in meas)
    return {"requests": len(meas), "warmup_requests": len(requests) - len(meas),
            "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "frames_per_s": len(meas) / wall, "mrays_per_s": rays / wall / 1e6, "wall_s": wall}
