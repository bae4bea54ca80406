"""Python binding over the C ABI: same call names, tensors in, tensors out.

PyTorch supplies device memory and streams only; every step of rendering
runs in libpowerfoam's HIP kernels.  There is no CPU fallback: calls raise
when the library is missing or no GPU is present.
"""
from __future__ import annotations

import ctypes as C
from typing import Dict, Iterable, List, Optional, Sequence

import numpy as np
import torch

from . import _lib as L

PARAM_FIELDS = ("p", "power", "radius", "normal", "occ_logit", "rgb", "tex")


def _stream_ptr(stream) -> int:
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream)


def _require_cuda():
    if not torch.cuda.is_available():
        raise RuntimeError("paper_2604_24994_amd needs a ROCm GPU (gfx950); none is visible")


def to_device_params(src, device="cuda") -> Dict[str, torch.Tensor]:
    """Cell parameters from any object or dict with the fields
    p, power, radius, normal, occ_logit, rgb, tex (numpy or torch) as
    contiguous float32 device tensors."""
    get = (lambda k: src[k]) if isinstance(src, dict) else (lambda k: getattr(src, k))
    out = {}
    for k in PARAM_FIELDS:
        t = torch.as_tensor(get(k))
        out[k] = t.to(device=device, dtype=torch.float32).contiguous()
    return out


def camera_struct(cam) -> L.PfCamera:
    """pf_camera from any object with the camera fields (see powerfoam.h)."""
    c = L.PfCamera()
    c.model = int(cam.model)
    c.width = int(cam.width)
    c.height = int(cam.height)
    m = np.asarray(cam.c2w, dtype=np.float32).reshape(12)
    for i in range(12):
        c.c2w[i] = float(m[i])
    for f in ("fx", "fy", "cx", "cy", "f_fish", "theta_max"):
        setattr(c, f, float(getattr(cam, f, 0.0)))
    return c


def _cams(cams) -> (L.PfCamera, int, List[tuple]):
    if not isinstance(cams, (list, tuple)):
        cams = [cams]
    arr = (L.PfCamera * len(cams))()
    shapes = []
    for i, cam in enumerate(cams):
        arr[i] = camera_struct(cam)
        shapes.append((int(cam.height), int(cam.width)))
    return arr, len(cams), shapes


class Scene:
    """A built scene: owns the pf_scene handle and keeps the parameter
    tensors it references alive."""

    def __init__(self, handle: int, params: Dict[str, torch.Tensor], consts: dict):
        self._h = C.c_void_p(handle)
        self.params = params
        self.consts = consts

    @property
    def handle(self) -> C.c_void_p:
        if not self._h:
            raise RuntimeError("scene was destroyed")
        return self._h

    def info(self) -> dict:
        inf = L.PfSceneInfo()
        L.check(L.load().pf_scene_info_get(self.handle, C.byref(inf)))
        return {"n": inf.n, "n_faces": inf.n_faces, "n_hidden": inf.n_hidden,
                "n_overflow": inf.n_overflow, "n_high_degree": inf.n_high_degree,
                "n_dropped": inf.n_dropped, "box_min": list(inf.box_min),
                "box_max": list(inf.box_max)}

    def adjacency(self, stream=None):
        """CSR (row [n+1], col [n_faces]) int32 device tensors."""
        inf = self.info()
        dev = self.params["p"].device
        row = torch.empty(inf["n"] + 1, dtype=torch.int32, device=dev)
        col = torch.empty(max(1, inf["n_faces"]), dtype=torch.int32, device=dev)
        L.check(L.load().pf_scene_adjacency(self.handle, C.c_void_p(row.data_ptr()),
                                            C.c_void_p(col.data_ptr()), C.c_void_p(_stream_ptr(stream))))
        return row, col[:inf["n_faces"]]

    def destroy(self):
        if self._h:
            L.load().pf_scene_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def build_scene(params, sigma_scale: float = 10.0, tau: float = 20.0, box=None, box_pad: float = 0.01,
                stream=None) -> Scene:
    """pf_build_scene.  ``params``: dict/object of cell arrays (moved to the
    GPU as float32 if needed).  ``box``: optional (min[3], max[3]) the domain
    box must contain (e.g. trace camera centres)."""
    _require_cuda()
    lib = L.load()
    t = to_device_params(params)
    n = int(t["p"].shape[0])
    k = int(t["tex"].shape[1])
    m = (int(t["tex"].shape[2]) - 3) // 6
    pp = L.PfParams(n=n, k_detail=k, m_axes=m, sigma_scale=float(sigma_scale), tau=float(tau))
    for f in PARAM_FIELDS:
        setattr(pp, f, t[f].data_ptr())
    opts = L.PfBuildOpts()
    opts.box_pad = float(box_pad)
    if box is None:
        opts.box_min[0], opts.box_max[0] = 1.0, -1.0
    else:
        for a in range(3):
            opts.box_min[a] = float(box[0][a])
            opts.box_max[a] = float(box[1][a])
    h = C.c_void_p()
    L.check(lib.pf_build_scene(C.byref(pp), C.byref(opts), C.c_void_p(_stream_ptr(stream)), C.byref(h)))
    return Scene(h.value, t, {"sigma_scale": sigma_scale, "tau": tau})


def update_scene(scene: Scene, params, stream=None) -> Scene:
    """pf_update_scene: rebuilds ``scene`` in place for new parameter values
    (same cell count); the scene then references the new tensors."""
    t = to_device_params(params)
    if int(t["p"].shape[0]) != int(scene.params["p"].shape[0]):
        raise ValueError("update_scene keeps the cell count; build a new scene instead")
    k = int(t["tex"].shape[1])
    m = (int(t["tex"].shape[2]) - 3) // 6
    pp = L.PfParams(n=int(t["p"].shape[0]), k_detail=k, m_axes=m, sigma_scale=float(scene.consts["sigma_scale"]),
                    tau=float(scene.consts["tau"]))
    for f in PARAM_FIELDS:
        setattr(pp, f, t[f].data_ptr())
    L.check(L.load().pf_update_scene(scene.handle, C.byref(pp), C.c_void_p(_stream_ptr(stream))))
    scene.params = t
    return scene


STORE, RECOMPUTE = 0, 1


def _opts(t_min: float, max_steps: int, state_mode: int = STORE, workspace_limit: int = 0,
          counters: Optional[torch.Tensor] = None) -> L.PfRenderOpts:
    if state_mode not in (STORE, RECOMPUTE):
        raise ValueError("state_mode must be STORE (0) or RECOMPUTE (1)")
    if counters is not None and (counters.dtype != torch.int64 or counters.numel() < 6 or not counters.is_cuda
                                 or not counters.is_contiguous()):
        raise ValueError("counters must be a contiguous int64 device tensor of at least 6 entries")
    return L.PfRenderOpts(t_min=float(t_min), max_steps=int(max_steps), state_mode=int(state_mode),
                          workspace_limit=int(workspace_limit),
                          counters=counters.data_ptr() if counters is not None else None)


def _alloc_images(shapes, device):
    total = sum(4 * h * w for h, w in shapes)
    buf = torch.empty(total, dtype=torch.float32, device=device)
    return buf


def _split(buf, shapes):
    out, off = [], 0
    for h, w in shapes:
        out.append(buf[off:off + 4 * h * w].view(h, w, 4))
        off += 4 * h * w
    return out


def render_raster(scene: Scene, cams, t_min: float = 1e-6, stream=None, out: Optional[torch.Tensor] = None,
                  counters: Optional[torch.Tensor] = None):
    """pf_render_raster: list of [H,W,4] float32 images (one per camera).
    counters: optional int64 device tensor [6] that the composite's work
    counters are added to (pixel-cell tests, sphere hits, contributions,
    (wave, cell) steps tested / with a piece / shaded)."""
    arr, nc, shapes = _cams(cams)
    buf = out if out is not None else _alloc_images(shapes, scene.params["p"].device)
    opts = _opts(t_min, 0, counters=counters)
    L.check(L.load().pf_render_raster(scene.handle, arr, nc, C.byref(opts), C.c_void_p(buf.data_ptr()),
                                      None, C.c_void_p(_stream_ptr(stream))))
    return _split(buf, shapes)


def render_trace(scene: Scene, cams, t_min: float = 1e-6, max_steps: int = 4096, stream=None,
                 out: Optional[torch.Tensor] = None, return_truncated: bool = False,
                 counters: Optional[torch.Tensor] = None):
    """pf_render_trace: list of [H,W,4] float32 images (one per camera).
    counters: optional int64 device tensor [6] that the walk's work counters
    are added to (rays, cells walked, pieces, contributions, exit faces
    scanned, most cells on one ray)."""
    arr, nc, shapes = _cams(cams)
    buf = out if out is not None else _alloc_images(shapes, scene.params["p"].device)
    opts = _opts(t_min, max_steps, counters=counters)
    trunc = C.c_int64(0)
    L.check(L.load().pf_render_trace(scene.handle, arr, nc, C.byref(opts), C.c_void_p(buf.data_ptr()),
                                     C.byref(trunc) if return_truncated else None, None,
                                     C.c_void_p(_stream_ptr(stream))))
    imgs = _split(buf, shapes)
    return (imgs, int(trunc.value)) if return_truncated else imgs


def render_trace_noalloc(scene: Scene, cams, out: torch.Tensor, t_min: float = 1e-6, max_steps: int = 4096,
                         stream=None, return_truncated: bool = False):
    """pf_render_trace_noalloc: the walk of ``render_trace`` with no device
    allocation (scratch in the library's fixed per-device array).  ``out``
    (caller-allocated float32 device tensor of 4 H W floats per camera,
    images back to back) is required.  Calls that overlap on one device
    race on the shared scratch."""
    arr, nc, shapes = _cams(cams)
    need = sum(4 * h * w for h, w in shapes)
    if out.dtype != torch.float32 or not out.is_cuda or not out.is_contiguous() or out.numel() < need:
        raise ValueError(f"out must be a contiguous float32 device tensor of at least {need} floats")
    opts = _opts(t_min, max_steps)
    trunc = C.c_int64(0)
    L.check(L.load().pf_render_trace_noalloc(scene.handle, arr, nc, C.byref(opts), C.c_void_p(out.data_ptr()),
                                             C.byref(trunc) if return_truncated else None,
                                             C.c_void_p(_stream_ptr(stream))))
    imgs = _split(out, shapes)
    return (imgs, int(trunc.value)) if return_truncated else imgs


class ForwardState:
    """pf_fwd_state handle of a forward (raster or walk, store or recompute
    mode)."""

    def __init__(self, handle: int, scene: Scene, shapes):
        self._h = C.c_void_p(handle)
        self.scene = scene
        self.shapes = shapes

    @property
    def handle(self) -> C.c_void_p:
        if not self._h:
            raise RuntimeError("forward state was released")
        return self._h

    def info(self) -> dict:
        nr, npx, mode = C.c_int64(0), C.c_int64(0), C.c_int32(0)
        L.check(L.load().pf_state_info(self.handle, C.byref(nr), C.byref(npx), C.byref(mode)))
        return {"records": int(nr.value), "pixels": int(npx.value),
                "mode": "store" if mode.value == STORE else "recompute"}

    def release(self):
        if self._h:
            L.load().pf_state_release(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.release()
        except Exception:
            pass


def render_raster_state(scene: Scene, cams, t_min: float = 1e-6, stream=None, out: Optional[torch.Tensor] = None,
                        state_mode: int = STORE, workspace_limit: int = 0):
    """pf_render_raster with a forward state: (flat RGBA buffer, ForwardState).
    ``workspace_limit``: bytes the records may occupy (store mode: past it
    the state keeps only the cameras; recompute mode: the backward's replay
    window)."""
    arr, nc, shapes = _cams(cams)
    buf = out if out is not None else _alloc_images(shapes, scene.params["p"].device)
    opts = _opts(t_min, 0, state_mode, workspace_limit)
    h = C.c_void_p()
    L.check(L.load().pf_render_raster(scene.handle, arr, nc, C.byref(opts), C.c_void_p(buf.data_ptr()),
                                      C.byref(h), C.c_void_p(_stream_ptr(stream))))
    return buf, ForwardState(h.value, scene, shapes)


def render_trace_state(scene: Scene, cams, t_min: float = 1e-6, max_steps: int = 4096, stream=None,
                       out: Optional[torch.Tensor] = None, state_mode: int = STORE, workspace_limit: int = 0):
    """pf_render_trace with a forward state: (flat RGBA buffer, ForwardState)."""
    arr, nc, shapes = _cams(cams)
    buf = out if out is not None else _alloc_images(shapes, scene.params["p"].device)
    opts = _opts(t_min, max_steps, state_mode, workspace_limit)
    h = C.c_void_p()
    L.check(L.load().pf_render_trace(scene.handle, arr, nc, C.byref(opts), C.c_void_p(buf.data_ptr()), None,
                                     C.byref(h), C.c_void_p(_stream_ptr(stream))))
    return buf, ForwardState(h.value, scene, shapes)


def connect_loss(scene: Scene, lam: float, grads: Optional[Dict[str, torch.Tensor]] = None, stream=None):
    """pf_connect_loss: ``lam * L_connect`` over the scene's sphere-overlap
    pairs; adds its gradient into grads['p'] / grads['radius'] (if given)
    and returns the value as a float64 device tensor [1]."""
    g = L.PfGrads()
    for f in ("p", "radius"):
        t = (grads or {}).get(f)
        if t is not None:
            if not (t.is_contiguous() and t.dtype == torch.float32 and t.shape == scene.params[f].shape):
                raise ValueError(f"gradient buffer {f} must be contiguous float32 shaped like the parameter")
            setattr(g, f, t.data_ptr())
    val = torch.zeros(1, dtype=torch.float64, device=scene.params["p"].device)
    L.check(L.load().pf_connect_loss(scene.handle, float(lam), C.byref(g), C.c_void_p(val.data_ptr()),
                                     C.c_void_p(_stream_ptr(stream))))
    return val


def query_workspace(scene: Scene, cams, what: int = 0, state_mode: int = STORE, workspace_limit: int = 0,
                    stream=None) -> int:
    """pf_query_workspace: upper bound on the device bytes the library asks
    for during a raster render (what 0), a render with a state of
    ``state_mode`` (1), or that render and its backward (2).  Runs the
    rasteriser's cull-and-count pass on ``stream`` and waits for it."""
    arr, nc, _ = _cams(cams)
    b = C.c_int64(0)
    opts = _opts(1e-6, 0, state_mode, workspace_limit)
    L.check(L.load().pf_query_workspace(scene.handle, arr, nc, int(what), C.byref(opts),
                                        C.c_void_p(_stream_ptr(stream)), C.byref(b)))
    return int(b.value)


_ALLOCATOR = {}   # the installed callbacks (kept alive while installed)


def use_torch_allocator(device=None) -> None:
    """Routes every device allocation of the library through PyTorch's
    caching allocator (pf_set_allocator), on the stream of each library call,
    so that one allocator owns all device memory.  A failed allocation makes
    the library call return OOM."""
    _require_cuda()
    dev = torch.cuda.current_device() if device is None else torch.device(device).index

    def _alloc(ctx, nbytes, stream):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), dev, int(stream or 0))
        except Exception:   # noqa: BLE001 - out of memory: the library reports OOM
            return None

    def _free(ctx, ptr, nbytes, stream):
        torch.cuda.caching_allocator_delete(int(ptr))

    a = L.PfAllocator(L.ALLOC_FN(_alloc), L.FREE_FN(_free), None)
    L.check(L.load().pf_set_allocator(C.byref(a)))
    _ALLOCATOR["active"] = a


def set_allocator(alloc_fn, free_fn) -> None:
    """Installs Python callables as the library's allocator:
    ``alloc_fn(nbytes, stream) -> int`` (device pointer, 0 on failure) and
    ``free_fn(ptr, nbytes, stream)``."""
    a = L.PfAllocator(L.ALLOC_FN(lambda ctx, n, st: alloc_fn(int(n), int(st or 0)) or None),
                      L.FREE_FN(lambda ctx, p, n, st: free_fn(int(p), int(n), int(st or 0))), None)
    L.check(L.load().pf_set_allocator(C.byref(a)))
    _ALLOCATOR["active"] = a


def use_library_allocator() -> None:
    """Restores the library's own block cache (pf_set_allocator(NULL))."""
    L.check(L.load().pf_set_allocator(None))
    _ALLOCATOR.pop("active", None)


def memory_stats(reset_peak: bool = False) -> dict:
    """pf_memory_stats: requested bytes of the library's device blocks in
    use, their high-water mark, and the bytes its cache holds."""
    live, peak, cached = C.c_int64(0), C.c_int64(0), C.c_int64(0)
    L.check(L.load().pf_memory_stats(C.byref(live), C.byref(peak), C.byref(cached), 1 if reset_peak else 0))
    return {"live": int(live.value), "peak": int(peak.value), "cached": int(cached.value)}


def backward(scene: Scene, state: ForwardState, d_rgba: torch.Tensor, grads: Dict[str, torch.Tensor],
             stream=None, lambda_normal: float = 0.0, contribution: Optional[torch.Tensor] = None,
             normal_loss: Optional[torch.Tensor] = None, pixel_error: Optional[torch.Tensor] = None,
             error: Optional[torch.Tensor] = None) -> None:
    """pf_backward: adds dL/dparams into ``grads`` (dict of float32 device
    tensors shaped like the parameters; missing keys are skipped).
    ``lambda_normal`` adds the normal loss; ``contribution`` (float32 [n]),
    ``normal_loss`` (float64 [1]) and, given the per-pixel ``pixel_error``,
    ``error`` (float32 [n]) receive the statistics (+=)."""
    d = d_rgba.contiguous()
    if d.dtype != torch.float32:
        raise TypeError("d_rgba must be float32")
    g = L.PfGrads()
    for f in PARAM_FIELDS:
        t = grads.get(f)
        if t is not None:
            if not (t.is_contiguous() and t.dtype == torch.float32 and t.shape == scene.params[f].shape):
                raise ValueError(f"gradient buffer {f} must be contiguous float32 shaped like the parameter")
            setattr(g, f, t.data_ptr())
    o = L.PfBackwardOpts(lambda_normal=float(lambda_normal))
    if contribution is not None:
        if not (contribution.is_contiguous() and contribution.dtype == torch.float32
                and contribution.numel() == scene.params["p"].shape[0]):
            raise ValueError("contribution must be a contiguous float32 tensor with one entry per cell")
        o.contribution = contribution.data_ptr()
    if normal_loss is not None:
        if not (normal_loss.dtype == torch.float64 and normal_loss.numel() >= 1):
            raise ValueError("normal_loss must be a float64 tensor")
        o.normal_loss = normal_loss.data_ptr()
    if (pixel_error is None) != (error is None):
        raise ValueError("pixel_error and error go together")
    if error is not None:
        if not (error.is_contiguous() and error.dtype == torch.float32
                and error.numel() == scene.params["p"].shape[0]):
            raise ValueError("error must be a contiguous float32 tensor with one entry per cell")
        pe = pixel_error.to(dtype=torch.float32).contiguous()
        if pe.numel() * 4 != d.numel():
            raise ValueError("pixel_error needs one value per pixel")
        o.pixel_error, o.error = pe.data_ptr(), error.data_ptr()
    L.check(L.load().pf_backward(scene.handle, state.handle, C.c_void_p(d.data_ptr()), C.byref(g), C.byref(o),
                                 C.c_void_p(_stream_ptr(stream))))


def steiner(params, z: torch.Tensor, lo_ratio: float = 2.0, hi_ratio: float = 6.0, cap: Optional[int] = None,
            stream=None) -> Dict[str, torch.Tensor]:
    """pf_steiner: Steiner cells for the walk.  ``z``: standard normal draws
    [rounds, n_cand, 3] (float32, moved to the GPU); ``params``: cell arrays
    (only p, power and radius are read).  Returns a dict of device tensors
    for the kept cells (p [A,3], power [A], radius [A], near [A] int32) and
    ``round_counts`` (list of ints)."""
    _require_cuda()
    lib = L.load()
    get = (lambda k: params[k]) if isinstance(params, dict) else (lambda k: getattr(params, k))
    t = {f: torch.as_tensor(get(f)).to(device="cuda", dtype=torch.float32).contiguous()
         for f in ("p", "power", "radius")}
    dev = t["p"].device
    zz = torch.as_tensor(z).to(device=dev, dtype=torch.float32).contiguous()
    if zz.dim() != 3 or zz.shape[2] != 3:
        raise ValueError("z must be shaped [rounds, n_cand, 3]")
    rounds, n_cand = int(zz.shape[0]), int(zz.shape[1])
    cap = rounds * n_cand if cap is None else int(cap)
    out_p = torch.empty((max(cap, 1), 3), dtype=torch.float32, device=dev)
    out_w = torch.empty(max(cap, 1), dtype=torch.float32, device=dev)
    out_r = torch.empty(max(cap, 1), dtype=torch.float32, device=dev)
    out_near = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
    pp = L.PfParams(n=int(t["p"].shape[0]), k_detail=0, m_axes=0)
    pp.p, pp.power, pp.radius = t["p"].data_ptr(), t["power"].data_ptr(), t["radius"].data_ptr()
    o = L.PfSteinerOpts(n_cand=n_cand, rounds=rounds, lo_ratio=float(lo_ratio), hi_ratio=float(hi_ratio))
    counts = (C.c_int64 * rounds)()
    n_out = C.c_int64(0)
    L.check(lib.pf_steiner(C.byref(pp), C.c_void_p(zz.data_ptr()), C.byref(o), cap, C.c_void_p(out_p.data_ptr()),
                           C.c_void_p(out_w.data_ptr()), C.c_void_p(out_r.data_ptr()),
                           C.c_void_p(out_near.data_ptr()), counts, C.byref(n_out),
                           C.c_void_p(_stream_ptr(stream))))
    a = int(n_out.value)
    return {"p": out_p[:a], "power": out_w[:a], "radius": out_r[:a], "near": out_near[:a],
            "round_counts": [int(c) for c in counts]}


def append_empty_cells(params, cells: Dict[str, torch.Tensor]) -> Dict[str, torch.Tensor]:
    """Scene arrays with ``cells`` (p, power, radius) appended as empty
    cells: zero density (occ_logit -inf), unit normal +z, zero colour and
    texture.  Such cells take part in the power diagram, so the walk crosses
    them, but never contribute to an image."""
    t = to_device_params(params)
    a = int(cells["p"].shape[0])
    dev = t["p"].device
    extra = {
        "p": cells["p"].to(dev, torch.float32).reshape(a, 3),
        "power": cells["power"].to(dev, torch.float32).reshape(a),
        "radius": cells["radius"].to(dev, torch.float32).reshape(a),
        "normal": torch.tensor([0.0, 0.0, 1.0], device=dev).expand(a, 3),
        "occ_logit": torch.full((a,), float("-inf"), device=dev),
        "rgb": torch.zeros((a, 3), device=dev),
        "tex": torch.zeros((a,) + tuple(t["tex"].shape[1:]), device=dev),
    }
    return {f: torch.cat([t[f], extra[f]]).contiguous() for f in PARAM_FIELDS}


def ema_update(ema: torch.Tensor, value: torch.Tensor, beta: float, stream=None) -> torch.Tensor:
    """pf_ema_update: ``ema = beta ema + (1 - beta) value`` in place
    (float32 device tensors of the same size)."""
    if not (ema.is_contiguous() and ema.dtype == torch.float32 and value.dtype == torch.float32
            and value.numel() == ema.numel()):
        raise ValueError("ema and value must be float32 tensors of the same size (ema contiguous)")
    v = value.contiguous()
    L.check(L.load().pf_ema_update(C.c_void_p(ema.data_ptr()), C.c_void_p(v.data_ptr()), ema.numel(), float(beta),
                                   C.c_void_p(_stream_ptr(stream))))
    return ema


def densify_prune(params, err_ema: torch.Tensor, contrib_ema: torch.Tensor, u: torch.Tensor, delta: torch.Tensor,
                  prune_below: float, spread: float, stream=None):
    """pf_densify_prune.  Returns (new cell arrays as a dict of device
    tensors, new error average, new contribution average, parent index per
    new cell).  ``u`` [n_new] uniforms, ``delta`` [n_new, 3] normal draws."""
    _require_cuda()
    t = to_device_params(params)
    n = int(t["p"].shape[0])
    dev = t["p"].device
    uu = torch.as_tensor(u).to(device=dev, dtype=torch.float32).contiguous().reshape(-1)
    dd = torch.as_tensor(delta).to(device=dev, dtype=torch.float32).contiguous().reshape(-1, 3)
    n_new = int(uu.numel())
    if dd.shape[0] < n_new:
        raise ValueError("delta needs one row per draw")
    ea = err_ema.to(device=dev, dtype=torch.float32).contiguous()
    ca = contrib_ema.to(device=dev, dtype=torch.float32).contiguous()
    if ea.numel() != n or ca.numel() != n:
        raise ValueError("err_ema and contrib_ema need one entry per cell")
    cap = n + n_new
    out = {f: torch.empty((cap,) + tuple(t[f].shape[1:]), dtype=torch.float32, device=dev) for f in PARAM_FIELDS}
    oe = torch.empty(cap, dtype=torch.float32, device=dev)
    oc = torch.empty(cap, dtype=torch.float32, device=dev)
    par = torch.empty(max(n_new, 1), dtype=torch.int32, device=dev)
    pp = L.PfParams(n=n, k_detail=int(t["tex"].shape[1]), m_axes=(int(t["tex"].shape[2]) - 3) // 6)
    for f in PARAM_FIELDS:
        setattr(pp, f, t[f].data_ptr())
    oa = L.PfCellArrays(**{f: out[f].data_ptr() for f in PARAM_FIELDS})
    o = L.PfDensifyOpts(n_new=n_new, prune_below=float(prune_below), spread=float(spread))
    nk, nd = C.c_int64(0), C.c_int64(0)
    L.check(L.load().pf_densify_prune(C.byref(pp), C.c_void_p(ea.data_ptr()), C.c_void_p(ca.data_ptr()),
                                      C.c_void_p(uu.data_ptr()), C.c_void_p(dd.data_ptr()), C.byref(o), C.byref(oa),
                                      C.c_void_p(oe.data_ptr()), C.c_void_p(oc.data_ptr()),
                                      C.c_void_p(par.data_ptr()), C.byref(nk), C.byref(nd),
                                      C.c_void_p(_stream_ptr(stream))))
    m = int(nk.value) + int(nd.value)
    return {f: out[f][:m] for f in PARAM_FIELDS}, oe[:m], oc[:m], par[:int(nd.value)]
