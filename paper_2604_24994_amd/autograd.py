"""torch.autograd.Function over the renderers: forward = pf_render_raster
or pf_render_trace with a forward state, backward = pf_backward (all HIP)."""
from __future__ import annotations

from typing import List, Optional

import torch

from .api import PARAM_FIELDS, STORE, Scene, backward, render_raster_state, render_trace_state


# record count of the most recent differentiable forward (for measurement)
LAST_FORWARD = {"records": 0, "mode": "store"}


class _RenderFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, scene: Scene, cams, walk: bool, t_min: float, state_mode: int, workspace_limit: int,
                lambda_normal: float, stats, *params):
        for f, t in zip(PARAM_FIELDS, params):
            if t.data_ptr() != scene.params[f].data_ptr():
                raise ValueError(f"parameter {f} is not the tensor the scene was built from")
        if walk:
            buf, state = render_trace_state(scene, cams, t_min=t_min, state_mode=state_mode,
                                            workspace_limit=workspace_limit)
        else:
            buf, state = render_raster_state(scene, cams, t_min=t_min, state_mode=state_mode,
                                             workspace_limit=workspace_limit)
        info = state.info()
        LAST_FORWARD["records"] = info["records"]
        LAST_FORWARD["mode"] = info["mode"]
        ctx.scene = scene
        ctx.state = state
        ctx.lambda_normal = lambda_normal
        ctx.stats = stats
        return buf

    @staticmethod
    def backward(ctx, g):
        scene, state, stats = ctx.scene, ctx.state, ctx.stats
        grads = {f: torch.zeros_like(scene.params[f]) for f in PARAM_FIELDS}
        contribution = normal_loss = error = pixel_error = None
        if stats is not None:
            dev = scene.params["p"].device
            contribution = torch.zeros(scene.params["p"].shape[0], dtype=torch.float32, device=dev)
            normal_loss = torch.zeros(1, dtype=torch.float64, device=dev)
            pixel_error = stats.get("pixel_error")
            if pixel_error is not None:
                error = torch.zeros_like(contribution)
        backward(scene, state, g.contiguous(), grads, lambda_normal=ctx.lambda_normal, contribution=contribution,
                 normal_loss=normal_loss, pixel_error=pixel_error, error=error)
        state.release()
        if stats is not None:
            stats["contribution"] = contribution
            stats["normal_loss"] = normal_loss
            if error is not None:
                stats["error"] = error
        return (None,) * 8 + tuple(grads[f] for f in PARAM_FIELDS)


def _render_diff(scene: Scene, cams, walk: bool, t_min: float, state_mode: int, workspace_limit: int,
                 lambda_normal: float, stats) -> List[torch.Tensor]:
    if not isinstance(cams, (list, tuple)):
        cams = [cams]
    p = scene.params
    flat = _RenderFn.apply(scene, cams, walk, t_min, state_mode, int(workspace_limit), float(lambda_normal), stats,
                           *[p[f] for f in PARAM_FIELDS])
    out, off = [], 0
    for c in cams:
        n = 4 * c.width * c.height
        out.append(flat[off:off + n].view(c.height, c.width, 4))
        off += n
    return out


def render_raster_diff(scene: Scene, cams, t_min: float = 1e-6, state_mode: int = STORE,
                       lambda_normal: float = 0.0, stats: Optional[dict] = None,
                       workspace_limit: int = 0) -> List[torch.Tensor]:
    """Differentiable raster render: list of [H,W,4] images whose gradient
    flows into ``scene.params`` (build the scene from leaf tensors with
    requires_grad=True).  state_mode RECOMPUTE keeps no records between the
    forward and the backward, which replays the forward in windows of at most
    ``workspace_limit`` bytes of records (0: 2 GiB); in STORE mode a forward
    whose records exceed a non-zero ``workspace_limit`` falls back to that.
    ``lambda_normal`` adds the normal loss of the rendered rays to the
    objective (its gradient joins the backward); a
    ``stats`` dict receives, after backward, 'contribution' (per-cell sum of
    T a) and 'normal_loss' (the unweighted loss value); if it holds a
    'pixel_error' tensor (one value per pixel of all images, set before the
    backward runs) it also receives 'error' (per-cell sum of T a e, the
    statistic densification averages).  The sparsity loss summed over cells
    is the sum of the A channel of the images."""
    return _render_diff(scene, cams, False, t_min, state_mode, workspace_limit, lambda_normal, stats)


def render_trace_diff(scene: Scene, cams, t_min: float = 1e-6, state_mode: int = STORE,
                      lambda_normal: float = 0.0, stats: Optional[dict] = None,
                      workspace_limit: int = 0) -> List[torch.Tensor]:
    """Differentiable ray-walk render (same images and gradients as the
    raster up to rounding)."""
    return _render_diff(scene, cams, True, t_min, state_mode, workspace_limit, lambda_normal, stats)
