"""torch.autograd.Function over the renderers: forward = pf_render_raster
or pf_render_trace with a forward state, backward = pf_backward (all HIP)."""
from __future__ import annotations

from typing import List

import torch

from .api import PARAM_FIELDS, STORE, Scene, backward, render_raster_state, render_trace_state


# record count of the most recent differentiable forward (for measurement)
LAST_FORWARD = {"records": 0}


class _RenderFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, scene: Scene, cams, walk: bool, t_min: float, state_mode: int, *params):
        for f, t in zip(PARAM_FIELDS, params):
            if t.data_ptr() != scene.params[f].data_ptr():
                raise ValueError(f"parameter {f} is not the tensor the scene was built from")
        if walk:
            buf, state = render_trace_state(scene, cams, t_min=t_min, state_mode=state_mode)
        else:
            buf, state = render_raster_state(scene, cams, t_min=t_min, state_mode=state_mode)
        LAST_FORWARD["records"] = state.info()["records"]
        ctx.scene = scene
        ctx.state = state
        return buf

    @staticmethod
    def backward(ctx, g):
        scene, state = ctx.scene, ctx.state
        grads = {f: torch.zeros_like(scene.params[f]) for f in PARAM_FIELDS}
        backward(scene, state, g.contiguous(), grads)
        state.release()
        return (None, None, None, None, None) + tuple(grads[f] for f in PARAM_FIELDS)


def _render_diff(scene: Scene, cams, walk: bool, t_min: float, state_mode: int) -> List[torch.Tensor]:
    if not isinstance(cams, (list, tuple)):
        cams = [cams]
    p = scene.params
    flat = _RenderFn.apply(scene, cams, walk, t_min, state_mode, *[p[f] for f in PARAM_FIELDS])
    out, off = [], 0
    for c in cams:
        n = 4 * c.width * c.height
        out.append(flat[off:off + n].view(c.height, c.width, 4))
        off += n
    return out


def render_raster_diff(scene: Scene, cams, t_min: float = 1e-6, state_mode: int = STORE) -> List[torch.Tensor]:
    """Differentiable raster render: list of [H,W,4] images whose gradient
    flows into ``scene.params`` (build the scene from leaf tensors with
    requires_grad=True).  state_mode RECOMPUTE keeps no records between the
    forward and the backward."""
    return _render_diff(scene, cams, False, t_min, state_mode)


def render_trace_diff(scene: Scene, cams, t_min: float = 1e-6, state_mode: int = STORE) -> List[torch.Tensor]:
    """Differentiable ray-walk render (same images and gradients as the
    raster up to rounding)."""
    return _render_diff(scene, cams, True, t_min, state_mode)
