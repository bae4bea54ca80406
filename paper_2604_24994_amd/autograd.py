"""torch.autograd.Function over the rasteriser: forward = pf_render_raster
with a forward state, backward = pf_backward (both HIP)."""
from __future__ import annotations

from typing import List

import torch

from .api import PARAM_FIELDS, Scene, backward, render_raster_state


# record count of the most recent differentiable forward (for measurement)
LAST_FORWARD = {"records": 0}


class _RasterFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, scene: Scene, cams, t_min: float, *params):
        for f, t in zip(PARAM_FIELDS, params):
            if t.data_ptr() != scene.params[f].data_ptr():
                raise ValueError(f"parameter {f} is not the tensor the scene was built from")
        buf, state = render_raster_state(scene, cams, t_min=t_min)
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
        return (None, None, None) + tuple(grads[f] for f in PARAM_FIELDS)


def render_raster_diff(scene: Scene, cams, t_min: float = 1e-6) -> List[torch.Tensor]:
    """Differentiable raster render: list of [H,W,4] images whose gradient
    flows into ``scene.params`` (build the scene from leaf tensors with
    requires_grad=True)."""
    if not isinstance(cams, (list, tuple)):
        cams = [cams]
    p = scene.params
    flat = _RasterFn.apply(scene, cams, t_min, *[p[f] for f in PARAM_FIELDS])
    out, off = [], 0
    for c in cams:
        n = 4 * c.width * c.height
        out.append(flat[off:off + n].view(c.height, c.width, 4))
        off += n
    return out
