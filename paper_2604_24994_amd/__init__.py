"""MI355X-native differentiable rendering of bounded power diagrams.

The compute path is libpowerfoam.so (HIP, gfx950) behind the C ABI in
include/powerfoam.h; this package is its Python binding.
"""
from .api import (ForwardState, Scene, backward, build_scene, camera_struct, render_raster, render_raster_state,
                  render_trace, to_device_params)
from .autograd import render_raster_diff

__all__ = ["ForwardState", "Scene", "backward", "build_scene", "camera_struct", "render_raster",
           "render_raster_state", "render_raster_diff", "render_trace", "to_device_params"]
