"""MI355X-native differentiable rendering of bounded power diagrams.

The compute path is libpowerfoam.so (HIP, gfx950) behind the C ABI in
include/powerfoam.h; this package is its Python binding.
"""
from .api import (RECOMPUTE, STORE, ForwardState, Scene, append_empty_cells, backward, build_scene, camera_struct,
                  connect_loss, densify_prune, ema_update, memory_stats, query_workspace, set_allocator, steiner,
                  render_raster, render_raster_state, render_trace, render_trace_noalloc, render_trace_state,
                  to_device_params,
                  update_scene, use_library_allocator, use_torch_allocator)
from .autograd import render_raster_diff, render_trace_diff

__all__ = ["RECOMPUTE", "STORE", "ForwardState", "Scene", "append_empty_cells", "backward", "build_scene", "camera_struct", "connect_loss", "densify_prune", "ema_update",
           "query_workspace", "render_raster", "render_raster_state", "render_raster_diff", "render_trace",
           "render_trace_state", "render_trace_diff", "render_trace_noalloc", "steiner", "to_device_params", "update_scene", "memory_stats",
           "set_allocator", "use_library_allocator", "use_torch_allocator"]
