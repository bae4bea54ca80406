"""MI355X-native differentiable rendering of bounded power diagrams.

The compute path is libpowerfoam.so (HIP, gfx950) behind the C ABI in
include/powerfoam.h; this package is its Python binding.
"""
from .api import Scene, build_scene, camera_struct, render_raster, render_trace, to_device_params

__all__ = ["Scene", "build_scene", "camera_struct", "render_raster", "render_trace", "to_device_params"]
