"""FP64 CPU oracle for bounded-power-diagram rendering.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously correct
restatement of what the renderer computes.  Only ``tests/``, the smoke check
in ``__graft_entry__.py`` and the CPU-baseline leg of ``bench.py`` may import
it; the GPU library never calls it, and it shares no code with the GPU path
(its only common dependency is the seeded input generator ``workloads``).

What it computes (all in float64, from the float32 inputs as given):

* power distance ``pow(x,i) = |x - p_i|^2 - w_i`` and the power cell
  ``Pi_i = {x : pow(x,i) <= pow(x,j) for all j}`` (Sec. 3.2; appendix B,
  power-distance and power-cell equations);
* the rendered cell ``Pi_i`` intersected with the sphere ``B(p_i, r_i)``
  (Sec. 3.2, bounded power diagram);
* the oriented dipole split with a soft-Voronoi displacement and the
  soft-Voronoi / Spherical-Voronoi radiance (Sec. 3.3, Sec. 3.4 Eq. svdisp and
  Eq. svrad);
* the exact segment-sum volume rendering ``C = sum_k T_k a_k c_k``
  (Sec. 3.1);
* the training regularisers of the supplementary material (normal,
  sparsity, connectivity) and the per-cell contribution statistic;
* the Steiner cells of the supplementary material (Alg. 1) that fill empty
  space for the walk;
* the per-cell error statistic, moving averages, pruning and multinomial
  densification of Sec. 3.5.

Two independent forms are provided: the brute-force walk (start cell by
argmin power distance over all sites, each exit by brute force over every
bisector plane) and the painter form (every cell's interval by brute force,
ordered by the power distance from the camera, appendix B theorem).  The
adjoint replays the walk's discrete decisions and differentiates the same
formulas with torch autograd in float64.

Parity-pinned parts and the pins are listed in the test modules
``tests/test_oracle_*.py``.
"""
from .camera import generate_rays, pixel_rays
from .cell import (bisector, onb, power_distance, shade, softplus, sphere_interval,
                   scene_tensors)
from .walk import render_walk, walk_records
from .painter import render_painter
from .adjoint import adjoint_gradients, loss_from_rgba
from .dense import dense_sample_ray
from .regularizers import connect_loss, normal_loss_value, regularized_gradients
from .steiner import evaluate_candidates, steiner_points
from .densify import cell_error, densify_prune, draw, ema

__all__ = [
    "generate_rays", "pixel_rays", "bisector", "onb", "power_distance", "shade",
    "softplus", "sphere_interval", "scene_tensors", "render_walk", "walk_records",
    "render_painter", "adjoint_gradients", "loss_from_rgba", "dense_sample_ray",
    "regularized_gradients", "normal_loss_value", "connect_loss", "evaluate_candidates", "steiner_points",
    "cell_error", "densify_prune", "draw", "ema",
]
