import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


def make_scene(p, power, radius, normal=None, occ_logit=None, rgb=None, tex=None,
               k=8, m=8, seed=0, sigma_scale=10.0, tau=20.0):
    """Hand-built scene for closed-form tests (float32 arrays)."""
    import workloads as W
    rng = np.random.default_rng(seed)
    p = np.asarray(p, dtype=np.float64).reshape(-1, 3)
    n = p.shape[0]
    if normal is None:
        normal = rng.normal(size=(n, 3))
        normal /= np.linalg.norm(normal, axis=1, keepdims=True)
    if occ_logit is None:
        occ_logit = rng.normal(size=n)
    if rgb is None:
        rgb = rng.uniform(size=(n, 3))
    if tex is None:
        tex = rng.normal(0, 0.1, size=(n, k, 3 + 6 * m))
    f32 = lambda a: np.ascontiguousarray(np.asarray(a), dtype=np.float32)
    return W.Scene(p=f32(p), power=f32(np.broadcast_to(power, (n,))), radius=f32(np.broadcast_to(radius, (n,))),
                   normal=f32(np.asarray(normal).reshape(n, 3)), occ_logit=f32(np.broadcast_to(occ_logit, (n,))),
                   rgb=f32(np.asarray(rgb).reshape(n, 3)), tex=f32(tex), sigma_scale=sigma_scale, tau=tau)


@pytest.fixture
def scene_factory():
    return make_scene


def grad_errors(g, ref):
    """Gradient errors against a reference (oracle) gradient, by the bar of
    the parity tests: per tensor ``|g - ref|_inf / |ref|_inf`` and per
    component ``max_c |g_c - ref_c| / max(|ref_c|, 1e-2 |ref|_inf)``.  Both
    must stay <= 1e-3."""
    g = np.asarray(g, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64).reshape(g.shape)
    scale = np.abs(ref).max()
    if scale == 0:
        return 0.0 if np.abs(g).max() == 0 else np.inf, 0.0 if np.abs(g).max() == 0 else np.inf
    err = np.abs(g - ref)
    per_tensor = err.max() / scale
    per_comp = (err / np.maximum(np.abs(ref), 1e-2 * scale)).max()
    return float(per_tensor), float(per_comp)


def worst_component(g, ref):
    """(flat index, g, ref, error ratio) of the component with the largest
    per-component error."""
    g = np.asarray(g, dtype=np.float64).reshape(-1)
    ref = np.asarray(ref, dtype=np.float64).reshape(-1)
    scale = np.abs(ref).max()
    ratio = np.abs(g - ref) / np.maximum(np.abs(ref), 1e-2 * scale) if scale > 0 else np.abs(g - ref)
    i = int(np.argmax(ratio))
    return i, float(g[i]), float(ref[i]), float(ratio[i])


def assert_grad_close(g, ref, name, tol=1e-3, log=print, may_vanish=False):
    """Per-tensor and per-component bars.  ``may_vanish``: the parameter has
    no influence in this configuration (e.g. the weight of a lone cell), so
    both gradients must be exactly zero."""
    if may_vanish and np.abs(np.asarray(ref)).max() == 0:
        log(f"  {name:10s} reference gradient is zero; GPU |g|max {np.abs(np.asarray(g)).max():.3e}")
        assert np.abs(np.asarray(g)).max() == 0, name
        return
    t, c = grad_errors(g, ref)
    i, gi, ri, _ = worst_component(g, ref)
    log(f"  {name:10s} |ref|max {np.abs(np.asarray(ref)).max():.4e}  rel {t:.3e}  per-component {c:.3e} "
        f"(worst at flat index {i}: {gi:.6e} vs {ri:.6e})")
    assert np.abs(np.asarray(ref)).max() > 0, name
    assert t <= tol, (name, t)
    assert c <= tol, (name, c)
