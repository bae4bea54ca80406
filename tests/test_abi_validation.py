"""The C-ABI boundary rejects bad arguments before it launches or allocates
anything: each call below must return its error status and leave the
matching message in pf_last_error.  No call reaches the GPU, so these run
on the host.  Pointers that the checks never dereference stand in for
device arrays."""
import ctypes as C
import math
import os

import pytest

from paper_2604_24994_amd import _lib as L

pytestmark = pytest.mark.skipif(not os.path.exists(L.LIB_PATH), reason="library not built")

PF_OK, PF_ERR_INVALID, PF_ERR_UNSUPPORTED = 0, 1, 4
FAKE = C.c_void_p(0x1000)   # never dereferenced by the checks exercised here


@pytest.fixture(scope="module")
def lib():
    return L.load()


def _err(lib):
    return lib.pf_last_error().decode()


def _params(n=10, k=8, m=8, sigma_scale=10.0, tau=20.0, null_field=None):
    p = L.PfParams(n=n, k_detail=k, m_axes=m, sigma_scale=sigma_scale, tau=tau)
    for f in ("p", "power", "radius", "normal", "occ_logit", "rgb", "tex"):
        setattr(p, f, 0 if f == null_field else 0x1000)
    return p


def _expect(lib, status, code, text):
    assert status == code, (status, _err(lib))
    assert text in _err(lib), _err(lib)


@pytest.mark.parametrize("kw,code,text", [
    (dict(n=0), PF_ERR_INVALID, "n must be >= 1"),
    (dict(n=1 << 30), PF_ERR_INVALID, "n must be < 2^30"),
    (dict(null_field="radius"), PF_ERR_INVALID, "a parameter array is NULL"),
    (dict(k=0), PF_ERR_INVALID, "k_detail and m_axes must be >= 1"),
    (dict(k=4), PF_ERR_UNSUPPORTED, "only k_detail = 8 and m_axes = 8"),
    (dict(sigma_scale=-1.0), PF_ERR_INVALID, "sigma_scale and tau must be finite"),
    (dict(tau=math.inf), PF_ERR_INVALID, "sigma_scale and tau must be finite"),
])
def test_build_scene_parameter_checks(lib, kw, code, text):
    out = C.c_void_p()
    p = _params(**kw)
    _expect(lib, lib.pf_build_scene(C.byref(p), None, None, C.byref(out)), code, text)
    assert out.value is None


def test_build_scene_null_arguments(lib):
    out = C.c_void_p()
    _expect(lib, lib.pf_build_scene(None, None, None, C.byref(out)), PF_ERR_INVALID, "params is NULL")
    p = _params()
    _expect(lib, lib.pf_build_scene(C.byref(p), None, None, None), PF_ERR_INVALID, "out is NULL")
    _expect(lib, lib.pf_update_scene(None, C.byref(p), None), PF_ERR_INVALID, "scene is NULL")


def _camera(**kw):
    c = L.PfCamera(model=0, width=16, height=16, fx=10.0, fy=10.0, cx=8.0, cy=8.0, f_fish=1.0, theta_max=1.0)
    for i, v in enumerate((1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, -3)):
        c.c2w[i] = v
    for k, v in kw.items():
        setattr(c, k, v)
    return c


@pytest.mark.parametrize("kw,text", [
    (dict(model=2), "camera model must be 0 or 1"),
    (dict(width=0), "camera size out of range"),
    (dict(width=1 << 16, height=1 << 16), "camera size out of range"),
    (dict(fx=0.0), "pinhole intrinsics must be finite"),
    (dict(cx=math.nan), "pinhole intrinsics must be finite"),
    (dict(model=1, theta_max=4.0), "fisheye needs f_fish > 0"),
    (dict(model=1, f_fish=0.0), "fisheye needs f_fish > 0"),
])
def test_render_camera_checks(lib, kw, text):
    cams = (L.PfCamera * 2)(_camera(), _camera(**kw))
    state = C.c_void_p(0x1)
    st = lib.pf_render_raster(FAKE, cams, 2, None, FAKE, C.byref(state), None)
    _expect(lib, st, PF_ERR_INVALID, "camera 1: " + text)
    assert state.value is None   # the state out-argument is cleared on error
    state = C.c_void_p(0x1)
    trunc = C.c_int64()
    st = lib.pf_render_trace(FAKE, cams, 2, None, FAKE, C.byref(trunc), C.byref(state), None)
    _expect(lib, st, PF_ERR_INVALID, "camera 1: " + text)
    assert state.value is None


def test_render_null_and_count_checks(lib):
    cams = (L.PfCamera * 1)(_camera())
    _expect(lib, lib.pf_render_raster(None, cams, 1, None, FAKE, None, None), PF_ERR_INVALID, "scene is NULL")
    _expect(lib, lib.pf_render_raster(FAKE, cams, 0, None, FAKE, None, None), PF_ERR_INVALID, "need ncam >= 1")
    _expect(lib, lib.pf_render_raster(FAKE, cams, 1, None, None, None, None), PF_ERR_INVALID, "rgba is NULL")
    bad = L.PfRenderOpts(t_min=1e-6, max_steps=0, state_mode=2)
    _expect(lib, lib.pf_render_raster(FAKE, cams, 1, C.byref(bad), FAKE, None, None), PF_ERR_INVALID,
            "state_mode must be 0 (store) or 1 (recompute)")
    n = C.c_int64()
    _expect(lib, lib.pf_query_workspace(FAKE, cams, 0, 0, None, None, C.byref(n)), PF_ERR_INVALID, "ncam < 1")
    _expect(lib, lib.pf_query_workspace(FAKE, cams, 1, 3, None, None, C.byref(n)), PF_ERR_INVALID,
            "what must be 0, 1 or 2")
    _expect(lib, lib.pf_query_workspace(FAKE, cams, 1, 1, C.byref(bad), None, C.byref(n)), PF_ERR_INVALID,
            "state_mode must be 0 or 1")
    neg = L.PfRenderOpts(t_min=1e-6, max_steps=0, state_mode=0, workspace_limit=-1)
    _expect(lib, lib.pf_query_workspace(FAKE, cams, 1, 1, C.byref(neg), None, C.byref(n)), PF_ERR_INVALID,
            "workspace_limit must be >= 0")
    _expect(lib, lib.pf_render_raster(FAKE, cams, 1, C.byref(neg), FAKE, None, None), PF_ERR_INVALID,
            "workspace_limit must be >= 0")


def test_backward_and_regulariser_checks(lib):
    g = L.PfGrads()
    _expect(lib, lib.pf_backward(None, FAKE, FAKE, C.byref(g), None, None), PF_ERR_INVALID, "NULL argument")
    _expect(lib, lib.pf_backward(FAKE, FAKE, FAKE, None, None, None), PF_ERR_INVALID, "NULL argument")
    loss = C.c_double()
    _expect(lib, lib.pf_connect_loss(FAKE, math.nan, C.byref(g), C.byref(loss), None), PF_ERR_INVALID,
            "lambda must be finite")
    n1, n2 = C.c_int64(), C.c_int64()
    _expect(lib, lib.pf_state_info(None, C.byref(n1), C.byref(n2), None), PF_ERR_INVALID, "NULL argument")


def _steiner(lib, p=None, rounds=6, n_cand=100, lo=2.0, hi=6.0, cap=10, outs=True, z=FAKE):
    o = L.PfSteinerOpts(n_cand=n_cand, rounds=rounds, lo_ratio=lo, hi_ratio=hi)
    n_out = C.c_int64(-7)
    arr = FAKE if outs else None
    st = lib.pf_steiner(C.byref(p if p is not None else _params()), z, C.byref(o), cap, arr, arr, arr, None, None,
                        C.byref(n_out), None)
    return st, n_out.value


@pytest.mark.parametrize("kw,text", [
    (dict(rounds=0), "rounds must be in 1 .. 64"),
    (dict(rounds=65), "rounds must be in 1 .. 64"),
    (dict(n_cand=0), "n_cand must be in 1 .. 2^31 - 1"),
    (dict(lo=7.0, hi=6.0), "lo_ratio <= hi_ratio"),
    (dict(hi=math.inf), "lo_ratio and hi_ratio must be finite"),
    (dict(cap=-1), "cap must be >= 0"),
    (dict(outs=False), "an output array is NULL"),
    (dict(z=None), "NULL argument"),
    (dict(p=_params(n=0)), "n must be in 1 .. 2^30 - 1"),
])
def test_steiner_checks(lib, kw, text):
    st, n_out = _steiner(lib, **kw)
    _expect(lib, st, PF_ERR_INVALID, text)


def test_ema_checks(lib):
    _expect(lib, lib.pf_ema_update(FAKE, FAKE, 10, 1.5, None), PF_ERR_INVALID, "beta must be in [0, 1]")
    _expect(lib, lib.pf_ema_update(FAKE, FAKE, 10, math.nan, None), PF_ERR_INVALID, "beta must be in [0, 1]")
    _expect(lib, lib.pf_ema_update(None, FAKE, 10, 0.5, None), PF_ERR_INVALID, "NULL argument or n < 0")
    _expect(lib, lib.pf_ema_update(FAKE, FAKE, -1, 0.5, None), PF_ERR_INVALID, "NULL argument or n < 0")
    # n = 0 is a no-op that succeeds without touching the arrays
    assert lib.pf_ema_update(FAKE, FAKE, 0, 0.5, None) == PF_OK


def _cell_arrays(null_field=None):
    a = L.PfCellArrays()
    for f in ("p", "power", "radius", "normal", "occ_logit", "rgb", "tex"):
        setattr(a, f, 0 if f == null_field else 0x1000)
    return a


@pytest.mark.parametrize("kw,text", [
    (dict(n_new=-1), "n_new must be >= 0"),
    (dict(n_new=1 << 30), "n + n_new < 2^30"),
    (dict(n_new=5, no_draws=True), "u and delta are needed for n_new > 0"),
    (dict(prune_below=math.inf), "prune_below and spread must be finite"),
    (dict(spread=math.nan), "prune_below and spread must be finite"),
    (dict(null_out="tex"), "an output array is NULL"),
])
def test_densify_checks(lib, kw, text):
    o = L.PfDensifyOpts(n_new=kw.get("n_new", 5), prune_below=kw.get("prune_below", 0.1),
                        spread=kw.get("spread", 0.5))
    p = _params()
    out = _cell_arrays(kw.get("null_out"))
    draws = None if kw.get("no_draws") else FAKE
    nk, nd = C.c_int64(), C.c_int64()
    st = lib.pf_densify_prune(C.byref(p), FAKE, FAKE, draws, draws, C.byref(o), C.byref(out), FAKE, FAKE, FAKE,
                              C.byref(nk), C.byref(nd), None)
    _expect(lib, st, PF_ERR_INVALID, text)


def test_profile_read_checks(lib):
    n = C.c_int32()
    _expect(lib, lib.pf_profile_read(None, 4, C.byref(n)), PF_ERR_INVALID, "NULL argument")
    _expect(lib, lib.pf_profile_read(None, 0, None), PF_ERR_INVALID, "NULL argument")


def test_allocator_and_memory_checks(lib):
    a = L.PfAllocator()
    _expect(lib, lib.pf_set_allocator(C.byref(a)), PF_ERR_INVALID, "alloc and free must both be set")
    _expect(lib, lib.pf_set_cache_limit(-1), PF_ERR_INVALID, "bytes must be >= 0")
    live, peak, cached = C.c_int64(-1), C.c_int64(-1), C.c_int64(-1)
    assert lib.pf_memory_stats(C.byref(live), C.byref(peak), C.byref(cached), 0) == PF_OK
    assert live.value >= 0 and peak.value >= live.value and cached.value >= 0
    assert lib.pf_set_allocator(None) == PF_OK
