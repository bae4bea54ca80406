"""The C-ABI library loads and exports every entry point the header declares
(no compute calls: these run without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2604_24994_amd", "libpowerfoam.so")


def _declared():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            src = open(os.path.join(ROOT, "include", fn)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names |= set(re.findall(r"\b(pf_[a-z_]+)\s*\(", src))
    return names


def test_header_declares_boundary():
    names = _declared()
    for n in ("pf_build_scene", "pf_update_scene", "pf_render_raster", "pf_render_trace", "pf_backward",
              "pf_query_workspace", "pf_connect_loss", "pf_steiner", "pf_ema_update", "pf_densify_prune",
              "pf_state_release", "pf_scene_destroy", "pf_last_error", "pf_set_allocator", "pf_set_cache_limit",
              "pf_memory_stats"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for n in sorted(_declared()):
        assert hasattr(lib, n), n


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_binding_struct_sizes_match_header_layout():
    from paper_2604_24994_amd import _lib as L
    assert ctypes.sizeof(L.PfCamera) == 4 * (3 + 12 + 6)
    assert ctypes.sizeof(L.PfParams) == 8 + 4 + 4 + 7 * 8 + 8
    assert ctypes.sizeof(L.PfRenderOpts) == 32       # float, int32, int32, int64, pointer
    assert ctypes.sizeof(L.PfAllocator) == 3 * 8
    assert ctypes.sizeof(L.PfSceneInfo) == 6 * 8 + 6 * 4
    assert ctypes.sizeof(L.PfSteinerOpts) == 8 + 4 * 4
    assert ctypes.sizeof(L.PfBackwardOpts) == 8 * 5
    assert ctypes.sizeof(L.PfDensifyOpts) == 16
    assert ctypes.sizeof(L.PfCellArrays) == 7 * 8
    lib = L.load()
    # argument errors are reported without touching a device
    h = ctypes.c_void_p()
    st = lib.pf_build_scene(None, None, None, ctypes.byref(h))
    assert st == L.PF_ERR_INVALID and b"NULL" in lib.pf_last_error()
    st = lib.pf_update_scene(None, None, None)
    assert st == L.PF_ERR_INVALID and b"pf_update_scene" in lib.pf_last_error()
    b = ctypes.c_int64(0)
    st = lib.pf_query_workspace(None, None, 0, 0, None, None, ctypes.byref(b))
    assert st == L.PF_ERR_INVALID and b"pf_query_workspace" in lib.pf_last_error()
    n_out = ctypes.c_int64(-1)
    o = L.PfSteinerOpts(n_cand=16, rounds=0, lo_ratio=2.0, hi_ratio=6.0)
    pp = L.PfParams(n=4)
    st = lib.pf_steiner(ctypes.byref(pp), ctypes.c_void_p(8), ctypes.byref(o), 0, None, None, None, None, None,
                        ctypes.byref(n_out), None)
    assert st == L.PF_ERR_INVALID and b"pf_steiner" in lib.pf_last_error()
    o.rounds = 6
    st = lib.pf_steiner(ctypes.byref(pp), ctypes.c_void_p(8), ctypes.byref(o), 0, None, None, None, None, None,
                        ctypes.byref(n_out), None)
    assert st == L.PF_ERR_INVALID and b"NULL" in lib.pf_last_error()   # p, power, radius not given
    st = lib.pf_ema_update(None, None, 4, ctypes.c_float(0.9), None)
    assert st == L.PF_ERR_INVALID and b"pf_ema_update" in lib.pf_last_error()
    st = lib.pf_ema_update(ctypes.c_void_p(8), ctypes.c_void_p(8), 4, ctypes.c_float(1.5), None)
    assert st == L.PF_ERR_INVALID and b"beta" in lib.pf_last_error()
    nk, nd = ctypes.c_int64(-1), ctypes.c_int64(-1)
    st = lib.pf_densify_prune(None, None, None, None, None, None, None, None, None, None, ctypes.byref(nk),
                              ctypes.byref(nd), None)
    assert st == L.PF_ERR_INVALID and b"pf_densify_prune" in lib.pf_last_error()
    st = lib.pf_render_trace_noalloc(None, None, 0, None, None, None, None)
    assert st == L.PF_ERR_INVALID and b"pf_render_trace_noalloc" in lib.pf_last_error()
