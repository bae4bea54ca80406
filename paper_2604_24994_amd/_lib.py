"""ctypes view of include/powerfoam.h (argument marshalling only)."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpowerfoam.so")

PF_OK, PF_ERR_INVALID, PF_ERR_OOM, PF_ERR_HIP, PF_ERR_UNSUPPORTED, PF_ERR_OVERFLOW = range(6)
STATUS_NAMES = {0: "OK", 1: "INVALID", 2: "OOM", 3: "HIP", 4: "UNSUPPORTED", 5: "OVERFLOW"}

EXPORTS = ("pf_build_scene", "pf_scene_info_get", "pf_scene_adjacency", "pf_scene_destroy",
           "pf_render_raster", "pf_render_trace", "pf_backward", "pf_state_release", "pf_last_error",
           "pf_profile_enable", "pf_profile_read", "pf_state_info", "pf_update_scene", "pf_query_workspace",
           "pf_connect_loss", "pf_steiner", "pf_ema_update", "pf_densify_prune", "pf_set_allocator",
           "pf_set_cache_limit", "pf_memory_stats", "pf_render_trace_noalloc")


class PfParams(C.Structure):
    _fields_ = [("n", C.c_int64), ("k_detail", C.c_int32), ("m_axes", C.c_int32),
                ("p", C.c_void_p), ("power", C.c_void_p), ("radius", C.c_void_p),
                ("normal", C.c_void_p), ("occ_logit", C.c_void_p), ("rgb", C.c_void_p),
                ("tex", C.c_void_p), ("sigma_scale", C.c_float), ("tau", C.c_float)]


class PfCamera(C.Structure):
    _fields_ = [("model", C.c_int32), ("width", C.c_int32), ("height", C.c_int32),
                ("c2w", C.c_float * 12), ("fx", C.c_float), ("fy", C.c_float),
                ("cx", C.c_float), ("cy", C.c_float), ("f_fish", C.c_float),
                ("theta_max", C.c_float)]


class PfBuildOpts(C.Structure):
    _fields_ = [("box_min", C.c_float * 3), ("box_max", C.c_float * 3), ("box_pad", C.c_float)]


class PfRenderOpts(C.Structure):
    _fields_ = [("t_min", C.c_float), ("max_steps", C.c_int32), ("state_mode", C.c_int32),
                ("workspace_limit", C.c_int64), ("counters", C.c_void_p)]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p)


class PfAllocator(C.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("ctx", C.c_void_p)]


class PfSceneInfo(C.Structure):
    _fields_ = [("n", C.c_int64), ("n_faces", C.c_int64), ("n_hidden", C.c_int64),
                ("n_overflow", C.c_int64), ("n_high_degree", C.c_int64), ("n_dropped", C.c_int64),
                ("box_min", C.c_float * 3),
                ("box_max", C.c_float * 3)]


class PfProfileEntry(C.Structure):
    _fields_ = [("name", C.c_char * 48), ("launches", C.c_int64), ("total_ms", C.c_double)]


class PfBackwardOpts(C.Structure):
    _fields_ = [("lambda_normal", C.c_float), ("contribution", C.c_void_p), ("normal_loss", C.c_void_p),
                ("pixel_error", C.c_void_p), ("error", C.c_void_p)]


class PfDensifyOpts(C.Structure):
    _fields_ = [("n_new", C.c_int64), ("prune_below", C.c_float), ("spread", C.c_float)]


class PfSteinerOpts(C.Structure):
    _fields_ = [("n_cand", C.c_int64), ("rounds", C.c_int32), ("lo_ratio", C.c_float),
                ("hi_ratio", C.c_float), ("reserved", C.c_int32)]


class PfGrads(C.Structure):
    _fields_ = [("p", C.c_void_p), ("power", C.c_void_p), ("radius", C.c_void_p),
                ("normal", C.c_void_p), ("occ_logit", C.c_void_p), ("rgb", C.c_void_p),
                ("tex", C.c_void_p)]


class PfCellArrays(C.Structure):
    _fields_ = [("p", C.c_void_p), ("power", C.c_void_p), ("radius", C.c_void_p),
                ("normal", C.c_void_p), ("occ_logit", C.c_void_p), ("rgb", C.c_void_p),
                ("tex", C.c_void_p)]


_lib = None


def load(path: str = LIB_PATH) -> C.CDLL:
    """Loads the HIP library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libpowerfoam.so not found at {path}; build it with "
                           f"`python -m paper_2604_24994_amd.build`")
    lib = C.CDLL(path)
    vp, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
    lib.pf_build_scene.argtypes = [C.POINTER(PfParams), C.POINTER(PfBuildOpts), vp, C.POINTER(vp)]
    lib.pf_scene_info_get.argtypes = [vp, C.POINTER(PfSceneInfo)]
    lib.pf_scene_adjacency.argtypes = [vp, vp, vp, vp]
    lib.pf_scene_destroy.argtypes = [vp]
    lib.pf_scene_destroy.restype = None
    lib.pf_render_raster.argtypes = [vp, C.POINTER(PfCamera), i32, C.POINTER(PfRenderOpts), vp,
                                     C.POINTER(vp), vp]
    lib.pf_render_trace.argtypes = [vp, C.POINTER(PfCamera), i32, C.POINTER(PfRenderOpts), vp,
                                    C.POINTER(i64), C.POINTER(vp), vp]
    lib.pf_render_trace_noalloc.argtypes = [vp, C.POINTER(PfCamera), i32, C.POINTER(PfRenderOpts), vp,
                                            C.POINTER(i64), vp]
    lib.pf_update_scene.argtypes = [vp, C.POINTER(PfParams), vp]
    lib.pf_query_workspace.argtypes = [vp, C.POINTER(PfCamera), i32, i32, C.POINTER(PfRenderOpts), vp,
                                       C.POINTER(i64)]
    lib.pf_set_allocator.argtypes = [C.POINTER(PfAllocator)]
    lib.pf_set_cache_limit.argtypes = [i64]
    lib.pf_memory_stats.argtypes = [C.POINTER(i64), C.POINTER(i64), C.POINTER(i64), i32]
    lib.pf_connect_loss.argtypes = [vp, C.c_float, C.POINTER(PfGrads), vp, vp]
    lib.pf_steiner.argtypes = [C.POINTER(PfParams), vp, C.POINTER(PfSteinerOpts), i64, vp, vp, vp, vp,
                               C.POINTER(i64), C.POINTER(i64), vp]
    lib.pf_ema_update.argtypes = [vp, vp, i64, C.c_float, vp]
    lib.pf_densify_prune.argtypes = [C.POINTER(PfParams), vp, vp, vp, vp, C.POINTER(PfDensifyOpts),
                                     C.POINTER(PfCellArrays), vp, vp, vp, C.POINTER(i64), C.POINTER(i64), vp]
    lib.pf_backward.argtypes = [vp, vp, vp, C.POINTER(PfGrads), C.POINTER(PfBackwardOpts), vp]
    lib.pf_state_release.argtypes = [vp]
    lib.pf_state_release.restype = None
    lib.pf_state_info.argtypes = [vp, C.POINTER(i64), C.POINTER(i64), C.POINTER(i32)]
    lib.pf_profile_enable.argtypes = [i32]
    lib.pf_profile_read.argtypes = [C.POINTER(PfProfileEntry), i32, C.POINTER(i32)]
    lib.pf_last_error.argtypes = []
    lib.pf_last_error.restype = C.c_char_p
    for name in EXPORTS:
        if name not in ("pf_scene_destroy", "pf_state_release", "pf_last_error"):
            getattr(lib, name).restype = C.c_int
    _lib = lib
    return lib


def profile_enable(on: bool = True) -> None:
    check(load().pf_profile_enable(1 if on else 0))


def profile_read() -> dict:
    """{kernel name: (launches, total ms)} since the last read (waits for
    the recorded events)."""
    buf = (PfProfileEntry * 64)()
    n = C.c_int32(0)
    check(load().pf_profile_read(buf, 64, C.byref(n)))
    return {buf[i].name.decode(): (int(buf[i].launches), float(buf[i].total_ms)) for i in range(n.value)}


class PowerFoamError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def check(status: int) -> None:
    if status != PF_OK:
        raise PowerFoamError(status, load().pf_last_error().decode(errors="replace"))
