"""ctypes loader for librtac.so (argument marshalling only).

The library is the product path: if it is missing the import fails loudly;
there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librtac.so")

P = ctypes.c_void_p
I32 = ctypes.c_int32
I64 = ctypes.c_int64
F32 = ctypes.c_float


class BuildParams(ctypes.Structure):
    _fields_ = [("leaf_size", I32)]


class TraceParams(ctypes.Structure):
    _fields_ = [("max_reflections", I32), ("max_path_length", F32), ("record_states", I32),
                ("fetch_threshold", I32), ("shade_threshold", I32), ("blocks_per_cu", I32),
                ("keep_order", I32), ("stats", P), ("rounds", I32), ("spill_threshold", I32),
                ("waves_per_simd", I32), ("kernel_event_start", P),
                ("kernel_event_stop", P), ("suspend_after", I32), ("min_beam_rays", I32),
                ("xcd_pools", I32), ("coop_queries", I32), ("record_rows", P), ("stack_depth", I32)]


class Job(ctypes.Structure):
    _fields_ = [("scene", I32), ("n_rcv", I32), ("n_rays", I64), ("src", F32 * 3), ("max_path_length", F32)]


# symbol -> (restype, argtypes); mirrors include/rtac.h
SIGNATURES = {
    "rt_build_tree": (ctypes.c_int, [P, I64, P, I64, P, P, ctypes.POINTER(BuildParams), P, ctypes.POINTER(P)]),
    "rt_rebuild_tree": (ctypes.c_int, [P, P, I64, P, I64, P, P, ctypes.POINTER(BuildParams), P]),
    "rt_scene_destroy": (ctypes.c_int, [P]),
    "rt_scene_info": (ctypes.c_int, [P, P, P]),
    "rt_fibonacci_directions": (ctypes.c_int, [I64, P, P]),
    "rt_icosahedral_directions": (ctypes.c_int, [I32, P, P]),
    "rt_directional_directions": (ctypes.c_int, [I64, ctypes.c_double, P, P, P]),
    "rt_trace_rays": (ctypes.c_int, [P, P, P, P, P, P, I64, P, I32, ctypes.POINTER(TraceParams), P, P, I64, P, P,
                                     P]),
    "rt_collect_image_sources": (ctypes.c_int, [P, P, P, I32, P, I64, I32, P, I64, P, P, P, P, P, I64, P, P]),
    "rt_assemble_ir": (ctypes.c_int, [P, P, P, P, P, I64, I32, I64, I32, P, P, F32, F32, I64, P, I32, P, P, P, P,
                                      P]),
    "rt_band_energy_adjoint": (ctypes.c_int, [P, P, P, P, P, I64, I32, I64, I32, P, I32, P, F32, F32, I64, P, P,
                                              P]),
    "rt_batch_create": (ctypes.c_int, [P, I32, P, I32, P, ctypes.POINTER(P)]),
    "rt_batch_destroy": (ctypes.c_int, [P]),
    "rt_batch_info": (ctypes.c_int, [P, P]),
    "rt_trace_batch": (ctypes.c_int, [P, P, ctypes.POINTER(TraceParams), P, P, I64, P, P, P]),
    "rt_collect_batch": (ctypes.c_int, [P, P, P, I32, P, I64, P, P, P, P, P, I64, P, P]),
    "rt_assemble_batch": (ctypes.c_int, [P, P, P, P, P, I64, I32, P, P, F32, F32, I64, P, I32, P, P, P, P, P]),
    "rt_adjoint_batch": (ctypes.c_int, [P, P, P, P, P, I64, I32, P, P, F32, F32, I64, P, P, P]),
    "rt_mlp_create": (ctypes.c_int, [P, I32, I64, ctypes.POINTER(P)]),
    "rt_mlp_destroy": (ctypes.c_int, [P]),
    "rt_mlp_info": (ctypes.c_int, [P, P]),
    "rt_mlp_forward": (ctypes.c_int, [P, P, P, P, I64, P, P]),
    "rt_mlp_backward": (ctypes.c_int, [P, P, P, I64, P, P, P, P, P, P]),
    "rt_mlp_adam": (ctypes.c_int, [I64, P, P, P, P, P, P, I32, F32, F32, F32, F32, P]),
    "rt_to_bf16": (ctypes.c_int, [P, I64, P, P]),
    "rt_hist_features": (ctypes.c_int, [P, I64, F32, F32, F32, P, P]),
    "rt_edc_db": (ctypes.c_int, [P, I64, I32, F32, P, P]),
    "rt_room_params": (ctypes.c_int, [P, I32, I64, F32, P, P]),
    "rt_room_params_noalloc": (ctypes.c_int, [P, I32, I64, F32, P, P]),
    "rt_debug_set_hash_bits": (ctypes.c_int, [ctypes.c_int]),
    "rt_debug_radix_sort": (ctypes.c_int, [P, P, I64, P, I32, I32, P]),
    "rt_last_error": (ctypes.c_char_p, []),
    "rt_version": (ctypes.c_char_p, []),
}

_lib = None


def load():
    """Load librtac.so and set every signature; raises if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("librtac.so is not built (run `python -c 'import __graft_entry__ as g; g.build()'` "
                          "or `python paper_1811_05784_amd/build.py`): %s" % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class RtError(RuntimeError):
    pass


def check(status: int, what: str):
    if status != 0:
        msg = load().rt_last_error().decode(errors="replace")
        raise RtError("%s failed (status %d): %s" % (what, status, msg))
