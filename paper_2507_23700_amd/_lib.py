"""ctypes loader for libarborx355.so (the HIP library behind include/arborx.h).

Loading fails loudly when the library has not been built: there is no CPU
fallback anywhere in this package.
"""
from __future__ import annotations

import ctypes
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libarborx355.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "arborx.h")

P, I32, I64, F32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_float

SIGNATURES = {
    "arborx_version": (ctypes.c_char_p, []),
    "arborx_last_error": (ctypes.c_char_p, []),
    "arborx_set_allocator": (I32, [P, P, P]),
    "arborx_set_tuning": (I32, [P]),
    "arborx_get_tuning": (I32, [P]),
    "arborx_set_tuning_op": (I32, [I32, P]),
    "arborx_get_tuning_op": (I32, [I32, P]),
    "arborx_autotune": (I32, [P, I32, P, I64, F32, I32, P, P, P]),
    "arborx_autotune_forest": (I32, [P, I32, P, I64, P, P, P, I32, I32, P, P, P]),
    "arborx_bvh_build": (I32, [P, I64, I32, I32, P, P]),
    "arborx_bvh_destroy": (I32, [P]),
    "arborx_bvh_info": (I32, [P, P, P, P, P, P]),
    "arborx_query_spatial": (I32, [P, P, I64, F32, P, P, I64, P, P]),
    "arborx_query_intersects": (I32, [P, P, I64, P, P, I64, P, P]),
    "arborx_query_knn": (I32, [P, P, I64, I32, P, P, P]),
    "arborx_query_knn_noalloc": (I32, [P, P, I64, I32, P, P, P]),
    "arborx_query_spatial_reduce": (I32, [P, P, I64, F32, I32, P, P, I32, P]),
    "arborx_query_spatial_count_up_to": (I32, [P, P, I64, F32, I32, P, P]),
    "arborx_query_match_distances": (I32, [P, P, P, I64, P, P, P, P]),
    "arborx_dbscan": (I32, [P, P, F32, I32, P, P]),
    "arborx_self_join_degree": (I32, [P, F32, P, P]),
    "arborx_query_ray_count": (I32, [P, P, I64, P, P]),
    "arborx_query_ray_intersect": (I32, [P, P, I64, P, P, I64, P, P]),
    "arborx_query_ray_intersect_begin": (I32, [P, P, I64, P, P, P, P]),
    "arborx_query_ray_ordered_intersect": (I32, [P, P, I64, P, P, P, I64, P, P]),
    "arborx_query_ray_ordered_intersect_begin": (I32, [P, P, I64, P, P, P, P]),
    "arborx_query_ray_nearest": (I32, [P, P, I64, I32, P, P, P]),
    "arborx_debug_radix_sort": (I32, [P, P, I64, I32, I32, I32, P]),
    "arborx_debug_morton64": (I32, [P, I64, I32, P, P, P]),
    "arborx_debug_tree_nodes": (I32, [P, P, P, P, P]),
    "arborx_debug_node_visits": (I32, [P, P, I64, F32, I32, I32, P, P]),
    "arborx_debug_valu_probe": (I32, [P, I32, I32, P]),
    "arborx_query_spatial_begin": (I32, [P, P, I64, F32, P, P, P, P]),
    "arborx_query_intersects_begin": (I32, [P, P, I64, P, P, P, P]),
    "arborx_query_finish": (I32, [P, P, I64]),
    "arborx_query_finish_unsorted": (I32, [P, P, I64]),
    "arborx_query_spatial_with_distances": (I32, [P, P, I64, F32, P, P, P, I64, P, P]),
    "arborx_query_spatial_with_distances_begin": (I32, [P, P, I64, F32, P, P, P, P]),
    "arborx_query_finish_with_distances": (I32, [P, P, P, I64]),
    "arborx_plan_destroy": (I32, [P]),
    "arborx_forest_build": (I32, [P, P, I32, I32, I32, P, P]),
    "arborx_forest_destroy": (I32, [P]),
    "arborx_forest_create": (I32, [I64, I32, I32, I32, P, P]),
    "arborx_forest_rebuild": (I32, [P, P, P, P]),
    "arborx_forest_info": (I32, [P, P, P, P, P, P]),
    "arborx_forest_reserve": (I32, [P, I64, P]),
    "arborx_forest_query_reduce": (I32, [P, P, I64, P, P, P, I32, I32, P, P, I32, P]),
    "arborx_forest_query_knn": (I32, [P, P, I64, P, P, I32, I32, P, P, P]),
    "arborx_chamfer_forward": (I32, [P, P, P, P, I32, P, P, P, P]),
    "arborx_chamfer_backward": (I32, [P, P, P, P, I32, P, P, P, P, P, P]),
    "arborx_profile_enable": (I32, [I32]),
    "arborx_profile_collect": (I32, [P, P, P, I32, P]),
}

_lib = None


class Tuning(ctypes.Structure):
    _fields_ = [("block", I32), ("order", I32), ("stack", I32), ("schedule", I32), ("build", I32),
                ("seed_mode", I32), ("node_format", I32),
                ("queries_per_thread", I32)]


def header_symbols() -> list[str]:
    """Names of every function include/arborx.h declares."""
    with open(HEADER) as f:
        text = f.read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[\w\s\*]+?\b(arborx_\w+)\s*\(", text, re.M)))


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2507_23700_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib
