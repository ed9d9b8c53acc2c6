"""C-ABI checks that need no GPU: the library loads, exports every declared
symbol, and rejects bad arguments on the host before any device work."""
import ctypes
import os

import pytest

import paper_2507_23700_amd as ax
from paper_2507_23700_amd import _lib, build

L = None


def setup_module(module):
    global L
    if not os.path.exists(_lib.LIB_PATH):
        build.build()
    L = _lib.lib()


def _has_gpu():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def test_every_declared_symbol_is_exported():
    names = _lib.header_symbols()
    assert len(names) >= 14
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(_lib.SIGNATURES)


def test_version_and_error_string():
    assert L.arborx_version().decode().startswith("arborx355")
    assert isinstance(L.arborx_last_error(), bytes)


P = ctypes.c_void_p
FAKE = P(0x1000)  # never dereferenced: validation fails first


def _err():
    return L.arborx_last_error().decode()


def test_build_argument_validation():
    out = P()
    assert L.arborx_bvh_build(FAKE, 10, 3, 0, None, None) == 1
    assert L.arborx_bvh_build(FAKE, -1, 3, 0, None, ctypes.byref(out)) == 1
    assert L.arborx_bvh_build(FAKE, 10, 0, 0, None, ctypes.byref(out)) == 1
    assert L.arborx_bvh_build(FAKE, 10, 11, 0, None, ctypes.byref(out)) == 1
    assert L.arborx_bvh_build(FAKE, 10, 3, 7, None, ctypes.byref(out)) == 1
    assert L.arborx_bvh_build(None, 10, 3, 0, None, ctypes.byref(out)) == 1
    assert "NULL" in _err()
    assert L.arborx_bvh_build(FAKE, 2 ** 31, 3, 0, None, ctypes.byref(out)) == 1
    assert L.arborx_bvh_build(FAKE, 10, 4, 0, None, ctypes.byref(out)) == 2
    assert out.value is None


def test_query_argument_validation():
    f = ctypes.c_float
    tot = ctypes.c_int64()
    assert L.arborx_query_spatial(None, FAKE, 1, f(1), FAKE, FAKE, 1, ctypes.byref(tot), None) == 1
    assert L.arborx_query_knn(None, FAKE, 1, 3, FAKE, FAKE, None) == 1
    assert L.arborx_query_spatial_reduce(None, FAKE, 1, f(1), 0, FAKE, None, 32, None) == 1
    assert L.arborx_query_spatial_count_up_to(None, FAKE, 1, f(1), 5, FAKE, None) == 1
    assert L.arborx_query_match_distances(None, FAKE, FAKE, 1, FAKE, FAKE, FAKE, None) == 1
    assert L.arborx_dbscan(None, FAKE, f(1), 2, FAKE, None) == 1
    assert L.arborx_query_ray_count(None, FAKE, 1, FAKE, None) == 1
    assert L.arborx_query_ray_nearest(None, FAKE, 1, 3, FAKE, FAKE, None) == 1
    assert L.arborx_query_intersects(None, FAKE, 1, FAKE, FAKE, 1, ctypes.byref(tot), None) == 1
    assert L.arborx_bvh_info(None, None, None, None, None, None) == 1
    assert L.arborx_debug_tree_nodes(None, FAKE, FAKE, FAKE, FAKE) == 1
    assert L.arborx_bvh_destroy(None) == 0
    plan = P()
    assert L.arborx_query_spatial_begin(None, FAKE, 1, f(1), FAKE, ctypes.byref(tot), ctypes.byref(plan), None) == 1
    assert L.arborx_query_intersects_begin(None, FAKE, 1, FAKE, ctypes.byref(tot), ctypes.byref(plan), None) == 1
    assert L.arborx_query_finish(None, FAKE, 1) == 1
    assert L.arborx_query_finish_unsorted(None, FAKE, 1) == 1
    assert L.arborx_plan_destroy(None) == 0


def test_tuning_validation_and_roundtrip():
    t = _lib.Tuning(128, 0, 8, 0, 1, 1, 1)
    assert L.arborx_set_tuning(ctypes.byref(t)) == 0
    g = _lib.Tuning()
    assert L.arborx_get_tuning(ctypes.byref(g)) == 0
    assert (g.block, g.order, g.stack, g.schedule, g.build, g.seed_mode, g.node_format) == (128, 0, 8, 0, 1, 1, 1)
    assert L.arborx_set_tuning(ctypes.byref(_lib.Tuning(100, 1, 0, 0, 0, 0, 0))) == 1
    assert L.arborx_set_tuning(ctypes.byref(_lib.Tuning(0, 1, 0, 0, 2, 0, 0))) == 1
    assert L.arborx_set_tuning(ctypes.byref(_lib.Tuning(0, 1, 0, 0, 0, 0, 3))) == 1
    assert L.arborx_set_tuning(ctypes.byref(_lib.Tuning(0, 1, 0, 0, 0, 0, 2))) == 0
    assert L.arborx_set_tuning(ctypes.byref(_lib.Tuning(0, 1, 0, 0, 0, 3, 0))) == 1
    assert L.arborx_set_tuning(ctypes.byref(_lib.Tuning(0, 1, 0, 0, 0, -1, 0))) == 1
    assert L.arborx_set_tuning(ctypes.byref(_lib.Tuning(0, 1, 0, 0, 0, 0, 0, 3))) == 1
    assert L.arborx_set_tuning(ctypes.byref(_lib.Tuning(0, 1, 12, 0, 0, 0, 0))) == 1
    assert L.arborx_set_tuning(None) == 0
    assert L.arborx_get_tuning(ctypes.byref(g)) == 0
    assert (g.block, g.order, g.stack, g.build, g.seed_mode, g.node_format, g.queries_per_thread) == (256, 1, 16, 0, 0, 1, 1)


def test_debug_entry_validation():
    assert L.arborx_debug_radix_sort(FAKE, FAKE, 10, 48, 0, 48, None) == 1
    assert L.arborx_debug_radix_sort(FAKE, FAKE, 10, 32, 0, 33, None) == 1
    assert L.arborx_debug_morton64(FAKE, 10, 5, FAKE, FAKE, None) == 2


@pytest.mark.skipif(_has_gpu(), reason="checks the no-GPU error path")
def test_valid_call_without_gpu_reports_device_error():
    out = P()
    assert L.arborx_bvh_build(FAKE, 10, 3, 0, None, ctypes.byref(out)) == 5
    assert "GPU" in _err()


def test_python_tuning_roundtrip():
    ax.arborx_set_tuning(block=64, stack=8, node_format=1)
    try:
        assert ax.arborx_get_tuning() == dict(block=64, order=1, stack=8, schedule=0, build=0, seed_mode=0, node_format=1,
                                              queries_per_thread=0)
        ax.arborx_set_tuning_op(ax.OP_KNN, block=128, seed_mode=1)
        assert ax.arborx_get_tuning_op(ax.OP_KNN)["seed_mode"] == 1
        assert ax.arborx_get_tuning_op(ax.OP_KNN)["node_format"] == 0
        assert ax.arborx_get_tuning_op(ax.OP_REDUCE)["node_format"] == 1
    finally:
        ax.arborx_reset_tuning()


def test_allocator_hook_validation():
    alloc = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)(lambda n, s, c: None)
    free = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)(lambda p, s, c: None)
    a, f = ctypes.cast(alloc, ctypes.c_void_p), ctypes.cast(free, ctypes.c_void_p)
    assert L.arborx_set_allocator(a, None, None) == 1
    assert L.arborx_set_allocator(None, f, None) == 1
    assert "both" in _err()
    assert L.arborx_set_allocator(a, f, None) == 0  # nothing is held: the hook may change
    assert L.arborx_set_allocator(None, None, None) == 0
    with pytest.raises(ValueError):
        ax.arborx_set_allocator(lambda n, s: 0)


def test_new_entry_point_validation():
    """Arguments of the pair search, per-match output, ray CSR, forest create/rebuild, forest
    autotuner, walk statistics and allocation-free kNN entry points fail on the host, before any
    device work."""
    f = ctypes.c_float
    tot = ctypes.c_int64()
    plan = P()
    out = P()
    assert L.arborx_self_join_degree(None, f(1), FAKE, None) == 1
    assert L.arborx_query_spatial_with_distances(None, FAKE, 1, f(1), FAKE, FAKE, FAKE, 1, ctypes.byref(tot), None) == 1
    assert L.arborx_query_spatial_with_distances_begin(None, FAKE, 1, f(1), FAKE, ctypes.byref(tot),
                                                       ctypes.byref(plan), None) == 1
    assert L.arborx_query_finish_with_distances(None, FAKE, FAKE, 1) == 1
    assert L.arborx_query_ray_intersect(None, FAKE, 1, FAKE, FAKE, 1, ctypes.byref(tot), None) == 1
    assert L.arborx_query_ray_intersect_begin(None, FAKE, 1, FAKE, ctypes.byref(tot), ctypes.byref(plan), None) == 1
    assert L.arborx_query_ray_ordered_intersect(None, FAKE, 1, FAKE, FAKE, FAKE, 1, ctypes.byref(tot), None) == 1
    assert L.arborx_query_ray_ordered_intersect_begin(None, FAKE, 1, FAKE, ctypes.byref(tot), ctypes.byref(plan),
                                                      None) == 1
    assert L.arborx_forest_create(10, 0, 3, 0, None, ctypes.byref(out)) == 1
    assert L.arborx_forest_create(-1, 2, 3, 0, None, ctypes.byref(out)) == 1
    assert L.arborx_forest_create(10, 2, 11, 0, None, ctypes.byref(out)) == 1
    assert L.arborx_forest_create(10, 2, 3, 5, None, ctypes.byref(out)) == 1
    assert L.arborx_forest_create(10, 2, 4, 0, None, ctypes.byref(out)) == 2
    assert L.arborx_forest_create(10, 2 ** 31 - 2, 3, 0, None, ctypes.byref(out)) == 1 and "trees" in _err()
    assert L.arborx_forest_create(10, 2, 3, 0, None, None) == 1
    assert L.arborx_forest_rebuild(None, FAKE, FAKE, None) == 1
    assert L.arborx_autotune_forest(None, 1, FAKE, 1, FAKE, FAKE, FAKE, 1, 1, None, None, None) == 1
    assert L.arborx_debug_node_visits(None, FAKE, 1, f(1), 0, 1, FAKE, None) == 1
    assert L.arborx_query_knn_noalloc(None, FAKE, 1, 3, FAKE, FAKE, None) == 1
    assert out.value is None
