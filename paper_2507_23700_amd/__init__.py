"""MI355X linear-BVH geometric search (the hot path of ArborX 2.0, arXiv 2507.23700).

A thin binding over the C ABI in include/arborx.h: functions carry the C names
and only marshal arguments (torch tensors in device memory, the current HIP
stream); every step runs in the library's HIP kernels.  The ``BVH`` class is a
convenience wrapper over the same calls.

Importing the package does not load the library; the first call does, and it
raises if ``libarborx355.so`` has not been built.
"""
from __future__ import annotations

import ctypes

from . import _lib

POINTS, BOXES = 0, 1
COUNT, COUNT_SUMDIST = 0, 1

OK, E_INVALID, E_UNSUPPORTED, E_NOMEM, E_CAPACITY, E_DEVICE = range(6)
_NAMES = {1: "E_INVALID", 2: "E_UNSUPPORTED", 3: "E_NOMEM", 4: "E_CAPACITY", 5: "E_DEVICE"}


class ArborXError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{_NAMES.get(status, status)}: {message}")
        self.status = status


def _check(st: int) -> None:
    if st != OK:
        raise ArborXError(st, _lib.lib().arborx_last_error().decode())


def _torch():
    import torch
    return torch


def _stream(stream):
    torch = _torch()
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _dev(t, dtype, name):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None and t.numel() > 0 else ctypes.c_void_p(0)


def version() -> str:
    return _lib.lib().arborx_version().decode()


_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)
_allocator = None  # the installed ctypes callbacks, kept alive while the library may call them


def arborx_set_allocator(alloc=None, free=None) -> None:
    """Take the library's device memory from ``alloc(nbytes, stream) -> int`` and return it to
    ``free(ptr, stream)`` (``stream`` is the raw stream handle as an int, 0 for the default
    stream); with no arguments the library's own stream-ordered pool is used again."""
    global _allocator
    if (alloc is None) != (free is None):
        raise ValueError("give both alloc and free, or neither")
    if alloc is None:
        _check(_lib.lib().arborx_set_allocator(None, None, None))
        _allocator = None
        return

    def a(nbytes, stream, ctx):
        try:
            return alloc(int(nbytes), stream or 0) or None
        except Exception:  # reported to the caller as ARBORX_E_NOMEM
            return None

    def f(ptr, stream, ctx):
        free(ptr, stream or 0)

    cbs = (_ALLOC_FN(a), _FREE_FN(f))
    _check(_lib.lib().arborx_set_allocator(ctypes.cast(cbs[0], ctypes.c_void_p), ctypes.cast(cbs[1], ctypes.c_void_p),
                                           None))
    _allocator = cbs


def use_torch_allocator(device=None) -> None:
    """Serve the library's device memory from PyTorch's caching allocator, so that trees, forests
    and per-call temporaries share torch's memory pool (and show in torch.cuda.memory_allocated)."""
    torch = _torch()
    dev = torch.cuda.current_device() if device is None else device
    arborx_set_allocator(lambda n, s: torch.cuda.caching_allocator_alloc(n, dev, s),
                         lambda p, s: torch.cuda.caching_allocator_delete(p))


def arborx_set_tuning(block=0, order=1, stack=0, schedule=0, build=0, seed_mode=0, node_format=0,
                      queries_per_thread=0) -> None:
    t = _lib.Tuning(block, order, stack, schedule, build, seed_mode, node_format, queries_per_thread)
    _check(_lib.lib().arborx_set_tuning(ctypes.byref(t)))


def arborx_reset_tuning() -> None:
    _check(_lib.lib().arborx_set_tuning(None))


def arborx_get_tuning() -> dict:
    t = _lib.Tuning()
    _check(_lib.lib().arborx_get_tuning(ctypes.byref(t)))
    return _tuning_dict(t)


OP_SPATIAL, OP_REDUCE, OP_KNN = 0, 1, 2


def _tuning_dict(t):
    return dict(block=t.block, order=t.order, stack=t.stack, schedule=t.schedule, build=t.build, seed_mode=t.seed_mode,
                node_format=t.node_format, queries_per_thread=t.queries_per_thread)


def arborx_set_tuning_op(op, block=0, order=1, stack=0, schedule=0, build=0, seed_mode=0, node_format=0,
                         queries_per_thread=0) -> None:
    t = _lib.Tuning(block, order, stack, schedule, build, seed_mode, node_format, queries_per_thread)
    _check(_lib.lib().arborx_set_tuning_op(op, ctypes.byref(t)))


def arborx_get_tuning_op(op) -> dict:
    t = _lib.Tuning()
    _check(_lib.lib().arborx_get_tuning_op(op, ctypes.byref(t)))
    return _tuning_dict(t)


def arborx_autotune(tree, op, queries, radius=0.0, k=1, stream=None):
    """Time the candidate schedules on these queries and keep the fastest for `op`: (tuning dict, ms)."""
    torch = _torch()
    q = _dev(queries, torch.float32, "queries")
    best = _lib.Tuning()
    ms = ctypes.c_double()
    _check(_lib.lib().arborx_autotune(tree.handle, op, _ptr(q), q.shape[0], ctypes.c_float(radius), k,
                                      ctypes.byref(best), ctypes.byref(ms), _stream(stream)))
    return _tuning_dict(best), ms.value


def arborx_autotune_forest(forest, op, queries, batch_offsets, batch_tree, batch_radius=None, k=1, stream=None):
    """Tune the forest queries of `op` (OP_REDUCE or OP_KNN) on these batches: (tuning dict, ms)."""
    torch = _torch()
    q = _dev(queries, torch.float32, "queries")
    bo = _dev(batch_offsets, torch.int64, "batch_offsets")
    bt = _dev(batch_tree, torch.int32, "batch_tree")
    br = _dev(batch_radius, torch.float32, "batch_radius") if batch_radius is not None else None
    best = _lib.Tuning()
    ms = ctypes.c_double()
    _check(_lib.lib().arborx_autotune_forest(forest.handle, op, _ptr(q), q.shape[0], _ptr(bo), _ptr(bt), _ptr(br),
                                             bt.shape[0], k, ctypes.byref(best), ctypes.byref(ms), _stream(stream)))
    return _tuning_dict(best), ms.value


class Tree:
    """Owns an arborx_tree handle; destroyed with the object."""

    def __init__(self, handle, n, dim, kind, values):
        self.handle, self.n, self.dim, self.kind = handle, n, dim, kind
        self._values = values  # keep the build input alive until the build has run

    def __del__(self):
        h = getattr(self, "handle", None)
        if h and _lib is not None and _lib._lib is not None:
            _lib._lib.arborx_bvh_destroy(h)
        self.handle = None


def arborx_bvh_build(values, kind=POINTS, stream=None) -> Tree:
    """values: float32 [n, dim] points or [n, 2, dim] boxes on the GPU."""
    torch = _torch()
    values = _dev(values, torch.float32, "values")
    if kind == POINTS and values.dim() != 2:
        raise ValueError("points must be [n, dim]")
    if kind == BOXES and (values.dim() != 3 or values.shape[1] != 2):
        raise ValueError("boxes must be [n, 2, dim]")
    n, dim = values.shape[0], values.shape[-1]
    h = ctypes.c_void_p()
    _check(_lib.lib().arborx_bvh_build(_ptr(values), n, dim, kind, _stream(stream), ctypes.byref(h)))
    return Tree(h, n, dim, kind, values)


def arborx_bvh_destroy(tree: Tree) -> None:
    if tree.handle:
        _check(_lib.lib().arborx_bvh_destroy(tree.handle))
        tree.handle = None


def arborx_bvh_info(tree: Tree) -> dict:
    n, dim, kind, height = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    b = (ctypes.c_float * 20)()
    _check(_lib.lib().arborx_bvh_info(tree.handle, ctypes.byref(n), ctypes.byref(dim), ctypes.byref(kind), b,
                                      ctypes.byref(height)))
    d = dim.value
    return dict(n=n.value, dim=d, kind=kind.value, lo=list(b[:d]), hi=list(b[d:2 * d]), height=height.value,
                empty=n.value == 0)


def _queries(tree, q, boxes):
    torch = _torch()
    q = _dev(q, torch.float32, "queries")
    want = (2, tree.dim) if boxes else (tree.dim,)
    if tuple(q.shape[1:]) != want:
        raise ValueError(f"queries must be [m, {', '.join(map(str, want))}]")
    return q


def _csr(begin, tree, q, extra, stream, ordered=True):
    """Count (begin), size indices exactly, fill (finish, or the unsorted finish when not
    ordered), release the plan."""
    torch = _torch()
    m = q.shape[0]
    offsets = torch.empty(m + 1, dtype=torch.int64, device=q.device)
    total = ctypes.c_int64()
    plan = ctypes.c_void_p()
    L = _lib.lib()
    _check(begin(tree.handle, _ptr(q), m, *extra, _ptr(offsets), ctypes.byref(total), ctypes.byref(plan),
                 _stream(stream)))
    try:
        indices = torch.empty(max(total.value, 1), dtype=torch.int32, device=q.device)
        finish = L.arborx_query_finish if ordered else L.arborx_query_finish_unsorted
        _check(finish(plan, _ptr(indices), indices.numel()))
    finally:
        L.arborx_plan_destroy(plan)
    return offsets, indices[:total.value]


def arborx_query_spatial(tree: Tree, queries, radius: float, stream=None, ordered=True):
    """Radius search: (offsets int64[m+1], indices int32[total]), rows ascending; with
    ordered=False each row in the order the walk found its matches (same sets)."""
    q = _queries(tree, queries, False)
    return _csr(_lib.lib().arborx_query_spatial_begin, tree, q, [ctypes.c_float(radius)], stream, ordered)


def arborx_query_intersects(tree: Tree, qboxes, stream=None, ordered=True):
    """Box-overlap search with [m, 2, dim] query boxes: CSR (offsets, indices); ordered as in
    arborx_query_spatial."""
    q = _queries(tree, qboxes, True)
    return _csr(_lib.lib().arborx_query_intersects_begin, tree, q, [], stream, ordered)


def arborx_query_knn(tree: Tree, queries, k: int, stream=None):
    """k nearest: (dist2 float32[m, k], indices int32[m, k]) in (d2, index) order, padded (+inf, -1)."""
    torch = _torch()
    q = _queries(tree, queries, False)
    m = q.shape[0]
    d2 = torch.empty((m, k), dtype=torch.float32, device=q.device)
    idx = torch.empty((m, k), dtype=torch.int32, device=q.device)
    _check(_lib.lib().arborx_query_knn(tree.handle, _ptr(q), m, k, _ptr(d2), _ptr(idx), _stream(stream)))
    return d2, idx


def arborx_query_knn_noalloc(tree: Tree, queries, k: int, dist2=None, indices=None, stream=None):
    """As arborx_query_knn, but the library allocates no device memory for the call (its query
    ordering runs in a static per-GPU scratch area; m <= ARBORX_NOALLOC_MAX_QUERIES).  Pass
    preallocated ``dist2`` float32[m, k] and ``indices`` int32[m, k] to keep the call free of
    torch allocations too."""
    torch = _torch()
    q = _queries(tree, queries, False)
    m = q.shape[0]
    if dist2 is None:
        dist2 = torch.empty((m, k), dtype=torch.float32, device=q.device)
    if indices is None:
        indices = torch.empty((m, k), dtype=torch.int32, device=q.device)
    _dev(dist2, torch.float32, "dist2")
    _dev(indices, torch.int32, "indices")
    if tuple(dist2.shape) != (m, k) or tuple(indices.shape) != (m, k):
        raise ValueError(f"dist2 and indices must be [{m}, {k}]")
    _check(_lib.lib().arborx_query_knn_noalloc(tree.handle, _ptr(q), m, k, _ptr(dist2), _ptr(indices),
                                               _stream(stream)))
    return dist2, indices


NOALLOC_MAX_QUERIES = 2097152  # ARBORX_NOALLOC_MAX_QUERIES in include/arborx.h


def arborx_query_spatial_reduce(tree: Tree, queries, radius: float, op=COUNT_SUMDIST, scale_bits=32, stream=None):
    """Fused radius reduce: counts int32[m] and (COUNT_SUMDIST) sum_fixed int64[m]."""
    torch = _torch()
    q = _queries(tree, queries, False)
    m = q.shape[0]
    counts = torch.empty(m, dtype=torch.int32, device=q.device)
    sums = torch.empty(m, dtype=torch.int64, device=q.device) if op == COUNT_SUMDIST else None
    _check(_lib.lib().arborx_query_spatial_reduce(tree.handle, _ptr(q), m, ctypes.c_float(radius), op, _ptr(counts),
                                                  _ptr(sums), scale_bits, _stream(stream)))
    return counts, sums


def arborx_query_match_distances(tree: Tree, values, queries, offsets, indices, stream=None):
    """Callback with output: float32 squared distance of every match of a radius CSR result."""
    torch = _torch()
    v = _dev(values, torch.float32, "values")
    want = (tree.n, 2, tree.dim) if tree.kind == BOXES else (tree.n, tree.dim)
    if tuple(v.shape) != want:
        raise ValueError(f"values must be the build input, shape {list(want)}")
    q = _queries(tree, queries, False)
    off = _dev(offsets, torch.int64, "offsets")
    if off.shape[0] != q.shape[0] + 1:
        raise ValueError("offsets must have m + 1 entries")
    idx = _dev(indices, torch.int32, "indices")
    out = torch.empty(idx.shape[0], dtype=torch.float32, device=q.device)
    _check(_lib.lib().arborx_query_match_distances(tree.handle, _ptr(v), _ptr(q), q.shape[0], _ptr(off), _ptr(idx),
                                                   _ptr(out), _stream(stream)))
    return out


def arborx_query_spatial_with_distances(tree: Tree, queries, radius: float, stream=None):
    """Callback with output: radius search returning (offsets, indices, squared distances) in CSR
    form, each distance written by the search's own walk beside its index."""
    torch = _torch()
    q = _queries(tree, queries, False)
    m = q.shape[0]
    offsets = torch.empty(m + 1, dtype=torch.int64, device=q.device)
    total = ctypes.c_int64()
    plan = ctypes.c_void_p()
    L = _lib.lib()
    _check(L.arborx_query_spatial_with_distances_begin(tree.handle, _ptr(q), m, ctypes.c_float(radius), _ptr(offsets),
                                                       ctypes.byref(total), ctypes.byref(plan), _stream(stream)))
    try:
        indices = torch.empty(max(total.value, 1), dtype=torch.int32, device=q.device)
        dist = torch.empty(max(total.value, 1), dtype=torch.float32, device=q.device)
        _check(L.arborx_query_finish_with_distances(plan, _ptr(indices), _ptr(dist), indices.numel()))
    finally:
        L.arborx_plan_destroy(plan)
    return offsets, indices[:total.value], dist[:total.value]


def arborx_query_ray_count(tree: Tree, rays, stream=None):
    """Number of values each ray meets; rays [m, 2, dim] = (origin, direction)."""
    torch = _torch()
    r = _queries(tree, rays, True)
    counts = torch.empty(r.shape[0], dtype=torch.int32, device=r.device)
    _check(_lib.lib().arborx_query_ray_count(tree.handle, _ptr(r), r.shape[0], _ptr(counts), _stream(stream)))
    return counts


def arborx_query_ray_intersect(tree: Tree, rays, stream=None):
    """Every value each ray meets (rays [m, 2, dim] = origin, direction): CSR (offsets, indices), rows ascending."""
    r = _queries(tree, rays, True)
    return _csr(_lib.lib().arborx_query_ray_intersect_begin, tree, r, [], stream)


def arborx_query_ray_ordered_intersect(tree: Tree, rays, stream=None):
    """The values each ray meets in the order met: CSR (offsets, indices, t_entry), rows by (t, index)."""
    torch = _torch()
    r = _queries(tree, rays, True)
    m = r.shape[0]
    offsets = torch.empty(m + 1, dtype=torch.int64, device=r.device)
    total = ctypes.c_int64()
    plan = ctypes.c_void_p()
    L = _lib.lib()
    _check(L.arborx_query_ray_ordered_intersect_begin(tree.handle, _ptr(r), m, _ptr(offsets), ctypes.byref(total),
                                                      ctypes.byref(plan), _stream(stream)))
    try:
        indices = torch.empty(max(total.value, 1), dtype=torch.int32, device=r.device)
        t = torch.empty(max(total.value, 1), dtype=torch.float32, device=r.device)
        _check(L.arborx_query_finish_with_distances(plan, _ptr(indices), _ptr(t), indices.numel()))
    finally:
        L.arborx_plan_destroy(plan)
    return offsets, indices[:total.value], t[:total.value]


def arborx_query_ray_nearest(tree: Tree, rays, k: int, stream=None):
    """The k values each ray meets first: (t_entry float32[m, k], indices int32[m, k]) by (t, index)."""
    torch = _torch()
    r = _queries(tree, rays, True)
    m = r.shape[0]
    t = torch.empty((m, k), dtype=torch.float32, device=r.device)
    idx = torch.empty((m, k), dtype=torch.int32, device=r.device)
    _check(_lib.lib().arborx_query_ray_nearest(tree.handle, _ptr(r), m, int(k), _ptr(t), _ptr(idx), _stream(stream)))
    return t, idx


def arborx_dbscan(tree: Tree, points, eps: float, min_pts: int, stream=None):
    """DBSCAN over the tree's points: int32 labels (cluster = smallest core index, border = its
    smallest-index core neighbour's cluster, noise = -1)."""
    torch = _torch()
    v = _dev(points, torch.float32, "points")
    if tree.kind != POINTS or tuple(v.shape) != (tree.n, tree.dim):
        raise ValueError(f"points must be the build input of a tree of points, shape [{tree.n}, {tree.dim}]")
    labels = torch.empty(tree.n, dtype=torch.int32, device=v.device)
    _check(_lib.lib().arborx_dbscan(tree.handle, _ptr(v), ctypes.c_float(eps), int(min_pts), _ptr(labels),
                                    _stream(stream)))
    return labels


def arborx_self_join_degree(tree: Tree, radius: float, stream=None):
    """Pair search over the tree's own points: int32 degree[i] = number of values j != i within
    radius of value i (every unordered pair is found once, by a walk over the later leaves)."""
    torch = _torch()
    if tree.kind != POINTS:
        raise ValueError("the self-join pairs the points of a tree built from points")
    deg = torch.empty(tree.n, dtype=torch.int32, device="cuda")
    _check(_lib.lib().arborx_self_join_degree(tree.handle, ctypes.c_float(radius), _ptr(deg), _stream(stream)))
    return deg


def arborx_query_spatial_count_up_to(tree: Tree, queries, radius: float, n_max: int, stream=None):
    """Early-terminating count: int32[m] = min(matches within radius, n_max)."""
    torch = _torch()
    q = _queries(tree, queries, False)
    m = q.shape[0]
    counts = torch.empty(m, dtype=torch.int32, device=q.device)
    _check(_lib.lib().arborx_query_spatial_count_up_to(tree.handle, _ptr(q), m, ctypes.c_float(radius), int(n_max),
                                                       _ptr(counts), _stream(stream)))
    return counts


def arborx_debug_radix_sort(keys, values, begin_bit=0, end_bit=None, stream=None):
    """In-place stable sort of (keys int64/int32 viewed as unsigned, values int32) by key bits."""
    torch = _torch()
    if keys.dtype not in (torch.int64, torch.int32):
        raise TypeError("keys must be int64 or int32 (bit patterns of unsigned keys)")
    _dev(keys, keys.dtype, "keys")
    _dev(values, torch.int32, "values")
    bits = 64 if keys.dtype == torch.int64 else 32
    end_bit = bits if end_bit is None else end_bit
    _check(_lib.lib().arborx_debug_radix_sort(_ptr(keys), _ptr(values), keys.numel(), bits, begin_bit, end_bit,
                                              _stream(stream)))


def arborx_debug_node_visits(tree: Tree, queries, radius=0.0, k=0, stream=None):
    """Node fetches per query: of the one-query-per-thread radius walk (k = 0) or of the kNN walk
    after its seeding (k >= 1).  int32[m]."""
    torch = _torch()
    q = _queries(tree, queries, False)
    v = torch.empty(q.shape[0], dtype=torch.int32, device=q.device)
    _check(_lib.lib().arborx_debug_node_visits(tree.handle, _ptr(q), q.shape[0], ctypes.c_float(radius),
                                               1 if k else 0, int(k), _ptr(v), _stream(stream)))
    return v


def arborx_debug_morton64(points, bounds, stream=None):
    """Morton-64 codes (as int64 bit patterns) of [n, dim] points under bounds [2, dim]."""
    torch = _torch()
    points = _dev(points, torch.float32, "points")
    bounds = _dev(bounds, torch.float32, "bounds")
    codes = torch.empty(points.shape[0], dtype=torch.int64, device=points.device)
    _check(_lib.lib().arborx_debug_morton64(_ptr(points), points.shape[0], points.shape[1], _ptr(bounds),
                                            _ptr(codes), _stream(stream)))
    return codes


def arborx_debug_tree_nodes(tree: Tree):
    """Host copies (child [nn,2] int32, lo [nn,2,dim], hi [nn,2,dim], root) of the tree's nodes."""
    import numpy as np
    nn = tree.n - 1 if tree.n > 1 else tree.n
    child = np.zeros((max(nn, 1), 2), dtype=np.int32)
    lo = np.zeros((max(nn, 1), 2, tree.dim), dtype=np.float32)
    hi = np.zeros_like(lo)
    root = ctypes.c_int32()
    _check(_lib.lib().arborx_debug_tree_nodes(tree.handle, child.ctypes.data_as(ctypes.c_void_p),
                                              lo.ctypes.data_as(ctypes.c_void_p), hi.ctypes.data_as(ctypes.c_void_p),
                                              ctypes.byref(root)))
    return child[:nn], lo[:nn], hi[:nn], root.value


# ---------------------------------------------------------------------------
# forest
# ---------------------------------------------------------------------------

class Forest:
    """Owns an arborx_forest handle; destroyed with the object.  Built by arborx_forest_build;
    .reduce / .knn / .reserve / .info call the forest entry points on it."""

    def __init__(self, handle, T, n, dim, kind, values):
        self.handle, self.T, self.n, self.dim, self.kind = handle, T, n, dim, kind
        self._values = values

    def info(self):
        return arborx_forest_info(self)

    def reserve(self, m, **kw):
        arborx_forest_reserve(self, m, **kw)

    def reduce(self, queries, batch_offsets, batch_tree, batch_radius, op=COUNT_SUMDIST, **kw):
        return arborx_forest_query_reduce(self, queries, batch_offsets, batch_tree, batch_radius, op, **kw)

    def knn(self, queries, batch_offsets, batch_tree, k, **kw):
        return arborx_forest_query_knn(self, queries, batch_offsets, batch_tree, k, **kw)

    def __del__(self):
        h = getattr(self, "handle", None)
        if h and _lib is not None and _lib._lib is not None:
            _lib._lib.arborx_forest_destroy(h)
        self.handle = None


def _host_i64(a):
    import numpy as np
    return np.ascontiguousarray(np.asarray(a, dtype=np.int64))


def arborx_forest_build(values, tree_offsets, kind=POINTS, stream=None) -> Forest:
    """values: packed float32 [n, dim] (or [n, 2, dim] boxes) on the GPU; tree_offsets: host ints [T+1]."""
    torch = _torch()
    values = _dev(values, torch.float32, "values")
    off = _host_i64(tree_offsets)
    T = len(off) - 1
    n, dim = values.shape[0], values.shape[-1]
    if T < 1 or off[-1] != n:
        raise ValueError("tree_offsets must have T+1 >= 2 entries ending at n")
    h = ctypes.c_void_p()
    _check(_lib.lib().arborx_forest_build(_ptr(values), off.ctypes.data_as(ctypes.c_void_p), T, dim, kind,
                                          _stream(stream), ctypes.byref(h)))
    return Forest(h, T, n, dim, kind, values)


def arborx_forest_create(n: int, T: int, dim: int, kind=POINTS, stream=None) -> Forest:
    """Allocate a forest for n values in T trees of dimension dim, built later (and in a captured
    graph, if wanted) by arborx_forest_rebuild."""
    h = ctypes.c_void_p()
    _check(_lib.lib().arborx_forest_create(int(n), int(T), int(dim), kind, _stream(stream), ctypes.byref(h)))
    return Forest(h, int(T), int(n), int(dim), kind, None)


def arborx_forest_rebuild(forest: Forest, values, tree_offsets, stream=None) -> None:
    """Build the forest's trees from device values [n, dim] (or [n, 2, dim]) and device int64
    tree_offsets [T+1]; kernels only, so it can be captured in a graph."""
    torch = _torch()
    values = _dev(values, torch.float32, "values")
    off = _dev(tree_offsets, torch.int64, "tree_offsets")
    if values.shape[0] != forest.n or values.shape[-1] != forest.dim or off.shape[0] != forest.T + 1:
        raise ValueError(f"values must be [{forest.n}, ..., {forest.dim}] and tree_offsets [{forest.T + 1}]")
    _check(_lib.lib().arborx_forest_rebuild(forest.handle, _ptr(values), _ptr(off), _stream(stream)))
    forest._values = values


def arborx_forest_info(forest: Forest) -> dict:
    import numpy as np
    T, n, dim = ctypes.c_int32(), ctypes.c_int64(), ctypes.c_int32()
    roots = np.zeros(forest.T, dtype=np.int32)
    heights = np.zeros(forest.T, dtype=np.int32)
    _check(_lib.lib().arborx_forest_info(forest.handle, ctypes.byref(T), ctypes.byref(n), ctypes.byref(dim),
                                         roots.ctypes.data_as(ctypes.c_void_p),
                                         heights.ctypes.data_as(ctypes.c_void_p)))
    return dict(T=T.value, n=n.value, dim=dim.value, roots=roots, heights=heights)


def arborx_forest_reserve(forest: Forest, m: int, stream=None) -> None:
    _check(_lib.lib().arborx_forest_reserve(forest.handle, int(m), _stream(stream)))


def _batches(queries, batch_offsets, batch_tree, dim):
    torch = _torch()
    q = _dev(queries, torch.float32, "queries")
    if q.dim() != 2 or q.shape[1] != dim:
        raise ValueError(f"queries must be [m, {dim}]")
    bo = _dev(batch_offsets, torch.int64, "batch_offsets")
    bt = _dev(batch_tree, torch.int32, "batch_tree")
    if bo.numel() != bt.numel() + 1:
        raise ValueError("batch_offsets must have B+1 entries")
    return q, bo, bt, bt.numel()


def arborx_forest_query_reduce(forest: Forest, queries, batch_offsets, batch_tree, batch_radius, op=COUNT_SUMDIST,
                               scale_bits=32, stream=None):
    """Per query: count (and fixed-point distance sum) within its batch's radius in its batch's tree."""
    torch = _torch()
    q, bo, bt, B = _batches(queries, batch_offsets, batch_tree, forest.dim)
    br = _dev(batch_radius, torch.float32, "batch_radius")
    m = q.shape[0]
    counts = torch.empty(m, dtype=torch.int32, device=q.device)
    sums = torch.empty(m, dtype=torch.int64, device=q.device) if op == COUNT_SUMDIST else None
    _check(_lib.lib().arborx_forest_query_reduce(forest.handle, _ptr(q), m, _ptr(bo), _ptr(bt), _ptr(br), B, op,
                                                 _ptr(counts), _ptr(sums), scale_bits, _stream(stream)))
    return counts, sums


def arborx_forest_query_knn(forest: Forest, queries, batch_offsets, batch_tree, k: int, stream=None):
    """Per query: k nearest in its batch's tree, indices local to that tree, padded (+inf, -1)."""
    torch = _torch()
    q, bo, bt, B = _batches(queries, batch_offsets, batch_tree, forest.dim)
    m = q.shape[0]
    d2 = torch.empty((m, k), dtype=torch.float32, device=q.device)
    idx = torch.empty((m, k), dtype=torch.int32, device=q.device)
    _check(_lib.lib().arborx_forest_query_knn(forest.handle, _ptr(q), m, _ptr(bo), _ptr(bt), B, k, _ptr(d2),
                                              _ptr(idx), _stream(stream)))
    return d2, idx


# ---------------------------------------------------------------------------
# Chamfer
# ---------------------------------------------------------------------------

def arborx_chamfer_forward(a, a_off, b, b_off, stream=None):
    """(loss float32[P], nn_ab int32[na], nn_ba int32[nb]); a_off, b_off host ints [P+1]."""
    torch = _torch()
    a = _dev(a, torch.float32, "a")
    b = _dev(b, torch.float32, "b")
    ao, bo = _host_i64(a_off), _host_i64(b_off)
    P = len(ao) - 1
    loss = torch.empty(P, dtype=torch.float32, device=a.device)
    nab = torch.empty(a.shape[0], dtype=torch.int32, device=a.device)
    nba = torch.empty(b.shape[0], dtype=torch.int32, device=a.device)
    _check(_lib.lib().arborx_chamfer_forward(_ptr(a), ao.ctypes.data_as(ctypes.c_void_p), _ptr(b),
                                             bo.ctypes.data_as(ctypes.c_void_p), P, _ptr(loss), _ptr(nab), _ptr(nba),
                                             _stream(stream)))
    return loss, nab, nba


def arborx_chamfer_backward(a, a_off, b, b_off, nn_ab, nn_ba, grad_loss, stream=None):
    """(grad_a float32[na, 3], grad_b float32[nb, 3]) with the forward's neighbours held fixed."""
    torch = _torch()
    a = _dev(a, torch.float32, "a")
    b = _dev(b, torch.float32, "b")
    g = _dev(grad_loss.contiguous(), torch.float32, "grad_loss")
    ao, bo = _host_i64(a_off), _host_i64(b_off)
    P = len(ao) - 1
    ga = torch.empty_like(a)
    gb = torch.empty_like(b)
    _check(_lib.lib().arborx_chamfer_backward(_ptr(a), ao.ctypes.data_as(ctypes.c_void_p), _ptr(b),
                                              bo.ctypes.data_as(ctypes.c_void_p), P, _ptr(nn_ab), _ptr(nn_ba),
                                              _ptr(g), _ptr(ga), _ptr(gb), _stream(stream)))
    return ga, gb


def _chamfer_function():
    torch = _torch()

    class ChamferFn(torch.autograd.Function):
        """Per-pair nearest-neighbour Chamfer loss; backward is the library's kernel."""

        @staticmethod
        def forward(ctx, a, b, a_off, b_off):
            loss, nab, nba = arborx_chamfer_forward(a.detach().contiguous(), a_off, b.detach().contiguous(), b_off)
            ctx.save_for_backward(a.detach(), b.detach(), nab, nba)
            ctx.offsets = (a_off, b_off)
            return loss

        @staticmethod
        def backward(ctx, grad_loss):
            a, b, nab, nba = ctx.saved_tensors
            ga, gb = arborx_chamfer_backward(a.contiguous(), ctx.offsets[0], b.contiguous(), ctx.offsets[1], nab, nba,
                                             grad_loss.float())
            return ga, gb, None, None

    return ChamferFn


_CHAMFER = None


def chamfer(a, a_off, b, b_off):
    """Differentiable per-pair Chamfer loss: a [na, 3], b [nb, 3] packed clouds, host offsets [P+1]."""
    global _CHAMFER
    if _CHAMFER is None:
        _CHAMFER = _chamfer_function()
    return _CHAMFER.apply(a, b, a_off, b_off)


class BVH:
    """Convenience wrapper: BVH(points) then .spatial / .intersects / .knn / .count / .count_sumdist."""

    def __init__(self, values, kind=POINTS, stream=None):
        self.tree = arborx_bvh_build(values, kind, stream)
        self.values = values

    def info(self):
        return arborx_bvh_info(self.tree)

    def size(self):
        return self.tree.n

    def empty(self):
        return self.tree.n == 0

    def bounds(self):
        i = self.info()
        return i["lo"], i["hi"]

    def spatial(self, queries, radius, **kw):
        return arborx_query_spatial(self.tree, queries, radius, **kw)

    def intersects(self, qboxes, **kw):
        return arborx_query_intersects(self.tree, qboxes, **kw)

    def knn(self, queries, k, **kw):
        return arborx_query_knn(self.tree, queries, k, **kw)

    def count(self, queries, radius, **kw):
        return arborx_query_spatial_reduce(self.tree, queries, radius, COUNT, **kw)[0]

    def spatial_with_distances(self, queries, radius, **kw):
        return arborx_query_spatial_with_distances(self.tree, queries, radius, **kw)

    def ray_count(self, rays, **kw):
        return arborx_query_ray_count(self.tree, rays, **kw)

    def ray_nearest(self, rays, k, **kw):
        return arborx_query_ray_nearest(self.tree, rays, k, **kw)

    def dbscan(self, eps, min_pts, **kw):
        return arborx_dbscan(self.tree, self.values, eps, min_pts, **kw)

    def count_up_to(self, queries, radius, n_max, **kw):
        return arborx_query_spatial_count_up_to(self.tree, queries, radius, n_max, **kw)

    def count_sumdist(self, queries, radius, scale_bits=32, **kw):
        return arborx_query_spatial_reduce(self.tree, queries, radius, COUNT_SUMDIST, scale_bits, **kw)
