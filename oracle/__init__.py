"""CPU brute-force oracle (TEST INFRASTRUCTURE ONLY).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import
this package.  The product path (the HIP library and its Python binding) never
imports, links or calls it, and shares no code with it; the seeded input
generators are the only thing both sides use.

The arithmetic lives in ``bruteforce.c`` (plain C, OpenMP over queries, built
with gcc ``-ffp-contract=off``).  This module compiles it on demand and wraps it
with numpy arrays.  Each function states the definition it computes; the
citations are to the ArborX 2.0 paper (arXiv 2507.23700):

* ``spatial`` / ``spatial_count``: radius query, CSR output (Section 2.1,
  original interface: indices plus offsets, the compressed-sparse-row format).
* ``intersects``: box-overlap spatial predicate (Section 2.1, new interface
  example with ``intersects``).
* ``knn``: nearest query, a query point and a number of neighbours (Section 2.1).
* ``reduce``: pure-callback query that stores nothing per match (Section 2.2,
  query form (1)); COUNT and COUNT plus a fixed-point distance sum.
* ``chamfer_forward`` / ``chamfer_backward``: nearest-neighbour Chamfer loss
  and its gradient in float64 (an addition to the paper's method; its
  definition is written out in ``bruteforce.c``).
* ``forest_*``: per batch, the query above against that batch's own tree.

Parity status: every function here is pinned by ``tests/test_oracle.py``
against hand-worked cases, scipy's k-d tree in float64, exact-rounding
emulation, invariants and finite differences; none is "parity unpinned".
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bruteforce.c")
LIB_PATH = os.path.join(_HERE, "_oracle.so")

CFLAGS = ["-O3", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
          "-fexcess-precision=standard", "-fno-finite-math-only"]

POINTS, BOXES = 0, 1
COUNT, COUNT_SUMDIST = 0, 1

_lib = None


def build(force: bool = True) -> str:
    """Compile bruteforce.c into _oracle.so with gcc."""
    if force or not os.path.exists(LIB_PATH):
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        P, I64, I32, F32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_float
        L.oracle_spatial_count.argtypes = [P, I64, I32, I32, P, I64, F32, P]
        L.oracle_spatial_fill.argtypes = [P, I64, I32, I32, P, I64, F32, P, P]
        L.oracle_intersects_count.argtypes = [P, I64, I32, I32, P, I64, P]
        L.oracle_intersects_fill.argtypes = [P, I64, I32, I32, P, I64, P, P]
        L.oracle_reduce.argtypes = [P, I64, I32, I32, P, I64, F32, I32, I32, P, P]
        L.oracle_count_up_to.argtypes = [P, I64, I32, I32, P, I64, F32, I32, P]
        L.oracle_match_distances.argtypes = [P, I64, I32, I32, P, I64, P, P, P]
        L.oracle_dbscan.argtypes = [P, I64, I32, F32, I32, P]
        L.oracle_self_join_degree.argtypes = [P, I64, I32, F32, P]
        L.oracle_self_join_pairs.argtypes = [P, I64, I32, F32, P, P]
        L.oracle_ray_count.argtypes = [P, I64, I32, I32, P, I64, P]
        L.oracle_ray_nearest.argtypes = [P, I64, I32, I32, P, I64, I32, P, P]
        L.oracle_ray_intersect.argtypes = [P, I64, I32, I32, P, I64, P, P]
        L.oracle_ray_ordered_intersect.argtypes = [P, I64, I32, I32, P, I64, P, P, P]
        L.oracle_knn.argtypes = [P, I64, I32, I32, P, I64, I32, P, P]
        L.oracle_chamfer_forward.argtypes = [P, P, P, P, I32, P, P, P]
        L.oracle_chamfer_backward.argtypes = [P, P, P, P, I32, P, P, P, P, P]
        for f in ("oracle_spatial_count", "oracle_spatial_fill", "oracle_intersects_count", "oracle_intersects_fill",
                  "oracle_reduce", "oracle_count_up_to", "oracle_self_join_degree", "oracle_self_join_pairs",
                  "oracle_ray_intersect", "oracle_ray_ordered_intersect", "oracle_knn", "oracle_chamfer_forward", "oracle_chamfer_backward",
                  "oracle_threads"):
            getattr(L, f).restype = ctypes.c_int
        _lib = L
    return _lib


def threads() -> int:
    """OpenMP threads the oracle runs with."""
    return int(lib().oracle_threads())


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _values(values, dim, kind):
    v = np.ascontiguousarray(values, dtype=np.float32)
    rows = v.shape[0] if v.ndim >= 1 else 0
    want = dim if kind == POINTS else 2 * dim
    if v.size != rows * want:
        raise ValueError("values must be [n][dim] points or [n][2][dim] boxes")
    return v, rows


def _queries(q, dim, per):
    q = np.ascontiguousarray(q, dtype=np.float32)
    m = q.shape[0]
    if q.size != m * per * dim:
        raise ValueError("bad query shape")
    return q, m


def spatial_count(values, queries, radius, dim=3, kind=POINTS):
    v, n = _values(values, dim, kind)
    q, m = _queries(queries, dim, 1)
    counts = np.zeros(m, dtype=np.int32)
    lib().oracle_spatial_count(_p(v), n, dim, kind, _p(q), m, np.float32(radius), _p(counts))
    return counts


def offsets_of(counts):
    """CSR offsets: offsets[0] = 0, offsets[i+1] = offsets[i] + counts[i]."""
    off = np.zeros(len(counts) + 1, dtype=np.int64)
    np.cumsum(counts, out=off[1:])
    return off


def spatial(values, queries, radius, dim=3, kind=POINTS):
    """Radius search (closed ball): (offsets int64[m+1], indices int32[total]) with ascending rows."""
    v, n = _values(values, dim, kind)
    q, m = _queries(queries, dim, 1)
    counts = spatial_count(v, q, radius, dim, kind)
    off = offsets_of(counts)
    idx = np.zeros(int(off[-1]), dtype=np.int32)
    lib().oracle_spatial_fill(_p(v), n, dim, kind, _p(q), m, np.float32(radius), _p(off), _p(idx))
    return off, idx


def intersects(values, qboxes, dim=3, kind=POINTS):
    """Box-overlap search: query boxes [m][2][dim]; CSR with ascending rows."""
    v, n = _values(values, dim, kind)
    q, m = _queries(qboxes, dim, 2)
    counts = np.zeros(m, dtype=np.int32)
    lib().oracle_intersects_count(_p(v), n, dim, kind, _p(q), m, _p(counts))
    off = offsets_of(counts)
    idx = np.zeros(int(off[-1]), dtype=np.int32)
    lib().oracle_intersects_fill(_p(v), n, dim, kind, _p(q), m, _p(off), _p(idx))
    return off, idx


def reduce(values, queries, radius, op=COUNT_SUMDIST, scale_bits=32, dim=3, kind=POINTS):
    """Pure-callback reduction: (counts int32[m], sum_fixed int64[m] or None)."""
    v, n = _values(values, dim, kind)
    q, m = _queries(queries, dim, 1)
    counts = np.zeros(m, dtype=np.int32)
    sums = np.zeros(m, dtype=np.int64)
    lib().oracle_reduce(_p(v), n, dim, kind, _p(q), m, np.float32(radius), op, scale_bits, _p(counts), _p(sums))
    return counts, (sums if op == COUNT_SUMDIST else None)


def ray_count(values, rays, dim=3, kind=POINTS):
    """Ray predicate (Section 2.5): number of values each ray o + t*d (t >= 0) meets; rays [m][2][dim]."""
    v, n = _values(values, dim, kind)
    r, m = _queries(rays, dim, 2)
    counts = np.zeros(m, dtype=np.int32)
    lib().oracle_ray_count(_p(v), n, dim, kind, _p(r), m, _p(counts))
    return counts


def ray_nearest(values, rays, k, dim=3, kind=POINTS):
    """The k values each ray meets first: (t float32[m][k], idx int32[m][k]) by (entry t, index)."""
    v, n = _values(values, dim, kind)
    r, m = _queries(rays, dim, 2)
    t = np.zeros((m, k), dtype=np.float32)
    idx = np.zeros((m, k), dtype=np.int32)
    lib().oracle_ray_nearest(_p(v), n, dim, kind, _p(r), m, k, _p(t), _p(idx))
    return t, idx


def ray_intersect(values, rays, dim=3, kind=POINTS):
    """Ray intersect (Section 2.5): every value each ray meets, CSR (offsets, indices) with ascending rows."""
    v, n = _values(values, dim, kind)
    r, m = _queries(rays, dim, 2)
    off = np.zeros(m + 1, dtype=np.int64)
    if lib().oracle_ray_intersect(_p(v), n, dim, kind, _p(r), m, _p(off), None) != 0:
        raise MemoryError("oracle_ray_intersect")
    idx = np.zeros(int(off[-1]), dtype=np.int32)
    lib().oracle_ray_intersect(_p(v), n, dim, kind, _p(r), m, _p(off), _p(idx))
    return off, idx


def ray_ordered_intersect(values, rays, dim=3, kind=POINTS):
    """Ray ordered intersect (Section 2.5): CSR rows in the order (entry t, index), with the entry
    parameters: (offsets, indices, t)."""
    v, n = _values(values, dim, kind)
    r, m = _queries(rays, dim, 2)
    off, _ = ray_intersect(values, rays, dim=dim, kind=kind)
    idx = np.zeros(int(off[-1]), dtype=np.int32)
    t = np.zeros(int(off[-1]), dtype=np.float32)
    lib().oracle_ray_ordered_intersect(_p(v), n, dim, kind, _p(r), m, _p(off), _p(idx), _p(t))
    return off, idx, t


def dbscan(points, eps, min_pts, dim=3):
    """DBSCAN (Section 2.4) by definition: int32 labels; a cluster is labelled by its smallest core
    index, a border point by its smallest-index core neighbour's cluster, noise by -1.  O(n^2)."""
    v, n = _values(points, dim, POINTS)
    labels = np.zeros(n, dtype=np.int32)
    if lib().oracle_dbscan(_p(v), n, dim, np.float32(eps), np.int32(min_pts), _p(labels)) != 0:
        raise MemoryError("oracle_dbscan")
    return labels


def self_join_degree(points, radius, dim=3):
    """Pair search (Section 2.6) as a self-join: int32 degree[i] = number of j != i with
    d2(p_i, p_j) <= fl(r*r)."""
    v, n = _values(points, dim, POINTS)
    deg = np.zeros(n, dtype=np.int32)
    lib().oracle_self_join_degree(_p(v), n, dim, np.float32(radius), _p(deg))
    return deg


def self_join_pairs(points, radius, dim=3):
    """The self-join's unordered pairs as upper-triangle CSR: row i = ascending j > i within r."""
    v, n = _values(points, dim, POINTS)
    off = np.zeros(n + 1, dtype=np.int64)
    lib().oracle_self_join_pairs(_p(v), n, dim, np.float32(radius), _p(off), None)
    idx = np.zeros(int(off[-1]), dtype=np.int32)
    lib().oracle_self_join_pairs(_p(v), n, dim, np.float32(radius), _p(off), _p(idx))
    return off, idx


def match_distances(values, queries, offsets, indices, dim=3, kind=POINTS):
    """Callback with output (Section 2.1, query call (2)): float32 squared distance of every CSR match."""
    v, n = _values(values, dim, kind)
    q, m = _queries(queries, dim, 1)
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    idx = np.ascontiguousarray(indices, dtype=np.int32)
    out = np.zeros(len(idx), dtype=np.float32)
    lib().oracle_match_distances(_p(v), n, dim, kind, _p(q), m, _p(off), _p(idx), _p(out))
    return out


def count_up_to(values, queries, radius, n_max, dim=3, kind=POINTS):
    """Early-terminating count (Section 2.2): each query stops at n_max matches; int32[m]."""
    v, n = _values(values, dim, kind)
    q, m = _queries(queries, dim, 1)
    counts = np.zeros(m, dtype=np.int32)
    lib().oracle_count_up_to(_p(v), n, dim, kind, _p(q), m, np.float32(radius), np.int32(n_max), _p(counts))
    return counts


def knn(values, queries, k, dim=3, kind=POINTS):
    """k nearest in the order (d2, index): (d2 float32[m][k], idx int32[m][k]), padded (+inf, -1)."""
    v, n = _values(values, dim, kind)
    q, m = _queries(queries, dim, 1)
    d2 = np.zeros((m, k), dtype=np.float32)
    idx = np.zeros((m, k), dtype=np.int32)
    if lib().oracle_knn(_p(v), n, dim, kind, _p(q), m, int(k), _p(d2), _p(idx)) != 0:
        raise ValueError("k must be positive")
    return d2, idx


def chamfer_forward(a, a_off, b, b_off):
    """(loss float64[P], nn_ab int32[sum nA], nn_ba int32[sum nB]) with local neighbour indices."""
    a = np.ascontiguousarray(a, dtype=np.float32)
    b = np.ascontiguousarray(b, dtype=np.float32)
    a_off = np.ascontiguousarray(a_off, dtype=np.int64)
    b_off = np.ascontiguousarray(b_off, dtype=np.int64)
    P = len(a_off) - 1
    loss = np.zeros(P, dtype=np.float64)
    nn_ab = np.zeros(int(a_off[-1]), dtype=np.int32)
    nn_ba = np.zeros(int(b_off[-1]), dtype=np.int32)
    lib().oracle_chamfer_forward(_p(a), _p(a_off), _p(b), _p(b_off), P, _p(loss), _p(nn_ab), _p(nn_ba))
    return loss, nn_ab, nn_ba


def chamfer_backward(a, a_off, b, b_off, nn_ab, nn_ba, grad_loss):
    """(grad_a float64[sum nA][3], grad_b float64[sum nB][3]) for fixed neighbour indices."""
    a = np.ascontiguousarray(a, dtype=np.float32)
    b = np.ascontiguousarray(b, dtype=np.float32)
    a_off = np.ascontiguousarray(a_off, dtype=np.int64)
    b_off = np.ascontiguousarray(b_off, dtype=np.int64)
    nn_ab = np.ascontiguousarray(nn_ab, dtype=np.int32)
    nn_ba = np.ascontiguousarray(nn_ba, dtype=np.int32)
    g = np.ascontiguousarray(grad_loss, dtype=np.float64)
    P = len(a_off) - 1
    ga = np.zeros((int(a_off[-1]), 3), dtype=np.float64)
    gb = np.zeros((int(b_off[-1]), 3), dtype=np.float64)
    lib().oracle_chamfer_backward(_p(a), _p(a_off), _p(b), _p(b_off), P, _p(nn_ab), _p(nn_ba), _p(g), _p(ga), _p(gb))
    return ga, gb


# ---------------------------------------------------------------------------
# forest: each batch against its own tree, local indices
# ---------------------------------------------------------------------------

def forest_reduce(values, tree_offsets, queries, batch_offsets, batch_tree, batch_radius, op=COUNT_SUMDIST,
                  scale_bits=32, batches=None):
    """Per batch b: reduce(queries of b, tree batch_tree[b], batch_radius[b]); optional batch subset."""
    m = int(batch_offsets[-1])
    counts = np.full(m, -1, dtype=np.int32)
    sums = np.full(m, -1, dtype=np.int64)
    for b in (range(len(batch_tree)) if batches is None else batches):
        t = int(batch_tree[b])
        v = values[tree_offsets[t]:tree_offsets[t + 1]]
        q0, q1 = int(batch_offsets[b]), int(batch_offsets[b + 1])
        c, s = reduce(v, queries[q0:q1], batch_radius[b], op, scale_bits)
        counts[q0:q1] = c
        if s is not None:
            sums[q0:q1] = s
    return counts, sums


def forest_knn(values, tree_offsets, queries, batch_offsets, batch_tree, k, batches=None):
    m = int(batch_offsets[-1])
    d2 = np.full((m, k), np.nan, dtype=np.float32)
    idx = np.full((m, k), -2, dtype=np.int32)
    for b in (range(len(batch_tree)) if batches is None else batches):
        t = int(batch_tree[b])
        v = values[tree_offsets[t]:tree_offsets[t + 1]]
        q0, q1 = int(batch_offsets[b]), int(batch_offsets[b + 1])
        d2[q0:q1], idx[q0:q1] = knn(v, queries[q0:q1], k)
    return d2, idx
