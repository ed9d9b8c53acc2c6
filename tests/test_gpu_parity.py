"""HIP path vs the CPU oracle, element by element, through the C ABI.

Integer outputs (indices, counts, fixed-point sums) and kNN distances must be
bit-identical: both sides compute float32 squared distances in the same
operation order without contraction, and every decision (radius test, kNN
order) is taken on those identical values.
"""
import numpy as np
import pytest

import oracle
import paper_2507_23700_amd as ax
from paper_2507_23700_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ax.arborx_reset_tuning()
    yield
    ax.arborx_reset_tuning()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    return t.cpu().numpy()


def check_spatial(tree, data, q, r, dim=3, kind=oracle.POINTS):
    off, idx = ax.arborx_query_spatial(tree, dev(q), float(r))
    o_off, o_idx = oracle.spatial(data, q, r, dim=dim, kind=kind)
    assert np.array_equal(host(off), o_off)
    assert np.array_equal(host(idx), o_idx)
    return o_off


def check_spatial_dist(tree, data, q, r, dim=3, kind=oracle.POINTS):
    """The callback-with-output form: (offsets, indices, distances) from one search, exact."""
    off, idx, d2 = ax.arborx_query_spatial_with_distances(tree, dev(q), float(r))
    o_off, o_idx = oracle.spatial(data, q, r, dim=dim, kind=kind)
    assert np.array_equal(host(off), o_off) and np.array_equal(host(idx), o_idx)
    assert np.array_equal(host(d2), oracle.match_distances(data, q, o_off, o_idx, dim=dim, kind=kind))
    return o_off


def check_knn(tree, data, q, k, dim=3, kind=oracle.POINTS):
    d2, ix = ax.arborx_query_knn(tree, dev(q), k)
    o_d2, o_ix = oracle.knn(data, q, k, dim=dim, kind=kind)
    assert np.array_equal(host(ix), o_ix)
    assert np.array_equal(host(d2), o_d2)


def check_reduce(tree, data, q, r, dim=3, kind=oracle.POINTS, sums=True):
    c, s = ax.arborx_query_spatial_reduce(tree, dev(q), float(r), ax.COUNT_SUMDIST)
    oc, os_ = oracle.reduce(data, q, r, dim=dim, kind=kind)
    assert np.array_equal(host(c), oc)
    if sums:  # fixed-point sums are only defined while the scaled distances fit in 63 bits
        assert np.array_equal(host(s), os_)
    c2, _ = ax.arborx_query_spatial_reduce(tree, dev(q), float(r), ax.COUNT)
    assert np.array_equal(host(c2), oc)


# ---------------------------------------------------------------------------
# components
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n", [1, 2, 4095, 4096, 4097, 100_003])
def test_radix_sort_stable_u64(n):
    g = np.random.default_rng(n)
    keys = g.integers(0, 1 << 63, size=n, dtype=np.int64)
    keys[::3] = keys[0]  # many equal keys
    keys[1::7] = g.integers(0, 50, size=len(keys[1::7]))
    vals = np.arange(n, dtype=np.int32)
    k, v = dev(keys), dev(vals)
    ax.arborx_debug_radix_sort(k, v, 0, 64)
    order = np.argsort(keys.view(np.uint64), kind="stable")
    assert np.array_equal(host(v), order.astype(np.int32))
    assert np.array_equal(host(k), keys[order])


def test_radix_sort_bit_range_u32():
    g = np.random.default_rng(5)
    n = 70_001
    keys = g.integers(0, 1 << 31, size=n, dtype=np.int64).astype(np.int32)
    vals = g.integers(0, 1 << 30, size=n, dtype=np.int64).astype(np.int32)
    k, v = dev(keys), dev(vals)
    ax.arborx_debug_radix_sort(k, v, 3, 20)
    sub = (keys.view(np.uint32) >> 3) & ((1 << 17) - 1)
    order = np.argsort(sub, kind="stable")
    assert np.array_equal(host(v), vals[order])


def _morton_ref(pts, lo, hi, dim):
    """Independent bit-loop encoder: cell of each coordinate, then bit interleave."""
    bits = 63 // dim
    ext = (hi - lo).astype(np.float32)
    inv = np.where(ext > 0, np.float32(1) / np.where(ext > 0, ext, 1), 0).astype(np.float32)
    u = ((pts - lo).astype(np.float32) * inv).astype(np.float32) * np.float32(1 << bits)
    cell = np.clip(np.floor(np.maximum(u, 0).astype(np.float64)), 0, (1 << bits) - 1).astype(np.uint64)
    code = np.zeros(len(pts), dtype=np.uint64)
    for b in range(bits - 1, -1, -1):
        for d in range(dim):
            code = (code << np.uint64(1)) | ((cell[:, d] >> np.uint64(b)) & np.uint64(1))
    return code


@pytest.mark.parametrize("dim", [2, 3, 6])
def test_morton64(dim):
    g = np.random.default_rng(dim)
    pts = g.random((5000, dim)).astype(np.float32)
    pts[0] = 0
    pts[1] = 1
    lo, hi = np.zeros(dim, np.float32), np.ones(dim, np.float32)
    codes = host(ax.arborx_debug_morton64(dev(pts), dev(np.stack([lo, hi])))).view(np.uint64)
    ref = _morton_ref(pts, lo, hi, dim)
    assert codes[0] == 0 and codes[1] == (1 << ((63 // dim) * dim)) - 1
    # quantisation may differ by float rounding of x*inv*2^b vs the reference only at cell edges
    assert np.mean(codes == ref) > 0.999


def _tree_invariants(tree, data, kind=oracle.POINTS):
    child, lo, hi, root = ax.arborx_debug_tree_nodes(tree)
    n, dim = tree.n, tree.dim
    if kind == oracle.POINTS:
        vlo = vhi = data
    else:
        vlo, vhi = data[:, 0], data[:, 1]
    seen_leaf = np.zeros(n, dtype=np.int32)
    seen_node = np.zeros(max(n - 1, 1), dtype=np.int32)
    stack = [(root, 0)]
    maxdepth = 0
    while stack:
        node, depth = stack.pop()
        seen_node[node] += 1
        for s in range(2):
            c = int(child[node, s])
            if c == -2 ** 31:
                continue
            if c < 0:
                j = ~c
                seen_leaf[j] += 1
                assert np.array_equal(lo[node, s], vlo[j]) and np.array_equal(hi[node, s], vhi[j])
                maxdepth = max(maxdepth, depth + 1)
            else:
                # the slot box is the exact union of the child's two slots
                cl = np.minimum(lo[c, 0], lo[c, 1]) if child[c, 1] != -2 ** 31 else lo[c, 0]
                ch = np.maximum(hi[c, 0], hi[c, 1]) if child[c, 1] != -2 ** 31 else hi[c, 0]
                assert np.array_equal(lo[node, s], cl) and np.array_equal(hi[node, s], ch)
                stack.append((c, depth + 1))
    assert np.all(seen_leaf == 1)
    assert np.all(seen_node == 1)
    info = ax.arborx_bvh_info(tree)
    assert info["height"] == maxdepth
    return child, lo, hi


def test_tree_invariants_and_repeatable_builds():
    cfg = inputs.config_small(n=30_000, m=10)
    data = cfg["data"]
    d = dev(data)
    t0 = ax.arborx_bvh_build(d)
    c0, l0, h0 = _tree_invariants(t0, data)
    info = ax.arborx_bvh_info(t0)
    assert info["n"] == 30_000 and info["dim"] == 3
    assert np.array_equal(np.float32(info["lo"]), data.min(0)) and np.array_equal(np.float32(info["hi"]), data.max(0))
    for _ in range(20):  # the hierarchy is a deterministic function of the input; races would show
        t = ax.arborx_bvh_build(d)
        c, l, h, _r = ax.arborx_debug_tree_nodes(t)
        assert np.array_equal(c, c0) and np.array_equal(l, l0) and np.array_equal(h, h0)


@pytest.mark.parametrize("n", [1023, 1024, 1025, 70_001])
def test_chunked_and_single_pass_builds_identical(n):
    g = np.random.default_rng(n)
    data = g.random((n, 3)).astype(np.float32)
    data[n // 3:n // 3 + n // 5] = data[1]  # equal codes across chunk borders
    d = dev(data)
    ax.arborx_set_tuning(build=1)
    try:
        ref = ax.arborx_debug_tree_nodes(ax.arborx_bvh_build(d))
    finally:
        ax.arborx_reset_tuning()
    t = ax.arborx_bvh_build(d)
    got = ax.arborx_debug_tree_nodes(t)
    for a, b in zip(ref, got):
        assert np.array_equal(a, b)
    _tree_invariants(t, data)
    g6 = g.random((n, 6)).astype(np.float32)
    d6 = dev(g6)
    ax.arborx_set_tuning(build=1)
    try:
        ref6 = ax.arborx_debug_tree_nodes(ax.arborx_bvh_build(d6))
    finally:
        ax.arborx_reset_tuning()
    t6 = ax.arborx_bvh_build(d6)
    for a, b in zip(ref6, ax.arborx_debug_tree_nodes(t6)):
        assert np.array_equal(a, b)
    _tree_invariants(t6, g6)


@pytest.mark.parametrize("n,dim,boxes", [(1025, 3, False), (70_001, 3, False), (5000, 6, False), (4000, 3, True),
                                         (1, 3, False)])
def test_quantized_nodes_both_builds(n, dim, boxes):
    # quantized nodes over trees from the single-pass and the chunked climb (equal codes across chunk borders,
    # box leaves refetched, a one-value tree): walks over them give the oracle's results
    g = np.random.default_rng(n + dim)
    c = g.random((n, dim)).astype(np.float32)
    c[n // 3:n // 3 + n // 5] = c[0]  # equal codes across chunk borders
    if boxes:
        h = (g.random((n, dim)) * 0.01).astype(np.float32)
        data, kind = np.ascontiguousarray(np.stack([c - h, c + h], axis=1)), oracle.BOXES
    else:
        data, kind = c, oracle.POINTS
    q = g.random((700, dim)).astype(np.float32)
    r = 0.05 if dim == 3 else 0.4
    for build in (1, 0):
        ax.arborx_set_tuning(build=build, node_format=1)
        try:
            t = ax.arborx_bvh_build(dev(data), ax.BOXES if boxes else ax.POINTS)
            check_spatial(t, data, q, r, dim=dim, kind=kind)
            check_knn(t, data, q, min(n, 7), dim=dim, kind=kind)
            if not boxes:
                check_reduce(t, data, q, r, dim=dim)
        finally:
            ax.arborx_reset_tuning()


def test_tree_invariants_duplicates_and_boxes():
    g = np.random.default_rng(1)
    data = g.random((3000, 3)).astype(np.float32)
    data[1000:2500] = data[7]  # long run of equal Morton codes
    _tree_invariants(ax.arborx_bvh_build(dev(data)), data)
    c = g.random((2000, 3)).astype(np.float32)
    h = (g.random((2000, 3)) * 0.02).astype(np.float32)
    boxes = np.ascontiguousarray(np.stack([c - h, c + h], axis=1))
    _tree_invariants(ax.arborx_bvh_build(dev(boxes), ax.BOXES), boxes, oracle.BOXES)


# ---------------------------------------------------------------------------
# parity with the oracle
# ---------------------------------------------------------------------------

def test_small_cube_all_queries():
    cfg = inputs.config_small()
    data, q, r = cfg["data"], cfg["queries"], cfg["radius"]
    tree = ax.arborx_bvh_build(dev(data))
    off = check_spatial(tree, data, q, r)
    assert off[-1] > 9 * len(q)
    check_knn(tree, data, q, cfg["k"])
    check_reduce(tree, data, q, r)


@pytest.mark.parametrize("k", [1, 2, 3, 8, 16, 17, 64])
def test_knn_k_values(k):
    cfg = inputs.config_small(n=5000, m=3000)
    tree = ax.arborx_bvh_build(dev(cfg["data"]))
    check_knn(tree, cfg["data"], cfg["queries"], k)


def test_shell_and_gmm6():
    s = inputs.config_paper("shell", n=40_000, m=5000)
    t = ax.arborx_bvh_build(dev(s["data"]))
    check_spatial(t, s["data"], s["queries"], inputs.radius_shell(40_000, 10.0))
    check_knn(t, s["data"], s["queries"], 16)
    g = inputs.config_gmm6(n=30_000, m=4000)
    r6 = inputs.radius_gmm(30_000, 20.0)
    t6 = ax.arborx_bvh_build(dev(g["data"]))
    check_spatial(t6, g["data"], g["queries"], r6, dim=6)
    check_knn(t6, g["data"], g["queries"], 8, dim=6)
    check_reduce(t6, g["data"], g["queries"], r6, dim=6)


@pytest.mark.parametrize("case", ["shell3", "gmm6", "dim2", "boxes", "duplicates"])
@pytest.mark.parametrize("node_format", [0, 1])
def test_knn_node_formats(case, node_format):
    # kNN on float and quantized nodes over ragged query counts, 2D/3D/6D,
    # box values and many equal points (ties decided by index)
    g = np.random.default_rng(404)
    dim, kind, k = 3, oracle.POINTS, 16
    if case == "shell3":
        s = inputs.config_paper("shell", n=30_000, m=3001)
        data, q = s["data"], s["queries"]
    elif case == "gmm6":
        s = inputs.config_gmm6(n=20_000, m=2003)
        data, q, dim, k = s["data"], s["queries"], 6, 8
    elif case == "dim2":
        data, q, dim, k = g.random((7000, 2)).astype(np.float32), g.random((902, 2)).astype(np.float32), 2, 5
    elif case == "boxes":
        c = g.random((6000, 3)).astype(np.float32)
        h = (g.random((6000, 3)) * 0.01).astype(np.float32)
        data, kind, k = np.ascontiguousarray(np.stack([c - h, c + h], axis=1)), oracle.BOXES, 10
        q = g.random((2001, 3)).astype(np.float32)
    else:  # many equal points: ties decided by index
        data = np.repeat(g.random((500, 3)).astype(np.float32), 8, axis=0)
        q = np.concatenate([data[::7], g.random((300, 3)).astype(np.float32)])
    ax.arborx_set_tuning(node_format=node_format)
    try:
        t = ax.arborx_bvh_build(dev(data), ax.BOXES if kind == oracle.BOXES else ax.POINTS)
        check_knn(t, data, q, k, dim=dim, kind=kind)
        check_knn(t, data, q[:3], 1, dim=dim, kind=kind)
    finally:
        ax.arborx_reset_tuning()


def test_dim2():
    g = np.random.default_rng(2)
    data = g.random((7000, 2)).astype(np.float32)
    q = g.random((900, 2)).astype(np.float32)
    t = ax.arborx_bvh_build(dev(data))
    check_spatial(t, data, q, 0.02, dim=2)
    check_knn(t, data, q, 5, dim=2)


def test_box_values_and_intersects():
    g = np.random.default_rng(3)
    c = g.random((6000, 3)).astype(np.float32)
    h = (g.random((6000, 3)) * 0.01).astype(np.float32)
    boxes = np.ascontiguousarray(np.stack([c - h, c + h], axis=1))
    q = g.random((2000, 3)).astype(np.float32)
    t = ax.arborx_bvh_build(dev(boxes), ax.BOXES)
    check_spatial(t, boxes, q, 0.03, kind=oracle.BOXES)
    check_knn(t, boxes, q, 10, kind=oracle.BOXES)
    check_reduce(t, boxes, q, 0.03, kind=oracle.BOXES)
    qc = g.random((1500, 3)).astype(np.float32)
    qh = (g.random((1500, 3)) * 0.03).astype(np.float32)
    qb = np.ascontiguousarray(np.stack([qc - qh, qc + qh], axis=1))
    off, idx = ax.arborx_query_intersects(t, dev(qb))
    o_off, o_idx = oracle.intersects(boxes, qb, kind=oracle.BOXES)
    assert np.array_equal(host(off), o_off) and np.array_equal(host(idx), o_idx)
    tp = ax.arborx_bvh_build(dev(c))
    off, idx = ax.arborx_query_intersects(tp, dev(qb))
    o_off, o_idx = oracle.intersects(c, qb)
    assert np.array_equal(host(off), o_off) and np.array_equal(host(idx), o_idx)


# ---------------------------------------------------------------------------
# edge cases
# ---------------------------------------------------------------------------

def test_empty_tree_and_empty_queries():
    q = np.random.default_rng(0).random((50, 3)).astype(np.float32)
    t = ax.arborx_bvh_build(torch.zeros((0, 3), dtype=torch.float32, device="cuda"))
    info = ax.arborx_bvh_info(t)
    assert info["empty"] and info["n"] == 0
    off, idx = ax.arborx_query_spatial(t, dev(q), 1.0)
    assert np.all(host(off) == 0) and idx.numel() == 0
    d2, ix = ax.arborx_query_knn(t, dev(q), 4)
    assert np.all(np.isinf(host(d2))) and np.all(host(ix) == -1)
    c, s = ax.arborx_query_spatial_reduce(t, dev(q), 1.0)
    assert np.all(host(c) == 0) and np.all(host(s) == 0)
    data = q[:10]
    t2 = ax.arborx_bvh_build(dev(data))
    e = torch.zeros((0, 3), dtype=torch.float32, device="cuda")
    off, idx = ax.arborx_query_spatial(t2, e, 1.0)
    assert host(off).tolist() == [0] and idx.numel() == 0
    d2, ix = ax.arborx_query_knn(t2, e, 3)
    assert d2.shape == (0, 3)


@pytest.mark.parametrize("n", [1, 2, 3, 5, 64, 65])
def test_tiny_trees(n):
    g = np.random.default_rng(n)
    data = g.random((n, 3)).astype(np.float32)
    q = g.random((300, 3)).astype(np.float32)
    t = ax.arborx_bvh_build(dev(data))
    check_spatial(t, data, q, 0.5)
    check_knn(t, data, q, 4)
    check_reduce(t, data, q, 0.5)
    check_spatial(t, data, q, float("inf"))


def test_all_equal_points_and_zero_radius():
    data = np.tile(np.float32([0.3, 0.6, 0.9]), (5000, 1))
    data[::10] += np.float32(1e-3)
    q = np.concatenate([data[:5], np.random.default_rng(1).random((20, 3)).astype(np.float32)])
    t = ax.arborx_bvh_build(dev(data))
    check_spatial(t, data, q, 0.0)  # exact duplicates only
    check_knn(t, data, q, 12)       # all ties: smallest indices first
    check_spatial(t, data, q, 1e-3)


def test_infinite_radius_long_rows():
    g = np.random.default_rng(4)
    data = g.random((9000, 3)).astype(np.float32)
    q = g.random((40, 3)).astype(np.float32)
    t = ax.arborx_bvh_build(dev(data))
    off = check_spatial(t, data, q, float("inf"))
    assert off[-1] == 9000 * 40
    check_spatial(t, data, q, 0.35)  # rows of a few thousand: workgroup sort
    check_spatial_dist(t, data, q, float("inf"))  # rows past the workgroup sort: radix path carries distances
    check_spatial_dist(t, data, q, 0.35)


def test_denormal_distances():
    data = np.array([[0, 0, 0], [1e-20, 0, 0], [0, 3e-20, 0], [1, 1, 1]], dtype=np.float32)
    q = np.array([[0, 0, 0], [1e-20, 1e-20, 0]], dtype=np.float32)
    t = ax.arborx_bvh_build(dev(data))
    check_knn(t, data, q, 4)
    check_spatial(t, data, q, 2e-20)
    check_reduce(t, data, q, 2e-20)


def test_capacity_protocol():
    cfg = inputs.config_small(n=2000, m=500)
    t = ax.arborx_bvh_build(dev(cfg["data"]))
    import ctypes
    from paper_2507_23700_amd import _lib
    q = dev(cfg["queries"])
    off = torch.empty(501, dtype=torch.int64, device="cuda")
    total = ctypes.c_int64()
    st = _lib.lib().arborx_query_spatial(t.handle, ctypes.c_void_p(q.data_ptr()), 500, ctypes.c_float(cfg["radius"]),
                                         ctypes.c_void_p(off.data_ptr()), None, 0, ctypes.byref(total), None)
    assert st == ax.E_CAPACITY
    o_off, o_idx = oracle.spatial(cfg["data"], cfg["queries"], cfg["radius"])
    assert total.value == o_off[-1] and np.array_equal(host(off), o_off)
    # the distance form follows the same protocol, and a missing distances buffer counts as too small
    L = _lib.lib()
    idx = torch.empty(int(o_off[-1]), dtype=torch.int32, device="cuda")
    d2 = torch.empty(int(o_off[-1]), dtype=torch.float32, device="cuda")
    args = (t.handle, ctypes.c_void_p(q.data_ptr()), 500, ctypes.c_float(cfg["radius"]), ctypes.c_void_p(off.data_ptr()))
    st = L.arborx_query_spatial_with_distances(*args, ctypes.c_void_p(idx.data_ptr()), None, idx.numel(),
                                               ctypes.byref(total), None)
    assert st == ax.E_CAPACITY and total.value == o_off[-1]
    st = L.arborx_query_spatial_with_distances(*args, ctypes.c_void_p(idx.data_ptr()), ctypes.c_void_p(d2.data_ptr()),
                                               idx.numel() - 1, ctypes.byref(total), None)
    assert st == ax.E_CAPACITY
    st = L.arborx_query_spatial_with_distances(*args, ctypes.c_void_p(idx.data_ptr()), ctypes.c_void_p(d2.data_ptr()),
                                               idx.numel(), ctypes.byref(total), None)
    assert st == ax.OK and np.array_equal(host(idx), o_idx)
    assert np.array_equal(host(d2), oracle.match_distances(cfg["data"], cfg["queries"], o_off, o_idx))
    # a plan begun without distances cannot give them
    plan = ctypes.c_void_p()
    assert L.arborx_query_spatial_begin(*args, ctypes.byref(total), ctypes.byref(plan), None) == ax.OK
    try:
        assert L.arborx_query_finish_with_distances(plan, ctypes.c_void_p(idx.data_ptr()),
                                                    ctypes.c_void_p(d2.data_ptr()), idx.numel()) == ax.E_INVALID
    finally:
        L.arborx_plan_destroy(plan)


@pytest.mark.parametrize("block,order,stack,schedule,node_format",
                         [(64, 1, 1, 0, 0), (128, 0, 2, 0, 0), (256, 1, 4, 0, 0), (256, 0, 64, 0, 0), (64, 0, 16, 0, 0),
                          (64, 1, 1, 0, 1), (256, 0, 64, 0, 1), (128, 1, 16, 0, 1),
                          (64, 1, 1, 0, 2), (256, 0, 64, 0, 2), (128, 1, 16, 0, 2), (256, 1, 4, 1, 2), (64, 1, 8, 2, 2),
                          (256, 1, 16, 1, 0), (64, 0, 16, 1, 0), (128, 1, 4, 1, 0),
                          (256, 1, 16, 2, 0), (64, 0, 16, 2, 0)])
def test_schedules_identical(block, order, stack, schedule, node_format):
    cfg = inputs.config_small(n=20_000, m=4000)
    data, q, r = cfg["data"], cfg["queries"], cfg["radius"]
    ax.arborx_set_tuning(block=block, order=order, stack=stack, schedule=schedule, node_format=node_format)
    try:
        t = ax.arborx_bvh_build(dev(data))
        check_spatial(t, data, q, r)
        check_spatial_dist(t, data, q, r)
        check_knn(t, data, q, 10)
        check_reduce(t, data, q, r)
    finally:
        ax.arborx_reset_tuning()


@pytest.mark.parametrize("nq", [1, 2, 4])
def test_query_packets_identical(nq):
    cfg = inputs.config_small(n=20_000, m=4001)  # a ragged last packet
    data, q, r = cfg["data"], cfg["queries"], cfg["radius"]
    t = ax.arborx_bvh_build(dev(data))
    for kw in (dict(queries_per_thread=nq), dict(queries_per_thread=nq, block=64, stack=2),
               dict(queries_per_thread=nq, order=0)):
        ax.arborx_set_tuning(**kw)
        try:
            check_reduce(t, data, q, r)
            check_reduce(t, data, q, 0.0)
            check_reduce(t, data, q[:3], float("inf"))
            check_spatial(t, data, q, r)
            check_spatial(t, data, q[:5], 0.3)  # rows longer than the register stash
            check_knn(t, data, q, 10)  # kNN ignores queries_per_thread: same rows under every setting
            check_knn(t, data, q[:6], 3)
        finally:
            ax.arborx_reset_tuning()
    g = np.random.default_rng(nq)
    for n in (1, 2, 5):
        small = g.random((n, 3)).astype(np.float32)
        ts = ax.arborx_bvh_build(dev(small))
        ax.arborx_set_tuning(queries_per_thread=nq)
        try:
            check_reduce(ts, small, q[:7], 0.4)
            check_spatial(ts, small, q[:7], 0.4)
            check_knn(ts, small, q[:7], 4)  # k above n: padded rows
        finally:
            ax.arborx_reset_tuning()


def test_stream_argument():
    cfg = inputs.config_small(n=3000, m=700)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        d = dev(cfg["data"])
        q = dev(cfg["queries"])
        t = ax.arborx_bvh_build(d, stream=s)
        d2, ix = ax.arborx_query_knn(t, q, 7, stream=s)
    s.synchronize()
    o_d2, o_ix = oracle.knn(cfg["data"], cfg["queries"], 7)
    assert np.array_equal(host(ix), o_ix)


def test_destroy_with_queries_in_flight():
    # destroying a tree orders the release of its memory after the work already
    # queued on every stream that used it; a new build may then reuse the memory
    cfg = inputs.config_small(n=50_000, m=20_000)
    other = np.random.default_rng(9).random((50_000, 3)).astype(np.float32)
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        d, q = dev(cfg["data"]), dev(cfg["queries"])
        t = ax.arborx_bvh_build(d, stream=side)
        c, s = ax.arborx_query_spatial_reduce(t, q, cfg["radius"], ax.COUNT_SUMDIST, stream=side)
        d2, ix = ax.arborx_query_knn(t, q, 8, stream=side)
    ax.arborx_bvh_destroy(t)
    t2 = ax.arborx_bvh_build(dev(other))
    c2, _ = ax.arborx_query_spatial_reduce(t2, dev(cfg["queries"]), cfg["radius"], ax.COUNT)
    side.synchronize()
    torch.cuda.synchronize()
    oc, os_ = oracle.reduce(cfg["data"], cfg["queries"], cfg["radius"])
    assert np.array_equal(host(c), oc) and np.array_equal(host(s), os_)
    o_d2, o_ix = oracle.knn(cfg["data"], cfg["queries"], 8)
    assert np.array_equal(host(ix), o_ix) and np.array_equal(host(d2), o_d2)
    oc2, _ = oracle.reduce(other, cfg["queries"], cfg["radius"])
    assert np.array_equal(host(c2), oc2)


def test_query_order_cache():
    # the tree reuses the traversal order of a repeated query array; results
    # never depend on it, also when the array changes in place
    cfg = inputs.config_small(n=30_000, m=8000)
    data, r = cfg["data"], cfg["radius"]
    t = ax.arborx_bvh_build(dev(data))
    qa = cfg["queries"]
    qb = np.random.default_rng(21).random((8000, 3)).astype(np.float32)
    q = dev(qa)
    check_reduce(t, data, qa, r)
    c, _ = ax.arborx_query_spatial_reduce(t, q, r, ax.COUNT)            # same array: reused order
    assert np.array_equal(host(c), oracle.reduce(data, qa, r)[0])
    q.copy_(dev(qb))                                                    # same address, new contents
    c, s = ax.arborx_query_spatial_reduce(t, q, r, ax.COUNT_SUMDIST)
    oc, os_ = oracle.reduce(data, qb, r)
    assert np.array_equal(host(c), oc) and np.array_equal(host(s), os_)
    d2, ix = ax.arborx_query_knn(t, q, 6)
    o_d2, o_ix = oracle.knn(data, qb, 6)
    assert np.array_equal(host(ix), o_ix) and np.array_equal(host(d2), o_d2)
    off, idx = ax.arborx_query_spatial(t, q, r)
    o_off, o_idx = oracle.spatial(data, qb, r)
    assert np.array_equal(host(off), o_off) and np.array_equal(host(idx), o_idx)
    side = torch.cuda.Stream()                                          # another stream, alternating arrays
    q2 = dev(qa)
    with torch.cuda.stream(side):
        for qq, ref in ((q2, qa), (q, qb), (q2, qa)):
            c, _ = ax.arborx_query_spatial_reduce(t, qq, r, ax.COUNT, stream=side)
            side.synchronize()
            assert np.array_equal(host(c), oracle.reduce(data, ref, r)[0])
    ax.arborx_bvh_destroy(t)
    torch.cuda.synchronize()


def test_plan_api_two_calls():
    import ctypes
    from paper_2507_23700_amd import _lib
    L = _lib.lib()
    cfg = inputs.config_small(n=6000, m=1500)
    t = ax.arborx_bvh_build(dev(cfg["data"]))
    q = dev(cfg["queries"])
    off = torch.empty(1501, dtype=torch.int64, device="cuda")
    total, plan = ctypes.c_int64(), ctypes.c_void_p()
    P = ctypes.c_void_p
    assert L.arborx_query_spatial_begin(t.handle, P(q.data_ptr()), 1500, ctypes.c_float(cfg["radius"]),
                                        P(off.data_ptr()), ctypes.byref(total), ctypes.byref(plan), None) == 0
    o_off, o_idx = oracle.spatial(cfg["data"], cfg["queries"], cfg["radius"])
    assert total.value == o_off[-1] and np.array_equal(host(off), o_off)
    small = torch.empty(max(total.value - 1, 1), dtype=torch.int32, device="cuda")
    assert L.arborx_query_finish(plan, P(small.data_ptr()), small.numel()) == ax.E_CAPACITY
    idx = torch.empty(total.value, dtype=torch.int32, device="cuda")
    assert L.arborx_query_finish(plan, P(idx.data_ptr()), idx.numel()) == 0
    torch.cuda.synchronize()
    assert L.arborx_plan_destroy(plan) == 0
    assert np.array_equal(host(idx), o_idx)


def test_rows_around_stash_size():
    # clustered data: row lengths spread across the in-register limit (16)
    g = np.random.default_rng(8)
    centres = g.random((300, 3))
    data = (centres[g.integers(0, 300, 20000)] + 0.004 * g.standard_normal((20000, 3))).astype(np.float32)
    q = (centres[g.integers(0, 300, 6000)] + 0.004 * g.standard_normal((6000, 3))).astype(np.float32)
    t = ax.arborx_bvh_build(dev(data))
    off = check_spatial(t, data, q, 0.007)
    lens = np.diff(off)
    assert (lens == 16).any() and (lens == 17).any() and (lens > 40).any() and (lens < 16).any()


@pytest.mark.parametrize("case", ["chains", "pool_runs_out", "wave", "rope", "quantized", "four_wide", "one_per_thread"])
def test_overflow_chains(case):
    # uniform points plus 20 dense blobs: queries near a blob centre have rows of several hundred matches,
    # kept in chains of many overflow chunks; with few queries the pool is small and runs out, and those
    # rows are walked a second time instead
    g = np.random.default_rng(11)
    hot = g.random((20, 3))
    blob = hot[g.integers(0, 20, 12000)] + 0.003 * g.standard_normal((12000, 3))
    data = np.concatenate([g.random((30000, 3)), blob]).astype(np.float32)
    near = lambda n: hot[g.integers(0, 20, n)] + 0.001 * g.standard_normal((n, 3))
    q = (near(60) if case == "pool_runs_out" else np.concatenate([g.random((20000, 3)), near(40)])).astype(np.float32)
    tuning = dict(wave=dict(schedule=1), rope=dict(schedule=2), quantized=dict(node_format=1),
                  four_wide=dict(node_format=2), one_per_thread=dict(queries_per_thread=1)).get(case, {})
    ax.arborx_set_tuning(**tuning)
    try:
        t = ax.arborx_bvh_build(dev(data))
        off = check_spatial(t, data, q, 0.01)
        check_spatial_dist(t, data, q, 0.01)  # distances through the stash, chunks and second walks
    finally:
        ax.arborx_reset_tuning()
    lens = np.diff(off)
    assert lens.max() > 16 + 5 * 31  # chains of several chunks
    assert (lens == 0).any() or case == "pool_runs_out"
    if case == "chains":  # box queries take the same path
        qb = np.ascontiguousarray(np.stack([q - 0.008, q + 0.008], axis=1))
        off_b, idx_b = ax.arborx_query_intersects(t, dev(qb))
        o_off, o_idx = oracle.intersects(data, qb)
        assert np.array_equal(host(off_b), o_off) and np.array_equal(host(idx_b), o_idx)
        assert np.diff(o_off).max() > 16 + 5 * 31


def check_spatial_unsorted(tree, data, q, r, dim=3, kind=oracle.POINTS, boxes=False):
    """The unsorted storage form: offsets exact, each row the oracle's set (compared sorted)."""
    if boxes:
        off, idx = ax.arborx_query_intersects(tree, dev(q), ordered=False)
        o_off, o_idx = oracle.intersects(data, q, dim=dim, kind=kind)
    else:
        off, idx = ax.arborx_query_spatial(tree, dev(q), float(r), ordered=False)
        o_off, o_idx = oracle.spatial(data, q, r, dim=dim, kind=kind)
    off, idx = host(off), host(idx)
    assert np.array_equal(off, o_off)
    rows = np.repeat(np.arange(len(off) - 1), np.diff(off))
    order = np.lexsort((idx, rows))  # sort inside each row
    assert np.array_equal(idx[order], o_idx)
    return off, idx


@pytest.mark.parametrize("case", ["cube", "gmm6", "long_rows", "pool_runs_out", "boxes", "wave"])
def test_spatial_unsorted(case):
    # rows in the order the walk found them: same offsets and the same set per row as the
    # oracle, through the stash (16 or 32 entries), overflow chains and second walks
    g = np.random.default_rng(23)
    dim, kind, boxes, tuning = 3, oracle.POINTS, False, {}
    if case == "gmm6":
        cfg = inputs.config_gmm6(n=20_000, m=2001)
        data, q, r, dim = cfg["data"], cfg["queries"], float(cfg["radius"]), 6
    elif case in ("long_rows", "pool_runs_out", "wave"):
        hot = g.random((20, 3))
        blob = hot[g.integers(0, 20, 12000)] + 0.003 * g.standard_normal((12000, 3))
        data = np.concatenate([g.random((30000, 3)), blob]).astype(np.float32)
        near = hot[g.integers(0, 20, 60)] + 0.001 * g.standard_normal((60, 3))
        q = (near if case == "pool_runs_out" else np.concatenate([g.random((20000, 3)), near])).astype(np.float32)
        r = 0.01
        tuning = dict(schedule=1) if case == "wave" else {}
    elif case == "boxes":
        data = g.random((20000, 3)).astype(np.float32)
        c = g.random((3001, 3)).astype(np.float32)
        q = np.ascontiguousarray(np.stack([c - 0.02, c + 0.02], axis=1)).astype(np.float32)
        r, boxes = 0.0, True
    else:
        cfg = inputs.config_small(n=20_000, m=4001)
        data, q, r = cfg["data"], cfg["queries"], float(cfg["radius"])
    ax.arborx_set_tuning(**tuning)
    try:
        t = ax.arborx_bvh_build(dev(data))
        off, _ = check_spatial_unsorted(t, data, q, r, dim=dim, kind=kind, boxes=boxes)
        if case in ("long_rows", "pool_runs_out"):
            assert np.diff(off).max() > 4096 or np.diff(off).max() > 16 + 5 * 31
        if case == "cube":  # r = 0 and an empty query set
            check_spatial_unsorted(t, data, q, 0.0)
            check_spatial_unsorted(t, data, q[:0], r)
    finally:
        ax.arborx_reset_tuning()


def test_spatial_unsorted_plans():
    # a plan begun with distances gives its indices unsorted (no distances); an ordered ray plan refuses
    import ctypes
    cfg = inputs.config_small(n=5000, m=500)
    data, q, r = cfg["data"], cfg["queries"], float(cfg["radius"])
    t = ax.arborx_bvh_build(dev(data))
    L = ax._lib.lib()
    qd = dev(q)
    off = torch.empty(len(q) + 1, dtype=torch.int64, device="cuda")
    total, plan = ctypes.c_int64(), ctypes.c_void_p()
    assert L.arborx_query_spatial_with_distances_begin(t.handle, ctypes.c_void_p(qd.data_ptr()), len(q),
                                                       ctypes.c_float(r), ctypes.c_void_p(off.data_ptr()),
                                                       ctypes.byref(total), ctypes.byref(plan), None) == ax.OK
    try:
        idx = torch.empty(max(total.value, 1), dtype=torch.int32, device="cuda")
        assert L.arborx_query_finish_unsorted(plan, ctypes.c_void_p(idx.data_ptr()), 0) == ax.E_CAPACITY
        assert L.arborx_query_finish_unsorted(plan, ctypes.c_void_p(idx.data_ptr()), idx.numel()) == ax.OK
        o_off, o_idx = oracle.spatial(data, q, r)
        h = host(idx)[:total.value]
        rows = np.repeat(np.arange(len(q)), np.diff(o_off))
        assert np.array_equal(host(off), o_off) and np.array_equal(h[np.lexsort((h, rows))], o_idx)
    finally:
        L.arborx_plan_destroy(plan)
    g = np.random.default_rng(5)
    rays = np.ascontiguousarray(np.stack([g.random((50, 3)), g.standard_normal((50, 3))], axis=1)).astype(np.float32)
    rd = dev(rays)
    off = torch.empty(51, dtype=torch.int64, device="cuda")
    assert L.arborx_query_ray_ordered_intersect_begin(t.handle, ctypes.c_void_p(rd.data_ptr()), 50,
                                                      ctypes.c_void_p(off.data_ptr()), ctypes.byref(total),
                                                      ctypes.byref(plan), None) == ax.OK
    try:
        idx = torch.empty(max(total.value, 1), dtype=torch.int32, device="cuda")
        assert L.arborx_query_finish_unsorted(plan, ctypes.c_void_p(idx.data_ptr()), idx.numel()) == ax.E_INVALID
    finally:
        L.arborx_plan_destroy(plan)


@pytest.mark.parametrize("k", [1, 16, 64])
def test_knn_seeding_off_identical(k):
    s = inputs.config_paper("shell", n=30_000, m=3000)
    t = ax.arborx_bvh_build(dev(s["data"]))
    check_knn(t, s["data"], s["queries"], k)
    for kw in (dict(seed_mode=1), dict(seed_mode=2), dict(schedule=1), dict(schedule=1, seed_mode=1),
               dict(schedule=1, seed_mode=2), dict(schedule=2), dict(node_format=1),
               dict(node_format=1, seed_mode=1), dict(node_format=1, seed_mode=2), dict(node_format=2),
               dict(node_format=2, seed_mode=1), dict(node_format=2, seed_mode=2)):
        ax.arborx_set_tuning(**kw)
        try:
            if "node_format" in kw:  # the format is stored when the tree is built
                t = ax.arborx_bvh_build(dev(s["data"]))
            check_knn(t, s["data"], s["queries"], k)
            check_spatial(t, s["data"], s["queries"], 0.01)
        finally:
            ax.arborx_reset_tuning()


def _both_node_forms(build, fn):
    for fmt in (0, 1, 2):
        ax.arborx_set_tuning(node_format=fmt)
        try:
            fn(build())
        finally:
            ax.arborx_reset_tuning()


@pytest.mark.parametrize("case", ["huge_extent", "denormal_extent", "offset_tiny_extent", "flat_dimension"])
def test_quantized_frames(case):
    # frames where 16-bit codes collapse, the extent leaves the float range or
    # the step underflows: decoded child boxes must still contain the true ones
    g = np.random.default_rng(11)
    x = g.random((6000, 3))
    y = g.random((500, 3))
    if case == "huge_extent":
        data, q, r = (x * 4e37 - 2e37).astype(np.float32), (y * 4e37 - 2e37).astype(np.float32), 3e36
        data[0, 0], data[1, 0] = np.float32(-3.3e38), np.float32(3.3e38)
    elif case == "denormal_extent":
        data, q, r = (x * 1e-39).astype(np.float32), (y * 1e-39).astype(np.float32), 0.0
    elif case == "offset_tiny_extent":
        data, q, r = (1e6 + x * 2e-2).astype(np.float32), (1e6 + y * 2e-2).astype(np.float32), 2e-3
    else:
        x[:, 2] = 0.25
        y[:, 2] = 0.25
        data, q, r = x.astype(np.float32), y.astype(np.float32), 0.02
    def run(t):
        check_spatial(t, data, q, r)
        check_knn(t, data, q, 9)
        check_reduce(t, data, q, r, sums=case != "huge_extent")
    _both_node_forms(lambda: ax.arborx_bvh_build(dev(data)), run)


def test_quantized_boxes_and_dims():
    g = np.random.default_rng(12)
    for dim in (2, 6):
        data = g.random((7000, dim)).astype(np.float32)
        q = g.random((400, dim)).astype(np.float32)
        r = 0.03 if dim == 2 else 0.3

        def run(t):
            check_spatial(t, data, q, r, dim=dim)
            check_knn(t, data, q, 5, dim=dim)
        _both_node_forms(lambda: ax.arborx_bvh_build(dev(data)), run)
    lo = g.random((5000, 3)).astype(np.float32)
    boxes = np.ascontiguousarray(np.stack([lo, lo + (0.02 * g.random((5000, 3))).astype(np.float32)], axis=1))
    q = g.random((300, 3)).astype(np.float32)
    def run_boxes(t):
        check_spatial(t, boxes, q, 0.01, kind=oracle.BOXES)
        check_knn(t, boxes, q, 6, kind=oracle.BOXES)
    _both_node_forms(lambda: ax.arborx_bvh_build(dev(boxes), kind=ax.BOXES), run_boxes)


@pytest.mark.parametrize("fmt", [1, 2])
def test_node_format_request_needs_that_build(fmt):
    cfg = inputs.config_small(n=3000, m=200)
    ax.arborx_set_tuning(node_format=0)  # a tree with float nodes only
    try:
        t = ax.arborx_bvh_build(dev(cfg["data"]))
    finally:
        ax.arborx_reset_tuning()
    # the library's defaults walk quantized nodes where a tree has them, float nodes where it has not
    check_spatial(t, cfg["data"], cfg["queries"], 0.05)
    check_reduce(t, cfg["data"], cfg["queries"], 0.05)
    check_knn(t, cfg["data"], cfg["queries"], 4)
    ax.arborx_set_tuning(node_format=fmt)
    try:
        with pytest.raises(ax.ArborXError, match="built without"):
            ax.arborx_query_knn(t, dev(cfg["queries"]), 4)
        with pytest.raises(ax.ArborXError, match="built without"):
            ax.arborx_query_spatial_reduce(t, dev(cfg["queries"]), 0.05, ax.COUNT)
        t2 = ax.arborx_bvh_build(dev(cfg["data"]))
        check_knn(t2, cfg["data"], cfg["queries"], 4)
    finally:
        ax.arborx_reset_tuning()
    check_knn(t2, cfg["data"], cfg["queries"], 4)  # float nodes are always there


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 7, 64, 65, 1000])
def test_four_wide_small_trees_and_duplicates(n):
    g = np.random.default_rng(100 + n)
    data = g.random((n, 3)).astype(np.float32)
    data[n // 2:] = data[0]  # duplicates
    q = np.concatenate([data[:3], g.random((200, 3)).astype(np.float32)])
    ax.arborx_set_tuning(node_format=2)
    try:
        t = ax.arborx_bvh_build(dev(data))
        for r in (0.0, 0.3, float("inf")):
            check_spatial(t, data, q, r)
        check_knn(t, data, q, min(5, n))
        check_knn(t, data, q, 9)
        check_reduce(t, data, q, 0.3)
    finally:
        ax.arborx_reset_tuning()


@pytest.mark.parametrize("case", ["cube", "clusters", "boxes_tree", "dim6", "tuned"])
def test_count_up_to(case):
    g = np.random.default_rng(31)
    kind, dim = oracle.POINTS, 3
    if case == "clusters":  # rows from 0 to several hundred matches
        hot = g.random((20, 3))
        data = np.concatenate([g.random((20000, 3)), hot[g.integers(0, 20, 8000)] + 0.003 * g.standard_normal((8000, 3))])
        data = data.astype(np.float32)
        q = np.concatenate([g.random((3000, 3)), hot[g.integers(0, 20, 200)]]).astype(np.float32)
        r = 0.01
    elif case == "boxes_tree":
        c = g.random((6000, 3)).astype(np.float32)
        h = (g.random((6000, 3)) * 0.01).astype(np.float32)
        data = np.ascontiguousarray(np.stack([c - h, c + h], axis=1))
        q, r, kind = g.random((2001, 3)).astype(np.float32), 0.03, oracle.BOXES
    elif case == "dim6":
        cfg = inputs.config_gmm6(n=20_000, m=2001)
        data, q, r, dim = cfg["data"], cfg["queries"], float(cfg["radius"]), 6
    else:
        cfg = inputs.config_small(n=20_000, m=4001)
        data, q, r = cfg["data"], cfg["queries"], float(cfg["radius"])
    if case == "tuned":
        ax.arborx_set_tuning(block=64, stack=2, order=0)
    try:
        t = ax.arborx_bvh_build(dev(data), ax.BOXES if kind == oracle.BOXES else ax.POINTS)
        full, _ = oracle.reduce(data, q, r, op=oracle.COUNT, dim=dim, kind=kind)
        for n_max in (0, 1, 2, 7, 16, 100, 2 ** 31 - 1):
            got = host(ax.arborx_query_spatial_count_up_to(t, dev(q), r, n_max))
            assert np.array_equal(got, oracle.count_up_to(data, q, r, n_max, dim=dim, kind=kind)), n_max
            assert np.array_equal(got, np.minimum(full, n_max))
        got = host(ax.arborx_query_spatial_count_up_to(t, dev(q), float("inf"), 50))
        assert np.all(got == min(50, len(data)))
    finally:
        ax.arborx_reset_tuning()
    e = ax.arborx_bvh_build(dev(np.zeros((0, dim), dtype=np.float32)))
    assert np.all(host(ax.arborx_query_spatial_count_up_to(e, dev(q[:, :dim] if q.ndim == 2 else q), 1.0, 3)) == 0)


@pytest.mark.parametrize("case", ["cube", "boxes", "dim6", "long_rows"])
def test_match_distances(case):
    g = np.random.default_rng(41)
    kind, dim = oracle.POINTS, 3
    if case == "boxes":
        c = g.random((6000, 3)).astype(np.float32)
        h = (g.random((6000, 3)) * 0.01).astype(np.float32)
        data = np.ascontiguousarray(np.stack([c - h, c + h], axis=1))
        q, r, kind = g.random((2001, 3)).astype(np.float32), 0.03, oracle.BOXES
    elif case == "dim6":
        cfg = inputs.config_gmm6(n=20_000, m=2001)
        data, q, r, dim = cfg["data"], cfg["queries"], float(cfg["radius"]), 6
    elif case == "long_rows":
        data, q, r = g.random((9000, 3)).astype(np.float32), g.random((50, 3)).astype(np.float32), 0.4
    else:
        cfg = inputs.config_small(n=20_000, m=4001)
        data, q, r = cfg["data"], cfg["queries"], float(cfg["radius"])
    bvh = ax.BVH(dev(data), ax.BOXES if kind == oracle.BOXES else ax.POINTS)
    off, idx, d2 = bvh.spatial_with_distances(dev(q), r)
    o_off, o_idx = oracle.spatial(data, q, r, dim=dim, kind=kind)
    assert np.array_equal(host(off), o_off) and np.array_equal(host(idx), o_idx)
    want = oracle.match_distances(data, q, o_off, o_idx, dim=dim, kind=kind)
    assert np.array_equal(host(d2), want)
    assert np.all(host(d2) <= np.float32(r) * np.float32(r))
    # the gather form over the same CSR result agrees with the walk's own output
    v = dev(data)
    assert np.array_equal(host(ax.arborx_query_match_distances(bvh.tree, v, dev(q), off, idx)), want)
    # every schedule and packet width of the count walk gives the same output
    for kw in (dict(schedule=1), dict(schedule=2), dict(queries_per_thread=1), dict(queries_per_thread=4)):
        ax.arborx_set_tuning(**kw)
        try:
            check_spatial_dist(bvh.tree, data, q, r, dim=dim, kind=kind)
        finally:
            ax.arborx_reset_tuning()


def _deepest_tree_points():
    """A comb with one split at every Morton code bit (cell coordinate 2^j in one
    dimension, 0 in the others, j = 0..20, bounds [0, 1]) above 2^14 copies of the
    origin (a position subtree of depth 14): about 78 levels, close to the deepest
    tree the build can make, where walks defer the most subtrees."""
    pts = [np.zeros(3)] * (1 << 14) + [np.ones(3)]
    for d in range(3):
        for j in range(21):
            p = np.zeros(3)
            p[d] = 2.0 ** (j - 21)
            pts.append(p)
    return np.array(pts, dtype=np.float32)


@pytest.mark.parametrize("tuning", [dict(stack=1), dict(stack=1, node_format=2), dict(stack=1, node_format=1),
                                    dict(stack=1, schedule=1), dict(stack=1, schedule=2),
                                    dict(stack=1, queries_per_thread=4)])
def test_deepest_tree_one_entry_ring(tuning):
    data = _deepest_tree_points()
    g = np.random.default_rng(77)
    q = np.concatenate([data[-70:], g.random((30, 3))]).astype(np.float32)
    ax.arborx_set_tuning(**tuning)
    try:
        t = ax.arborx_bvh_build(dev(data))
        h = ax.arborx_bvh_info(t)["height"]
        assert 70 <= h <= 95
        for r in (float("inf"), 2.0 ** -20, 0.0):  # every value deferred and found again at r = inf
            check_spatial(t, data, q, r)
            check_reduce(t, data, q, r)
            for n_max in (1, 40):  # the early-terminating walk stops with deferred subtrees left
                got = host(ax.arborx_query_spatial_count_up_to(t, dev(q), r, n_max))
                assert np.array_equal(got, oracle.count_up_to(data, q, r, n_max))
        check_knn(t, data, q, 64)
        check_knn(t, data, q, 3)
    finally:
        ax.arborx_reset_tuning()


def test_node_visit_statistics():
    # an infinite radius visits every internal node exactly once; kNN visits at least the root
    cfg = inputs.config_small(n=5000, m=300)
    t = ax.arborx_bvh_build(dev(cfg["data"]))
    v = host(ax.arborx_debug_node_visits(t, dev(cfg["queries"]), radius=float("inf")))
    assert np.all(v == 4999)
    v = host(ax.arborx_debug_node_visits(t, dev(cfg["queries"]), radius=float(cfg["radius"])))
    assert np.all(v >= 1) and v.mean() < 200
    vk = host(ax.arborx_debug_node_visits(t, dev(cfg["queries"]), k=10))
    assert np.all(vk >= 1) and np.all(vk <= 4999)


def test_with_distances_edge_cases():
    empty = ax.arborx_bvh_build(dev(np.zeros((0, 3), dtype=np.float32)))
    q = np.random.default_rng(3).random((20, 3)).astype(np.float32)
    off, idx, d2 = ax.arborx_query_spatial_with_distances(empty, dev(q), 0.5)
    assert np.all(host(off) == 0) and idx.numel() == 0 and d2.numel() == 0
    data = np.concatenate([q[:5], q[:5], np.random.default_rng(4).random((200, 3))]).astype(np.float32)
    t = ax.arborx_bvh_build(dev(data))
    check_spatial_dist(t, data, q, 0.0)  # exact duplicates only, at distance 0
    off, idx, d2 = ax.arborx_query_spatial_with_distances(t, dev(q[:0]), 0.1)
    assert off.numel() == 1 and idx.numel() == 0
