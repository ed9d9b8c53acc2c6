"""Pair search (the self-join of a tree's points, each pair met once by a walk
over the later leaves) and DBSCAN built on it (core points from the pair
counts, clusters by a lock-free union-find, border points to their
smallest-index core neighbour), against the brute-force definitions in the
oracle, element by element."""
import numpy as np
import pytest

import oracle
import paper_2507_23700_amd as ax

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ax.arborx_reset_tuning()
    yield
    ax.arborx_reset_tuning()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def clustered(n, dim, seed, noise=0.15):
    g = np.random.default_rng(seed)
    k = max(2, n // 150)
    centres = g.random((k, dim)) * 10
    m = int(n * (1 - noise))
    pts = np.concatenate([centres[g.integers(0, k, m)] + 0.25 * g.standard_normal((m, dim)),
                          g.random((n - m, dim)) * 10])
    return np.ascontiguousarray(pts.astype(np.float32))


def check(pts, eps, min_pts):
    bvh = ax.BVH(dev(pts))
    got = bvh.dbscan(eps, min_pts).cpu().numpy()
    want = oracle.dbscan(pts, eps, min_pts, dim=pts.shape[1])
    assert np.array_equal(got, want), (eps, min_pts)
    return got


def test_hand_worked_line():
    pts = np.array([[0, 0, 0], [1, 0, 0], [2, 0, 0], [10, 0, 0], [11, 0, 0], [20, 0, 0]], dtype=np.float32)
    assert list(check(pts, 1.5, 2)) == [0, 0, 0, 3, 3, -1]
    assert list(check(pts, 1.5, 3)) == [1, 1, 1, -1, -1, -1]
    assert list(check(pts, 1.5, 1)) == [0, 0, 0, 3, 3, 5]


@pytest.mark.parametrize("eps,min_pts", [(0.3, 6), (0.3, 1), (0.2, 10), (0.6, 4), (100.0, 5), (0.0, 2)])
def test_clustered_3d(eps, min_pts):
    pts = clustered(6000, 3, 1)
    pts[::97] = pts[1::97][: len(pts[::97])]  # exact duplicates: eps = 0 still links them
    lab = check(pts, eps, min_pts)
    if eps == 100.0:
        assert np.all(lab == 0)


@pytest.mark.parametrize("dim", [2, 6])
def test_other_dims(dim):
    check(clustered(5000, dim, 2 + dim), 0.35 if dim == 2 else 0.6, 5)


def test_large_and_tuned():
    pts = clustered(40_000, 3, 7)
    check(pts, 0.15, 8)
    ax.arborx_set_tuning(block=64, stack=2, order=0)
    check(pts, 0.15, 8)


def test_empty_and_tiny():
    e = ax.BVH(dev(np.zeros((0, 3), dtype=np.float32)))
    assert e.dbscan(1.0, 2).numel() == 0
    one = np.array([[0.5, 0.5, 0.5]], dtype=np.float32)
    assert list(check(one, 1.0, 1)) == [0] and list(check(one, 1.0, 2)) == [-1]


def test_rejects_box_trees():
    boxes = np.zeros((4, 2, 3), dtype=np.float32)
    t = ax.arborx_bvh_build(dev(boxes), ax.BOXES)
    with pytest.raises(ValueError):
        ax.arborx_dbscan(t, dev(np.zeros((4, 3), dtype=np.float32)), 1.0, 2)


def check_degree(pts, r):
    bvh = ax.BVH(dev(pts))
    got = ax.arborx_self_join_degree(bvh.tree, r).cpu().numpy()
    want = oracle.self_join_degree(pts, r, dim=pts.shape[1])
    assert np.array_equal(got, want), r
    return got


def test_self_join_hand_worked():
    pts = np.array([[0, 0, 0], [1, 0, 0], [2, 0, 0], [10, 0, 0], [11, 0, 0], [20, 0, 0]], dtype=np.float32)
    assert list(check_degree(pts, 1.5)) == [1, 2, 1, 1, 1, 0]
    assert list(check_degree(pts, 1.0)) == [1, 2, 1, 1, 1, 0]
    assert list(check_degree(pts, float(np.nextafter(np.float32(1), np.float32(0))))) == [0] * 6
    assert list(check_degree(pts, float("inf"))) == [5] * 6


@pytest.mark.parametrize("dim,r", [(2, 0.3), (3, 0.25), (3, 0.0), (3, 3.0), (6, 0.5)])
def test_self_join_clustered(dim, r):
    pts = clustered(7000, dim, 30 + dim)
    pts[::89] = pts[1::89][: len(pts[::89])]  # exact duplicates pair at r = 0
    deg = check_degree(pts, r)
    assert deg.sum() % 2 == 0


@pytest.mark.parametrize("n", [0, 1, 2, 3, 64, 65, 1000])
def test_self_join_small_trees(n):
    g = np.random.default_rng(n)
    pts = g.random((n, 3)).astype(np.float32)
    pts[n // 2:] = pts[:n - n // 2]
    if n == 0:
        bvh = ax.BVH(dev(pts))
        assert ax.arborx_self_join_degree(bvh.tree, 1.0).numel() == 0
        return
    for r in (0.0, 0.2, float("inf")):
        check_degree(pts, r)


def test_self_join_uniform_cube_matches_count():
    g = np.random.default_rng(5)
    pts = g.random((60_000, 3)).astype(np.float32)
    r = 0.02
    bvh = ax.BVH(dev(pts))
    deg = ax.arborx_self_join_degree(bvh.tree, r)
    c, _ = ax.arborx_query_spatial_reduce(bvh.tree, dev(pts), r, ax.COUNT)
    assert torch.equal(deg + 1, c)  # a point's partners are its radius matches without itself
    sample = g.choice(len(pts), 3000, replace=False)
    want = oracle.spatial_count(pts, pts[sample], r) - 1
    assert np.array_equal(deg.cpu().numpy()[sample], want)


def test_self_join_rejects_boxes_and_bad_radius():
    boxes = np.zeros((4, 2, 3), dtype=np.float32)
    t = ax.arborx_bvh_build(dev(boxes), ax.BOXES)
    with pytest.raises(ValueError):
        ax.arborx_self_join_degree(t, 1.0)
    p = ax.arborx_bvh_build(dev(np.zeros((4, 3), dtype=np.float32)))
    with pytest.raises(ax.ArborXError):
        ax.arborx_self_join_degree(p, float("nan"))


@pytest.mark.parametrize("tuning", [dict(schedule=2), dict(queries_per_thread=1), dict(queries_per_thread=2),
                                    dict(queries_per_thread=4), dict(block=64, stack=1),
                                    dict(queries_per_thread=1, node_format=1),
                                    dict(queries_per_thread=1, node_format=1, block=64, stack=1)])
def test_pair_walk_forms_identical(tuning):
    pts = clustered(9000, 3, 61)
    pts[::53] = pts[1::53][: len(pts[::53])]
    ax.arborx_set_tuning(**tuning)
    check_degree(pts, 0.2)
    check(pts, 0.2, 6)
    check(pts, 0.35, 1)
    p6 = clustered(4000, 6, 62)
    check_degree(p6, 0.6)
    check(p6, 0.6, 5)


def test_self_join_line_closed_form():
    # n points spaced 1 apart on a line: at r = 1.5 the ends pair once and every other point twice
    n = 5000
    pts = np.zeros((n, 3), dtype=np.float32)
    pts[:, 0] = np.arange(n, dtype=np.float32)
    deg = check_degree(pts, 1.5)
    assert deg[0] == 1 and deg[-1] == 1 and np.all(deg[1:-1] == 2)
    lab = check(pts, 1.5, 3)  # interior points are core, the two ends border: one cluster, smallest core index 1
    assert np.all(lab == 1)
