"""Ray predicates over the hierarchy (hit count; first k hits by entry
parameter; all hits, ascending or in the order met, with entry parameters)
against the brute-force oracle, bit for bit."""
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


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def random_boxes(n, dim, g, size=0.05):
    c = g.random((n, dim)).astype(np.float32)
    h = (g.random((n, dim)) * size + 0.002).astype(np.float32)
    return np.ascontiguousarray(np.stack([c - h, c + h], axis=1))


def random_rays(m, dim, g, axis_share=0.2):
    o = (g.random((m, dim)) * 1.4 - 0.2).astype(np.float32)
    d = g.standard_normal((m, dim)).astype(np.float32)
    d[g.random((m, dim)) < axis_share] = 0.0  # rays parallel to some axes
    d[np.all(d == 0, axis=1), 0] = 1.0
    return np.ascontiguousarray(np.stack([o, d], axis=1))


def check(values, rays, k, dim, kind):
    t = ax.arborx_bvh_build(dev(values), ax.BOXES if kind == oracle.BOXES else ax.POINTS)
    c = ax.arborx_query_ray_count(t, dev(rays)).cpu().numpy()
    assert np.array_equal(c, oracle.ray_count(values, rays, dim=dim, kind=kind))
    te, ix = ax.arborx_query_ray_nearest(t, dev(rays), k)
    o_t, o_ix = oracle.ray_nearest(values, rays, k, dim=dim, kind=kind)
    assert np.array_equal(ix.cpu().numpy(), o_ix) and np.array_equal(te.cpu().numpy(), o_t)
    check_all_hits(t, values, rays, dim, kind)
    return c


def check_all_hits(tree, values, rays, dim, kind):
    off, idx = ax.arborx_query_ray_intersect(tree, dev(rays))
    o_off, o_idx = oracle.ray_intersect(values, rays, dim=dim, kind=kind)
    assert np.array_equal(off.cpu().numpy(), o_off) and np.array_equal(idx.cpu().numpy(), o_idx)
    off2, idx2, te = ax.arborx_query_ray_ordered_intersect(tree, dev(rays))
    o_off2, o_idx2, o_t = oracle.ray_ordered_intersect(values, rays, dim=dim, kind=kind)
    assert np.array_equal(off2.cpu().numpy(), o_off2) and np.array_equal(idx2.cpu().numpy(), o_idx2)
    assert np.array_equal(te.cpu().numpy(), o_t)
    return o_off


@pytest.mark.parametrize("k", [1, 3, 16, 40])
def test_boxes_3d(k):
    g = np.random.default_rng(k)
    c = check(random_boxes(8000, 3, g), random_rays(3001, 3, g), k, 3, oracle.BOXES)
    assert c.max() > k and (c == 0).any()


@pytest.mark.parametrize("dim", [2, 6])
def test_other_dims(dim):
    g = np.random.default_rng(dim)
    check(random_boxes(5000, dim, g, 0.08), random_rays(1501, dim, g), 8, dim, oracle.BOXES)


def test_hand_worked_and_ties():
    boxes = np.array([[[i, 0, 0], [i + 1, 1, 1]] for i in range(5)], dtype=np.float32)
    rays = np.array([[(-1, 0.5, 0.5), (1, 0, 0)], [(2.5, 0.5, 0.5), (2, 0, 0)], [(1, 0.5, -1), (0, 0, 1)],
                     [(-1, 0.5, 0.5), (-1, 0, 0)], [(0.5, 2, -1), (0, 0, 1)]], dtype=np.float32)
    c = check(boxes, rays, 3, 3, oracle.BOXES)
    assert list(c) == [5, 3, 2, 0, 0]
    dup = np.repeat(random_boxes(300, 3, np.random.default_rng(5)), 3, axis=0)  # equal entry parameters
    check(dup, random_rays(400, 3, np.random.default_rng(6)), 10, 3, oracle.BOXES)


def test_points_and_empty():
    pts = np.array([[0, 0, 0], [1, 0, 0], [1, 1, 0], [3, 0, 0]], dtype=np.float32)
    rays = np.array([[(-2, 0, 0), (0.5, 0, 0)], [(1, 1, 5), (0, 0, -1)]], dtype=np.float32)
    c = check(pts, rays, 4, 3, oracle.POINTS)
    assert list(c) == [3, 1]
    e = ax.arborx_bvh_build(dev(np.zeros((0, 3), dtype=np.float32)))
    te, ix = ax.arborx_query_ray_nearest(e, dev(rays), 2)
    assert np.all(ix.cpu().numpy() == -1) and np.all(np.isinf(te.cpu().numpy()))
    assert np.all(ax.arborx_query_ray_count(e, dev(rays)).cpu().numpy() == 0)


@pytest.mark.parametrize("tuning", [dict(schedule=1), dict(schedule=2), dict(node_format=1), dict(node_format=2),
                                    dict(block=64, stack=1, order=0)])
def test_all_hits_every_schedule(tuning):
    g = np.random.default_rng(71)
    boxes, rays = random_boxes(6000, 3, g, 0.06), random_rays(1200, 3, g)
    ax.arborx_set_tuning(**tuning)
    try:
        t = ax.arborx_bvh_build(dev(boxes), ax.BOXES)
        check_all_hits(t, boxes, rays, 3, oracle.BOXES)
    finally:
        ax.arborx_reset_tuning()


def test_all_hits_long_rows():
    # big overlapping boxes: rows past the register stash, the overflow chunks, the wavefront and
    # workgroup sorts, and past the workgroup sort (radix path, ordered by entry parameter in two passes)
    g = np.random.default_rng(72)
    c = g.random((9000, 3)).astype(np.float32)
    h = (g.random((9000, 3)) * 0.3 + 0.2).astype(np.float32)
    boxes = np.ascontiguousarray(np.stack([c - h, c + h], axis=1))
    rays = np.concatenate([random_rays(300, 3, g), random_rays(20, 3, g, axis_share=0.0)])
    t = ax.arborx_bvh_build(dev(boxes), ax.BOXES)
    lens = np.diff(check_all_hits(t, boxes, rays, 3, oracle.BOXES))
    # box sizes spread over two decades: rows from a few to about a thousand hits
    h2 = (np.exp(g.uniform(np.log(0.005), np.log(0.5), (9000, 1))) * (0.5 + g.random((9000, 3)))).astype(np.float32)
    boxes2 = np.ascontiguousarray(np.stack([c - h2, c + h2], axis=1))
    t2 = ax.arborx_bvh_build(dev(boxes2), ax.BOXES)
    lens = np.concatenate([lens, np.diff(check_all_hits(t2, boxes2, rays, 3, oracle.BOXES))])
    assert lens.max() > 4096 and ((lens > 16) & (lens <= 64)).any() and ((lens > 64) & (lens <= 4096)).any()


def test_all_hits_empty_tree_and_no_rays():
    e = ax.arborx_bvh_build(dev(np.zeros((0, 3), dtype=np.float32)))
    rays = random_rays(5, 3, np.random.default_rng(1))
    off, idx = ax.arborx_query_ray_intersect(e, dev(rays))
    assert np.all(off.cpu().numpy() == 0) and idx.numel() == 0
    off, idx, te = ax.arborx_query_ray_ordered_intersect(e, dev(rays))
    assert np.all(off.cpu().numpy() == 0) and te.numel() == 0
    t = ax.arborx_bvh_build(dev(random_boxes(50, 3, np.random.default_rng(2))), ax.BOXES)
    off, idx, te = ax.arborx_query_ray_ordered_intersect(t, dev(np.zeros((0, 2, 3), dtype=np.float32)))
    assert off.numel() == 1 and off.item() == 0
