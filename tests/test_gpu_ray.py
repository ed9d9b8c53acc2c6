"""Ray predicates over the hierarchy (hit count; first k hits by entry
parameter) against the brute-force oracle, bit for bit."""
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
    return c


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
