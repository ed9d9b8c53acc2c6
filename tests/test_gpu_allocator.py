"""Device memory from a caller's allocator (PyTorch's caching allocator): same
results as the library's own pool, memory accounted by torch while a tree lives
and handed back in full once it is destroyed."""
import gc

import numpy as np
import pytest

import oracle
import paper_2507_23700_amd as ax
from paper_2507_23700_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    gc.collect()
    torch.cuda.synchronize()
    yield
    gc.collect()
    torch.cuda.synchronize()
    ax.arborx_set_allocator()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    return t.cpu().numpy()


def run_all(tree, q, r, k, stream=None):
    off, idx = ax.arborx_query_spatial(tree, q, r, stream=stream)
    c, s = ax.arborx_query_spatial_reduce(tree, q, r, ax.COUNT_SUMDIST, stream=stream)
    d2, ix = ax.arborx_query_knn(tree, q, k, stream=stream)
    return [off, idx, c, s, d2, ix]


def same(got, expect):
    return all(np.array_equal(host(g), e) for g, e in zip(got, expect))


def test_torch_allocator_results_and_accounting():
    cfg = inputs.config_small(n=20_000, m=3001)
    data, q, r = cfg["data"], cfg["queries"], float(cfg["radius"])
    d, qd = dev(data), dev(q)
    o_off, o_idx = oracle.spatial(data, q, r)
    oc, os_ = oracle.reduce(data, q, r)
    od2, oix = oracle.knn(data, q, 10)
    expect = [o_off, o_idx, oc, os_, od2, oix]

    ax.use_torch_allocator()
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    t = ax.arborx_bvh_build(d)
    torch.cuda.synchronize()
    held = torch.cuda.memory_allocated() - base
    assert held >= 20_000 * (64 + 16)  # nodes and leaves at least, now in torch's pool
    out = run_all(t, qd, r, 10)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        out2 = run_all(t, qd, r, 10, stream=side)
    side.synchronize()
    torch.cuda.synchronize()
    assert same(out, expect) and same(out2, expect)
    del out, out2, t
    gc.collect()
    ax.arborx_set_allocator()  # waits for blocks that the side stream used, then hands them back
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == base


def test_allocator_change_needs_no_live_structures():
    d = dev(np.random.default_rng(0).random((500, 3), dtype=np.float32))
    t = ax.arborx_bvh_build(d)
    with pytest.raises(ax.ArborXError) as e:
        ax.use_torch_allocator()
    assert e.value.status == ax.E_INVALID
    del t
    gc.collect()
    ax.use_torch_allocator()
    t = ax.arborx_bvh_build(d)
    with pytest.raises(ax.ArborXError):
        ax.arborx_set_allocator()
    del t
    gc.collect()
    ax.arborx_set_allocator()


def test_failing_allocator_reports_nomem_and_leaks_nothing():
    d = dev(np.random.default_rng(1).random((5000, 3), dtype=np.float32))
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    calls = {"alloc": 0, "free": 0}
    dev_index = torch.cuda.current_device()

    def alloc(n, s):
        calls["alloc"] += 1
        if calls["alloc"] > 3:  # the first few blocks of the build succeed, then memory "runs out"
            return 0
        return torch.cuda.caching_allocator_alloc(n, dev_index, s)

    def free(p, s):
        calls["free"] += 1
        torch.cuda.caching_allocator_delete(p)

    ax.arborx_set_allocator(alloc, free)
    with pytest.raises(ax.ArborXError) as e:
        ax.arborx_bvh_build(d)
    assert e.value.status == ax.E_NOMEM
    gc.collect()
    ax.arborx_set_allocator()  # nothing of the failed build is still held
    torch.cuda.synchronize()
    assert calls["free"] == 3
    assert torch.cuda.memory_allocated() == base


def test_torch_allocator_forest_and_chamfer():
    g = np.random.default_rng(2)
    sizes = [700, 0, 1200, 5]
    vals = np.ascontiguousarray(np.concatenate([inputs.cube(s, 3, g) for s in sizes]))
    toff = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    bsz = [300, 50, 0, 90]
    qs = np.ascontiguousarray(np.concatenate([inputs.cube(s, 3, g) for s in bsz]))
    boff = np.concatenate([[0], np.cumsum(bsz)]).astype(np.int64)
    btree = np.array([0, 2, 1, 3], dtype=np.int32)
    brad = np.full(4, 0.07, dtype=np.float32)
    oc, os_ = oracle.forest_reduce(vals, toff, qs, boff, btree, brad)
    od2, oix = oracle.forest_knn(vals, toff, qs, boff, btree, 4)
    ax.use_torch_allocator()
    f = ax.arborx_forest_build(dev(vals), toff)
    c, s = ax.arborx_forest_query_reduce(f, dev(qs), dev(boff), dev(btree), dev(brad), ax.COUNT_SUMDIST)
    d2, ix = ax.arborx_forest_query_knn(f, dev(qs), dev(boff), dev(btree), 4)
    assert np.array_equal(host(c), oc) and np.array_equal(host(s), os_)
    assert np.array_equal(host(d2), od2) and np.array_equal(host(ix), oix)
    c2, s2 = f.reduce(dev(qs), dev(boff), dev(btree), dev(brad))  # the handle's convenience methods
    d22, ix2 = f.knn(dev(qs), dev(boff), dev(btree), 4)
    assert np.array_equal(host(c2), oc) and np.array_equal(host(s2), os_) and np.array_equal(host(ix2), oix)
    assert f.info()["T"] == 4
    a = dev(inputs.cube(900, 3, g))
    b = dev(inputs.cube(1100, 3, g))
    a_off = np.array([0, 400, 900], dtype=np.int64)
    b_off = np.array([0, 600, 1100], dtype=np.int64)
    loss, nn_ab, nn_ba = ax.arborx_chamfer_forward(a, a_off, b, b_off)
    o_loss, o_ab, o_ba = oracle.chamfer_forward(host(a), a_off, host(b), b_off)
    assert np.array_equal(host(nn_ab), o_ab) and np.array_equal(host(nn_ba), o_ba)
    np.testing.assert_allclose(host(loss), o_loss, rtol=1e-6)
    del f
    gc.collect()
