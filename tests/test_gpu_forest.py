"""Forest and Chamfer paths vs the CPU oracle and vs the single-tree path."""
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


def small_forest(seed=0):
    """Uneven trees (one empty, one single value) and batches (one empty, one aimed at the empty tree)."""
    g = np.random.default_rng(seed)
    sizes = [3000, 0, 1, 1500, 700, 5000, 2]
    vals = [inputs.cube(s, 3, g) if t % 2 == 0 else inputs.shell(s, g) for t, s in enumerate(sizes)]
    toff = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    bsizes = [400, 0, 250, 900, 30, 600, 128, 77]
    btree = np.array([0, 3, 1, 5, 2, 3, 6, 4], dtype=np.int32)
    qs = []
    for b, s in enumerate(bsizes):
        t = btree[b]
        qs.append(inputs.cube(s, 3, g) if t % 2 == 0 else inputs.shell(s, g))
    boff = np.concatenate([[0], np.cumsum(bsizes)]).astype(np.int64)
    brad = np.array([0.06 if btree[b] % 2 == 0 else 0.08 for b in range(len(bsizes))], dtype=np.float32)
    return dict(values=np.ascontiguousarray(np.concatenate(vals)), tree_offsets=toff,
                queries=np.ascontiguousarray(np.concatenate(qs)), batch_offsets=boff, batch_tree=btree,
                batch_radius=brad)


def run_forest(f, cfg, k):
    fo = ax.arborx_forest_build(dev(cfg["values"]), cfg["tree_offsets"])
    q, bo, bt, br = dev(cfg["queries"]), dev(cfg["batch_offsets"]), dev(cfg["batch_tree"]), dev(cfg["batch_radius"])
    c, s = ax.arborx_forest_query_reduce(fo, q, bo, bt, br, ax.COUNT_SUMDIST)
    c0, _ = ax.arborx_forest_query_reduce(fo, q, bo, bt, br, ax.COUNT)
    d2, ix = ax.arborx_forest_query_knn(fo, q, bo, bt, k)
    return fo, host(c), host(s), host(c0), host(d2), host(ix)


@pytest.mark.parametrize("k,tuning", [(1, {}), (8, {}), (16, {}), (1, dict(node_format=1)),
                                      (8, dict(node_format=1)), (8, dict(seed_mode=2)), (16, dict(seed_mode=1)),
                                      (1, dict(node_format=2)), (8, dict(node_format=2)),
                                      (16, dict(node_format=2, seed_mode=2)), (8, dict(queries_per_thread=1)),
                                      (1, dict(queries_per_thread=2)), (16, dict(queries_per_thread=4))])
def test_forest_vs_oracle(k, tuning):
    cfg = small_forest(k)
    ax.arborx_set_tuning(**tuning)  # before the build: it decides what is stored
    try:
        fo, c, s, c0, d2, ix = run_forest(None, cfg, k)
    finally:
        ax.arborx_reset_tuning()
    oc, os_ = oracle.forest_reduce(cfg["values"], cfg["tree_offsets"], cfg["queries"], cfg["batch_offsets"],
                                   cfg["batch_tree"], cfg["batch_radius"])
    od2, oix = oracle.forest_knn(cfg["values"], cfg["tree_offsets"], cfg["queries"], cfg["batch_offsets"],
                                 cfg["batch_tree"], k)
    assert np.array_equal(c, oc) and np.array_equal(s, os_) and np.array_equal(c0, oc)
    assert np.array_equal(ix, oix) and np.array_equal(d2, od2)
    info = ax.arborx_forest_info(fo)
    assert info["T"] == 7 and info["roots"][1] == -1 and info["heights"][2] == 1


def test_forest_equals_per_tree_path():
    cfg = inputs.forest(trees=10, tree_lo=200, tree_hi=20_000, batches=40, batch_lo=10, batch_hi=3000, cfg=50)
    k = cfg["k"]
    fo, c, s, c0, d2, ix = run_forest(None, cfg, k)
    toff, boff, bt, br = cfg["tree_offsets"], cfg["batch_offsets"], cfg["batch_tree"], cfg["batch_radius"]
    trees = [ax.arborx_bvh_build(dev(cfg["values"][toff[t]:toff[t + 1]])) for t in range(len(toff) - 1)]
    for b in range(len(bt)):
        q = dev(cfg["queries"][boff[b]:boff[b + 1]])
        pc, ps = ax.arborx_query_spatial_reduce(trees[bt[b]], q, float(br[b]), ax.COUNT_SUMDIST)
        pd, pi = ax.arborx_query_knn(trees[bt[b]], q, k)
        sl = slice(boff[b], boff[b + 1])
        assert np.array_equal(host(pc), c[sl]) and np.array_equal(host(ps), s[sl])
        assert np.array_equal(host(pi), ix[sl]) and np.array_equal(host(pd), d2[sl])
    # and a sample of batches against the oracle
    sel = list(range(0, len(bt), 7))
    oc, os_ = oracle.forest_reduce(cfg["values"], toff, cfg["queries"], boff, bt, br, batches=sel)
    od2, oix = oracle.forest_knn(cfg["values"], toff, cfg["queries"], boff, bt, k, batches=sel)
    for b in sel:
        sl = slice(boff[b], boff[b + 1])
        assert np.array_equal(c[sl], oc[sl]) and np.array_equal(s[sl], os_[sl]) and np.array_equal(ix[sl], oix[sl])


def test_forest_query_in_hip_graph():
    cfg = small_forest(3)
    fo = ax.arborx_forest_build(dev(cfg["values"]), cfg["tree_offsets"])
    q, bo, bt, br = dev(cfg["queries"]), dev(cfg["batch_offsets"]), dev(cfg["batch_tree"]), dev(cfg["batch_radius"])
    torch.cuda.synchronize()
    ref_c, ref_s = ax.arborx_forest_query_reduce(fo, q, bo, bt, br, ax.COUNT_SUMDIST)
    ref_d, ref_i = ax.arborx_forest_query_knn(fo, q, bo, bt, 8)
    ax.arborx_forest_reserve(fo, q.shape[0])
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            out = ax.arborx_forest_query_reduce(fo, q, bo, bt, br, ax.COUNT_SUMDIST, stream=s)
            outk = ax.arborx_forest_query_knn(fo, q, bo, bt, 8, stream=s)
    for rep in range(3):
        out[0].fill_(-7)
        outk[1].fill_(-7)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(host(out[0]), host(ref_c)), rep
        assert np.array_equal(host(out[1]), host(ref_s)), rep
        assert np.array_equal(host(outk[1]), host(ref_i)), rep
        assert np.array_equal(host(outk[0]), host(ref_d)), rep
        ax.arborx_forest_query_knn(fo, q, bo, bt, 4)  # eager work between replays
        torch.cuda.synchronize()


def _forest_contents(rep, n, T, m):
    """New contents of the same sizes for a replay: n values split anew into T trees (some empty,
    some of one value), and m new queries with the fixed batch layout."""
    g = np.random.default_rng(500 + rep)
    cuts = np.sort(g.integers(0, n + 1, T - 1))
    cuts[: rep % 3] = 0  # leading empty trees on some replays
    toff = np.concatenate([[0], cuts, [n]]).astype(np.int64)
    vals = inputs.cube(n, 3, g) if rep % 2 == 0 else inputs.shell(n, g)
    return np.ascontiguousarray(vals), toff, np.ascontiguousarray(inputs.cube(m, 3, g))


@pytest.mark.parametrize("tuning", [{}, dict(node_format=1), dict(node_format=2)])
def test_forest_build_and_queries_in_one_hip_graph(tuning):
    cfg = small_forest(4)
    n, T, m = len(cfg["values"]), len(cfg["tree_offsets"]) - 1, len(cfg["queries"])
    ax.arborx_set_tuning(**tuning)
    try:
        fo = ax.arborx_forest_create(n, T, 3)
        v, off = dev(cfg["values"]), dev(cfg["tree_offsets"])
        q, bo, bt, br = dev(cfg["queries"]), dev(cfg["batch_offsets"]), dev(cfg["batch_tree"]), dev(cfg["batch_radius"])
        ax.arborx_forest_reserve(fo, m)
        torch.cuda.synchronize()
        s = torch.cuda.Stream()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.stream(s):
            with torch.cuda.graph(g, stream=s):  # build, reduce and kNN: one graph, nothing allocated
                ax.arborx_forest_rebuild(fo, v, off, stream=s)
                out = ax.arborx_forest_query_reduce(fo, q, bo, bt, br, ax.COUNT_SUMDIST, stream=s)
                outk = ax.arborx_forest_query_knn(fo, q, bo, bt, 8, stream=s)
        for rep in range(4):
            vals, toff, qs = _forest_contents(rep, n, T, m)
            v.copy_(dev(vals))
            off.copy_(dev(toff))
            q.copy_(dev(qs))
            out[0].fill_(-7)
            outk[1].fill_(-7)
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            # the eager build of the same contents gives the same answers, bit for bit
            ref = ax.arborx_forest_build(dev(vals), toff)
            rc, rs = ax.arborx_forest_query_reduce(ref, dev(qs), bo, bt, br, ax.COUNT_SUMDIST)
            rd, ri = ax.arborx_forest_query_knn(ref, dev(qs), bo, bt, 8)
            torch.cuda.synchronize()
            assert np.array_equal(host(out[0]), host(rc)) and np.array_equal(host(out[1]), host(rs)), rep
            assert np.array_equal(host(outk[1]), host(ri)) and np.array_equal(host(outk[0]), host(rd)), rep
            sel = list(range(0, len(cfg["batch_tree"]), 2))
            oc, os_ = oracle.forest_reduce(vals, toff, qs, cfg["batch_offsets"], cfg["batch_tree"],
                                           cfg["batch_radius"], batches=sel)
            od2, oix = oracle.forest_knn(vals, toff, qs, cfg["batch_offsets"], cfg["batch_tree"], 8, batches=sel)
            for b in sel:
                sl = slice(cfg["batch_offsets"][b], cfg["batch_offsets"][b + 1])
                assert np.array_equal(host(out[0])[sl], oc[sl]) and np.array_equal(host(out[1])[sl], os_[sl])
                assert np.array_equal(host(outk[1])[sl], oix[sl]) and np.array_equal(host(outk[0])[sl], od2[sl])
            ax.arborx_forest_query_knn(ref, dev(qs), bo, bt, 4)  # eager work between replays
            del ref
            torch.cuda.synchronize()
        del g
    finally:
        ax.arborx_reset_tuning()


def test_forest_rebuild_sanitizes_offsets():
    # offsets that are not a valid split are made one on the device: never out of range
    cfg = small_forest(5)
    n, T = len(cfg["values"]), len(cfg["tree_offsets"]) - 1
    fo = ax.arborx_forest_create(n, T, 3)
    bad = np.array([5, -3, 2000, 1500, n + 100, 7000, 9000, 3], dtype=np.int64)
    ax.arborx_forest_rebuild(fo, dev(cfg["values"]), dev(bad))
    fixed = np.concatenate([[0], np.maximum.accumulate(np.clip(bad[1:T], 0, n)), [n]]).astype(np.int64)
    fixed[1:T] = np.maximum.accumulate(fixed[1:T])
    ref = ax.arborx_forest_build(dev(cfg["values"]), fixed)
    q, bo, bt, br = dev(cfg["queries"]), dev(cfg["batch_offsets"]), dev(cfg["batch_tree"]), dev(cfg["batch_radius"])
    a = ax.arborx_forest_query_reduce(fo, q, bo, bt, br, ax.COUNT_SUMDIST)
    b = ax.arborx_forest_query_reduce(ref, q, bo, bt, br, ax.COUNT_SUMDIST)
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])
    info = ax.arborx_forest_info(fo)
    assert info["n"] == n and info["T"] == T


def test_chamfer_forward_backward_vs_oracle():
    cfg = inputs.chamfer_pairs(pairs=12, lo=50, hi=3000, cfg=60)
    a, ao, b, bo = cfg["a"], cfg["a_off"], cfg["b"], cfg["b_off"]
    loss, nab, nba = ax.arborx_chamfer_forward(dev(a), ao, dev(b), bo)
    o_loss, o_ab, o_ba = oracle.chamfer_forward(a, ao, b, bo)
    assert np.array_equal(host(nab), o_ab) and np.array_equal(host(nba), o_ba)
    np.testing.assert_allclose(host(loss), o_loss, rtol=1e-6)
    gl = np.linspace(0.5, 2.0, 12).astype(np.float32)
    ga, gb = ax.arborx_chamfer_backward(dev(a), ao, dev(b), bo, nab, nba, dev(gl))
    oga, ogb = oracle.chamfer_backward(a, ao, b, bo, o_ab, o_ba, gl.astype(np.float64))
    ga, gb = host(ga), host(gb)
    for p in range(12):
        ref = np.concatenate([oga[ao[p]:ao[p + 1]].ravel(), ogb[bo[p]:bo[p + 1]].ravel()])
        got = np.concatenate([ga[ao[p]:ao[p + 1]].ravel(), gb[bo[p]:bo[p + 1]].ravel()])
        assert np.max(np.abs(got - ref)) <= 1e-5 * np.max(np.abs(ref))


def test_chamfer_autograd_and_finite_differences():
    cfg = inputs.chamfer_pairs(pairs=3, lo=64, hi=64, cfg=61)
    a, ao, b, bo = cfg["a"], cfg["a_off"], cfg["b"], cfg["b_off"]
    ta = dev(a).requires_grad_(True)
    tb = dev(b).requires_grad_(True)
    w = torch.tensor([1.0, -0.5, 2.0], device="cuda")
    loss = ax.chamfer(ta, ao, tb, bo)
    (loss * w).sum().backward()
    ga, gb = host(ta.grad), host(tb.grad)
    _, nab, nba = ax.arborx_chamfer_forward(dev(a), ao, dev(b), bo)
    nab, nba = host(nab), host(nba)
    h = 1e-4
    for p in range(3):
        A = a[ao[p]:ao[p + 1]].astype(np.float64)
        B = b[bo[p]:bo[p + 1]].astype(np.float64)
        n1, n2 = nab[ao[p]:ao[p + 1]], nba[bo[p]:bo[p + 1]]

        def L_fixed(A_):  # the loss with the forward pass's neighbour assignment held fixed
            return ((A_ - B[n1]) ** 2).sum() + ((B - A_[n2]) ** 2).sum()

        def L_free(A_):
            d = ((A_[:, None, :] - B[None, :, :]) ** 2).sum(-1)
            return d.min(1).sum() + d.min(0).sum(), d.argmin(1), d.argmin(0)

        d64 = ((A[:, None, :] - B[None, :, :]) ** 2).sum(-1)
        same = np.array_equal(d64.argmin(1), n1) and np.array_equal(d64.argmin(0), n2)
        fd = np.zeros_like(A)
        fd_free = np.full_like(A, np.nan)
        for i in range(len(A)):
            for d in range(3):
                Ap, Am = A.copy(), A.copy()
                Ap[i, d] += h
                Am[i, d] -= h
                fd[i, d] = float(w[p]) * (L_fixed(Ap) - L_fixed(Am)) / (2 * h)
                lp, a1p, a2p = L_free(Ap)
                lm, a1m, a2m = L_free(Am)
                # the free loss is differentiable here only if the assignment is the same at x +- h
                if same and all(np.array_equal(x, y) for x, y in ((a1p, n1), (a1m, n1), (a2p, n2), (a2m, n2))):
                    fd_free[i, d] = float(w[p]) * (lp - lm) / (2 * h)
        g = ga[ao[p]:ao[p + 1]]
        assert np.max(np.abs(g - fd)) <= 1e-5 * np.max(np.abs(fd))
        ok = ~np.isnan(fd_free)
        assert ok.mean() > 0.9 or not same
        if ok.any():
            assert np.max(np.abs(g[ok] - fd_free[ok])) <= 1e-5 * np.max(np.abs(fd_free[ok]))
    assert np.abs(ga.sum(0) + gb.sum(0)).max() < 1e-3


def test_autotune_keeps_results(tmp_path, monkeypatch):
    cfg = inputs.config_small(n=20_000, m=20_000)
    data, q, r = cfg["data"], cfg["queries"], cfg["radius"]
    t = ax.arborx_bvh_build(dev(data))
    dq = dev(q)
    monkeypatch.setenv("ARBORX_TUNING_CACHE", str(tmp_path / "tuning.jsonl"))
    try:
        for op in (ax.OP_REDUCE, ax.OP_KNN, ax.OP_SPATIAL):
            base = ax.arborx_get_tuning_op(op)
            best, ms = ax.arborx_autotune(t, op, dq, radius=float(r), k=10)
            # the winner is timing-dependent; it must be one of the documented candidates:
            # thread (0), wavefront-packet (1) or, for the radius walks only, rope (2) schedules
            assert ms > 0 and best["block"] in (64, 128, 256, base["block"])
            assert best["schedule"] in ((0, 1) if op == ax.OP_KNN else (0, 1, 2))
            assert best["stack"] in (8, 16, 32, base["stack"]) and best["order"] in (0, 1)
            assert best["node_format"] in (0, 1, 2) and best["queries_per_thread"] in (0, 1, 2, 4)
            assert best["seed_mode"] in (0, 1, 2)
            assert ax.arborx_get_tuning_op(op) == best
        best2, ms2 = ax.arborx_autotune(t, ax.OP_KNN, dq, radius=float(r), k=10)
        assert ms2 == -1.0 and best2 == ax.arborx_get_tuning_op(ax.OP_KNN)
        c, s = ax.arborx_query_spatial_reduce(t, dq, float(r))
        oc, os_ = oracle.reduce(data, q, r)
        assert np.array_equal(host(c), oc) and np.array_equal(host(s), os_)
        d2, ix = ax.arborx_query_knn(t, dq, 10)
        o_d2, o_ix = oracle.knn(data, q, 10)
        assert np.array_equal(host(ix), o_ix) and np.array_equal(host(d2), o_d2)
        off, idx = ax.arborx_query_spatial(t, dq, float(r))
        o_off, o_idx = oracle.spatial(data, q, r)
        assert np.array_equal(host(off), o_off) and np.array_equal(host(idx), o_idx)
    finally:
        ax.arborx_reset_tuning()


def test_autotune_forest_keeps_results(tmp_path, monkeypatch):
    cfg = small_forest(6)
    ax.arborx_set_tuning(node_format=2)  # build the four-wide nodes too, so that format is a candidate
    try:
        fo = ax.arborx_forest_build(dev(cfg["values"]), cfg["tree_offsets"])
    finally:
        ax.arborx_reset_tuning()
    q, bo, bt, br = dev(cfg["queries"]), dev(cfg["batch_offsets"]), dev(cfg["batch_tree"]), dev(cfg["batch_radius"])
    monkeypatch.setenv("ARBORX_TUNING_CACHE", str(tmp_path / "forest_tuning.jsonl"))
    try:
        for op in (ax.OP_REDUCE, ax.OP_KNN):
            base = ax.arborx_get_tuning_op(op)
            best, ms = ax.arborx_autotune_forest(fo, op, q, bo, bt, br, k=8)
            assert ms > 0 and best["stack"] in (4, 8, 16, 32, base["stack"])
            assert best["node_format"] in (0, 2) and best["queries_per_thread"] in (0, 1, 2, 4)
            assert best["seed_mode"] in (0, 1, 2) and ax.arborx_get_tuning_op(op) == best
        best2, ms2 = ax.arborx_autotune_forest(fo, ax.OP_KNN, q, bo, bt, br, k=8)
        assert ms2 == -1.0 and best2 == ax.arborx_get_tuning_op(ax.OP_KNN)
        c, s = ax.arborx_forest_query_reduce(fo, q, bo, bt, br, ax.COUNT_SUMDIST)
        d2, ix = ax.arborx_forest_query_knn(fo, q, bo, bt, 8)
        oc, os_ = oracle.forest_reduce(cfg["values"], cfg["tree_offsets"], cfg["queries"], cfg["batch_offsets"],
                                       cfg["batch_tree"], cfg["batch_radius"])
        od2, oix = oracle.forest_knn(cfg["values"], cfg["tree_offsets"], cfg["queries"], cfg["batch_offsets"],
                                     cfg["batch_tree"], 8)
        assert np.array_equal(host(c), oc) and np.array_equal(host(s), os_)
        assert np.array_equal(host(ix), oix) and np.array_equal(host(d2), od2)
    finally:
        ax.arborx_reset_tuning()


def test_forest_create_edge_cases():
    # no values at all: every tree empty, reductions zero, kNN padded
    fo = ax.arborx_forest_create(0, 3, 3)
    ax.arborx_forest_rebuild(fo, torch.zeros((0, 3), dtype=torch.float32, device="cuda"),
                             dev(np.zeros(4, dtype=np.int64)))
    q = dev(np.random.default_rng(1).random((10, 3)).astype(np.float32))
    bo, bt = dev(np.array([0, 4, 10], dtype=np.int64)), dev(np.array([2, 0], dtype=np.int32))
    c, s = ax.arborx_forest_query_reduce(fo, q, bo, bt, dev(np.array([1.0, 1.0], dtype=np.float32)), ax.COUNT_SUMDIST)
    d2, ix = ax.arborx_forest_query_knn(fo, q, bo, bt, 3)
    assert np.all(host(c) == 0) and np.all(host(s) == 0) and np.all(host(ix) == -1) and np.all(np.isinf(host(d2)))
    # one tree holding everything, then rebuilt as two: same forest object
    g = np.random.default_rng(2)
    vals = g.random((3000, 3)).astype(np.float32)
    fo = ax.arborx_forest_create(3000, 2, 3)
    v = dev(vals)
    for toff in (np.array([0, 3000, 3000]), np.array([0, 1234, 3000]), np.array([0, 0, 3000])):
        ax.arborx_forest_rebuild(fo, v, dev(toff.astype(np.int64)))
        bo2, bt2 = np.array([0, 5, 10], dtype=np.int64), np.array([0, 1], dtype=np.int32)
        d2, ix = ax.arborx_forest_query_knn(fo, q, dev(bo2), dev(bt2), 4)
        od2, oix = oracle.forest_knn(vals, toff, host(q), bo2, bt2, 4)
        assert np.array_equal(host(ix), oix) and np.array_equal(host(d2), od2)
