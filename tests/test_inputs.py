"""Seeded workload generators: reproducibility and the neighbour counts they are sized for."""
import hashlib

import numpy as np
from scipy.spatial import cKDTree

from paper_2507_23700_amd import inputs


def _h(a):
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def test_reproducible_and_float32():
    a = inputs.config_small(n=1000, m=100)
    b = inputs.config_small(n=1000, m=100)
    assert a["data"].dtype == np.float32 and a["data"].shape == (1000, 3)
    assert _h(a["data"]) == _h(b["data"]) and _h(a["queries"]) == _h(b["queries"])
    assert _h(a["data"]) != _h(a["queries"][:100])


def test_radii_closed_forms():
    assert abs(float(inputs.radius_cube(20_000, 10.0)) - 0.049237251) < 1e-7
    assert abs(float(inputs.radius_cube(10_000_000, 10.0)) - 6.2035047e-3) < 1e-9
    assert abs(float(inputs.radius_shell(10_000_000, 10.0)) - 2.3852e-3) < 1e-7
    assert abs(float(inputs.radius_gmm(2_000_000, 20.0)) - 0.016154) < 1e-6


def _mean_count(data, q, r):
    return np.mean([len(x) for x in cKDTree(data).query_ball_point(q, float(r))])


def test_mean_neighbour_counts():
    c = inputs.config_small()
    assert abs(_mean_count(c["data"], c["queries"][:3000], c["radius"]) - 9.45) < 0.4
    s = inputs.config_paper("shell", n=400_000, m=2000)
    assert abs(_mean_count(s["data"], s["queries"], s["radius"]) - 10.0) < 0.6
    g = inputs.config_gmm6(n=400_000, m=2000)
    assert abs(_mean_count(g["data"], g["queries"], g["radius"]) - 20.0) < 1.5


def test_chamfer_and_forest_shapes():
    c = inputs.chamfer_pairs(pairs=3, lo=50, hi=80)
    assert c["a"].shape == (c["a_off"][-1], 3) and c["b"].shape == (c["b_off"][-1], 3)
    assert np.all(np.diff(c["a_off"]) >= 50) and np.all(np.diff(c["a_off"]) <= 80)
    f = inputs.forest(trees=4, tree_lo=100, tree_hi=1000, batches=8, batch_lo=10, batch_hi=100)
    assert f["values"].shape[0] == f["tree_offsets"][-1]
    assert f["queries"].shape[0] == f["batch_offsets"][-1]
    assert f["batch_tree"].min() >= 0 and f["batch_tree"].max() < 4
    assert f["batch_radius"].dtype == np.float32
