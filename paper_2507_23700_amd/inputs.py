"""Seeded synthetic workloads for the geometric-search hot path.

This module only draws random inputs and computes workload parameters (radii
chosen for a target mean neighbour count).  It holds none of the search
arithmetic: both the HIP path and the CPU oracle consume what it produces, and
neither is imported here.

Every array is drawn in float64 from ``numpy.random.default_rng`` seeded with
``SeedSequence([250723700, cfg, role, sub])`` (role 0 = data values, 1 =
queries, 2 = auxiliary draws such as centres, axes or sizes) and rounded once
to float32.  Radii are computed in float64 and rounded once to float32.

Workloads (the paper measures on a ~37M-point cosmology set, Table 1 in
Section 2.6, which is not available; these stand in for it at its scale):

* ``cube``   : uniform in the unit cube [0,1)^D.
* ``shell``  : hollow unit sphere, uniform directions, radial noise 1e-3.
* ``gmm``    : 64-component isotropic Gaussian mixture in [0,1)^D, sigma 0.02.
* ``chamfer_pairs`` : noisy random-ellipsoid surface clouds, packed per pair.
* ``forest`` : many uneven trees (half cube, half shell) and query batches.
"""
from __future__ import annotations

import math

import numpy as np

ROOT_SEED = 250723700


def rng(cfg: int, role: int, sub: int = 0) -> np.random.Generator:
    """Generator for (configuration, role, sub-stream)."""
    return np.random.default_rng(np.random.SeedSequence([ROOT_SEED, cfg, role, sub]))


def _f32(x: np.ndarray) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(x, dtype=np.float64).astype(np.float32))


# --------------------------------------------------------------------------
# point distributions
# --------------------------------------------------------------------------

def cube(n: int, dim: int, g: np.random.Generator) -> np.ndarray:
    """n points uniform in [0,1)^dim, float32 [n, dim]."""
    return _f32(g.random((n, dim)))


def shell(n: int, g: np.random.Generator, noise: float = 1e-3) -> np.ndarray:
    """n points on the unit sphere (direction g/|g|, g ~ N(0,I3)) scaled by 1+noise*eps."""
    v = g.standard_normal((n, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    v *= (1.0 + noise * g.standard_normal((n, 1)))
    return _f32(v)


def gmm_centres(dim: int, g: np.random.Generator, components: int = 64) -> np.ndarray:
    return g.random((components, dim))


def gmm(n: int, centres: np.ndarray, g: np.random.Generator, sigma: float = 0.02) -> np.ndarray:
    """n points: a uniformly chosen centre plus sigma*N(0,I)."""
    comp = g.integers(0, centres.shape[0], size=n)
    return _f32(centres[comp] + sigma * g.standard_normal((n, centres.shape[1])))


# --------------------------------------------------------------------------
# radii for a target mean neighbour count K (workload recipe, not the method)
# --------------------------------------------------------------------------

def radius_cube(n: int, k_mean: float, dim: int = 3) -> np.float32:
    """Ball volume = k_mean / n in the unit cube (boundary loss ignored)."""
    unit_ball = math.pi ** (dim / 2) / math.gamma(dim / 2 + 1)
    return np.float32((k_mean / (n * unit_ball)) ** (1.0 / dim))


def radius_shell(n: int, k_mean: float, noise: float = 1e-3) -> np.float32:
    """Locally planar shell of area 4*pi and radial N(0, noise^2) thickness.

    The expected count for a query drawn from the same shell is
    (n/4) * [(r^2 - s^2)(2 Phi(r/s) - 1) + 2 r s phi(r/s)] with s = sqrt(2)*noise.
    """
    from scipy.optimize import brentq
    from scipy.stats import norm
    s = math.sqrt(2.0) * noise

    def f(r):
        a = r / s
        return (n / 4.0) * ((r * r - s * s) * (2 * norm.cdf(a) - 1) + 2 * r * s * norm.pdf(a)) - k_mean
    return np.float32(brentq(f, 1e-9, 2.0))


def radius_gmm(n: int, k_mean: float, dim: int = 6, components: int = 64, sigma: float = 0.02) -> np.float32:
    """Same-component pairs: |q-p|^2 / (2 sigma^2) ~ chi^2_dim."""
    from scipy.stats import chi2
    x = chi2.ppf(k_mean * components / n, dim)
    return np.float32(sigma * math.sqrt(2.0 * x))


# --------------------------------------------------------------------------
# configurations
# --------------------------------------------------------------------------

def config_small(n: int = 20_000, m: int = 20_000):
    """3D uniform cube, radius for ~10 neighbours, kNN k = 10."""
    return dict(workload=f"cube3d_n{n}_m{m}", data=cube(n, 3, rng(1, 0)), queries=cube(m, 3, rng(1, 1)),
                radius=radius_cube(n, 10.0), k=10)


def config_paper(dist: str = "cube", n: int = 10_000_000, m: int | None = None):
    """3D paper-scale: 'cube' (filled unit cube) or 'shell' (hollow sphere); ~10 neighbours; k = 16."""
    m = n if m is None else m
    if dist == "cube":
        data, queries, r = cube(n, 3, rng(2, 0, 0)), cube(m, 3, rng(2, 1, 0)), radius_cube(n, 10.0)
    elif dist == "shell":
        data, queries, r = shell(n, rng(2, 0, 1)), shell(m, rng(2, 1, 1)), radius_shell(n, 10.0)
    else:
        raise ValueError(dist)
    return dict(workload=f"{dist}3d_n{n}_m{m}", data=data, queries=queries, radius=r, k=16)


def config_gmm6(n: int = 2_000_000, m: int | None = None):
    """6D 64-component Gaussian mixture; ~20 neighbours; k = 8."""
    m = n if m is None else m
    c = gmm_centres(6, rng(3, 2))
    return dict(workload=f"gmm6d_n{n}_m{m}", data=gmm(n, c, rng(3, 0)), queries=gmm(m, c, rng(3, 1)),
                radius=radius_gmm(n, 20.0), k=8)


def random_rotation(g: np.random.Generator) -> np.ndarray:
    """Haar rotation: QR of a Gaussian 3x3 with sign and determinant fixed."""
    q, r = np.linalg.qr(g.standard_normal((3, 3)))
    q = q * np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


def ellipsoid_cloud(n: int, g: np.random.Generator, noise: float = 0.01) -> np.ndarray:
    axes = g.uniform(0.5, 1.5, size=3)
    rot = random_rotation(g)
    u = g.standard_normal((n, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    pts = (u * axes) @ rot.T + noise * g.standard_normal((n, 3))
    return _f32(pts)


def chamfer_pairs(pairs: int = 256, lo: int = 1000, hi: int = 65536, cfg: int = 4):
    """Packed clouds: a [sum nA, 3], a_off [P+1] int64, b, b_off; each cloud its own ellipsoid."""
    gs = rng(cfg, 2)
    na = gs.integers(lo, hi + 1, size=pairs)
    nb = gs.integers(lo, hi + 1, size=pairs)
    a = [ellipsoid_cloud(int(na[p]), rng(cfg, 0, p)) for p in range(pairs)]
    b = [ellipsoid_cloud(int(nb[p]), rng(cfg, 1, p)) for p in range(pairs)]
    a_off = np.concatenate([[0], np.cumsum(na)]).astype(np.int64)
    b_off = np.concatenate([[0], np.cumsum(nb)]).astype(np.int64)
    return dict(workload=f"chamfer_p{pairs}_n{lo}-{hi}", a=np.ascontiguousarray(np.concatenate(a)), a_off=a_off,
                b=np.ascontiguousarray(np.concatenate(b)), b_off=b_off)


def _log_uniform_int(g, lo, hi, size):
    return np.rint(np.exp(g.uniform(math.log(lo), math.log(hi), size=size))).astype(np.int64)


def forest(trees: int = 64, tree_lo: int = 10_000, tree_hi: int = 4_000_000, batches: int = 4096,
           batch_lo: int = 100, batch_hi: int = 1_000_000, cfg: int = 5):
    """Forest of uneven trees (even index: cube, odd: shell) and query batches aimed at random trees.

    Each batch's queries follow its target tree's distribution and its radius is the
    ~10-neighbour closed form for that tree's size and distribution.
    """
    ga = rng(cfg, 2)
    tsize = _log_uniform_int(ga, tree_lo, tree_hi, trees)
    bsize = _log_uniform_int(ga, batch_lo, batch_hi, batches)
    btree = ga.integers(0, trees, size=batches).astype(np.int32)
    vals = [cube(int(tsize[t]), 3, rng(cfg, 0, t)) if t % 2 == 0 else shell(int(tsize[t]), rng(cfg, 0, t))
            for t in range(trees)]
    qs = [cube(int(bsize[b]), 3, rng(cfg, 1, b)) if btree[b] % 2 == 0 else shell(int(bsize[b]), rng(cfg, 1, b))
          for b in range(batches)]
    tr = np.array([radius_cube(int(tsize[t]), 10.0) if t % 2 == 0 else radius_shell(int(tsize[t]), 10.0)
                   for t in range(trees)], dtype=np.float32)
    return dict(workload=f"forest_t{trees}_b{batches}",
                values=np.ascontiguousarray(np.concatenate(vals)),
                tree_offsets=np.concatenate([[0], np.cumsum(tsize)]).astype(np.int64),
                queries=np.ascontiguousarray(np.concatenate(qs)),
                batch_offsets=np.concatenate([[0], np.cumsum(bsize)]).astype(np.int64),
                batch_tree=btree, batch_radius=np.ascontiguousarray(tr[btree]), k=8)
