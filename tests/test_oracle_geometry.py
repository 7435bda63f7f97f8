"""Pins of the oracle's closest-point queries (the distance step of Alg. 1) against
closed forms and dense sampling of the boundary."""
import math

import numpy as np
import pytest

from paper_2201_13240_amd import workloads as W


def _prob(geom, dim):
    z = W.field_const(0.0)
    return W.make_problem(dim, geom, W.field_const(1.0), z, z, z, z)


def test_ball_distance(oracle):
    for dim in (2, 3):
        c = np.array([0.1, -0.2, 0.3])[:dim]
        prob = _prob(W.geom_ball(c, 2.0), dim)
        pts = np.random.default_rng(0).uniform(-0.8, 0.8, size=(200, dim))
        d, xb = oracle.distance(prob, pts)
        np.testing.assert_allclose(d, 2.0 - np.linalg.norm(pts - c, axis=1), rtol=1e-14, atol=1e-15)
        np.testing.assert_allclose(np.linalg.norm(xb - c, axis=1), 2.0, rtol=1e-14)
        np.testing.assert_allclose(np.linalg.norm(xb - pts, axis=1), d, rtol=1e-12, atol=1e-14)


def test_box_distance(oracle):
    lo, hi = np.array([0.0, -1.0, 2.0]), np.array([1.0, 0.5, 4.0])
    for dim in (2, 3):
        prob = _prob(W.geom_box(lo[:dim], hi[:dim]), dim)
        pts = np.random.default_rng(1).uniform(lo[:dim], hi[:dim], size=(300, dim))
        d, xb = oracle.distance(prob, pts)
        ref = np.minimum(pts - lo[:dim], hi[:dim] - pts).min(1)
        np.testing.assert_allclose(d, ref, rtol=1e-14, atol=1e-15)
        np.testing.assert_allclose(np.linalg.norm(xb - pts, axis=1), d, rtol=1e-12, atol=1e-14)


def test_regular_polygon_inradius(oracle):
    for n in (3, 7, 64):
        th = 2 * math.pi * np.arange(n) / n
        prob = _prob(W.geom_polygon(np.c_[np.cos(th), np.sin(th)]), 2)
        d, _ = oracle.distance(prob, np.zeros((1, 2)))
        assert d[0] == pytest.approx(math.cos(math.pi / n), rel=1e-14)


def _dense_boundary_polygon(V, m=400):
    a, b = V, np.roll(V, -1, 0)
    t = np.linspace(0, 1, m)[None, :, None]
    return (a[:, None, :] * (1 - t) + b[:, None, :] * t).reshape(-1, 2)


def test_star_polygon_against_dense_sampling(oracle):
    geom = W.star_polygon(np.random.default_rng(2), 64, 8, 0.3)
    prob = _prob(geom, 2)
    pts = W.sample_inside(np.random.default_rng(3), geom, 2, 100)
    d, xb = oracle.distance(prob, pts)
    S = _dense_boundary_polygon(geom["vertices"])
    dd = np.sqrt(((pts[:, None, :] - S[None, :, :]) ** 2).sum(-1)).min(1)
    seg = np.max(np.linalg.norm(np.roll(geom["vertices"], -1, 0) - geom["vertices"], axis=1))
    assert np.all(d <= dd + 1e-12)
    assert np.all(dd - d <= seg / 399 + 1e-12)
    np.testing.assert_allclose(np.linalg.norm(xb - pts, axis=1), d, rtol=1e-12)


def test_trimesh_against_dense_sampling(oracle):
    geom = W.icosphere(np.random.default_rng(4), subdiv=1, noise=0.1)
    prob = _prob(geom, 3)
    pts = np.random.default_rng(5).uniform(-0.5, 0.5, size=(60, 3))
    d, xb = oracle.distance(prob, pts)
    V, F = geom["vertices"], geom["triangles"]
    m = 60
    i, j = np.meshgrid(np.arange(m + 1), np.arange(m + 1), indexing="ij")
    keep = i + j <= m
    b1, b2 = (i[keep] / m), (j[keep] / m)
    b0 = 1 - b1 - b2
    S = (V[F[:, 0]][:, None, :] * b0[None, :, None] + V[F[:, 1]][:, None, :] * b1[None, :, None]
         + V[F[:, 2]][:, None, :] * b2[None, :, None]).reshape(-1, 3)
    dd = np.array([np.sqrt(((S - p) ** 2).sum(1)).min() for p in pts])
    edge = np.max(np.linalg.norm(V[F[:, 1]] - V[F[:, 0]], axis=1))
    assert np.all(d <= dd + 1e-12)
    assert np.all(dd - d <= 2 * edge / m)
    np.testing.assert_allclose(np.linalg.norm(xb - pts, axis=1), d, rtol=1e-12)
    # a projection closest point is where the offset is normal to the face
    for p, q in zip(pts, xb):
        assert np.all(np.abs(np.linalg.norm(S - q, axis=1).min()) < 2 * edge / m)


def _near_boundary_and_inside(rng, prob, n):
    """Interior samples plus points pushed towards the boundary (small and large distances)."""
    dim = prob["dim"]
    pts = W.sample_inside(rng, prob["geometry"], dim, n)
    return np.concatenate([pts, 0.98 * pts, 0.5 * pts, pts + 0.2])


@pytest.mark.parametrize("which", ["star256", "star4096", "ico20480"])
def test_bvh_distance_equals_brute_force(oracle, which):
    """The oracle's BVH (timing mode, Sec. 7.1) returns exactly the brute-force minimum
    distance, at interior points, points near the boundary and points outside it."""
    rng = np.random.default_rng(11)
    if which == "ico20480":
        g = W.icosphere(np.random.default_rng(3000), 5, 0.1)
        dim, n = 3, 300
    else:
        g = W.star_polygon(np.random.default_rng(2000), 256 if which == "star256" else 4096)
        dim, n = 2, 1000
    prob = _prob(g, dim)
    pts = _near_boundary_and_inside(rng, prob, n)
    d0, x0 = oracle.distance(prob, pts, bvh=False)
    d1, x1 = oracle.distance(prob, pts, bvh=True)
    assert np.array_equal(d0, d1)
    # where primitives tie (a closest point on a shared edge or vertex), another primitive
    # may give it, with other rounding
    np.testing.assert_allclose(np.linalg.norm(x1 - pts, axis=1), d1, rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(x1, x0, rtol=0, atol=1e-12)


def test_bvh_walk_equals_brute_force_walk(oracle):
    """A walk in timing mode makes the same distance queries as in correctness mode (the
    distances are identical), so step counts and estimates agree."""
    c = W.config2(n_grid=64)
    prob, pts = c["problems"][0], c["points"][0][:40]
    sb = 12.0
    a = oracle.solve(prob, pts, 64, sb, seed=3, bvh=False)
    b = oracle.solve(prob, pts, 64, sb, seed=3, bvh=True)
    assert np.array_equal(a["steps"], b["steps"])
    np.testing.assert_allclose(a["sum"], b["sum"], rtol=1e-12, atol=1e-12)
