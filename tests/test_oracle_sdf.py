"""Pins of the oracle's SDF/CSG domains (Sec. 7.2: the domain as a list of CSG operations
on signed distance fields) against the oracle's explicit ball and box geometry, closed
forms of the distance to unions, intersections and differences, dense sampling of the
boundary, and harmonic boundary data (u = g on any domain)."""
import math

import numpy as np
import pytest

from paper_2201_13240_amd import workloads as W

Z = W.field_const(0.0)
ONE = W.field_const(1.0)
U, I, S = W.SDF_UNION, W.SDF_INTERSECT, W.SDF_SUBTRACT


def _prob(geom, dim, **fields):
    f = dict(alpha=ONE, psi=Z, sigma=Z, source=Z, boundary=Z)
    f.update(fields)
    return W.make_problem(dim, geom, f["alpha"], f["psi"], f["sigma"], f["source"], f["boundary"], 1e-4)


def _box_pts(rng, lo, hi, n):
    return rng.uniform(lo, hi, size=(n, len(lo)))


@pytest.mark.parametrize("dim", [2, 3])
def test_single_ball_matches_ball_geometry(oracle, dim):
    c = np.array([0.1, -0.2, 0.3])[:dim]
    sdf = W.geom_sdf([W.sdf_row(U, "ball", c, [2.0])], c - 2, c + 2)
    pts = np.random.default_rng(0).uniform(-0.9, 0.9, size=(300, dim))
    d1, x1 = oracle.distance(_prob(sdf, dim), pts)
    d2, x2 = oracle.distance(_prob(W.geom_ball(c, 2.0), dim), pts)
    np.testing.assert_allclose(d1, d2, rtol=1e-14, atol=1e-15)
    np.testing.assert_allclose(x1, x2, rtol=1e-14, atol=1e-14)


@pytest.mark.parametrize("dim", [2, 3])
def test_box_and_halfspace_intersection_match_box_geometry(oracle, dim):
    lo, hi = np.array([0.0, -1.0, 2.0])[:dim], np.array([1.0, 0.5, 4.0])[:dim]
    pts = _box_pts(np.random.default_rng(1), lo, hi, 400)
    d0, x0 = oracle.distance(_prob(W.geom_box(lo, hi), dim), pts)
    box = W.geom_sdf([W.sdf_row(U, "box", (lo + hi) / 2, (hi - lo) / 2)], lo, hi)
    rows = []
    for i in range(dim):
        n = np.zeros(dim)
        n[i] = 2.5   # unnormalised normals: the field divides by |n|
        rows.append(W.sdf_row(U if i == 0 else I, "halfspace", n, [2.5 * hi[i]]))
        rows.append(W.sdf_row(I, "halfspace", -n, [-2.5 * lo[i]]))
    planes = W.geom_sdf(rows, lo, hi)
    for g in (box, planes):
        d, x = oracle.distance(_prob(g, dim), pts)
        np.testing.assert_allclose(d, d0, rtol=0, atol=1e-14)
        np.testing.assert_allclose(x, x0, rtol=0, atol=1e-14)


def test_square_with_round_hole(oracle):
    geom = W.geom_sdf([W.sdf_row(U, "box", [0, 0], [1, 1]), W.sdf_row(S, "ball", [0.2, 0.1], [0.3])],
                      [-1, -1], [1, 1])
    rng = np.random.default_rng(2)
    pts = _box_pts(rng, [-1, -1], [1, 1], 2000)
    pts = pts[W.inside_mask(geom, pts)]
    d, xb = oracle.distance(_prob(geom, 2), pts)
    c = np.array([0.2, 0.1])
    r = np.linalg.norm(pts - c, axis=1)
    face = (1 - np.abs(pts)).min(1)
    np.testing.assert_allclose(d, np.minimum(face, r - 0.3), rtol=0, atol=1e-14)
    hole = r - 0.3 < face
    proj = c + 0.3 * (pts - c) / r[:, None]
    np.testing.assert_allclose(xb[hole], proj[hole], rtol=0, atol=1e-14)
    # outer faces: the coordinate of the nearest face is set to +-1
    ax = np.argmin(1 - np.abs(pts), axis=1)
    o = ~hole
    np.testing.assert_allclose(np.abs(xb[o, ax[o]]), 1.0, rtol=0, atol=1e-14)


def test_cube_with_box_hole_outside_box_distance(oracle):
    """Subtracting a box uses the box field outside it: the distance to the nearest point
    of the hole (clamping)."""
    hl, hh = np.array([-0.3, -0.2, -0.1]), np.array([0.3, 0.4, 0.2])
    geom = W.geom_sdf([W.sdf_row(U, "box", [0, 0, 0], [1, 1, 1]),
                       W.sdf_row(S, "box", (hl + hh) / 2, (hh - hl) / 2)], [-1] * 3, [1] * 3)
    pts = _box_pts(np.random.default_rng(3), [-1] * 3, [1] * 3, 3000)
    pts = pts[W.inside_mask(geom, pts)]
    d, xb = oracle.distance(_prob(geom, 3), pts)
    q = np.clip(pts, hl, hh)
    dh = np.linalg.norm(pts - q, axis=1)
    face = (1 - np.abs(pts)).min(1)
    np.testing.assert_allclose(d, np.minimum(face, dh), rtol=0, atol=1e-14)
    hole = dh < face
    np.testing.assert_allclose(xb[hole], q[hole], rtol=0, atol=1e-13)


def test_union_distance_is_a_lower_bound(oracle):
    """Two overlapping disks: -f = max of the two disk distances never exceeds the true
    distance to the union's boundary (dense sampling of the exposed arcs) and equals it
    where the nearer exposed arc belongs to the deeper disk."""
    c1, c2, r1, r2 = np.array([-0.4, 0.0]), np.array([0.5, 0.1]), 0.7, 0.6
    geom = W.geom_sdf([W.sdf_row(U, "ball", c1, [r1]), W.sdf_row(U, "ball", c2, [r2])], [-1.2, -0.7], [1.2, 0.8])
    rng = np.random.default_rng(4)
    pts = _box_pts(rng, [-1.2, -0.7], [1.2, 0.8], 3000)
    pts = pts[W.inside_mask(geom, pts)][:400]
    d, xb = oracle.distance(_prob(geom, 2), pts)
    t = np.linspace(0, 2 * math.pi, 20000, endpoint=False)
    arcs = []
    for c, r, co, ro in ((c1, r1, c2, r2), (c2, r2, c1, r1)):
        p = c + r * np.c_[np.cos(t), np.sin(t)]
        arcs.append(p[np.linalg.norm(p - co, axis=1) >= ro])
    B = np.concatenate(arcs)
    true = np.sqrt(((pts[:, None, :] - B[None, :, :]) ** 2).sum(-1)).min(1)
    assert np.all(d > 0)
    assert np.all(d <= true + 1e-12)
    # sampling resolution of the arcs bounds how far the dense distance overestimates
    h = 2 * math.pi * max(r1, r2) / 20000
    assert np.mean(np.abs(d - true) < h) > 0.5
    # the exit point lies on the deciding circle
    on = np.minimum(np.abs(np.linalg.norm(xb - c1, axis=1) - r1), np.abs(np.linalg.norm(xb - c2, axis=1) - r2))
    assert np.all(on < 1e-14)


def _expcos(p):
    return np.exp(p[:, 0]) * np.cos(p[:, 1])


def csg_scenes():
    return {
        "annulus": (W.geom_sdf([W.sdf_row(U, "ball", [0, 0], [1.0]), W.sdf_row(S, "ball", [0.1, 0], [0.35])],
                               [-1, -1], [1, 1]), 2),
        "two-disks": (W.geom_sdf([W.sdf_row(U, "ball", [-0.4, 0], [0.7]), W.sdf_row(U, "ball", [0.5, 0.1], [0.6])],
                                 [-1.1, -0.7], [1.1, 0.8]), 2),
        "cut-square": (W.geom_sdf([W.sdf_row(U, "box", [0, 0], [1, 0.8]),
                                   W.sdf_row(I, "halfspace", [1, 1], [0.9]),
                                   W.sdf_row(S, "box", [-0.4, -0.3], [0.2, 0.15])], [-1, -0.8], [1, 0.8]), 2),
        "cube-minus-ball": (W.geom_sdf([W.sdf_row(U, "box", [0, 0, 0], [1, 1, 1]),
                                        W.sdf_row(S, "ball", [0.3, 0.2, 0.1], [0.45])], [-1] * 3, [1] * 3), 3),
    }


@pytest.mark.parametrize("name", ["annulus", "two-disks", "cut-square", "cube-minus-ball"])
def test_harmonic_data_on_csg_domains(oracle, name):
    geom, dim = csg_scenes()[name]
    prob = _prob(geom, dim, boundary=W.field_manufactured("expcos"))
    rng = np.random.default_rng(5)
    pts = W.sample_inside(rng, geom, dim, 6)
    r = oracle.solve(prob, pts, 3000, 0.0, seed=6)
    z = (r["mean"] - _expcos(pts)) / np.maximum(r["se"], 1e-10)
    assert np.all(np.abs(z) < 4.5), (name, z)


@pytest.mark.parametrize("dim", [2, 3])
def test_sdf_ball_walk_equals_ball_walk(oracle, dim):
    """The same screened problem on the explicit ball and on a one-row SDF ball: the walks
    draw the same numbers and differ only by rounding of the distance."""
    sdf = W.geom_sdf([W.sdf_row(U, "ball", np.zeros(dim), [1.0])], -np.ones(dim), np.ones(dim))
    kw = dict(sigma=W.field_const(9.0), source=W.field_const(2.0), boundary=W.field_manufactured("expcos"))
    pts = W.sample_inside(np.random.default_rng(7), W.geom_ball(np.zeros(dim), 1.0), dim, 8)
    a = oracle.solve(_prob(W.geom_ball(np.zeros(dim), 1.0), dim, **kw), pts, 500, 12.0, seed=8)
    b = oracle.solve(_prob(sdf, dim, **kw), pts, 500, 12.0, seed=8)
    np.testing.assert_allclose(b["mean"], a["mean"], rtol=1e-9, atol=1e-12)
    assert np.array_equal(a["steps"], b["steps"])
