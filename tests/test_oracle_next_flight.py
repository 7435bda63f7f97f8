"""Pins of the oracle's next-flight walk (Sec. 5.2, supplemental Alg. 2) and of its
off-centred Green's function and Poisson kernel approximations (supplemental Sec. 1.2).

The approximations are not exact off the centre of the ball (the supplement says so),
so they are pinned where the mathematics fixes them: exactly at the centre; exactly in
the harmonic limit for points on a line through the centre (the image construction of
the disk and ball); and by first-order convergence to the exact Bessel series of the
off-centred kernels as the offset goes to zero. The walk is pinned exactly where it
uses only centred kernels (sigma_bar = sigma' constant) and in the harmonic case."""
import math

import numpy as np
import pytest
from scipy import special

from paper_2201_13240_amd import workloads as WL

Z = WL.field_const(0.0)
ONE = WL.field_const(1.0)


def series_poisson(dim, a, theta, R, sb, terms=60):
    """Exact Poisson kernel of the ball for Lap - sb at distance a from the centre, angle
    theta to the boundary point: the separable solution sum of I_n(k a)/I_n(k R) cos(n
    theta) (2D) or of (2n+1) i_n(k a)/i_n(k R) P_n(cos theta) (3D), normalised so that a
    constant boundary value is reproduced."""
    k = math.sqrt(sb)
    if dim == 2:
        tot = special.iv(0, a * k) / special.iv(0, R * k)
        for n in range(1, terms):
            tot += 2 * math.cos(n * theta) * special.iv(n, a * k) / special.iv(n, R * k)
        return tot / (2 * math.pi * R)
    tot = 0.0
    for n in range(terms):
        tot += ((2 * n + 1) * special.eval_legendre(n, math.cos(theta)) * special.spherical_in(n, a * k)
                / special.spherical_in(n, R * k))
    return tot / (4 * math.pi * R * R)


def series_green(dim, rl, rg, theta, R, sb, terms=14):
    """Exact off-centred Green's function of the ball (addition theorems of the screened
    free-space kernel minus the regular part that vanishes on the sphere); rl < rg."""
    k = math.sqrt(sb)
    tot = 0.0
    for n in range(terms):
        if dim == 2:
            t = special.iv(n, rl * k) * (special.kv(n, rg * k) - special.kv(n, R * k) / special.iv(n, R * k)
                                         * special.iv(n, rg * k))
            tot += (1 if n == 0 else 2) * math.cos(n * theta) * t
        else:
            t = special.spherical_in(n, rl * k) * (special.spherical_kn(n, rg * k) - special.spherical_kn(n, R * k)
                                                   / special.spherical_in(n, R * k) * special.spherical_in(n, rg * k))
            tot += (2 * n + 1) * special.eval_legendre(n, math.cos(theta)) * t
    if dim == 2:
        return tot / (2 * math.pi)
    return tot * (2 * k / math.pi) / (4 * math.pi)


def on_circle(dim, r, theta):
    p = np.zeros(dim)
    p[0], p[1] = r * math.cos(theta), r * math.sin(theta)
    return p


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("sb", [0.5, 4.0, 60.0])
def test_kernels_at_the_centre(oracle, dim, sb):
    """At the centre: P equals the exact series, G equals the exact series, and
    sigma_bar * int_B G + int_dB P = 1 (constant solution), by quadrature of the oracle's
    own G over the radius."""
    R = 0.7
    u = np.zeros(dim)
    for th in (0.0, 1.3, math.pi):
        z = on_circle(dim, R, th)
        p = oracle.nf_kernel("poisson", dim, u, z, R, sb)[0]
        assert p == pytest.approx(series_poisson(dim, 0.0, th, R, sb), rel=1e-13)
        y = on_circle(dim, 0.45, th)
        g = oracle.nf_kernel("green", dim, u, y, R, sb)[0]
        assert g == pytest.approx(series_green(dim, 0.0, 0.45, th, R, sb), rel=1e-12)
    # identity: integral of G over the ball (radial quadrature in r = R t^2, which
    # smooths the logarithmic singularity at the centre) and P over the sphere
    x, w = np.polynomial.legendre.leggauss(200)
    t = 0.5 * (x + 1)
    r = R * t * t
    pts = np.zeros((r.size, dim))
    pts[:, 0] = r
    g = oracle.nf_kernel("green", dim, np.zeros((r.size, dim)), pts, R, sb)
    shell = 2 * math.pi * r if dim == 2 else 4 * math.pi * r * r
    vol = float(np.sum(0.5 * w * 2 * R * t * shell * g))
    area = 2 * math.pi * R if dim == 2 else 4 * math.pi * R * R
    p = oracle.nf_kernel("poisson", dim, u, on_circle(dim, R, 0.4), R, sb)[0]
    assert sb * vol + area * p == pytest.approx(1.0, rel=1e-9)


@pytest.mark.parametrize("dim", [2, 3])
def test_kernels_harmonic_limit_on_the_axis(oracle, dim):
    """sigma_bar = 0 (and sigma_bar -> 0 through the Bessel forms): for x, y, z on one line
    through the centre the approximations equal the exact harmonic Green's function (image
    point R^2 u/|u|^2) and Poisson kernel of the disk or ball."""
    R = 1.3
    for a in (0.2, 0.6, 1.1):
        u = on_circle(dim, a, 0.0)
        ustar = R * R * u / (a * a)
        for side in (0.0, math.pi):
            z = on_circle(dim, R, side)
            dz = np.linalg.norm(z - u)
            exact_p = (R * R - a * a) / (2 * math.pi * R * dz ** 2) if dim == 2 else \
                (R * R - a * a) / (4 * math.pi * R * dz ** 3)
            for sb, rel in ((0.0, 1e-13), (1e-12, 1e-5)):
                assert oracle.nf_kernel("poisson", dim, u, z, R, sb)[0] == pytest.approx(exact_p, rel=rel)
            for b in (0.1, 0.9):
                y = on_circle(dim, b, side)
                w = np.linalg.norm(y - u)
                img = a * np.linalg.norm(y - ustar) / R
                exact_g = math.log(img / w) / (2 * math.pi) if dim == 2 else (1 / w - 1 / img) / (4 * math.pi)
                got = oracle.nf_kernel("green", dim, u, y, R, 0.0)[0]
                assert got == pytest.approx(exact_g, rel=1e-12, abs=1e-14)
                got = oracle.nf_kernel("green", dim, u, y, R, 1e-12)[0]
                assert got == pytest.approx(exact_g, rel=1e-5)


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("sbR2", [1.0, 10.0])
def test_kernels_converge_to_exact_series_at_first_order(oracle, dim, sbR2):
    """Off the centre the approximations differ from the exact series; the difference
    vanishes linearly with the offset (halving the offset halves it)."""
    R = 1.0
    sb = sbR2 / (R * R)
    errs_p, errs_g = [], []
    for a in (0.004, 0.008, 0.016):
        ep, eg = 0.0, 0.0
        for th in (0.0, 0.9, 2.2, math.pi):
            u = on_circle(dim, a, 0.0)
            z = on_circle(dim, R, th)
            ex = series_poisson(dim, a, th, R, sb)
            ep = max(ep, abs(oracle.nf_kernel("poisson", dim, u, z, R, sb)[0] / ex - 1))
            y = on_circle(dim, 0.6, th)
            ex = series_green(dim, a, 0.6, th, R, sb)
            eg = max(eg, abs(oracle.nf_kernel("green", dim, u, y, R, sb)[0] / ex - 1))
        errs_p.append(ep)
        errs_g.append(eg)
    for errs in (errs_p, errs_g):
        assert errs[0] < 0.05
        for e1, e2 in zip(errs, errs[1:]):
            assert 1.6 < e2 / e1 < 2.4, errs


def screened_ball_solution(dim, sig, f0, r, R=1.0):
    k = math.sqrt(sig)
    if dim == 2:
        return (f0 / sig) * (1 - special.i0(k * r) / special.i0(k * R))
    ratio = np.where(r > 0, R * np.sinh(k * np.maximum(r, 1e-300)) / (np.maximum(r, 1e-300) * np.sinh(k * R)),
                     k * R / np.sinh(k * R))
    return (f0 / sig) * (1 - ratio)


@pytest.mark.parametrize("dim", [2, 3])
def test_next_flight_exact_when_sigma_bar_equals_sigma(oracle, dim):
    """Constant sigma = sigma_bar: every throughput factor vanishes, so each ball uses the
    centred kernels only and the walk is an exact estimator of the screened Poisson
    solution (I0 / sinh closed forms)."""
    sig, f0 = 9.0, 3.0
    centre = [0.0] * dim
    prob = WL.make_problem(dim, WL.geom_ball(centre, 1.0), ONE, Z, WL.field_const(sig), WL.field_const(f0),
                           WL.field_const(0.0), 1e-5)
    pts = np.zeros((4, dim))
    pts[:, 0] = [0.0, 0.3, -0.5, 0.7]
    pts[:, 1] = [0.0, 0.2, 0.4, -0.1]
    o = oracle.solve(prob, pts, 40000, sig, seed=3, variant=2)
    exact = screened_ball_solution(dim, sig, f0, np.linalg.norm(pts, axis=1))
    z = (o["mean"] - exact) / o["se"]
    assert np.all(np.abs(z) < 4), z
    assert o["counters"][3] > 0


def test_next_flight_harmonic_data(oracle):
    """sigma = sigma_bar = 0: the walk is plain walk on spheres; u = e^x cos y is
    reproduced (within the epsilon-shell bias and 4 standard errors)."""
    prob = WL.make_problem(2, WL.geom_ball([0.0, 0.0], 1.0), ONE, Z, Z, Z, WL.field_manufactured("expcos"), 1e-5)
    pts = np.array([[0.0, 0.0], [0.4, -0.3], [-0.6, 0.5]])
    o = oracle.solve(prob, pts, 20000, 0.0, seed=4, variant=2)
    exact = np.exp(pts[:, 0]) * np.cos(pts[:, 1])
    assert np.all(np.abs(o["mean"] - exact) < 4 * o["se"] + 1e-3)


def test_next_flight_distance_queries_do_not_depend_on_sigma_bar(oracle):
    """Every ball ends on its sphere, so the number of distance queries per walk has the
    law of plain walk on spheres whatever sigma_bar is (Sec. 5.2); delta tracking needs
    more queries as sigma_bar grows."""
    prob = WL.make_problem(2, WL.geom_ball([0.0, 0.0], 1.0), ONE, Z, WL.field_const(2.0), WL.field_const(1.0),
                           WL.field_const(0.0), 1e-3)
    pts = np.array([[0.1, 0.2]])
    n = 20000
    means, ses = [], []
    for sb in (2.0, 50.0):
        o = oracle.solve(prob, pts, n, sb, seed=5, variant=2)
        means.append(o["steps"][0] / n)
    o = oracle.solve(prob, pts, n, 50.0, seed=5, variant=0)
    dt_steps = o["steps"][0] / n
    # walk-on-spheres step counts in a disk with epsilon 1e-3: mean about 10, sd about 5
    assert abs(means[0] - means[1]) < 4 * 6.0 * math.sqrt(2.0 / n)
    assert dt_steps > 2 * means[1]


def test_exact_kernels_match_independent_series(oracle):
    """The oracle's exact series kernels (ratio recurrences in logarithms, free-space part
    in closed form) against scipy's Bessel functions summed term by term."""
    for dim in (2, 3):
        for sb in (1.0, 30.0):
            for th in (0.0, 1.0, 3.0):
                u = on_circle(dim, 0.3, 0.0)
                v = on_circle(dim, 0.9, th)
                g = oracle.nf_kernel("green_exact", dim, u, v, 1.0, sb)[0]
                assert g == pytest.approx(series_green(dim, 0.3, 0.9, th, 1.0, sb, terms=60), rel=1e-11)
                p = oracle.nf_kernel("poisson_exact", dim, u, on_circle(dim, 1.0, th), 1.0, sb)[0]
                assert p == pytest.approx(series_poisson(dim, 0.3, th, 1.0, sb), rel=1e-11)


@pytest.mark.parametrize("sb", [13.5, 30.0])
def test_next_flight_with_exact_kernels_is_unbiased(oracle, sb):
    """With the exact off-centred kernels the unrolled series of Alg. 2 is an unbiased
    estimator for any sigma_bar >= sigma', so constant-sigma screened Poisson in the disk
    is reproduced with sigma_bar above sigma. This pins the throughput, roulette and source
    bookkeeping of the walk, which the approximate-kernel walk shares."""
    sig, f0 = 9.0, 3.0
    prob = WL.make_problem(2, WL.geom_ball([0.0, 0.0], 1.0), ONE, Z, WL.field_const(sig), WL.field_const(f0),
                           WL.field_const(0.0), 1e-5)
    pts = np.array([[0.0, 0.0], [0.3, 0.2], [-0.5, 0.4], [0.7, -0.1]])
    o = oracle.solve(prob, pts, 10000, sb, seed=3, variant=3)
    exact = screened_ball_solution(2, sig, f0, np.linalg.norm(pts, axis=1))
    z = (o["mean"] - exact) / o["se"]
    assert np.all(np.abs(z) < 4), z


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("sb", [0.0, 2.0, 30.0])
def test_gradient_kernels_match_derivatives_of_the_exact_series(oracle, dim, sb):
    """grad_x G(x, y) and grad_x P(x, z) at the centre (supplemental Sec. 1.3, used by the
    gradient estimator of supplemental Sec. 2) against central differences in x of the
    exact off-centred kernels (or of the harmonic image formulas when sigma_bar = 0)."""
    R, h = 0.9, 1e-5

    def green(u, v):
        if sb > 0:
            return oracle.nf_kernel("green_exact", dim, u, v, R, sb)[0]
        # harmonic: the image construction, G = Phi(|v - u|) - Phi(|u| |v - u*| / R), u* = R^2 u/|u|^2
        a = np.linalg.norm(u)
        img = R if a == 0 else a * np.linalg.norm(v - R * R * u / (a * a)) / R
        w = np.linalg.norm(v - u)
        return np.log(img / w) / (2 * np.pi) if dim == 2 else (1 / w - 1 / img) / (4 * np.pi)

    def poisson(u, v):
        if sb > 0:
            return oracle.nf_kernel("poisson_exact", dim, u, v, R, sb)[0]
        w = np.linalg.norm(v - u)
        a2 = float(u @ u)
        return (R * R - a2) / (2 * np.pi * R * w ** 2) if dim == 2 else (R * R - a2) / (4 * np.pi * R * w ** 3)

    rng = np.random.default_rng(dim + int(sb))
    for _ in range(4):
        d = rng.normal(size=dim)
        d /= np.linalg.norm(d)
        y = d * R * rng.uniform(0.2, 0.8)
        z = rng.normal(size=dim)
        z = z / np.linalg.norm(z) * R
        ratio_g = oracle.grad_ratio("green", dim, y, R, sb)
        ratio_p = oracle.grad_ratio("poisson", dim, z, R, sb)
        for i in range(dim):
            e = np.zeros(dim)
            e[i] = h
            fd = (green(e, y) - green(-e, y)) / (2 * h)
            assert fd == pytest.approx(ratio_g[i] * green(0 * e, y), rel=1e-5, abs=1e-7)
            fd = (poisson(e, z) - poisson(-e, z)) / (2 * h)
            assert fd == pytest.approx(ratio_p[i] * poisson(0 * e, z), rel=1e-5, abs=1e-7)


def test_next_flight_with_exact_kernels_variable_coefficients(oracle):
    """Variable coefficients inside every ball (alpha = 1 + 0.02 sin sin, drift potential
    psi = sin(pi x / 2), so gamma varies by about 1 across the disk and sigma' in about
    [1.1, 5.1]) at a small s = R sqrt(sigma_bar) (< 2.5, where the throughput has finite
    variance): with the exact off-centred kernels the walk reproduces the manufactured
    u = e^x cos y. This pins the gamma weights of the boundary and source terms and the
    sigma' of the throughput for varying coefficients."""
    alpha = WL.field_fourier([[1.0, -1.0], [1.0, 1.0]], [0.01, -0.01], [0.0, 0.0], transform="affine",
                             c0=1.0, c1=1.0)
    psi = WL.field_fourier([[0.25, 0.0]], [1.0], [-math.pi / 2])
    prob = WL.make_problem(2, WL.geom_ball([0.0, 0.0], 1.0), alpha, psi, WL.field_const(3.0),
                           WL.field_manufactured("expcos"), WL.field_manufactured("expcos"), 1e-4)
    g = WL.grid_points(256, -1.0, 1.0)
    mn, mx = oracle.sigma_prime_range(prob, g[WL.inside_mask(prob["geometry"], g)])
    assert 1.0 < mn and mx < 6.0
    pts = np.array([[0.0, 0.0], [0.3, -0.4], [-0.6, 0.5], [0.5, 0.5]])
    exact = np.exp(pts[:, 0]) * np.cos(pts[:, 1])
    o = oracle.solve(prob, pts, 10000, mx, seed=5, variant=3)
    z = (o["mean"] - exact) / o["se"]
    assert np.all(np.abs(z) < 4), z
