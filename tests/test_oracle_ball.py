"""Pins of the oracle's ball kernels (supplemental Sec. 1.1 and 1.4): the centred
screened-Poisson Green's function, its integral |G|, the Poisson-kernel identity, and
the radial law used to sample y ~ G/|G|. References are built independently from
scipy.special Bessel functions and numerical quadrature."""
import math

import numpy as np
import pytest
from scipy import integrate, special

S_VALUES = [1e-3, 0.05, 0.5, 1.0, 2.0, 4.0, 10.0, 30.0, 55.0]


@pytest.mark.parametrize("which,ref", [("i0", special.i0), ("i1", special.i1),
                                       ("k0", special.k0), ("k1", special.k1)])
def test_bessel_matches_scipy(oracle, which, ref):
    for x in np.geomspace(1e-6, 300.0, 120):
        a, b = oracle.bessel(which, x), float(ref(x))
        assert abs(a - b) <= 1e-12 * abs(b), (which, x, a, b)


def green(dim, r, R, sigma):
    """Centred Green's function of Laplace - sigma on the ball (supp. Sec. 1.1)."""
    k = math.sqrt(sigma)
    if dim == 2:
        if sigma == 0:
            return math.log(R / r) / (2 * math.pi)
        return (special.k0(k * r) - special.k0(k * R) / special.i0(k * R) * special.i0(k * r)) / (2 * math.pi)
    if sigma == 0:
        return (1 / r - 1 / R) / (4 * math.pi)
    return (math.exp(-k * r) / r - math.exp(-k * R) / R * (math.sinh(k * r) / (k * r)) * (k * R / math.sinh(k * R))) / (4 * math.pi)


def gnorm_quad(dim, R, sigma):
    if dim == 2:
        f = lambda r: 2 * math.pi * r * green(2, r, R, sigma)
    else:
        f = lambda r: 4 * math.pi * r * r * green(3, r, R, sigma)
    pts = [R / math.sqrt(sigma)] if sigma > 0 and 1 / math.sqrt(sigma) < R else None
    return integrate.quad(f, 0, R, limit=400, epsabs=0, epsrel=1e-13, points=pts)[0]


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("R,sigma", [(0.3, 2.0), (1.0, 50.0), (2.0, 0.01), (0.5, 1e4), (1.0, 0.0)])
def test_gnorm_matches_quadrature(oracle, dim, R, sigma):
    q = gnorm_quad(dim, R, sigma)
    g = oracle.ball_gnorm(dim, R, sigma)
    assert abs(g - q) <= 1e-9 * q, (g, q)


def test_gnorm_harmonic_limits(oracle):
    for R in (0.1, 1.0, 3.0):
        assert oracle.ball_gnorm(2, R, 0.0) == pytest.approx(R * R / 4, rel=1e-15)
        assert oracle.ball_gnorm(3, R, 0.0) == pytest.approx(R * R / 6, rel=1e-15)
        # continuity across the small-s switch of the oracle
        for dim, c in ((2, 4), (3, 6)):
            lo = oracle.ball_gnorm(dim, R, (0.99e-4 / R) ** 2)
            hi = oracle.ball_gnorm(dim, R, (1.01e-4 / R) ** 2)
            assert abs(lo - hi) <= 1e-7 * R * R / c


@pytest.mark.parametrize("dim", [2, 3])
def test_poisson_kernel_identity(oracle, dim):
    # P = -dG/dr at r = R (inward normal derivative) equals (1 - sigma |G|)/|dB|
    for R, sigma in ((0.7, 3.0), (1.0, 40.0), (0.2, 0.5)):
        h = 1e-6 * R
        # second-order one-sided difference for dG/dr at r = R
        dGdr = (3 * green(dim, R, R, sigma) - 4 * green(dim, R - h, R, sigma) + green(dim, R - 2 * h, R, sigma)) / (2 * h)
        area = 2 * math.pi * R if dim == 2 else 4 * math.pi * R * R
        pb = sigma * oracle.ball_gnorm(dim, R, sigma)
        assert -dGdr == pytest.approx((1 - pb) / area, rel=1e-5)
        assert 0 < pb < 1


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("s", S_VALUES + [0.0])
def test_radial_cdf_matches_quadrature(oracle, dim, s):
    R = 1.0
    sigma = s * s
    norm = gnorm_quad(dim, R, sigma)
    w = (lambda r: 2 * math.pi * r * green(2, r, R, sigma)) if dim == 2 else \
        (lambda r: 4 * math.pi * r * r * green(3, r, R, sigma))
    for t in (0.01, 0.1, 0.3, 0.5, 0.8, 0.99):
        q = integrate.quad(w, 0, t, limit=400, epsabs=0, epsrel=1e-12)[0] / norm
        c = oracle.radial_cdf(dim, s, t)
        assert abs(c - q) <= 2e-8 + 1e-8 * q, (dim, s, t, c, q)
        # density is the derivative of the CDF
        # (the central difference itself carries ~1e-16/(s^2 h) round-off at small s)
        h = 1e-4 / max(1.0, s)
        fd = (oracle.radial_cdf(dim, s, t + h) - oracle.radial_cdf(dim, s, t - h)) / (2 * h)
        assert oracle.radial_pdf(dim, s, t) == pytest.approx(fd, rel=1e-5, abs=2e-6 if s >= 0.01 else 1e-5)
    assert oracle.radial_cdf(dim, s, 1.0) == 1.0 and oracle.radial_cdf(dim, s, 0.0) == 0.0


def test_radial_harmonic_special_cases(oracle):
    # sigma -> 0: 2D law t^2 (1 - 2 ln t) (density 4 t ln(1/t)); 3D Beta(2, 2)
    for t in (0.05, 0.3, 0.7, 0.95):
        assert oracle.radial_cdf(2, 0.0, t) == pytest.approx(t * t * (1 - 2 * math.log(t)), rel=1e-14)
        assert oracle.radial_cdf(3, 0.0, t) == pytest.approx(3 * t * t - 2 * t ** 3, rel=1e-14)
        # small but nonzero s approaches the harmonic law
        assert oracle.radial_cdf(2, 2e-3, t) == pytest.approx(t * t * (1 - 2 * math.log(t)), rel=1e-5)
        assert oracle.radial_cdf(3, 2e-3, t) == pytest.approx(3 * t * t - 2 * t ** 3, rel=1e-5)


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("s", [1e-4, 0.1, 1.0, 4.0, 10.0, 55.0])
def test_radial_quantile_inverts_and_ks(oracle, dim, s):
    from scipy import stats
    rng = np.random.default_rng(11)
    u = rng.uniform(size=3000)
    t = np.array([oracle.radial_quantile(dim, s, x) for x in u])
    back = np.array([oracle.radial_cdf(dim, s, x) for x in t])
    # the closed-form CDF carries ~1e-16/s^2 round-off, which bounds the inversion accuracy
    assert np.max(np.abs(back - u)) < max(1e-12, 2e-15 / s**2)
    # KS against the quadrature CDF (independent of the oracle's closed form)
    R, sigma = 1.0, s * s
    norm = gnorm_quad(dim, R, sigma)
    w = (lambda r: 2 * math.pi * r * green(2, r, R, sigma)) if dim == 2 else \
        (lambda r: 4 * math.pi * r * r * green(3, r, R, sigma))
    grid = np.linspace(0, 1, 201)
    cdf = np.concatenate([[0.0], np.cumsum([integrate.quad(w, a, b, epsrel=1e-12)[0]
                                            for a, b in zip(grid[:-1], grid[1:])])]) / norm
    ks = stats.kstest(t, lambda x: np.interp(x, grid, cdf))
    assert ks.pvalue > 1e-3
