"""GPU parity of each step of the walk against the FP64 oracle, through the C ABI's
diagnostic entry points (they run the walker's own device functions)."""
import math

import numpy as np
import pytest
from scipy import special, stats

from paper_2201_13240_amd import workloads as WL
from tests.gpu_common import dev, torch_cuda

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def W():
    torch_cuda()
    from paper_2201_13240_amd import wos
    wos.lib()
    return wos


def test_philox_bit_exact(W, oracle):
    torch = torch_cuda()
    rng = np.random.default_rng(1)
    ctr = rng.integers(0, 2**32, size=(4096, 4), dtype=np.uint64).astype(np.uint32)
    key = int(rng.integers(0, 2**63))
    out = W.philox(torch.as_tensor(ctr.view(np.int32), device="cuda"), key).cpu().numpy().view(np.uint32)
    for i in range(0, 4096, 97):
        ref = oracle.philox(ctr[i].tolist(), [key & 0xFFFFFFFF, key >> 32])
        assert out[i].tolist() == ref


@pytest.mark.parametrize("precision,tol", [("fp64", 5e-15), ("fp32", 3e-6)])
def test_scaled_bessel(W, precision, tol):
    x = np.concatenate([np.geomspace(1e-6, 0.999, 300), np.linspace(1.0, 9.0, 400), np.geomspace(8.0, 2e4, 300)])
    xi = dev(x)
    i0e = W.eval_bessel("i0e", xi, precision).cpu().numpy()
    k0e = W.eval_bessel("k0e", xi, precision).cpu().numpy()
    np.testing.assert_allclose(i0e, special.i0e(x), rtol=tol)
    np.testing.assert_allclose(k0e, special.k0e(x), rtol=tol * (20 if precision == "fp32" else 2))
    # order 1 (off-centred Poisson kernel of the next-flight walk)
    i1e = W.eval_bessel("i1e", xi, precision).cpu().numpy()
    k1e = W.eval_bessel("k1e", xi, precision).cpu().numpy()
    np.testing.assert_allclose(i1e, special.i1e(x), rtol=tol * 2)
    np.testing.assert_allclose(k1e, special.k1e(x), rtol=tol * (20 if precision == "fp32" else 2))


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("sb", [0.0, 0.3, 4.0, 60.0, 3000.0])
def test_offcentred_kernels_match_oracle(W, oracle, dim, precision, sb):
    """G(x, y)|B| and P(x, z)|dB| of the next-flight walk (supplemental Sec. 1.2
    approximations) against the oracle's at uniform points of the ball; the error is
    measured against the kernel scale (R^2 for G|B|, 1 for P|dB|)."""
    rng = np.random.default_rng(int(10 * sb) + dim)
    R, n = 0.8, 4000
    d = rng.normal(size=(n, dim))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    u = d * (R * rng.uniform(0, 1, (n, 1)) ** (1 / dim))
    d2 = rng.normal(size=(n, dim))
    d2 /= np.linalg.norm(d2, axis=1, keepdims=True)
    v = d2 * (R * rng.uniform(0, 1, (n, 1)) ** (1 / dim))
    z = d2 * R
    g = W.eval_offcentred("green", dim, R, sb, dev(u), dev(v), precision).cpu().numpy()
    p = W.eval_offcentred("poisson", dim, R, sb, dev(u), dev(z), precision).cpu().numpy()
    vol = np.pi * R * R if dim == 2 else 4 / 3 * np.pi * R ** 3
    area = 2 * np.pi * R if dim == 2 else 4 * np.pi * R * R
    g_ref = oracle.nf_kernel("green", dim, u, v, R, sb) * vol
    p_ref = oracle.nf_kernel("poisson", dim, u, z, R, sb) * area
    tol = 1e-9 if precision == "fp64" else 1e-3
    eg = np.abs(g - g_ref) / np.maximum(np.abs(g_ref), 1e-3 * R * R)
    ep = np.abs(p - p_ref) / np.maximum(np.abs(p_ref), 1e-6)
    assert eg.max() < tol and ep.max() < tol, (eg.max(), ep.max())
    assert np.median(eg) < tol / 100 and np.median(ep) < tol / 100


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("precision,tol", [("fp64", 1e-13), ("fp32", 2e-6)])
def test_ball_normalisation(W, oracle, dim, precision, tol):
    s = np.concatenate([[0.0], np.geomspace(1e-4, 80.0, 200)])
    out = W.eval_ball(dim, dev(s), precision).cpu().numpy()
    for si, (pb, g) in zip(s, out):
        if si == 0:
            assert pb == 0 and g == pytest.approx(1 / (2 * dim), rel=1e-7)
            continue
        ref_pb = oracle.ball_pb(dim, si)
        # the oracle forms 1 - 1/I0(s) (1 - s/sinh s) directly: ~4e-16/P_B relative round-off,
        # and uses the leading term s^2/(2n) below s = 1e-4 (relative error ~s^2/8)
        rel = tol + 4e-16 / ref_pb + (si * si if si < 1e-4 else 0.0)
        assert pb == pytest.approx(ref_pb, rel=rel), (si, pb, ref_pb)
        # |G| of the unit ball = P_B / sigma_bar, sigma_bar = s^2
        assert g == pytest.approx(oracle.ball_gnorm(dim, 1.0, si * si), rel=rel)


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("s", [0.0, 1e-3, 0.5, 1.9, 2.1, 2.5, 6.0, 20.0, 55.0])
def test_green_sampler_matches_oracle_law(W, oracle, dim, precision, s):
    n = 100000
    t, trials = W.sample_radius(dim, s, n, seed=17, precision=precision)
    t = t.cpu().numpy()
    assert np.all((t > 0) & (t <= 1))
    ks = stats.kstest(t, lambda x: oracle.radial_cdf_many(dim, s, np.atleast_1d(x)))
    assert ks.pvalue > 1e-4, (dim, precision, s, ks)
    # expected proposals per sample: <= 1.8 by the envelope bounds (1 for the harmonic law)
    mean_trials = trials.item() / n
    assert 1.0 <= mean_trials < (1.02 if s == 0 and dim == 2 else 1.85)


CONFIGS = {
    "cfg1": lambda: WL.config1()["problems"][0],
    "cfg2": lambda: WL.config2(n_grid=8)["problems"][0],
    "cfg3": lambda: WL.config3(n_grid=4, subdiv=2)["problems"][0],
    "cfg5": lambda: WL.config5(n_grid=8)["problems"][0],
}


def _points(prob, n, seed=0):
    rng = np.random.default_rng(seed)
    return WL.sample_inside(rng, prob["geometry"], prob["dim"], n)


@pytest.mark.parametrize("name", sorted(CONFIGS))
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_coefficients_match_oracle(W, oracle, name, precision):
    prob = CONFIGS[name]()
    h = W.Problem(prob, sigma_bar=1.0)
    pts = _points(prob, 3000)
    if name == "cfg5":   # include points inside the steep layer
        pts[:500, 0] = 0.5 + np.linspace(-0.03, 0.03, 500)
    got = W.eval_coefficients(h, dev(pts), precision).cpu().numpy()
    ref = oracle.coefficients(prob, pts)
    # columns: alpha, gamma, sigma', f, f', g
    scale = np.maximum(np.abs(ref).max(0), 1.0)
    if precision == "fp64":
        np.testing.assert_allclose(got, ref, rtol=1e-10, atol=1e-10 * scale.max())
    else:
        err = np.abs(got - ref) / scale[None, :]
        assert np.max(err) < 2e-4, (name, np.max(err, 0))


GEOMS = {
    "disk": lambda: WL.make_problem(2, WL.geom_ball([0.1, -0.2], 1.3), *[WL.field_const(1.0)] * 5),
    "box3": lambda: WL.make_problem(3, WL.geom_box([0, 0, 0], [1, 2, 0.5]), *[WL.field_const(1.0)] * 5),
    "ball3": lambda: WL.make_problem(3, WL.geom_ball([0, 0, 0], 1.0), *[WL.field_const(1.0)] * 5),
    "star256": lambda: WL.config2(n_grid=8)["problems"][0],
    "star4096": lambda: WL.make_problem(2, WL.star_polygon(np.random.default_rng(9), 4096), *[WL.field_const(1.0)] * 5),
    "ico20480": lambda: WL.make_problem(3, WL.icosphere(np.random.default_rng(3000), 5, 0.1), *[WL.field_const(1.0)] * 5),
}


@pytest.mark.parametrize("name", sorted(GEOMS))
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_distance_matches_oracle(W, oracle, name, precision):
    prob = GEOMS[name]()
    if prob["alpha"]["base"] != "none":
        for k in ("alpha", "psi", "sigma", "source", "boundary"):
            prob[k] = WL.field_const(1.0)
    h = W.Problem(prob, sigma_bar=1.0)
    pts = _points(prob, 400 if name == "ico20480" else 3000, seed=4)
    d, xb = W.eval_distance(h, dev(pts), precision)
    d, xb = d.cpu().numpy(), xb.cpu().numpy()
    rd, rxb = oracle.distance(prob, pts)
    tol = 1e-12 if precision == "fp64" else 2e-6
    np.testing.assert_allclose(d, rd, atol=tol * 4)
    # the closest point is unique almost surely; it must lie at distance d
    np.testing.assert_allclose(np.linalg.norm(xb - pts, axis=1), rd, atol=tol * 8)
    np.testing.assert_allclose(xb, rxb, atol=1e-6 if precision == "fp64" else 5e-4)


@pytest.mark.parametrize("name", ["disk", "box3", "star256", "ico20480"])
def test_classify_matches_generator(W, name):
    prob = GEOMS[name]()
    for k in ("alpha", "psi", "sigma", "source", "boundary"):
        prob[k] = WL.field_const(1.0)
    h = W.Problem(prob, sigma_bar=1.0)
    rng = np.random.default_rng(5)
    V = prob["geometry"].get("vertices")
    lo, hi = (V.min(0), V.max(0)) if V is not None else (-2 * np.ones(prob["dim"]), 2 * np.ones(prob["dim"]))
    pts = rng.uniform(lo - 0.1, hi + 0.1, size=(3000 if name != "ico20480" else 500, prob["dim"]))
    got = W.classify(h, dev(pts)).cpu().numpy().astype(bool)
    ref = WL.inside_mask(prob["geometry"], pts)
    assert np.mean(got == ref) == 1.0


def test_sigma_bar_default_matches_oracle(W, oracle):
    prob = WL.config1()["problems"][0]
    h = W.Problem(prob, sigma_bar_grid=512)
    info = h.info()
    g = WL.grid_points(512, -1, 1)
    g = g[WL.inside_mask(prob["geometry"], g)]
    mn, mx = oracle.sigma_prime_range(prob, g)
    assert info["sigma_prime_min"] == pytest.approx(mn, rel=1e-9)
    assert info["sigma_prime_max"] == pytest.approx(mx, rel=1e-9)
    assert info["sigma_bar"] == pytest.approx(max(mx, 0) - min(mn, 0), rel=1e-9)
