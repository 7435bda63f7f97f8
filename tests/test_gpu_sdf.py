"""GPU walks on SDF/CSG domains (Sec. 7.2) through the C ABI: distance and exit point per
query against the oracle, inside classification, whole solves against the oracle and
against exact solutions (manufactured and harmonic data hold on any domain), next
flight, gradients, and progressive accumulation of one walk per point per frame."""
import numpy as np
import pytest

from paper_2201_13240_amd import workloads as WL
from tests.gpu_common import dev, gpu_solve, gpu_solve_grad, torch_cuda
from tests.parity import assert_parity
from tests.test_oracle_sdf import csg_scenes

pytestmark = pytest.mark.gpu

Z = WL.field_const(0.0)
ONE = WL.field_const(1.0)
SCENES = csg_scenes()


@pytest.fixture(scope="module")
def W():
    torch_cuda()
    from paper_2201_13240_amd import wos
    wos.lib()
    return wos


def tol(precision):
    return 1e-12 if precision == "fp64" else 2e-6


def _prob(geom, dim, sigma=Z, source=Z, boundary=Z, alpha=ONE, eps=1e-4):
    return WL.make_problem(dim, geom, alpha, Z, sigma, source, boundary, eps)


def _expcos(p):
    return np.exp(p[:, 0]) * np.cos(p[:, 1])


@pytest.mark.parametrize("name", list(SCENES))
def test_distance_and_exit_point_match_oracle(W, oracle, name):
    geom, dim = SCENES[name]
    prob = _prob(geom, dim)
    h = W.Problem(prob, sigma_bar=0.0)
    pts = WL.sample_inside(np.random.default_rng(1), geom, dim, 3000)
    d_o, x_o = oracle.distance(prob, pts)
    for precision, atol in (("fp64", 1e-12), ("fp32", 1e-5)):
        d, xb = W.eval_distance(h, dev(pts), precision)
        np.testing.assert_allclose(d.cpu().numpy(), d_o, rtol=0, atol=atol, err_msg=f"{name} {precision}")
        np.testing.assert_allclose(xb.cpu().numpy(), x_o, rtol=0, atol=atol, err_msg=f"{name} {precision}")


@pytest.mark.parametrize("name", list(SCENES))
def test_classification_matches_set_membership(W, oracle, name):
    geom, dim = SCENES[name]
    prob = _prob(geom, dim)
    h = W.Problem(prob, sigma_bar=0.0)
    lo, hi = geom["lo"], geom["hi"]
    pts = np.random.default_rng(2).uniform(lo - 0.1, hi + 0.1, size=(20000, dim))
    d, _ = oracle.distance(prob, pts)
    pts = pts[np.abs(d) > 1e-9]
    got = W.classify(h, dev(pts)).cpu().numpy().astype(bool)
    assert np.array_equal(got, WL.inside_mask(geom, pts))


def test_manufactured_variable_coefficients_cut_square(W, oracle):
    """alpha = 1 + 0.5 sin(2 pi x) sin(2 pi y), sigma = 1, f and g from u = e^x cos y:
    the exact solution on the CSG domain is u itself."""
    geom, dim = SCENES["cut-square"]
    alpha = WL.config1()["problems"][0]["alpha"]
    prob = _prob(geom, 2, sigma=ONE, source=WL.field_manufactured("expcos"),
                 boundary=WL.field_manufactured("expcos"), alpha=alpha)
    h = W.Problem(prob)
    pts = WL.sample_inside(np.random.default_rng(3), geom, 2, 48)
    o = oracle.solve(prob, pts, 1024, h.sigma_bar, seed=31)
    for precision in ("fp64", "fp32"):
        r = gpu_solve(W, h, pts, 1024, precision, seed=32)
        assert_parity(r["mean"], r["se"], o["mean"], o["se"], f"cut square vs oracle {precision}", tol(precision))
        gs, os_ = r["steps"].sum(), o["steps"].sum()
        assert abs(gs / os_ - 1) < 0.05, (gs, os_)
    r = gpu_solve(W, h, pts, 16384, "fp32", seed=33)
    ex = _expcos(pts)
    assert_parity(r["mean"], r["se"], ex, 0 * ex, "cut square vs exact", tol("fp32"))


def test_screened_cube_minus_ball(W, oracle):
    geom, dim = SCENES["cube-minus-ball"]
    prob = _prob(geom, 3, sigma=WL.field_const(4.0), source=WL.field_manufactured("expcos"),
                 boundary=WL.field_manufactured("expcos"))
    h = W.Problem(prob, sigma_bar=6.0)
    pts = WL.sample_inside(np.random.default_rng(4), geom, 3, 32)
    o = oracle.solve(prob, pts, 1024, 6.0, seed=41)
    for precision in ("fp64", "fp32"):
        r = gpu_solve(W, h, pts, 1024, precision, seed=42)
        assert_parity(r["mean"], r["se"], o["mean"], o["se"], f"cube minus ball vs oracle {precision}",
                      tol(precision))
    r = gpu_solve(W, h, pts, 16384, "fp32", seed=43)
    ex = _expcos(pts)
    assert_parity(r["mean"], r["se"], ex, 0 * ex, "cube minus ball vs exact", tol("fp32"))


@pytest.mark.parametrize("name", ["two-disks", "annulus"])
def test_harmonic_data_and_gradient(W, name):
    geom, dim = SCENES[name]
    prob = _prob(geom, 2, boundary=WL.field_manufactured("expcos"))
    h = W.Problem(prob)
    pts = WL.sample_inside(np.random.default_rng(5), geom, 2, 64)
    r = gpu_solve_grad(W, h, pts, 8192, "fp32", seed=51)
    ex = _expcos(pts)
    assert_parity(r["mean"], r["se"], ex, 0 * ex, f"{name} harmonic", tol("fp32"))
    gex = np.c_[np.exp(pts[:, 0]) * np.cos(pts[:, 1]), -np.exp(pts[:, 0]) * np.sin(pts[:, 1])]
    assert_parity(r["grad_mean"].ravel(), r["grad_se"].ravel(), gex.ravel(), 0 * gex.ravel(),
                  f"{name} gradient", tol("fp32"))


def test_next_flight_matches_oracle(W, oracle):
    geom, dim = SCENES["annulus"]
    prob = _prob(geom, 2, sigma=WL.field_const(9.0), source=WL.field_const(3.0),
                 boundary=WL.field_manufactured("expcos"))
    h = W.Problem(prob, sigma_bar=12.0)
    pts = WL.sample_inside(np.random.default_rng(6), geom, 2, 40)
    o = oracle.solve(prob, pts, 1024, 12.0, seed=61, variant=2)
    for precision in ("fp64", "fp32"):
        r = gpu_solve(W, h, pts, 1024, precision, seed=62, variant=2)
        assert_parity(r["mean"], r["se"], o["mean"], o["se"], f"next flight annulus {precision}", tol(precision))


def test_progressive_frames_equal_one_solve(W):
    """Sec. 7.2 accumulates one walk per point per frame. A plan of one walk per point
    replayed for 32 frames with walk offsets 0..31 adds up to one solve of 32 walks."""
    torch = torch_cuda()
    geom, dim = SCENES["cut-square"]
    alpha = WL.config1()["problems"][0]["alpha"]
    prob = _prob(geom, 2, sigma=ONE, source=WL.field_manufactured("expcos"),
                 boundary=WL.field_manufactured("expcos"), alpha=alpha)
    h = W.Problem(prob)
    g = WL.grid_points(64, -1.0, 1.0)
    P = dev(g[WL.inside_mask(geom, g)])
    acc = W.Accumulators(P.shape[0])
    plan = W.Plan([(h, P, acc, 0)], W.options(precision="fp32", walks=1, seed=0))
    means = []
    for frame in range(32):
        plan.launch(seed=77, walk_offset_add=frame)
        if frame in (0, 7, 31):
            m, _ = W.finalize(acc)
            means.append(m.cpu().numpy())
    torch.cuda.synchronize()
    ref = W.Accumulators(P.shape[0])
    W.solve([(h, P, ref, 0)], W.options(precision="fp32", walks=32, seed=77))
    torch.cuda.synchronize()
    np.testing.assert_allclose(acc.sum.cpu().numpy(), ref.sum.cpu().numpy(), rtol=1e-12, atol=1e-12)
    assert np.array_equal(acc.n_steps.cpu().numpy(), ref.n_steps.cpu().numpy())
    assert np.all(acc.n_walks.cpu().numpy() == 32)
    # the running estimate converges: error after 32 frames well below that after 1
    ex = _expcos(P.cpu().numpy())
    e = [np.sqrt(np.mean((m - ex) ** 2)) for m in means]
    assert e[2] < 0.5 * e[0], e


def test_cube_minus_ball_next_flight_and_gradient(W, oracle):
    """3D CSG domain: next flight against the oracle's next flight (screened data), and the
    gradient estimator against the exact gradient of harmonic data u = e^x cos y."""
    geom, dim = SCENES["cube-minus-ball"]
    prob = _prob(geom, 3, sigma=WL.field_const(4.0), source=WL.field_const(1.0),
                 boundary=WL.field_manufactured("expcos"))
    h = W.Problem(prob, sigma_bar=6.0)
    pts = WL.sample_inside(np.random.default_rng(9), geom, 3, 32)
    o = oracle.solve(prob, pts, 1024, 6.0, seed=91, variant=2)
    for precision in ("fp64", "fp32"):
        r = gpu_solve(W, h, pts, 1024, precision, seed=92, variant=2)
        assert_parity(r["mean"], r["se"], o["mean"], o["se"], f"next flight cube minus ball {precision}",
                      tol(precision))
    harm = _prob(geom, 3, boundary=WL.field_manufactured("expcos"))
    hh = W.Problem(harm)
    r = gpu_solve_grad(W, hh, pts, 8192, "fp32", seed=93)
    ex = _expcos(pts)
    assert_parity(r["mean"], r["se"], ex, 0 * ex, "cube minus ball harmonic", tol("fp32"))
    gex = np.c_[np.exp(pts[:, 0]) * np.cos(pts[:, 1]), -np.exp(pts[:, 0]) * np.sin(pts[:, 1]), 0 * pts[:, 0]]
    assert_parity(r["grad_mean"].ravel(), r["grad_se"].ravel(), gex.ravel(), 0 * gex.ravel(),
                  "cube minus ball gradient", tol("fp32"))
