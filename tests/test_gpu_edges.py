"""Edge cases of the GPU path through the C ABI: empty batch items next to full ones, a
single walk per point, query points inside the epsilon shell (Alg. 1 ends the walk at
once with g at the closest boundary point), an epsilon shell that covers the whole
domain, and tile tails that do not fill a wavefront."""
import numpy as np
import pytest

from paper_2201_13240_amd import workloads as WL
from tests.gpu_common import dev, gpu_solve, torch_cuda

pytestmark = pytest.mark.gpu

Z = WL.field_const(0.0)
ONE = WL.field_const(1.0)


@pytest.fixture(scope="module")
def W():
    torch_cuda()
    from paper_2201_13240_amd import wos
    wos.lib()
    return wos


def screened_disk(eps=1e-4):
    return WL.make_problem(2, WL.geom_ball([0.0, 0.0], 1.0), ONE, Z, WL.field_const(4.0), WL.field_const(1.0),
                           WL.field_manufactured("expcos"), eps)


def test_empty_items_next_to_full_ones(W):
    torch = torch_cuda()
    h = W.Problem(screened_disk())
    pts = WL.sample_inside(np.random.default_rng(1), WL.geom_ball([0.0, 0.0], 1.0), 2, 100)
    P = dev(pts)
    E = dev(np.zeros((0, 2)))
    alone = W.Accumulators(100)
    W.solve([(h, P, alone, 1)], W.options(precision="fp32", walks=64, seed=4))
    mixed = [W.Accumulators(0), W.Accumulators(100), W.Accumulators(0)]
    W.solve([(h, E, mixed[0], 0), (h, P, mixed[1], 1), (h, E, mixed[2], 2)],
            W.options(precision="fp32", walks=64, seed=4))
    only_empty = W.Accumulators(0)
    W.solve([(h, E, only_empty, 0)], W.options(precision="fp32", walks=64, seed=4))
    torch.cuda.synchronize()
    assert np.array_equal(mixed[1].sum.cpu().numpy(), alone.sum.cpu().numpy())
    assert np.array_equal(mixed[1].n_steps.cpu().numpy(), alone.n_steps.cpu().numpy())


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_single_walk_per_point(W, precision):
    h = W.Problem(screened_disk())
    pts = WL.sample_inside(np.random.default_rng(2), WL.geom_ball([0.0, 0.0], 1.0), 2, 77)
    r = gpu_solve(W, h, pts, 1, precision, seed=5)
    assert np.all(r["n"] == 1) and np.all(np.isfinite(r["mean"]))
    assert np.all(np.isnan(r["se"]))          # no spread from one sample
    assert np.all(r["steps"] >= 1)


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_points_in_the_epsilon_shell_end_at_once(W, precision):
    """A point closer than epsilon to the circle: every walk makes one distance query and
    returns g at the closest boundary point (Alg. 1), so the spread is zero."""
    eps = 1e-3
    h = W.Problem(screened_disk(eps))
    th = np.linspace(0.0, 2 * np.pi, 50, endpoint=False)
    r_in = 1.0 - np.array([0.0, 1e-5, 5e-4, 9e-4] * 13)[:50]
    pts = np.c_[r_in * np.cos(th), r_in * np.sin(th)]
    inside = np.linalg.norm(pts, axis=1) < 1.0
    pts = pts[inside]
    r = gpu_solve(W, h, pts, 32, precision, seed=6)
    assert np.all(r["steps"] == 32)
    xb = pts / np.linalg.norm(pts, axis=1, keepdims=True)
    g = np.exp(xb[:, 0]) * np.cos(xb[:, 1])
    tol = 1e-12 if precision == "fp64" else 2e-6
    np.testing.assert_allclose(r["mean"], g, rtol=tol, atol=tol)
    # identical samples: the one-pass variance (sum_sq/n - mean^2) leaves only its rounding,
    # about sqrt(1e-16) of the mean
    assert np.all(r["se"] <= 1e-7 * np.abs(g) + 1e-12)


def test_epsilon_shell_covering_the_domain(W):
    """epsilon above the inradius: every point is in the shell, every walk is one query."""
    h = W.Problem(screened_disk(eps=1.5))
    pts = WL.sample_inside(np.random.default_rng(3), WL.geom_ball([0.0, 0.0], 1.0), 2, 200)
    r = gpu_solve(W, h, pts, 16, "fp32", seed=7)
    assert np.all(r["steps"] == 16)
    assert np.all(r["counters"][1:3] == 0)


@pytest.mark.parametrize("n", [1, 63, 65, 129])
def test_tile_tails(W, n):
    """Point counts that leave a partly filled tile and wavefront: the sums equal those of
    the same points solved as part of a larger batch (per-walk values depend only on
    seed, problem, point and walk)."""
    torch = torch_cuda()
    h = W.Problem(screened_disk())
    pts = WL.sample_inside(np.random.default_rng(8), WL.geom_ball([0.0, 0.0], 1.0), 2, 200)
    big = W.Accumulators(200)
    W.solve([(h, dev(pts), big, 0)], W.options(precision="fp32", walks=3, seed=9, block_size=64, tile_walks=64))
    small = W.Accumulators(n)
    W.solve([(h, dev(pts[:n]), small, 0)], W.options(precision="fp32", walks=3, seed=9, block_size=64,
                                                     tile_walks=64))
    torch.cuda.synchronize()
    assert np.array_equal(small.sum.cpu().numpy(), big.sum.cpu().numpy()[:n])


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_sums_are_exact_sums_of_the_walks(W, precision):
    """The per-point sums (Sec. 3.1, eqs. 17-18) are exact: each walk's estimate is added
    as a fixed-point number with integer atomics, so a solve of N walks returns the exact
    sum of the N estimates rounded once (within one unit in the last place), whatever the
    order in which the walks ended. The estimates are taken one by one from N solves of
    one walk each (walk_offset j), whose sums are the estimates themselves."""
    from fractions import Fraction
    torch = torch_cuda()
    h = W.Problem(screened_disk(1e-3))
    pts = WL.sample_inside(np.random.default_rng(12), WL.geom_ball([0.0, 0.0], 1.0), 2, 40)
    P = dev(pts)
    n_w = 24
    single = []
    for j in range(n_w):
        a = W.Accumulators(40)
        W.solve([(h, P, a, 0)], W.options(precision=precision, walks=1, seed=3, walk_offset=j))
        single.append(a)
    full = W.Accumulators(40)
    W.solve([(h, P, full, 0)], W.options(precision=precision, walks=n_w, seed=3, block_size=64, tile_walks=64))
    torch.cuda.synchronize()
    v = np.stack([a.sum.cpu().numpy() for a in single])       # [walk][point]
    q = np.stack([a.sum_sq.cpu().numpy() for a in single])
    assert np.array_equal(q, v * v)                           # one walk: v^2 exactly
    got, got_sq = full.sum.cpu().numpy(), full.sum_sq.cpu().numpy()
    for i in range(40):
        exact = float(sum(Fraction(float(x)) for x in v[:, i]))
        exact_sq = float(sum(Fraction(float(x)) * Fraction(float(x)) for x in v[:, i]))
        assert abs(got[i] - exact) <= np.spacing(abs(exact)), (i, got[i], exact)
        assert abs(got_sq[i] - exact_sq) <= np.spacing(abs(exact_sq)), (i, got_sq[i], exact_sq)
    assert np.array_equal(full.n_steps.cpu().numpy(), sum(a.n_steps.cpu().numpy() for a in single))
