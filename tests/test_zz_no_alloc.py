"""wos_solve_static (no device allocation, scratch in the library's static array) against
wos_solve through the C ABI: the same walks and exact sums, so the outputs agree bit for
bit, on two calls in a row, the second with fewer points (the array keeps the first
call's contents, which the second must not see); a job whose walks per point do not fit
at once runs in several launches and agrees to rounding; a job too large for the array
is rejected before any work."""
import numpy as np
import pytest

from paper_2201_13240_amd import workloads as WL
from tests.gpu_common import dev, torch_cuda

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def W():
    torch_cuda()
    from paper_2201_13240_amd import wos
    wos.lib()
    return wos


def _outputs(acc):
    return [t.cpu().numpy() for t in (acc.sum, acc.sum_sq, acc.n_walks, acc.n_steps, acc.counters)]


def _both(W, entries_pts, handles, walks, precision, **kw):
    """Runs wos_solve and wos_solve_static on the same items; returns both outputs."""
    torch = torch_cuda()
    out = []
    for fn in (W.solve, W.solve_static):
        accs = [W.Accumulators(P.shape[0]) for P in entries_pts]
        fn([(h, P, a, i) for i, (h, P, a) in enumerate(zip(handles, entries_pts, accs))],
           W.options(precision=precision, walks=walks, seed=11, **kw))
        torch.cuda.synchronize()
        out.append([_outputs(a) for a in accs])
    return out


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_static_matches_solve_twice_second_smaller(W, precision):
    c = WL.config4(n_problems=3, min_pts=500, max_pts=3000, max_edges=512)
    handles = [W.Problem(p) for p in c["problems"]]
    pts = [dev(q) for q in c["points"]]
    for k, cut in enumerate((None, 0.4)):
        P = pts if cut is None else [q[: max(1, int(cut * q.shape[0]))] for q in pts[:2]]
        a, b = _both(W, P, handles[: len(P)], 96 if k == 0 else 40, precision)
        for ia, ib in zip(a, b):
            for x, y in zip(ia, ib):
                assert np.array_equal(x, y, equal_nan=True)
        assert all(np.all(ia[2] == (96 if k == 0 else 40)) for ia in a)


def test_static_with_gradients_matches_solve(W):
    torch = torch_cuda()
    c = WL.config1(n_grid=24)
    h = W.Problem(c["problems"][0])
    P = dev(c["points"][0])
    res = []
    for fn in (W.solve, W.solve_static):
        acc = W.Accumulators(P.shape[0], grad_dim=2)
        fn([(h, P, acc, 0)], W.options(precision="fp32", walks=128, seed=3))
        torch.cuda.synchronize()
        res.append([t.cpu().numpy() for t in (acc.sum, acc.grad_sum, acc.grad_sum_sq, acc.n_steps)])
    for x, y in zip(*res):
        assert np.array_equal(x, y)


def test_static_splits_walks_that_do_not_fit(W):
    """300,000 points x 2048 walks at tiles of 64 walks need 32 slots of 128 bytes per
    point, far beyond the array: the static path runs the walks in several launches; each
    launch rounds its exact sums once, so the sums agree with wos_solve to rounding and
    the step counts exactly."""
    torch = torch_cuda()
    g = WL.geom_ball([0.0, 0.0], 1.0)
    prob = WL.make_problem(2, g, WL.field_const(1.0), WL.field_const(0.0), WL.field_const(4.0),
                           WL.field_const(1.0), WL.field_manufactured("expcos"), 1e-3)
    h = W.Problem(prob)
    P = dev(WL.sample_inside(np.random.default_rng(4), g, 2, 300000))
    (a,), (b,) = _both(W, [P], [h], 2048, "fp32", tile_walks=64)
    np.testing.assert_allclose(b[0], a[0], rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(b[1], a[1], rtol=1e-13, atol=1e-13)
    assert np.array_equal(a[2], b[2]) and np.array_equal(a[3], b[3])
    del P
    torch.cuda.synchronize()


def test_static_rejects_a_job_too_large(W):
    """1.5 million points need more than the 128 MiB array: refused before any work, and
    the outputs are left untouched."""
    torch = torch_cuda()
    h = W.Problem(WL.make_problem(2, WL.geom_ball([0.0, 0.0], 1.0), WL.field_const(1.0), WL.field_const(0.0),
                                  WL.field_const(0.0), WL.field_const(0.0), WL.field_const(1.0), 1e-3))
    P = torch.zeros((1500000, 2), dtype=torch.float64, device="cuda")
    acc = W.Accumulators(P.shape[0])
    with pytest.raises(W.WosError, match="static scratch"):
        W.solve_static([(h, P, acc, 0)], W.options(precision="fp32", walks=4, seed=1))
    torch.cuda.synchronize()
    assert float(acc.n_walks.sum().item()) == 0.0
