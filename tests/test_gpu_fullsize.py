"""Parity at the workloads' full sizes, in the launch configuration the benchmark times:
one autotuned plan over every query point of the workload, replayed as a captured graph,
with the oracle computing a random sample of the points one by one (its own walks, the
same count per point), compared per point within the statistical bound of
tests/parity.py.

* star polygon, 256 edges: 124,319 points x 1024 walks, FP32 and FP64 (the benchmark pass);
* perturbed icosphere, 20,480 triangles: 676,691 points on the z = 0 slice x 256 walks, FP32;
* batch of 64 polygons (16-4096 edges): 2.65e6 points x 512 walks in one plan, FP32;
* high-contrast square: 65,536 points x 1024 walks with Russian roulette, FP32, FP32
  with compensated sums and FP64."""
import numpy as np
import pytest

from paper_2201_13240_amd import workloads as WL
from tests.gpu_common import dev, torch_cuda
from tests.parity import assert_parity

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def W():
    torch_cuda()
    from paper_2201_13240_amd import wos
    wos.lib()
    return wos


def tol(precision):
    return 1e-12 if precision == "fp64" else 2e-6


def plan_solve(W, items, walks, precision, seed, **kw):
    """items: [(problem handle, points)]; one plan over all of them, one replay."""
    torch = torch_cuda()
    entries = []
    for i, (h, pts) in enumerate(items):
        P = dev(pts)
        entries.append((h, P, W.Accumulators(P.shape[0]), i))
    plan = W.Plan(entries, W.options(precision=precision, walks=walks, seed=0, **kw))
    plan.launch(seed=seed)
    out = []
    for _, _, acc, _ in entries:
        mean, se = W.finalize(acc)
        torch.cuda.synchronize()
        out.append((mean.cpu().numpy(), se.cpu().numpy(), acc.counters.cpu().numpy()))
    plan.close()
    return out


def test_star_polygon_full(W, oracle):
    c = WL.config2()
    prob, pts = c["problems"][0], c["points"][0]
    assert pts.shape[0] == 124319
    h = W.Problem(prob)
    idx = np.random.default_rng(20).choice(pts.shape[0], 64, replace=False)
    o = oracle.solve(prob, pts[idx], 1024, h.sigma_bar, seed=21)
    for precision in ("fp32", "fp64"):
        (mean, se, cnt), = plan_solve(W, [(h, pts)], 1024, precision, seed=22)
        assert np.all(np.isfinite(mean)) and cnt[0] == 0 and cnt[1] == 0
        assert_parity(mean[idx], se[idx], o["mean"], o["se"], f"star polygon full {precision}", tol(precision))


def test_icosphere_slice_full(W, oracle):
    c = WL.config3()
    prob, pts = c["problems"][0], c["points"][0]
    assert pts.shape[0] == 676691
    h = W.Problem(prob)
    idx = np.random.default_rng(30).choice(pts.shape[0], 16, replace=False)
    o = oracle.solve(prob, pts[idx], 256, h.sigma_bar, seed=31)
    (mean, se, cnt), = plan_solve(W, [(h, pts)], 256, "fp32", seed=32)
    assert np.all(np.isfinite(mean)) and cnt[0] == 0 and cnt[1] == 0
    assert_parity(mean[idx], se[idx], o["mean"], o["se"], "icosphere full fp32", tol("fp32"))


def test_batch_of_64_polygons_full(W, oracle):
    c = WL.config4()
    assert len(c["problems"]) == 64
    handles = [W.Problem(p) for p in c["problems"]]
    res = plan_solve(W, list(zip(handles, c["points"])), 512, "fp32", seed=42)
    rng = np.random.default_rng(40)
    gm, gs, om, os_ = [], [], [], []
    for i, (p, pts, h, (mean, se, cnt)) in enumerate(zip(c["problems"], c["points"], handles, res)):
        assert np.all(np.isfinite(mean)) and cnt[0] == 0 and cnt[1] == 0
        idx = rng.choice(pts.shape[0], 2, replace=False)
        o = oracle.solve(p, pts[idx], 512, h.sigma_bar, seed=41, problem_index=i)
        gm.append(mean[idx])
        gs.append(se[idx])
        om.append(o["mean"])
        os_.append(o["se"])
    assert_parity(np.concatenate(gm), np.concatenate(gs), np.concatenate(om), np.concatenate(os_),
                  "64-polygon batch full fp32", tol("fp32"))


def test_high_contrast_square_full(W, oracle):
    c = WL.config5()
    prob, pts = c["problems"][0], c["points"][0]
    assert pts.shape[0] == 65536
    h = W.Problem(prob)
    idx = np.random.default_rng(50).choice(pts.shape[0], 32, replace=False)
    o = oracle.solve(prob, pts[idx], 1024, h.sigma_bar, seed=51, russian_roulette=True)
    for precision in ("fp32", "fp32c", "fp64"):
        (mean, se, cnt), = plan_solve(W, [(h, pts)], 1024, precision, seed=52, russian_roulette=True)
        assert np.all(np.isfinite(mean)) and cnt[0] == 0 and cnt[1] == 0
        assert_parity(mean[idx], se[idx], o["mean"], o["se"], f"high-contrast square full {precision}",
                      tol(precision))
