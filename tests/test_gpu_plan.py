"""Plans: set-up times and the persistent cache of tuned launch shapes (the batched
schedule's autotuner, Sec. 3.1: walks are independent, so any shape gives the same
result)."""
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


def _plan(W, h, P, **kw):
    # 1024 walks per point on the 64^2 disk grid: more walks than the autotuner's sample
    # (eight per resident lane), so that the plan tunes its variant if no earlier plan did
    acc = W.Accumulators(P.shape[0])
    return W.Plan([(h, P, acc, 0)], W.options(precision="fp32", walks=1024, seed=3, **kw)), acc


def test_problem_setup_times(W):
    c = WL.config2(n_grid=64)
    h = W.Problem(c["problems"][0])
    t = h.setup_times()
    assert t["geometry_ms"] > 0 and t["sigma_bar_ms"] > 0 and t["upload_ms"] > 0
    assert all(np.isfinite(v) and v < 60e3 for v in t.values())


def test_tune_cache_round_trip(W, tmp_path):
    """A plan with the automatic shape tunes its walker variant (or finds it tuned); the
    saved file holds that variant; a file that names another shape for it makes the next
    plan use that shape without tuning, and the results do not depend on the shape."""
    torch = torch_cuda()
    c = WL.config1(n_grid=64)
    h = W.Problem(c["problems"][0])
    P = dev(c["points"][0])
    plan, acc = _plan(W, h, P)
    info0 = plan.info()
    st = plan.setup_times()
    assert st["build_ms"] > 0 and (st["tune_ms"] > 0) == st["tuned_here"]
    plan.launch(seed=5)
    ref = acc.sum.cpu().numpy().copy()
    plan.close()
    path = tmp_path / "tuned.txt"
    n = W.tune_cache_save(path)
    lines = [ln.split() for ln in path.read_text().splitlines() if not ln.startswith("#")]
    assert n == len(lines) >= 1
    # the disk's FP32 delta-tracking single-problem variant: dim 2, geometry 0, mode 0, batch 0
    mine = [ln for ln in lines if ln[2:8] == ["0", "0", "2", "0", "0", "0"]]
    assert len(mine) == 1 and [int(mine[0][8]), int(mine[0][9])] == [info0["block_size"], info0["tile_walks"]]
    # another shape for that variant, loaded from a file
    other = (128, 512) if (info0["block_size"], info0["tile_walks"]) != (128, 512) else (64, 1024)
    mine[0][8], mine[0][9] = str(other[0]), str(other[1])
    path.write_text("\n".join(" ".join(ln) for ln in lines) + "\n")
    assert W.tune_cache_load(path) >= 1
    plan, acc = _plan(W, h, P)
    assert (plan.info()["block_size"], plan.info()["tile_walks"]) == other
    assert plan.setup_times()["tuned_here"] is False and plan.setup_times()["tune_ms"] == 0
    plan.launch(seed=5)
    torch.cuda.synchronize()
    assert np.array_equal(acc.sum.cpu().numpy(), ref)    # exact sums: shape-independent
    plan.close()
    # restore the tuned shape for the tests that follow
    mine[0][8], mine[0][9] = str(info0["block_size"]), str(info0["tile_walks"])
    path.write_text("\n".join(" ".join(ln) for ln in lines) + "\n")
    W.tune_cache_load(path)
