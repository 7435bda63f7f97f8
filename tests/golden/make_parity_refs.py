"""Writes the oracle references of the full-size parity tests (tests/golden/parity_*.npz).

Calls only the FP64 CPU oracle (oracle/oracle.py) and the seeded input generators
(paper_2201_13240_amd/workloads.py); nothing here comes from the GPU library. For each
workload at its full size it draws a seeded random sample of the query points, fixes
sigma_bar by the oracle's own sampling of sigma' (the default rule max(sigma'_max, 0) -
min(sigma'_min, 0) of Sec. 5.1 / Sec. 7.1, over a dense grid of interior points), and runs
the oracle's walks (Sec. 5.1, supplemental Alg. 1) at the sampled points as B batches,
twice, with independent seeds:

* run A (seed 1000 + k): the reference the GPU is compared with;
* run B (seed 2000 + k): a second oracle run of the same points, for the null
  calibration of the parity rule (tests/test_parity_rule.py).

Usage: python tests/golden/make_parity_refs.py [name ...]   (default: all workloads)
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_2201_13240_amd import workloads as WL  # noqa: E402

BATCHES = 32


def oracle_sigma_bar(prob, n_grid=512):
    """sigma_bar by the oracle: max(sigma'_max, 0) - min(sigma'_min, 0) over the interior
    points of an n_grid^2 (2D) or (n_grid/8)^3 (3D) grid over the bounding box."""
    g = prob["geometry"]
    dim = prob["dim"]
    lo, hi = WL._bbox(g, dim)
    if dim == 2:
        xs = [np.linspace(lo[i], hi[i], n_grid) for i in range(2)]
        P = np.stack(np.meshgrid(*xs, indexing="xy"), -1).reshape(-1, 2)
    else:
        m = n_grid // 8
        xs = [np.linspace(lo[i], hi[i], m) for i in range(3)]
        P = np.stack(np.meshgrid(*xs, indexing="ij"), -1).reshape(-1, 3)
    P = np.ascontiguousarray(P[WL.inside_mask(g, P)])
    return float(O.sigma_bar_default(prob, P))


# name -> (config builder, sample points per problem, walks per batch, solve options, seed of the sample)
WORKLOADS = {
    "star256": (WL.config2, 256, 64, {}, 20),
    "ico20480": (WL.config3, 128, 16, {"bvh": True}, 30),
    "batch64": (WL.config4, 4, 16, {"bvh": True}, 40),
    "square_rr": (WL.config5, 128, 32, {"russian_roulette": True}, 50),
}


def make(name):
    builder, per_problem, wpb, opts, sample_seed = WORKLOADS[name]
    c = builder()
    rng = np.random.default_rng(sample_seed)
    rec = {"idx": [], "problem": [], "sigma_bar": [], "run_a": [], "run_b": []}
    t0 = time.time()
    for k, (prob, pts) in enumerate(zip(c["problems"], c["points"])):
        inside = np.flatnonzero(WL.inside_mask(prob["geometry"], pts))
        idx = np.sort(rng.choice(inside, per_problem, replace=False))
        sb = oracle_sigma_bar(prob)
        opt = dict(opts, problem_index=k)
        a = O.solve_batches(prob, pts[idx], BATCHES, wpb, sb, seed=1000 + k, **opt)["batch_means"]
        b = O.solve_batches(prob, pts[idx], BATCHES, wpb, sb, seed=2000 + k, **opt)["batch_means"]
        rec["idx"].append(idx)
        rec["problem"].append(np.full(per_problem, k))
        rec["sigma_bar"].append(sb)
        rec["run_a"].append(a)
        rec["run_b"].append(b)
    out = os.path.join(HERE, f"parity_{name}.npz")
    np.savez_compressed(out, idx=np.concatenate(rec["idx"]), problem=np.concatenate(rec["problem"]),
                        sigma_bar=np.array(rec["sigma_bar"]), run_a=np.concatenate(rec["run_a"], 1),
                        run_b=np.concatenate(rec["run_b"], 1), walks_per_batch=wpb, batches=BATCHES,
                        options=json.dumps(opts))
    print(f"{name}: {sum(len(i) for i in rec['idx'])} points x {BATCHES} x {wpb} walks, twice, "
          f"{time.time() - t0:.1f} s -> {out}", flush=True)


if __name__ == "__main__":
    for name in (sys.argv[1:] or list(WORKLOADS)):
        make(name)
