"""Writes the oracle reference of the RMSE-versus-walks sweep on the high-contrast square
(tests/golden/sweep_square_rr.npz).

Calls only the FP64 CPU oracle (oracle/oracle.py) and the seeded input generators
(paper_2201_13240_amd/workloads.py); nothing here comes from the GPU library. The
workload is the high-contrast unit square (alpha jumping from 1 to 100 across a tanh
layer of width 0.01, drift (50, 0), sigma in [100, 1000]) with the static weight window's
Russian roulette (Sec. 6). At a seeded random sample of its 256 x 256 query points the
oracle runs WALKS walks per point (Sec. 5.1, supplemental Alg. 1) with the sigma_bar it
fixes by its own sampling of sigma' (as tests/golden/make_parity_refs.py does), and stores
the per-point mean and standard error (Sec. 3.1, eqs. 17-18).

Usage: python tests/golden/make_sweep_ref.py [threads]
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, HERE)

from make_parity_refs import oracle_sigma_bar  # noqa: E402
from oracle import oracle as O  # noqa: E402
from paper_2201_13240_amd import workloads as WL  # noqa: E402

POINTS = 48
WALKS = 32768
SEED_SAMPLE = 60
SEED_WALKS = 3000


def main():
    threads = int(sys.argv[1]) if len(sys.argv) > 1 else 0
    c = WL.config5()
    prob, pts = c["problems"][0], c["points"][0]
    inside = np.flatnonzero(WL.inside_mask(prob["geometry"], pts))
    idx = np.sort(np.random.default_rng(SEED_SAMPLE).choice(inside, POINTS, replace=False))
    sb = oracle_sigma_bar(prob)
    t0 = time.time()
    o = O.solve(prob, pts[idx], WALKS, sb, seed=SEED_WALKS, russian_roulette=True, threads=threads)
    out = os.path.join(HERE, "sweep_square_rr.npz")
    np.savez_compressed(out, idx=idx, sigma_bar=np.array([sb]), mean=o["mean"], se=o["se"], walks=WALKS,
                        steps=o["steps"])
    print(f"{POINTS} points x {WALKS} walks, {time.time() - t0:.1f} s, median se {np.median(o['se']):.2e} -> {out}",
          flush=True)


if __name__ == "__main__":
    main()
