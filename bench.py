"""Benchmark of the delta-tracking walk on spheres on one MI355X.

Workload: the 256-edge star polygon problem with random alpha, drift and sigma fields
(Gaussian-bump f and g), all query points of a 512 x 512 grid inside the domain, 1024
walks per point. One "step" of this benchmark is one full pass of the hot path over
that batch: a captured hipGraph replay of [tile-counter reset, persistent walker,
per-point reduction]. The metric is walk steps (distance queries) per second; points
per second at RMSE 1e-2 against the FP64 oracle is derived from the measured per-walk
variance. Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--walks", type=int, default=1024)
    ap.add_argument("--grid", type=int, default=512)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp32c", "fp64"])
    ap.add_argument("--fp64-steps", type=int, default=1, help="timed passes of the FP64 walker")
    ap.add_argument("--cpu-points", type=int, default=48, help="oracle sample size (0: skip)")
    ap.add_argument("--cpu-walks", type=int, default=1024)
    ap.add_argument("--no-events", action="store_true")
    return ap.parse_args()

# ----------------------------------------------------------------------------- cost model
# Algorithmic floating-point operations of one event of the walk (FMA = 2, add / sub /
# mul / div / min / max / compare = 1; sqrt, exp, log, sin and cos are counted apart as
# transcendental operations). The counts follow the arithmetic of the device functions
# in csrc/wos_device.h for the 2D FP32 walker; event totals come from the event-counting
# build of the walker (wos_count_events), so the FLOP figure is measured work times
# fixed per-event weights.

def _field_cost(f, dim, derivs):
    """(flops, transcendentals) of one evaluation of a field, with or without gradient and
    Laplacian."""
    b = f["base"]
    fl, tr = 0, 0
    if b == "fourier":
        n = len(f["a"])
        per = (2 * dim - 1) + 3 + 1 + ((3 + 2 * dim + 2) if derivs else 0)   # phase, value, sum, derivatives
        fl += n * per
        tr += n * (2 if derivs else 1)                                        # sin and cos, or cos only
    elif b == "bumps":
        n = len(f["amps"])
        per = dim + (2 * dim - 1) + 3 + ((2 * dim + 4) if derivs else 0)
        fl += n * per
        tr += n
    elif b in ("tanh", "tanh_drift"):
        fl += 12 if derivs else 6
        tr += 2
    if f["transform"] == "exp":
        fl += 2 + ((4 * dim + 4) if derivs else 0)
        tr += 1
    else:
        fl += 2 + ((dim + 1) if derivs else 0)
    return fl, tr


def event_weights(prob):
    dim = prob["dim"]
    af, at = _field_cost(prob["alpha"], dim, True)
    pf, pt = _field_cost(prob["psi"], dim, True) if prob["psi"]["base"] != "none" else (0, 0)
    sf, st = _field_cost(prob["sigma"], dim, False)
    if prob["source"]["base"] == "manufactured":
        ff, ft = 12 + 4 * dim, 3
    else:
        ff, ft = _field_cost(prob["source"], dim, False)
    coef = af + pf + sf + ff + (9 + 3 * dim) + (8 + 2 * dim) + 4     # ln-alpha derivatives, gamma, sigma'
    coef_t = at + pt + st + ft + (0 if prob["alpha"]["transform"] == "exp" else 1)
    ga_f = _field_cost(prob["alpha"], dim, False)
    ps_f = _field_cost(prob["psi"], dim, False) if prob["psi"]["base"] != "none" else (0, 0)
    gamma_only = (ga_f[0] + ps_f[0] + 2, ga_f[1] + ps_f[1])
    bf, bt = _field_cost(prob["boundary"], dim, False) if prob["boundary"]["base"] != "manufactured" else (6, 3)
    seg = 21 if dim == 2 else 75                                         # segment / triangle distance
    node = 2 * (3 * dim) + 2                                             # two child boxes + ordering
    W = {
        # per distance query: sqrt, epsilon test, ball radius
        "steps": (3, 1),
        "bvh_nodes": (node, 0),
        "grid_cells": (2 * dim + 4, 0),                                  # cell index of the query point
        "prims": (seg, 0),
        # per sampled ball: normalisation (series), direction, y, mu, coefficients at y, source
        "sampled": (73 + 2 + 5 + 1 + coef + 5, 1 + 2 + coef_t + 1),
        "ball_large_s": (42, 2),                                         # Chebyshev instead of series
        "trials": (78, 3),                                               # harmonic-law proposal
        "trials_free": (37, 1),                                          # free-space proposal, extra
        "volume": (3, 0),
        "exit": (6, 2),
        "terminal": (12 + bf + 4, bt + 1),
        "gamma_evals": gamma_only,
        "rr_draws": (4, 0),
    }
    return W


def algorithmic_work(events, prob):
    W = event_weights(prob)
    ev = dict(events)
    ev["sampled"] = ev["steps"] - ev["terminal"]
    flops = sum(W[k][0] * ev[k] for k in W)
    trans = sum(W[k][1] * ev[k] for k in W)
    return flops, trans


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}); "
              "the walk is embarrassingly parallel and would shard by walk range, see DESIGN.md",
              file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_2201_13240_amd import wos
    from paper_2201_13240_amd import workloads as WL

    torch.cuda.set_device(0)
    c = WL.config2(n_grid=args.grid)
    prob, pts = c["problems"][0], c["points"][0]
    n_pts = pts.shape[0]
    h = wos.Problem(prob)
    P = torch.as_tensor(pts, dtype=torch.float64, device="cuda")

    def run(precision, steps, warmup, walks):
        acc = wos.Accumulators(n_pts)
        plan = wos.Plan([(h, P, acc, 0)], wos.options(precision=precision, walks=walks, seed=0))
        for w in range(warmup):
            plan.launch(seed=1000 + w, walk_offset_add=0)
        torch.cuda.synchronize()
        for t in (acc.sum, acc.sum_sq, acc.n_walks, acc.n_steps, acc.counters):
            t.zero_()
        stream = torch.cuda.current_stream()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(steps):
            ev[k][0].record(stream)
            plan.launch(seed=k, walk_offset_add=k * walks)
            ev[k][1].record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ms = [a.elapsed_time(b) for a, b in ev]
        mean, se = wos.finalize(acc)
        torch.cuda.synchronize()
        info = plan.info()
        plan.close()
        print(f"bench: {precision} {steps} timed passes, ms/pass {np.round(ms, 2).tolist()}", file=sys.stderr,
              flush=True)
        return {"wall_s": wall, "ms": ms, "steps": int(acc.n_steps.sum().item()),
                "walks": int(acc.n_walks.sum().item()), "mean": mean.cpu().numpy(), "se": se.cpu().numpy(),
                "counters": acc.counters.cpu().numpy().tolist(), "plan": info}

    r32 = run(args.precision, args.steps, args.warmup, args.walks)

    # algorithmic work per distance query from the event-counting walker on a sample of
    # the same workload (every 8th query point, 64 walks each)
    sub = P[::8].contiguous()
    acc_c = wos.Accumulators(sub.shape[0])
    events = wos.count_events([(h, sub, acc_c, 0)], wos.options(precision=args.precision, walks=64, seed=99))
    flops_ev, trans_ev = algorithmic_work(events, prob)
    flops_per_step = flops_ev / events["steps"]
    trans_per_step = trans_ev / events["steps"]
    steps_per_pass = r32["steps"] / args.steps
    achieved = flops_per_step * steps_per_pass / (np.mean(r32["ms"]) / 1e3) / 1e12
    peak = 157.3 if args.precision != "fp64" else 78.6
    roofline = {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak,
                "traffic": None, "flops_per_step": flops_per_step, "transcendentals_per_step": trans_per_step,
                "events_per_step": {k: v / events["steps"] for k, v in events.items()}}
    r64 = run("fp64", args.fp64_steps, 0, args.walks) if args.fp64_steps > 0 else None
    ms_step = float(np.mean(r32["ms"]))
    steps_per_s = r32["steps"] / (sum(r32["ms"]) / 1e3)
    walks_per_pt = args.walks * args.steps

    # per-walk variance -> walks needed for RMSE 1e-2 (Sec. 3.1: RMSE = sqrt(mean var / N))
    var_walk = (r32["se"] ** 2) * walks_per_pt
    n_star = float(np.mean(var_walk)) / 1e-4
    t_walk_pass = (sum(r32["ms"]) / 1e3) / walks_per_pt          # seconds per walk per point (all points)
    pts_per_s_rmse = n_pts / (n_star * t_walk_pass)
    out64 = {}
    if r64 is not None:
        s64 = r64["steps"] / (sum(r64["ms"]) / 1e3)
        t64 = (sum(r64["ms"]) / 1e3) / (args.walks * args.fp64_steps)
        var64 = (r64["se"] ** 2) * args.walks * args.fp64_steps
        n64 = float(np.mean(var64)) / 1e-4
        out64 = {"fp64_steps_per_s": s64, "fp64_ms_per_step": float(np.mean(r64["ms"])),
                 "fp64_points_per_s_at_rmse_1e-2": n_pts / (n64 * t64)}

    # CPU baseline: the FP64 oracle on a bounded sample of the same workload; its
    # estimates are the reference for the RMSE of the GPU walkers at those points.
    cpu = None
    rmse = {}
    if args.cpu_points > 0:
        from oracle import oracle as O
        idx = np.random.default_rng(0).choice(n_pts, args.cpu_points, replace=False)
        threads = os.cpu_count() or 1
        t0 = time.perf_counter()
        o = O.solve(prob, pts[idx], args.cpu_walks, h.sigma_bar, seed=77, threads=threads)
        dt = time.perf_counter() - t0
        cpu = {"value": float(o["steps"].sum() / dt), "unit": "walk steps/s", "cores": threads,
               "kind": "oracle",
               "sample": f"{args.cpu_points} random query points x {args.cpu_walks} walks of the same workload, "
                         f"{dt:.1f} s"}
        for name, r in (("fp32", r32), ("fp64", r64)):
            if r is None:
                continue
            d2 = (r["mean"][idx] - o["mean"]) ** 2 - o["se"] ** 2
            rmse[name] = {"rmse_vs_oracle": float(math.sqrt(max(np.mean(d2), 0.0))),
                          "mean_se_gpu": float(np.mean(r["se"][idx])), "mean_se_oracle": float(np.mean(o["se"]))}

    line = {
        "metric": "walk steps/s and query pts/s at RMSE 1e-2 vs FP64 oracle (FP32 vs FP64 GPU)",
        "value": steps_per_s,
        "unit": "walk steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp32": "f32", "fp32c": "f32", "fp64": "f64"}[args.precision],
        "data": "synthetic",
        "config": {"workload": "star polygon 256 edges, 512x512 grid inside the domain, random alpha/drift/sigma "
                               "fields, Gaussian-bump f and g",
                   "query_points": n_pts, "walks_per_point": args.walks, "precision": args.precision,
                   "sigma_bar": h.sigma_bar, "plan": r32["plan"]},
        "points_per_s_at_rmse_1e-2": pts_per_s_rmse,
        "walks_for_rmse_1e-2": n_star,
        "steps_per_walk": r32["steps"] / r32["walks"],
        "counters": r32["counters"],
        "roofline": roofline,
        "cpu_baseline": cpu,
        "rmse": rmse,
    }
    line.update(out64)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
