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
    ap.add_argument("--fp32c-steps", type=int, default=1,
                    help="timed passes of the FP32 walker with compensated per-walk sums")
    ap.add_argument("--ttr", type=int, default=1,
                    help="also measure time to RMSE 1e-2 by doubling walks per point (0: skip)")
    ap.add_argument("--cpu-points", type=int, default=96, help="oracle sample size (0: skip)")
    ap.add_argument("--cpu-walks", type=int, default=8192)
    ap.add_argument("--no-events", action="store_true")
    ap.add_argument("--variants", type=int, default=1,
                    help="also time next flight against delta tracking on the high-contrast square (0: skip)")
    ap.add_argument("--extras", type=int, default=1,
                    help="also time gradients, weight-window splitting and an SDF/CSG scene (0: skip)")
    ap.add_argument("--shape", default="auto",
                    help="walker launch shape: 'auto' (the plan autotunes block size and tile length) or "
                         "BLOCKxTILE, e.g. 256x256 (profiling runs pin the tuned shape so that no tuning "
                         "dispatches enter the kernel statistics)")
    # profiling helpers (each does only this and exits)
    ap.add_argument("--copy-probe", action="store_true",
                    help="run one 1 GiB device-to-device copy: the calibration kernel for FETCH_SIZE/WRITE_SIZE")
    ap.add_argument("--summarize-trace", nargs="+", metavar=("DB", "SUBSTR"),
                    help="print the kernel table of a rocprofv3 --kernel-trace --stats results.db")
    ap.add_argument("--summarize-pmc", nargs="+", metavar=("SUBSTR", "DB"),
                    help="print per-dispatch counter values of matching kernels from rocprofv3 --pmc results.db files")
    ap.add_argument("--write-traffic", nargs=4, metavar=("WALKER_FETCH_DB", "WALKER_WRITE_DB", "COPY_FETCH_DB",
                                                         "COPY_WRITE_DB"),
                    help="write profiles/walker_star256_traffic.json from four --pmc runs")
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


# ----------------------------------------------------------------------------- HBM traffic
# Measured HBM bytes of the walker come from rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE,
# KiB per dispatch) of this benchmark, committed as JSON under profiles/ together with
# the same counters read for a copy of known size (the calibration factors) and a hash of
# the device sources the counters were taken with. A changed kernel makes them stale:
# traffic is then reported as null.
DEVICE_SOURCES = ("wos_kernels.hip", "wos_device.h", "wos_types.h", "bessel_tables.h")


def device_source_hash():
    import hashlib
    h = hashlib.sha256()
    for name in DEVICE_SOURCES:
        with open(os.path.join(ROOT, "paper_2201_13240_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def walker_kernel_name(precision):
    """Name of the delta-tracking walker on the 2-D polygon domain as the profiler reports it."""
    return "walker_kernel_%s<2, 2, false, 0>" % precision


def traffic_of(kernel):
    path = os.path.join(ROOT, "profiles", "walker_star256_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("device_source_hash") != device_source_hash():
        return None
    k = rec.get("kernels", {}).get(kernel)
    if k is None:
        return None
    cal = rec["copy_calibration"]
    fetch = k["FETCH_SIZE_KiB"] * 1024 * cal["fetch_bytes_per_counted_byte"]
    write = k["WRITE_SIZE_KiB"] * 1024 * cal["write_bytes_per_counted_byte"]
    return {"bytes_per_launch": fetch + write, "fetch_bytes": fetch, "write_bytes": write,
            "source": "profiles/walker_star256_traffic.json"}


# ----------------------------------------------------------------------------- profile summaries
def summarize_trace(db, pattern=""):
    """Kernel table of a rocprofv3 --kernel-trace --stats database (durations there are in
    microseconds)."""
    import sqlite3
    cur = sqlite3.connect(db).cursor()
    rows = list(cur.execute("select name, total_calls, total_duration, average, percentage from top_kernels"))
    out = ["| kernel | calls | total ms | average ms | % |", "|---|---|---|---|---|"]
    for name, calls, tot, avg, pct in rows:
        if pattern and pattern not in name:
            continue
        out.append(f"| `{name.split('(')[0]}` | {calls} | {tot / 1e3:.3f} | {avg / 1e3:.3f} | {pct:.2f} |")
    return "\n".join(out)


def pmc_values(pattern, dbs):
    """Counter values per dispatch (mean over the matching dispatches of each run) of the
    kernels whose name contains `pattern`, with the kernel's resource figures."""
    import sqlite3
    from collections import defaultdict
    vals = defaultdict(float)
    info = {}
    for db in dbs:
        cur = sqlite3.connect(db).cursor()
        q = ("select kernel_name, dispatch_id, counter_name, value, vgpr_count, sgpr_count, scratch_size, grid_size, "
             "workgroup_size from counters_collection")
        per_dispatch = defaultdict(lambda: defaultdict(float))
        for name, did, cname, v, vg, sg, scr, grid, wg in cur.execute(q):
            if pattern not in name:
                continue
            per_dispatch[did][cname] += v
            info = {"kernel": name.split("(")[0], "vgpr": vg, "sgpr": sg, "scratch": scr, "grid": grid,
                    "workgroup": wg}
        n = max(1, len(per_dispatch))
        for d in per_dispatch.values():
            for k, v in d.items():
                vals[k] += v / n
    return dict(vals), info


def summarize_pmc(pattern, dbs):
    vals, info = pmc_values(pattern, dbs)
    lines = [f"kernel `{info.get('kernel')}`: grid {info.get('grid')}, workgroup {info.get('workgroup')}, "
             f"VGPRs {info.get('vgpr')}, SGPRs {info.get('sgpr')}, scratch {info.get('scratch')} B/lane", "",
             "| counter | value per dispatch |", "|---|---|"]
    for k in sorted(vals):
        lines.append(f"| {k} | {vals[k]:.6g} |")
    return "\n".join(lines)


def write_traffic(walker_fetch, walker_write, copy_fetch, copy_write):
    copy_bytes = float(1 << 30)
    cf = pmc_values("copyBuffer", [copy_fetch])[0]["FETCH_SIZE"]
    cw = pmc_values("copyBuffer", [copy_write])[0]["WRITE_SIZE"]
    rec = {"device_source_hash": device_source_hash(),
           "copy_calibration": {"copy_bytes": copy_bytes, "FETCH_SIZE_KiB": cf, "WRITE_SIZE_KiB": cw,
                                "fetch_bytes_per_counted_byte": copy_bytes / (cf * 1024),
                                "write_bytes_per_counted_byte": copy_bytes / (cw * 1024)},
           "kernels": {}}
    for prec in ("fp32", "fp64"):
        name = walker_kernel_name(prec)
        f = pmc_values(name, [walker_fetch])[0].get("FETCH_SIZE")
        w = pmc_values(name, [walker_write])[0].get("WRITE_SIZE")
        if f is not None and w is not None:
            rec["kernels"][name] = {"FETCH_SIZE_KiB": f, "WRITE_SIZE_KiB": w}
    path = os.path.join(ROOT, "profiles", "walker_star256_traffic.json")
    with open(path, "w") as fh:
        json.dump(rec, fh, indent=1)
    print(json.dumps(rec, indent=1))


def copy_probe():
    import torch
    n = 1 << 28   # float32 elements: 1 GiB
    a = torch.ones(n, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    print("copied bytes", n * 4, flush=True)


def compare_variants(wos, WL, args):
    """Next flight (Sec. 5.2) against delta tracking (Sec. 5.1) on the high-contrast unit
    square: 65,536 query points, sigma_bar about 1.2e4, where delta tracking takes many
    short steps. Both FP32 at the same walks per point, one captured plan each; reports
    pass time, distance queries per walk, per-walk variance, points per second at RMSE
    1e-2 from that variance, and how far the two means are apart in combined standard
    errors. On this problem sigma' < 0 in places and R sqrt(sigma_bar) is large, where
    next flight's in-ball series has no finite variance, so only its time and distance
    queries compare directly."""
    import torch
    c = WL.config5()
    prob, pts = c["problems"][0], c["points"][0]
    n = pts.shape[0]
    h = wos.Problem(prob)
    P = torch.as_tensor(pts, dtype=torch.float64, device="cuda")
    walks = 256
    out = {"workload": "unit square, alpha tanh jump 1..100, omega = (50, 0), sigma in [100, 1000], "
                       "256x256 points", "walks_per_point": walks, "sigma_bar": h.sigma_bar}
    res = {}
    for name, variant, rr in (("delta_tracking", 0, True), ("next_flight", 2, False)):
        acc = wos.Accumulators(n)
        plan = wos.Plan([(h, P, acc, 0)], wos.options(precision="fp32", walks=walks, seed=0, variant=variant,
                                                      russian_roulette=rr))
        plan.launch(seed=99)
        torch.cuda.synchronize()
        for t in (acc.sum, acc.sum_sq, acc.n_walks, acc.n_steps, acc.counters):
            t.zero_()
        ms = []
        for k in range(3):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            plan.launch(seed=k, walk_offset_add=k * walks)
            b.record()
            torch.cuda.synchronize()
            ms.append(a.elapsed_time(b))
        mean, se = wos.finalize(acc)
        torch.cuda.synchronize()
        plan.close()
        nw = float(acc.n_walks[0].item())
        var = float(np.mean((se.cpu().numpy() ** 2) * nw))
        t_walk = (np.mean(ms) / 1e3) / walks
        res[name] = (mean.cpu().numpy(), se.cpu().numpy())
        out[name] = {"ms_per_pass": float(np.mean(ms)),
                     "distance_queries_per_walk": float(acc.n_steps.sum().item()) / (nw * n),
                     "ball_samples_per_walk": float(acc.counters[3].item()) / (nw * n),
                     "per_walk_variance": var,
                     "points_per_s_at_rmse_1e-2": n / ((var / 1e-4) * t_walk)}
        print(f"bench: {name} on the high-contrast square, ms/pass {np.round(ms, 2).tolist()}", file=sys.stderr,
              flush=True)
    (m0, s0), (m1, s1) = res["delta_tracking"], res["next_flight"]
    z = (m1 - m0) / np.sqrt(s0 ** 2 + s1 ** 2)
    out["mean_abs_z_next_flight_vs_delta_tracking"] = float(np.mean(np.abs(z)))
    out["mean_abs_difference"] = float(np.mean(np.abs(m1 - m0)))
    return out


def _timed_plan(wos, torch, prob_handle, P, opt_kw, walks, reps, grad_dim=0):
    """Creates a plan of one item, warms it up, then times `reps` graph replays with HIP
    events on the current stream; returns timings and the accumulated statistics."""
    n = P.shape[0]
    acc = wos.Accumulators(n, grad_dim=grad_dim)
    plan = wos.Plan([(prob_handle, P, acc, 0)], wos.options(walks=walks, seed=0, **opt_kw))
    plan.launch(seed=999)
    torch.cuda.synchronize()
    for t in (acc.sum, acc.sum_sq, acc.n_walks, acc.n_steps, acc.counters, acc.grad_sum, acc.grad_sum_sq):
        if t is not None:
            t.zero_()
    ms = []
    for k in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        plan.launch(seed=k, walk_offset_add=k * walks)
        b.record()
        torch.cuda.synchronize()
        ms.append(a.elapsed_time(b))
    mean, se = wos.finalize(acc)
    torch.cuda.synchronize()
    nw = float(acc.n_walks[0].item())
    steps = float(acc.n_steps.sum().item())
    se_np = se.cpu().numpy()
    var = float(np.mean((se_np ** 2) * nw))
    info = plan.info()
    plan.close()
    t_walk = (np.mean(ms) / 1e3) / walks
    return {"ms_per_pass": float(np.mean(ms)), "steps_per_s": steps / (sum(ms) / 1e3),
            "distance_queries_per_walk": steps / (nw * n), "per_walk_variance": var,
            "points_per_s_at_rmse_1e-2": n / ((var / 1e-4) * t_walk), "plan": info,
            "_mean": mean.cpu().numpy(), "_se": se_np}


def time_to_rmse(wos, torch, prob_handle, P, ref_idx, ref_mean, ref_se, precision, max_walks=65536):
    """Doubles the walks per point from 64 until the RMSE against the reference at the
    reference points is at most 1e-2 (RMSE^2 = mean squared difference minus the mean
    squared standard error of the reference); returns that run's walks, RMSE and graph
    replay time, and query points per second over all points."""
    walks = 64
    while True:
        r = _timed_plan(wos, torch, prob_handle, P, {"precision": precision}, walks, 1)
        d2 = float(np.mean((r["_mean"][ref_idx] - ref_mean) ** 2) - np.mean(np.asarray(ref_se) ** 2))
        rmse = math.sqrt(max(d2, 0.0))
        if rmse <= 1e-2 or walks >= max_walks:
            return {"walks": walks, "rmse": rmse, "ms": r["ms_per_pass"],
                    "points_per_s": P.shape[0] / (r["ms_per_pass"] / 1e3), "reached": rmse <= 1e-2}
        walks *= 2


def measure_extras(wos, WL):
    """Throughput of the rows beyond the plain delta-tracking walk, FP32, each against the
    plain walk on the same workload: gradients (supplemental Sec. 2) on the star polygon;
    weight-window splitting (Sec. 6) on the manufactured disk, where sigma' < 0 lets
    null-collision weights grow; an SDF/CSG scene (Sec. 7.2); and the other workload
    shapes: the batch of 64 polygon problems in one plan and the 3D mesh walker."""
    import torch
    out = {}
    # gradient estimates: the star-polygon workload at 256 walks per point
    c = WL.config2(n_grid=512)
    prob, pts = c["problems"][0], c["points"][0]
    h = wos.Problem(prob)
    P = torch.as_tensor(pts, dtype=torch.float64, device="cuda")
    plain = _timed_plan(wos, torch, h, P, {"precision": "fp32"}, 256, 3)
    grad = _timed_plan(wos, torch, h, P, {"precision": "fp32"}, 256, 3, grad_dim=2)
    out["gradient"] = {"workload": "star polygon 256 edges, 512x512 grid inside, 256 walks per point",
                       "plain_ms_per_pass": plain["ms_per_pass"], "gradient_ms_per_pass": grad["ms_per_pass"],
                       "overhead": grad["ms_per_pass"] / plain["ms_per_pass"] - 1.0}
    print(f"bench: gradient overhead {out['gradient']['overhead']:.3f}", file=sys.stderr, flush=True)
    del P
    # splitting: manufactured disk on a 256x256 grid, window [0.5, 1.5]
    c = WL.config1(n_grid=256)
    prob, pts = c["problems"][0], c["points"][0]
    h = wos.Problem(prob)
    P = torch.as_tensor(pts, dtype=torch.float64, device="cuda")
    rr = _timed_plan(wos, torch, h, P, {"precision": "fp32", "russian_roulette": True, "ww_lo": 0.5}, 256, 3)
    sp = _timed_plan(wos, torch, h, P, {"precision": "fp32", "russian_roulette": True, "ww_lo": 0.5,
                                        "ww_hi": 1.5}, 256, 3)
    for r in (rr, sp):
        r.pop("_mean")
        r.pop("_se")
    out["splitting"] = {"workload": "manufactured disk, 256x256 grid inside, sigma_bar %.4g, 256 walks per point"
                                    % h.sigma_bar, "roulette_only": rr, "roulette_and_splitting": sp}
    print("bench: splitting pts/s at RMSE 1e-2 %.3e (roulette only %.3e)"
          % (sp["points_per_s_at_rmse_1e-2"], rr["points_per_s_at_rmse_1e-2"]), file=sys.stderr, flush=True)
    del P
    # SDF/CSG scene
    c = WL.config6(n_grid=256)
    prob, pts = c["problems"][0], c["points"][0]
    h = wos.Problem(prob)
    P = torch.as_tensor(pts, dtype=torch.float64, device="cuda")
    sdf = _timed_plan(wos, torch, h, P, {"precision": "fp32"}, 256, 3)
    sdf.pop("_mean")
    sdf.pop("_se")
    out["sdf"] = {"workload": "square with 24 round and 8 box holes (33 CSG rows), star-polygon fields, "
                              "256x256 grid inside, 256 walks per point", "query_points": int(P.shape[0]), **sdf}
    print(f"bench: sdf steps/s {sdf['steps_per_s']:.3e}", file=sys.stderr, flush=True)
    del P
    # the batch of 64 polygon problems (16-4096 edges, 2.65e6 points) in one plan
    c = WL.config4()
    entries, n_total = [], 0
    for i, (p, q) in enumerate(zip(c["problems"], c["points"])):
        Q = torch.as_tensor(q, dtype=torch.float64, device="cuda")
        entries.append((wos.Problem(p), Q, wos.Accumulators(Q.shape[0]), i))
        n_total += Q.shape[0]
    plan = wos.Plan(entries, wos.options(precision="fp32", walks=512, seed=0))
    plan.launch(seed=999)
    torch.cuda.synchronize()
    for _, _, acc, _ in entries:
        acc.n_steps.zero_()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    plan.launch(seed=1, walk_offset_add=512)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b)
    steps = sum(float(acc.n_steps.sum().item()) for _, _, acc, _ in entries)
    out["batch64"] = {"workload": "64 star polygons with 16-4096 edges, log-uniform 1k-256k points each, 512 walks "
                                  "per point, one plan", "query_points": n_total, "ms_per_pass": ms,
                      "steps_per_s": steps / (ms / 1e3), "plan": plan.info()}
    plan.close()
    del entries
    print(f"bench: 64-problem batch steps/s {out['batch64']['steps_per_s']:.3e}", file=sys.stderr, flush=True)
    # 3D mesh walker on a slice of the perturbed icosphere (20,480 triangles)
    c = WL.config3(n_grid=256)
    prob, pts = c["problems"][0], c["points"][0]
    h = wos.Problem(prob)
    P = torch.as_tensor(pts, dtype=torch.float64, device="cuda")
    ico = _timed_plan(wos, torch, h, P, {"precision": "fp32"}, 64, 2)
    ico.pop("_mean")
    ico.pop("_se")
    out["icosphere"] = {"workload": "perturbed icosphere, 20,480 triangles, 256x256 slice grid inside, 64 walks per "
                                    "point", "query_points": int(P.shape[0]), **ico}
    print(f"bench: icosphere steps/s {ico['steps_per_s']:.3e}", file=sys.stderr, flush=True)
    return out


def main():
    args = parse()
    if args.summarize_trace:
        print(summarize_trace(*args.summarize_trace[:2]))
        return
    if args.summarize_pmc:
        print(summarize_pmc(args.summarize_pmc[0], args.summarize_pmc[1:]))
        return
    if args.write_traffic:
        write_traffic(*args.write_traffic)
        return
    if args.copy_probe:
        copy_probe()
        return
    if args.gpus != 1:
        print(f"bench.py: the benchmark runs on one GPU only (asked for --gpus {args.gpus}); "
              "the walks are independent and would shard by walk range, one process per GPU",
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
        shape = {} if args.shape == "auto" else dict(zip(("block_size", "tile_walks"),
                                                         map(int, args.shape.lower().split("x"))))
        plan = wos.Plan([(h, P, acc, 0)], wos.options(precision=precision, walks=walks, seed=0, **shape))
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
        n_steps = int(acc.n_steps.sum().item())
        n_walks = int(acc.n_walks.sum().item())
        print(f"bench: {precision} {steps} timed passes, ms/pass {np.round(ms, 2).tolist()}", file=sys.stderr,
              flush=True)
        # the walker alone: the same pass issued as separate launches with HIP events
        # around the walker kernel on the stream it runs on
        walker_ms = []
        for k in range(steps):
            wm, _ = plan.time(seed=500 + k, walk_offset_add=k * walks, stream=stream)
            walker_ms.append(wm)
        torch.cuda.synchronize()
        timed_steps = int(acc.n_steps.sum().item()) - n_steps
        print(f"bench: {precision} walker ms/launch {np.round(walker_ms, 2).tolist()}", file=sys.stderr, flush=True)
        mean, se = wos.finalize(acc)
        torch.cuda.synchronize()
        info = plan.info()
        plan.close()
        return {"wall_s": wall, "ms": ms, "steps": n_steps, "walks": n_walks,
                "walker_ms": walker_ms, "walker_steps": timed_steps,
                "walks_total": int(acc.n_walks.sum().item()),
                "mean": mean.cpu().numpy(), "se": se.cpu().numpy(),
                "counters": acc.counters.cpu().numpy().tolist(), "plan": info}

    r32 = run(args.precision, args.steps, args.warmup, args.walks)

    # algorithmic work per distance query and lane occupancy from the event-counting
    # walker over one full pass of the same workload (same shape as the timed plan)
    if args.no_events:
        events = {k: 1 for k in wos.EVENT_NAMES}   # profiling runs: no event-counting launch
    else:
        acc_c = wos.Accumulators(n_pts)
        events = wos.count_events([(h, P, acc_c, 0)],
                                  wos.options(precision=args.precision, walks=args.walks, seed=99,
                                              block_size=r32["plan"]["block_size"],
                                              tile_walks=r32["plan"]["tile_walks"]))
        del acc_c
    flops_ev, trans_ev = algorithmic_work(events, prob)
    flops_per_step = flops_ev / events["steps"]
    trans_per_step = trans_ev / events["steps"]
    # per walker launch: algorithmic flops per step x steps of one launch, over the
    # walker's own average launch duration
    steps_per_launch = r32["walker_steps"] / len(r32["walker_ms"])
    walker_ms = float(np.mean(r32["walker_ms"]))
    achieved = flops_per_step * steps_per_launch / (walker_ms / 1e3) / 1e12
    peak = 157.3 if args.precision != "fp64" else 78.6
    traffic = traffic_of(walker_kernel_name(args.precision))
    roofline = {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak,
                "traffic": traffic["bytes_per_launch"] if traffic else None, "traffic_detail": traffic,
                "kernel": walker_kernel_name(args.precision), "kernel_ms": walker_ms,
                "flops_per_step": flops_per_step, "transcendentals_per_step": trans_per_step,
                "events_per_step": {k: v / events["steps"] for k, v in events.items()}}
    if not args.no_events:
        # lane occupancy of the walker's lockstep iterations (event-counting build)
        roofline["lanes_holding_a_walk"] = events["active_lane_iterations"] / events["lane_iterations"]
        roofline["lanes_evaluating_coefficients"] = events["coefficient_lane_iterations"] / events["lane_iterations"]
    r64 = run("fp64", args.fp64_steps, 0, args.walks) if args.fp64_steps > 0 else None
    r32c = run("fp32c", args.fp32c_steps, 0, args.walks) if args.fp32c_steps > 0 else None
    ms_step = float(np.mean(r32["ms"]))
    steps_per_s = r32["steps"] / (sum(r32["ms"]) / 1e3)
    walks_per_pt = args.walks * args.steps

    # per-walk variance -> walks needed for RMSE 1e-2 (Sec. 3.1: RMSE = sqrt(mean var / N))
    var_walk = (r32["se"] ** 2) * (r32["walks_total"] / n_pts)
    n_star = float(np.mean(var_walk)) / 1e-4
    t_walk_pass = (sum(r32["ms"]) / 1e3) / walks_per_pt          # seconds per walk per point (all points)
    pts_per_s_rmse = n_pts / (n_star * t_walk_pass)
    out64 = {}
    if r64 is not None:
        s64 = r64["steps"] / (sum(r64["ms"]) / 1e3)
        t64 = (sum(r64["ms"]) / 1e3) / (args.walks * args.fp64_steps)
        var64 = (r64["se"] ** 2) * (r64["walks_total"] / n_pts)
        n64 = float(np.mean(var64)) / 1e-4
        out64 = {"fp64_steps_per_s": s64, "fp64_ms_per_step": float(np.mean(r64["ms"])),
                 "fp64_points_per_s_at_rmse_1e-2": n_pts / (n64 * t64)}
    if r32c is not None:
        out64.update({"fp32c_steps_per_s": r32c["steps"] / (sum(r32c["ms"]) / 1e3),
                      "fp32c_ms_per_step": float(np.mean(r32c["ms"]))})

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
        # the same oracle on one thread, over a twelfth of the points
        n1 = max(1, args.cpu_points // 12)
        t0 = time.perf_counter()
        o1 = O.solve(prob, pts[idx[:n1]], args.cpu_walks, h.sigma_bar, seed=78, threads=1)
        dt1 = time.perf_counter() - t0
        cpu["single_thread"] = {"value": float(o1["steps"].sum() / dt1), "cores": 1,
                                "sample": f"{n1} of those points x {args.cpu_walks} walks, {dt1:.1f} s"}
        for name, r in (("fp32", r32), ("fp32c", r32c), ("fp64", r64)):
            if r is None:
                continue
            d2 = (r["mean"][idx] - o["mean"]) ** 2 - o["se"] ** 2
            rmse[name] = {"rmse_vs_oracle": float(math.sqrt(max(np.mean(d2), 0.0))),
                          "mean_se_gpu": float(np.mean(r["se"][idx])), "mean_se_oracle": float(np.mean(o["se"]))}

    # time to RMSE 1e-2, walks doubled from 64: on this workload against the oracle's
    # sample, and on the manufactured disk against its exact solution u = e^x cos y
    ttr = {}
    if args.ttr:
        if args.cpu_points > 0:
            ttr["star_polygon_vs_oracle_sample"] = {
                prec: time_to_rmse(wos, torch, h, P, idx, o["mean"], o["se"], prec) for prec in ("fp32", "fp32c", "fp64")}
        c1 = WL.config1()
        h1 = wos.Problem(c1["problems"][0])
        p1 = c1["points"][0]
        P1 = torch.as_tensor(p1, dtype=torch.float64, device="cuda")
        ex = np.exp(p1[:, 0]) * np.cos(p1[:, 1])
        all1 = np.arange(p1.shape[0])
        ttr["manufactured_disk_vs_exact"] = {
            prec: time_to_rmse(wos, torch, h1, P1, all1, ex, np.zeros_like(ex), prec) for prec in ("fp32", "fp32c", "fp64")}
        print("bench: time to RMSE 1e-2 " + json.dumps(ttr), file=sys.stderr, flush=True)

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
        "time_to_rmse_1e-2": ttr,
    }
    line.update(out64)
    if args.variants:
        line["next_flight_vs_delta_tracking"] = compare_variants(wos, WL, args)
    if args.extras:
        line["extras"] = measure_extras(wos, WL)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
