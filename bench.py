"""Benchmark of the delta-tracking walk on spheres on one MI355X.

Workload: the 256-edge star polygon problem with random alpha, drift and sigma fields
(Gaussian-bump f and g), all query points of a 512 x 512 grid inside the domain, 1024
walks per point. One "step" of this benchmark is one full pass of the hot path over
that batch: a captured hipGraph replay of [tile-counter reset, persistent walker,
per-point exact sums]. The metric is walk steps (distance queries) per second; points
per second at RMSE 1e-2 against the FP64 oracle is derived from the measured per-walk
variance. Beside it the line reports the walker's vector-ALU roofline, the FP64 walker,
the FP32 rounding error against the FP64 walker on common random numbers, the FP64 CPU
oracle as a baseline, time to RMSE 1e-2, next flight against delta tracking, the RMSE
against the oracle versus walks per point on the high-contrast square, set-up times, and
the throughput and roofline of every other walker (gradients, splitting, an SDF scene,
the 64-problem batch, the full icosphere slice). Prints one JSON line.
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
                    help="also time next flight against delta tracking on a screened disk and on the high-contrast "
                         "square (0: skip)")
    ap.add_argument("--extras", type=int, default=1,
                    help="also time (with rooflines) the FP64 walker, gradients, weight-window splitting, an SDF/CSG "
                         "scene, the 64-problem batch and the full icosphere slice (0: skip)")
    ap.add_argument("--fp32-error", type=int, default=1,
                    help="FP32 against FP64 on common random numbers (0: skip)")
    ap.add_argument("--sweep", type=int, default=1,
                    help="RMSE against the oracle versus walks per point on the high-contrast square (0: skip)")
    ap.add_argument("--tune-cache", default="",
                    help="file of tuned launch shapes: loaded before the runs if it exists, written after them")
    ap.add_argument("--shape", default="auto",
                    help="walker launch shape: 'auto' (the plan autotunes block size and tile length) or "
                         "BLOCKxTILE, e.g. 256x256 (profiling runs pin the tuned shape so that no tuning "
                         "dispatches enter the kernel statistics)")
    # profiling helpers (each does only this and exits)
    ap.add_argument("--copy-probe", action="store_true",
                    help="run one 1 GiB device-to-device copy: the calibration kernel for FETCH_SIZE/WRITE_SIZE")
    ap.add_argument("--batch-only", action="store_true",
                    help="run one pass of the 64-problem batch (512 walks per point, --shape or autotuned) "
                         "after one warm-up pass: the profiling run for the batch's own counters")
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


def _coefficient_costs(prob):
    """(flops, transcendentals) of the coefficient program at one point, of gamma alone,
    and of the boundary field."""
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
    return (coef, coef_t), gamma_only, (bf, bt)


def _geometry_costs(prob):
    dim = prob["dim"]
    seg = 21 if dim == 2 else 75                                         # segment / triangle distance
    node = 2 * (3 * dim) + 2                                             # two child boxes + ordering
    return {"steps": (3, 1),                                             # per query: sqrt, epsilon test, radius
            "bvh_nodes": (node, 0),
            "grid_cells": (2 * dim + 4, 0),                              # cell index of the query point
            "prims": (seg, 0)}


def event_weights(prob):
    """Per-event (flops, transcendentals) of the delta-tracking walk (Sec. 5.1, Alg. 1)."""
    (coef, coef_t), gamma_only, (bf, bt) = _coefficient_costs(prob)
    W = _geometry_costs(prob)
    W.update({
        # per sampled ball: normalisation (series), direction, y, mu, coefficients at y, source
        "sampled": (73 + 2 + 5 + 1 + coef + 5, 1 + 2 + coef_t + 1),
        "ball_large_s": (42, 2),                                         # Chebyshev instead of series
        "trials": (78, 3),                                               # harmonic-law proposal
        "trials_free": (37, 1),                                          # free-space proposal, extra
        # below s = 3.5 (2D) or 4 (3D): the harmonic draw mapped to t0^a (a, ln t0, t0^a),
        # in 2D the Bessel values unscaled, the envelope constant (closed form or 12-term
        # polynomial) and the acceptance test with t0^(2a - 2) = t^2 / t0^2
        "trials_power": (33, 2) if prob["dim"] == 2 else (26, 2),
        "volume": (3, 0),
        "exit": (6, 2),
        "terminal": (12 + bf + 4, bt + 1),
        "gamma_evals": gamma_only,
        "rr_draws": (4, 0),
    })
    return W


def nf_event_weights(prob):
    """Per-event (flops, transcendentals) of the next-flight walk (Sec. 5.2, supplemental
    Alg. 2). A ball (a distance query that does not end the walk) takes the centred ball
    terms and its exit direction; an inner point (counted as a proposal, events[3]) takes a
    uniform point in the ball, the coefficients there, the off-centred Green's function (two
    radial profiles of about 45 flops and 2 exponentials each), the source and throughput
    updates, the off-centred Poisson kernel at the exit point (two profiles) and the
    throughput roulette."""
    (coef, coef_t), gamma_only, (bf, bt) = _coefficient_costs(prob)
    dim = prob["dim"]
    W = _geometry_costs(prob)
    green = 4 * dim + 5 + 2 * 45, 1 + 2 * 2                               # nf_green_vol
    poisson = 4 * dim + 11 + 2 * 45, 1 + 2 * 2                            # nf_poisson_area
    W.update({
        "sampled": (73 + 2 + 6, 1 + 2),                                  # ball terms, exit direction
        "ball_large_s": (42, 2),
        "trials": (8 + dim + coef + green[0] + 6 + 3 + poisson[0] + 3, 3 + coef_t + green[1] + 1 + poisson[1]),
        "terminal": (12 + bf + 4, bt + 1),
        "gamma_evals": gamma_only,
    })
    return W


def algorithmic_work(events, prob, next_flight=False):
    W = nf_event_weights(prob) if next_flight else event_weights(prob)
    ev = dict(events)
    ev["sampled"] = ev["steps"] - ev["terminal"]
    ev["trials_power"] = ev["trials"] - ev["trials_free"]
    flops = sum(W[k][0] * ev[k] for k in W)
    trans = sum(W[k][1] * ev[k] for k in W)
    return flops, trans


# ----------------------------------------------------------------------------- HBM traffic
# Measured HBM bytes of the walker come from rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE,
# KiB per dispatch) of this benchmark, committed as JSON under profiles/ together with
# the same counters read for a copy of known size (the calibration factors) and a hash of
# the device sources the counters were taken with. A changed kernel makes them stale:
# traffic is then reported as null.
DEVICE_SOURCES = ("wos_walker.h", "wos_walker_f32_2d.hip", "wos_walker_f64_2d.hip", "wos_kernels.hip", "wos_device.h",
                  "wos_types.h", "bessel_tables.h", "proposal_bound.h")


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


def batch_only(wos, torch, WL, shape_arg):
    """One warm-up and one timed pass of the 64-problem batch in one plan (the extras
    workload), so that counter runs see only its walker dispatches."""
    c = WL.config4()
    entries = []
    for i, (p, q) in enumerate(zip(c["problems"], c["points"])):
        Q = torch.as_tensor(q, dtype=torch.float64, device="cuda")
        entries.append((wos.Problem(p), Q, wos.Accumulators(Q.shape[0]), i))
    shape = {} if shape_arg == "auto" else dict(zip(("block_size", "tile_walks"),
                                                    map(int, shape_arg.lower().split("x"))))
    plan = wos.Plan(entries, wos.options(precision="fp32", walks=512, seed=0, **shape))
    for k in range(2):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan.launch(seed=k, walk_offset_add=0)
        torch.cuda.synchronize()
        print(f"batch pass {k}: {(time.perf_counter() - t0) * 1e3:.1f} ms, plan {plan.info()}", flush=True)


def copy_probe():
    import torch
    n = 1 << 28   # float32 elements: 1 GiB
    a = torch.ones(n, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    print("copied bytes", n * 4, flush=True)


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


def measure_extras(wos, torch, WL, setup):
    """Throughput and vector-ALU roofline of every other walker the benchmark times, FP32
    unless stated: the FP64 walker on the star polygon; gradients (supplemental Sec. 2) on
    the star polygon; weight-window splitting (Sec. 6) on the manufactured disk, where
    sigma' < 0 lets null-collision weights grow; an SDF/CSG scene (Sec. 7.2); the batch of
    64 polygon problems in one plan; and the 3D mesh walker on the perturbed icosphere's
    z = 0 slice at its full size (676,691 points x 256 walks). `setup` collects the set-up
    time of each problem."""
    out = {}

    def problem(name, prob, **kw):
        t0 = time.perf_counter()
        h = wos.Problem(prob, **kw)
        setup[name] = {"problem_create_ms": (time.perf_counter() - t0) * 1e3, **h.setup_times()}
        return h

    def one(h, pts, grad_dim=0):
        P = torch.as_tensor(pts, dtype=torch.float64, device="cuda")
        return [(h, P, wos.Accumulators(P.shape[0], grad_dim=grad_dim), 0)]

    c = WL.config2(n_grid=512)
    prob, pts = c["problems"][0], c["points"][0]
    h = problem("star_polygon_again", prob)
    out["fp64_star"] = {"workload": "star polygon 256 edges, 512x512 grid inside, 1024 walks per point, FP64",
                        **_strip(measure_walker(wos, torch, one(h, pts), {"precision": "fp64"}, 1024, 2, prob,
                                                label="FP64 star polygon"))}
    plain = _strip(measure_walker(wos, torch, one(h, pts), {"precision": "fp32"}, 256, 3, prob, label="plain 256"))
    grad = _strip(measure_walker(wos, torch, one(h, pts, 2), {"precision": "fp32"}, 256, 3, prob,
                                 label="gradient 256"))
    out["gradient"] = {"workload": "star polygon 256 edges, 512x512 grid inside, 256 walks per point",
                       "plain": plain, "with_gradient": grad,
                       "overhead": grad["ms_per_pass"] / plain["ms_per_pass"] - 1.0}
    # splitting: manufactured disk on a 256x256 grid, window [0.5, 1.5]
    c = WL.config1(n_grid=256)
    prob, pts = c["problems"][0], c["points"][0]
    h = problem("manufactured_disk", prob)
    rr = _strip(measure_walker(wos, torch, one(h, pts), {"precision": "fp32", "russian_roulette": True,
                                                         "ww_lo": 0.5}, 256, 3, prob, label="roulette"))
    sp = _strip(measure_walker(wos, torch, one(h, pts), {"precision": "fp32", "russian_roulette": True,
                                                         "ww_lo": 0.5, "ww_hi": 1.5}, 256, 3, prob,
                               label="roulette and splitting"))
    out["splitting"] = {"workload": "manufactured disk, 256x256 grid inside, sigma_bar %.4g, 256 walks per point"
                                    % h.sigma_bar, "roulette_only": rr, "roulette_and_splitting": sp}
    # SDF/CSG scene
    c = WL.config6(n_grid=256)
    prob, pts = c["problems"][0], c["points"][0]
    h = problem("sdf_scene", prob)
    out["sdf"] = {"workload": "square with 24 round and 8 box holes (33 CSG rows), star-polygon fields, "
                              "256x256 grid inside, 256 walks per point",
                  **_strip(measure_walker(wos, torch, one(h, pts), {"precision": "fp32"}, 256, 3, prob,
                                          label="sdf"))}
    # the batch of 64 polygon problems (16-4096 edges, 2.65e6 points) in one plan
    c = WL.config4()
    t0 = time.perf_counter()
    entries = []
    for i, (p, q) in enumerate(zip(c["problems"], c["points"])):
        Q = torch.as_tensor(q, dtype=torch.float64, device="cuda")
        entries.append((wos.Problem(p), Q, wos.Accumulators(Q.shape[0]), i))
    setup["batch64"] = {"problems_create_ms": (time.perf_counter() - t0) * 1e3,
                        "geometry_ms": sum(e[0].setup_times()["geometry_ms"] for e in entries),
                        "sigma_bar_ms": sum(e[0].setup_times()["sigma_bar_ms"] for e in entries)}
    out["batch64"] = {"workload": "64 star polygons with 16-4096 edges, log-uniform 1k-256k points each, 512 walks "
                                  "per point, one plan",
                      **_strip(measure_walker(wos, torch, entries, {"precision": "fp32"}, 512, 1, c["problems"][0],
                                              label="64-problem batch"))}
    del entries
    # 3D mesh walker on the perturbed icosphere's slice (20,480 triangles), full size
    c = WL.config3()
    prob, pts = c["problems"][0], c["points"][0]
    h = problem("icosphere", prob)
    out["icosphere"] = {"workload": "perturbed icosphere, 20,480 triangles, 1024x1024 slice grid inside, 256 walks "
                                    "per point",
                        **_strip(measure_walker(wos, torch, one(h, pts), {"precision": "fp32"}, 256, 2, prob,
                                                label="icosphere"))}
    return out


def _zero(acc):
    for t in (acc.sum, acc.sum_sq, acc.n_walks, acc.n_steps, acc.counters, acc.grad_sum, acc.grad_sum_sq):
        if t is not None:
            t.zero_()


def measure_walker(wos, torch, entries, opt_kw, walks, reps, weights_prob, next_flight=False, events=True,
                   label=""):
    """One plan over `entries` (one item per problem), replayed `reps` times (graph replays,
    HIP events on the current stream) and then timed `reps` times as separate launches with
    HIP events around the walker kernel (wos_plan_time). With `events`, the event-counting
    build runs the same job once in the plan's launch shape and gives the algorithmic
    flops per distance query (per-event weights of `weights_prob`); achieved = flops per
    step x steps per walker launch / the walker's mean launch time."""
    t0 = time.perf_counter()
    plan = wos.Plan(entries, wos.options(walks=walks, seed=0, **opt_kw))
    plan_wall_ms = (time.perf_counter() - t0) * 1e3
    setup = plan.setup_times()
    info = plan.info()
    plan.launch(seed=999)
    torch.cuda.synchronize()
    for _, _, acc, _ in entries:
        _zero(acc)
    stream = torch.cuda.current_stream()
    ms = []
    for k in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        plan.launch(seed=k, walk_offset_add=k * walks)
        b.record(stream)
        torch.cuda.synchronize()
        ms.append(a.elapsed_time(b))
    n_pts = sum(int(P.shape[0]) for _, P, _, _ in entries)
    steps = sum(float(acc.n_steps.sum().item()) for _, _, acc, _ in entries)
    var, nw = [], 0.0
    means = []
    for _, _, acc, _ in entries:
        mean, se = wos.finalize(acc)
        torch.cuda.synchronize()
        nw = float(acc.n_walks[0].item()) if acc.n_walks.numel() else nw
        se_np = se.cpu().numpy()
        var.append((se_np ** 2) * nw)
        means.append((mean.cpu().numpy(), se_np))
    var = np.concatenate(var)
    var_mean = float(np.nanmean(var))
    walker_ms, steps_w = [], 0.0
    for _, _, acc, _ in entries:
        _zero(acc)
    for k in range(reps):
        wm, _ = plan.time(seed=500 + k, walk_offset_add=k * walks, stream=stream)
        walker_ms.append(wm)
    torch.cuda.synchronize()
    steps_w = sum(float(acc.n_steps.sum().item()) for _, _, acc, _ in entries)
    plan.close()
    t_walk = (np.mean(ms) / 1e3) / walks
    out = {"query_points": n_pts, "walks_per_point": walks, "ms_per_pass": float(np.mean(ms)),
           "steps_per_s": steps / (sum(ms) / 1e3), "distance_queries_per_walk": steps / (reps * walks * n_pts),
           "per_walk_variance": var_mean, "points_per_s_at_rmse_1e-2": n_pts / ((var_mean / 1e-4) * t_walk),
           "plan": info, "setup_ms": {"plan_create": plan_wall_ms, **setup}}
    if events:
        accs = [(h, P, wos.Accumulators(P.shape[0], grad_dim=(acc.grad_sum.shape[1] if acc.grad_sum is not None
                                                              else 0)), i) for h, P, acc, i in entries]
        ev = wos.count_events(accs, wos.options(walks=walks, seed=99, block_size=info["block_size"],
                                                tile_walks=info["tile_walks"], **opt_kw))
        del accs
        flops, trans = algorithmic_work(ev, weights_prob, next_flight)
        fps = flops / ev["steps"]
        wms = float(np.mean(walker_ms))
        prec = opt_kw.get("precision", "fp32")
        peak = 78.6 if prec.startswith("fp64") else 157.3
        ach = fps * (steps_w / reps) / (wms / 1e3) / 1e12
        out["roofline"] = {"bound": "alu", "achieved": ach, "peak": peak, "unit": "TFLOP/s", "frac": ach / peak,
                           "kernel_ms": wms, "flops_per_step": fps, "transcendentals_per_step": trans / ev["steps"],
                           "lanes_holding_a_walk": ev["active_lane_iterations"] / ev["lane_iterations"],
                           "lanes_evaluating_coefficients": ev["coefficient_lane_iterations"] / ev["lane_iterations"]}
    out["_means"] = means
    if label:
        print(f"bench: {label}: {out['ms_per_pass']:.2f} ms/pass, {out['steps_per_s']:.3e} steps/s"
              + (f", {out['roofline']['frac']:.3f} of peak" if events else ""), file=sys.stderr, flush=True)
    return out


def _strip(d):
    d.pop("_means", None)
    return d


def max_ball_s(wos, h, P):
    """Largest s = R sqrt(sigma_bar) of a first ball: the largest distance to the boundary
    over the query points (FP64 distance queries) times sqrt(sigma_bar)."""
    d, _ = wos.eval_distance(h, P, precision="fp64")
    return float(d.max().item()) * math.sqrt(max(h.sigma_bar, 0.0))


def compare_variants(wos, torch, WL):
    """Next flight (Sec. 5.2) against delta tracking (Sec. 5.1), FP32, same walks per point.

    * screened disk (sigma' = sigma in [0.5, 3.5], s < 2 in every ball): both walks have
      finite variance, so time, distance queries and query points per second at RMSE 1e-2
      compare directly; the mean difference in combined standard errors shows the bias of
      the off-centred kernel approximations (supplemental Sec. 1.2).
    * high-contrast square (sigma' changes sign, s up to about 50): next flight takes far
      fewer distance queries, but its in-ball series has no finite variance there, so its
      points per second at RMSE 1e-2 is reported as null with the reason."""
    out = {}
    for name, cfg, walks in (("screened_disk", WL.config7(), 1024), ("high_contrast_square", WL.config5(), 256)):
        prob, pts = cfg["problems"][0], cfg["points"][0]
        h = wos.Problem(prob)
        P = torch.as_tensor(pts, dtype=torch.float64, device="cuda")
        info = h.info()
        s_max = max_ball_s(wos, h, P)
        rec = {"query_points": int(P.shape[0]), "walks_per_point": walks, "sigma_bar": info["sigma_bar"],
               "sigma_prime_range": [info["sigma_prime_min"], info["sigma_prime_max"]], "max_s": s_max}
        res = {}
        for vname, variant, rr in (("delta_tracking", 0, name == "high_contrast_square"), ("next_flight", 2, False)):
            r = measure_walker(wos, torch, [(h, P, wos.Accumulators(P.shape[0]), 0)],
                               {"precision": "fp32", "variant": variant, "russian_roulette": rr}, walks, 3, prob,
                               next_flight=variant == 2, label=f"{vname} on the {name}")
            res[vname] = r.pop("_means")[0]
            rec[vname] = r
        valid = info["sigma_prime_min"] >= 0 and s_max < 2.0
        if not valid:
            rec["next_flight"]["points_per_s_at_rmse_1e-2"] = None
            rec["next_flight"]["note"] = (
                "null: sigma' < 0 somewhere (a throughput factor can exceed one) and s = R sqrt(sigma_bar) reaches "
                f"{s_max:.3g} > 2, where the second moment of the in-ball series diverges; its sample variance "
                "does not estimate a finite variance")
        (m0, s0), (m1, s1) = res["delta_tracking"], res["next_flight"]
        z = (m1 - m0) / np.sqrt(s0 ** 2 + s1 ** 2)
        rec["mean_abs_z_next_flight_vs_delta_tracking"] = float(np.nanmean(np.abs(z)))
        rec["mean_z_next_flight_vs_delta_tracking"] = float(np.nanmean(z))
        rec["mean_abs_difference"] = float(np.nanmean(np.abs(m1 - m0)))
        rec["next_flight_valid"] = bool(valid)
        out[name] = rec
        del P, h
    return out


def fp32_error(wos, torch, h, P, walks, single_walk_passes=8, russian_roulette=False):
    """Rounding error of the FP32 walker (Sec. 3.1's estimator, eqs. 17-18) on common random
    numbers: the FP64 walker drawing the FP32 walker's uniforms (WOS_FP64_FP32_DRAWS) runs
    the same walks from the same uniforms, so the per-point means differ only by rounding
    along paths that coincide, plus the walks whose paths part when rounding flips a
    branch. Reports the RMSE over all points of (FP32 - FP64) and (FP32 compensated - FP64)
    with its standard error (delta method over the points), and from single-walk passes
    the fraction of walks whose step counts differ or whose estimates differ by more than
    1e-4 max(1, |v|)."""
    n = int(P.shape[0])
    means = {}
    for prec in ("fp32", "fp32c", "fp64_fp32draws"):
        acc = wos.Accumulators(n)
        plan = wos.Plan([(h, P, acc, 0)], wos.options(precision=prec, walks=walks, seed=0,
                                                      russian_roulette=russian_roulette))
        plan.launch(seed=4242)
        torch.cuda.synchronize()
        means[prec] = (acc.sum / acc.n_walks.double()).cpu().numpy()
        plan.close()
    out = {"workload_points": n, "walks_per_point": walks}
    for name in ("fp32", "fp32c"):
        d = means[name] - means["fp64_fp32draws"]
        d = d[np.isfinite(d)]
        d2 = d * d
        msd = float(np.mean(d2))
        rmse = math.sqrt(msd)
        se_msd = float(np.std(d2, ddof=1) / math.sqrt(d2.size))
        out[f"{name}_minus_fp64"] = {"rmse": rmse, "rmse_se": se_msd / (2 * rmse) if rmse > 0 else 0.0,
                                     "max_abs": float(np.max(np.abs(d))), "median_abs": float(np.median(np.abs(d)))}
    # walk by walk: single-walk passes of both walkers
    vals = {}
    for prec in ("fp32", "fp64_fp32draws"):
        acc = wos.Accumulators(n)
        plan = wos.Plan([(h, P, acc, 0)], wos.options(precision=prec, walks=1, seed=0, block_size=256,
                                                      tile_walks=64, russian_roulette=russian_roulette))
        v, st = [], []
        for k in range(single_walk_passes):
            _zero(acc)
            plan.launch(seed=4242, walk_offset_add=k)
            torch.cuda.synchronize()
            v.append(acc.sum.cpu().numpy().copy())
            st.append(acc.n_steps.cpu().numpy().copy())
        plan.close()
        vals[prec] = (np.concatenate(v), np.concatenate(st))
    (v32, s32), (v64, s64) = vals["fp32"], vals["fp64_fp32draws"]
    ok = np.isfinite(v32) & np.isfinite(v64)
    v32, v64, s32, s64 = v32[ok], v64[ok], s32[ok], s64[ok]
    steps_differ = s32 != s64
    value_differ = np.abs(v32 - v64) > 1e-4 * np.maximum(1.0, np.abs(v64))
    same = ~(steps_differ | value_differ)
    out["single_walks"] = {
        "walks": int(v32.size), "diverged_fraction": float(np.mean(~same)),
        "steps_differ_fraction": float(np.mean(steps_differ)),
        "rms_difference_of_coinciding_walks": float(np.sqrt(np.mean((v32[same] - v64[same]) ** 2))),
        "rms_difference_of_diverged_walks": float(np.sqrt(np.mean((v32[~same] - v64[~same]) ** 2)))
        if np.any(~same) else 0.0}
    return out


def rmse_vs_reference(m, se, ref_mean, ref_se):
    """Raw RMSE of estimates m (standard errors se) against a reference (ref_mean, ref_se)
    at the same points, and the part of it that the two Monte Carlo errors do not explain:
    excess = mean((m - ref)^2) - mean(se^2 + ref_se^2), with its standard error over the
    points. No clamping: a negative excess means the difference is all noise."""
    d2 = (np.asarray(m) - np.asarray(ref_mean)) ** 2
    noise = np.asarray(se) ** 2 + np.asarray(ref_se) ** 2
    ex = d2 - noise
    return {"rmse_raw": float(math.sqrt(np.mean(d2))), "rms_noise": float(math.sqrt(np.mean(noise))),
            "excess_ms": float(np.mean(ex)), "excess_ms_se": float(np.std(ex, ddof=1) / math.sqrt(ex.size)),
            "points": int(ex.size)}


def rmse_sweep(wos, torch, WL, walks_list=(64, 128, 256, 512, 1024, 2048, 4096, 8192, 16384), replicates=32):
    """RMSE against the FP64 oracle versus walks per point on the high-contrast square with
    Russian roulette (Sec. 3.1 eq. 18: RMSE ~ N^-1/2; Sec. 6), for FP32, FP32 with
    compensated per-walk sums and FP64. The reference is the oracle at a seeded sample of
    48 points (tests/golden/sweep_square_rr.npz, written by tests/golden/make_sweep_ref.py
    from the oracle alone, 32,768 walks per point); the curve is taken over the sampled
    points whose reference standard error is at most 2.5e-3, and, split into the part the
    two Monte Carlo errors explain and the excess, over all 48. Single walks are heavy-tailed
    there (null-collision weights above one where sigma' < 0), so each N is run as
    `replicates` independent estimates (items of one plan with their own Philox streams,
    walks added in doublings) and the mean squared error is their average:
    MSE(N) = mean over replicates and points of (m - ref)^2 - mean(ref_se^2); beside it the
    median over replicates, which a rare heavy walk does not move. Query points per second
    come from a full pass over all 65,536 points at 1024 walks."""
    path = os.path.join(ROOT, "tests", "golden", "sweep_square_rr.npz")
    if not os.path.exists(path):
        return None
    ref = np.load(path, allow_pickle=False)
    c = WL.config5()
    prob, pts = c["problems"][0], c["points"][0]
    h = wos.Problem(prob, sigma_bar=float(ref["sigma_bar"][0]))
    idx_all = np.asarray(ref["idx"])
    sel = np.asarray(ref["se"]) <= 2.5e-3
    rmean_all, rse_all = np.asarray(ref["mean"]), np.asarray(ref["se"])
    Psel = torch.as_tensor(pts[idx_all], dtype=torch.float64, device="cuda")
    Pall = torch.as_tensor(pts, dtype=torch.float64, device="cuda")
    out = {"workload": "high-contrast unit square, 65,536 points, Russian roulette",
           "reference_points": int(sel.sum()), "sampled_points": int(sel.size),
           "reference_walks": int(ref["walks"]), "reference_max_se": float(rse_all[sel].max()),
           "replicates": replicates, "walks": list(walks_list), "curves": {}}
    ref_var_sel = float(np.mean(rse_all[sel] ** 2))
    for prec in ("fp32", "fp32c", "fp64"):
        # time per walk and point over the whole grid
        r = measure_walker(wos, torch, [(h, Pall, wos.Accumulators(Pall.shape[0]), 0)],
                           {"precision": prec, "russian_roulette": True}, 1024, 1, prob, events=False)
        t_walk = (r["ms_per_pass"] / 1e3) / 1024
        entries = [(h, Psel, wos.Accumulators(Psel.shape[0]), k) for k in range(replicates)]
        done, curve = 0, []
        for N in walks_list:
            plan = wos.Plan(entries, wos.options(precision=prec, walks=N - done, seed=0, walk_offset=done,
                                                 russian_roulette=True))
            plan.launch(seed=77)
            torch.cuda.synchronize()
            plan.close()
            done = N
            m = np.stack([(acc.sum / acc.n_walks.double()).cpu().numpy() for _, _, acc, _ in entries])
            d2 = (m - rmean_all[None, :]) ** 2                        # [replicate][point]
            mse_r = d2[:, sel].mean(1) - ref_var_sel
            mse = float(mse_r.mean())
            mse_se = float(mse_r.std(ddof=1) / math.sqrt(replicates))
            all_r = d2.mean(1) - float(np.mean(rse_all ** 2))
            # the median over replicates, which one rare heavy walk does not move
            med = float(np.median(mse_r))
            curve.append({"walks": N, "rmse": math.sqrt(max(mse, 0.0)), "mse": mse, "mse_se": mse_se,
                          "rmse_median_replicate": math.sqrt(max(med, 0.0)),
                          "rmse_all_sampled": math.sqrt(max(float(all_r.mean()), 0.0)),
                          "mse_all_sampled_se": float(all_r.std(ddof=1) / math.sqrt(replicates)),
                          "points_per_s": Pall.shape[0] / (N * t_walk)})
        ok = [e for e in curve if e["mse"] > 2 * e["mse_se"]]
        slope = (float(np.polyfit([math.log(e["walks"]) for e in ok], [0.5 * math.log(e["mse"]) for e in ok], 1)[0])
                 if len(ok) >= 3 else None)
        okm = [e for e in curve if e["rmse_median_replicate"] > 0]
        slope_med = (float(np.polyfit([math.log(e["walks"]) for e in okm],
                                      [math.log(e["rmse_median_replicate"]) for e in okm], 1)[0])
                     if len(okm) >= 3 else None)
        reached = [e for e in curve if e["rmse"] <= 1e-2]
        out["curves"][prec] = {"points": curve, "loglog_slope": slope, "loglog_slope_median_replicate": slope_med,
                               "seconds_per_walk_and_point": t_walk,
                               "walks_to_rmse_1e-2": reached[0]["walks"] if reached else None,
                               "points_per_s_at_rmse_1e-2": reached[0]["points_per_s"] if reached else None}
        print(f"bench: sweep {prec}: slope {slope} (median replicate {slope_med}), "
              f"rmse at {curve[0]['walks']} walks {curve[0]['rmse']:.3e}, "
              f"at {curve[-1]['walks']} walks {curve[-1]['rmse']:.3e}", file=sys.stderr, flush=True)
    # common random numbers at 1024 walks over all points: what compensation changes
    # against the FP64 walk
    out["common_random_numbers_1024"] = fp32_error(wos, torch, h, Pall, 1024, single_walk_passes=2,
                                                   russian_roulette=True)
    return out


def host_cpu():
    """Model name of the host CPU and the threads the oracle may use (the process's CPU
    share, at most 16)."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    return model, min(cores, 16)


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
    if args.batch_only:
        batch_only(wos, torch, WL, args.shape)
        return
    if args.tune_cache and os.path.exists(args.tune_cache):
        print(f"bench: {wos.tune_cache_load(args.tune_cache)} tuned shapes loaded", file=sys.stderr, flush=True)
    c = WL.config2(n_grid=args.grid)
    prob, pts = c["problems"][0], c["points"][0]
    n_pts = pts.shape[0]
    t0 = time.perf_counter()
    h = wos.Problem(prob)
    setup = {"star_polygon": {"problem_create_ms": (time.perf_counter() - t0) * 1e3, **h.setup_times()}}
    P = torch.as_tensor(pts, dtype=torch.float64, device="cuda")

    def run(precision, steps, warmup, walks):
        acc = wos.Accumulators(n_pts)
        shape = {} if args.shape == "auto" else dict(zip(("block_size", "tile_walks"),
                                                         map(int, args.shape.lower().split("x"))))
        t0 = time.perf_counter()
        plan = wos.Plan([(h, P, acc, 0)], wos.options(precision=precision, walks=walks, seed=0, **shape))
        plan_ms = (time.perf_counter() - t0) * 1e3
        for w in range(warmup):
            plan.launch(seed=1000 + w, walk_offset_add=0)
        torch.cuda.synchronize()
        _zero(acc)
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
        info = plan.info()
        print(f"bench: {precision} walker ms/launch {np.round(walker_ms, 2).tolist()}, plan {info}", file=sys.stderr,
              flush=True)
        mean, se = wos.finalize(acc)
        torch.cuda.synchronize()
        st = plan.setup_times()
        plan.close()
        return {"wall_s": wall, "ms": ms, "steps": n_steps, "walks": n_walks,
                "walker_ms": walker_ms, "walker_steps": timed_steps,
                "walks_total": int(acc.n_walks.sum().item()),
                "mean": mean.cpu().numpy(), "se": se.cpu().numpy(),
                "counters": acc.counters.cpu().numpy().tolist(), "plan": info,
                "setup_ms": {"plan_create": plan_ms, **st}}

    r32 = run(args.precision, args.steps, args.warmup, args.walks)
    setup["star_polygon"]["plan_" + args.precision] = r32["setup_ms"]

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

    # rounding error of the FP32 walker against the FP64 walker on common random numbers
    fp32err = fp32_error(wos, torch, h, P, args.walks) if args.fp32_error else None
    if fp32err:
        print("bench: FP32 - FP64 on common random numbers " + json.dumps(fp32err), file=sys.stderr, flush=True)

    # CPU baseline: the FP64 oracle (timing mode: its own BVH for closest points) on a
    # bounded sample of the same workload; its estimates are also the reference for the
    # RMSE of the GPU walkers at those points.
    cpu = None
    rmse = {}
    if args.cpu_points > 0:
        from oracle import oracle as O
        model, threads = host_cpu()
        idx = np.random.default_rng(0).choice(n_pts, args.cpu_points, replace=False)
        t0 = time.perf_counter()
        o = O.solve(prob, pts[idx], args.cpu_walks, h.sigma_bar, seed=77, threads=threads, bvh=True)
        dt = time.perf_counter() - t0
        cpu = {"value": float(o["steps"].sum() / dt), "unit": "walk steps/s", "cores": threads,
               "kind": "oracle", "cpu_model": model,
               "sample": f"{args.cpu_points} random query points x {args.cpu_walks} walks of the same workload, "
                         f"{dt:.1f} s; FP64 oracle with its own BVH for closest points (timing mode)"}
        # the same oracle on one thread, over a twelfth of the points
        n1 = max(1, args.cpu_points // 12)
        t0 = time.perf_counter()
        o1 = O.solve(prob, pts[idx[:n1]], args.cpu_walks, h.sigma_bar, seed=78, threads=1, bvh=True)
        dt1 = time.perf_counter() - t0
        cpu["single_thread"] = {"value": float(o1["steps"].sum() / dt1), "cores": 1,
                                "sample": f"{n1} of those points x {args.cpu_walks} walks, {dt1:.1f} s"}
        for name, r in (("fp32", r32), ("fp32c", r32c), ("fp64", r64)):
            if r is None:
                continue
            rmse[name] = rmse_vs_reference(r["mean"][idx], r["se"][idx], o["mean"], o["se"])

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
        "fp32_error_vs_fp64": fp32err,
        "rmse_vs_oracle_sample": rmse,
        "time_to_rmse_1e-2": ttr,
    }
    line.update(out64)
    if args.variants:
        line["next_flight_vs_delta_tracking"] = compare_variants(wos, torch, WL)
    if args.sweep:
        line["rmse_sweep_high_contrast_square"] = rmse_sweep(wos, torch, WL)
    if args.extras:
        line["extras"] = measure_extras(wos, torch, WL, setup)
    line["setup_ms"] = setup
    if args.tune_cache:
        wos.tune_cache_save(args.tune_cache)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
