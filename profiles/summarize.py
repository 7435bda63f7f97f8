"""Summarises rocprofv3 result databases (kernel trace and --pmc runs) as a short text
table for profiles/. Usage:

    python profiles/summarize.py trace <results.db> [kernel-substring]
    python profiles/summarize.py pmc <kernel-substring> <results.db> [<results.db> ...]
"""
import sqlite3
import sys
from collections import defaultdict


def trace(db, pattern=""):
    cur = sqlite3.connect(db).cursor()
    rows = list(cur.execute("select name, total_calls, total_duration, average, percentage from top_kernels"))
    out = ["| kernel | calls | total ms | average ms | % |", "|---|---|---|---|---|"]
    for name, calls, tot, avg, pct in rows:
        if pattern and pattern not in name:
            continue
        short = name.split("(")[0]
        out.append(f"| `{short}` | {calls} | {tot / 1e6:.3f} | {avg / 1e6:.3f} | {pct:.2f} |")
    return "\n".join(out)


def pmc(pattern, dbs):
    vals = defaultdict(float)
    info = {}
    for db in dbs:
        cur = sqlite3.connect(db).cursor()
        q = ("select kernel_name, dispatch_id, counter_name, value, vgpr_count, sgpr_count, scratch_size, grid_size, "
             "workgroup_size, duration from counters_collection")
        per_dispatch = defaultdict(lambda: defaultdict(float))
        for name, did, cname, v, vg, sg, scr, grid, wg, dur in cur.execute(q):
            if pattern not in name:
                continue
            per_dispatch[did][cname] += v
            info = {"kernel": name.split("(")[0], "vgpr": vg, "sgpr": sg, "scratch": scr, "grid": grid,
                    "workgroup": wg}
        # average over the dispatches of this run
        n = max(1, len(per_dispatch))
        for d in per_dispatch.values():
            for k, v in d.items():
                vals[k] += v / n
    lines = [f"kernel `{info.get('kernel')}`: grid {info.get('grid')}, workgroup {info.get('workgroup')}, "
             f"VGPRs {info.get('vgpr')}, SGPRs {info.get('sgpr')}, scratch {info.get('scratch')} B/lane", "",
             "| counter | value per dispatch |", "|---|---|"]
    for k in sorted(vals):
        lines.append(f"| {k} | {vals[k]:.6g} |")
    return "\n".join(lines), vals


if __name__ == "__main__":
    if sys.argv[1] == "trace":
        print(trace(sys.argv[2], sys.argv[3] if len(sys.argv) > 3 else ""))
    else:
        print(pmc(sys.argv[2], sys.argv[3:])[0])
