"""Summarise a rocprofv3 kernel-trace database (rocpd SQLite output): per
kernel total time, dispatch count and average duration, optionally per grid
size, as short text for the profiles/ folder.

python -m paper_1904_03317_amd.profsummary <results.db> [--by-grid PATTERN [--last N]] [--per-iteration]

--last N: beside each grid's average over all its dispatches, the average
of its last N dispatches (bench.py's timed repetitions of one level
operator come last for each precision).

--per-iteration: kernel time per CG iteration inside the last timed solve of
each precision, delimited by the update_xr dispatches (one per iteration).
"""
import argparse
import collections
import re
import sqlite3


def short(name):
    name = re.sub(r"\(.*$", "", name)
    return name.replace("void gmg::dev::", "").replace("gmg::dev::", "")


def summarize(db_path, top=30, by_grid=None, last=20):
    db = sqlite3.connect(db_path)
    rows = db.execute("select name, duration, grid_x, start, end from kernels order by start").fetchall()
    out = []
    agg = collections.defaultdict(lambda: [0, 0])
    for n, d, gx, s, e in rows:
        a = agg[short(n)]
        a[0] += 1
        a[1] += d
    tot = sum(v[1] for v in agg.values())
    out.append(f"dispatches {len(rows)}, total kernel time {tot / 1e6:.3f} ms")
    out.append(f"{'total_ms':>10} {'share':>6} {'count':>7} {'avg_us':>10}  kernel")
    for k, v in sorted(agg.items(), key=lambda kv: -kv[1][1])[:top]:
        out.append(f"{v[1] / 1e6:10.3f} {100 * v[1] / tot:5.1f}% {v[0]:7d} {v[1] / v[0] / 1e3:10.2f}  {k}")
    if by_grid:
        g = collections.defaultdict(list)
        for n, d, gx, s, e in rows:
            if by_grid in short(n):
                g[gx].append(d)
        out.append("")
        out.append(f"per grid size, kernels matching '{by_grid}':")
        for gx in sorted(g):
            v = g[gx]
            t = v[-last:]
            out.append(f"  grid_x {gx:10d} threads: n={len(v):5d} avg {sum(v) / len(v) / 1e3:9.2f} us "
                       f"min {min(v) / 1e3:9.2f} us, last {len(t)} avg {sum(t) / len(t) / 1e3:9.2f} us")
    return "\n".join(out)


def per_iteration(db_path, top=24, solves=(("FP64-MG", 24, 35), ("FP32-MG", 60, 71))):
    """Kernels between the update_xr dispatches a..b (bench.py with --steps 2
    --warmup 1: dispatches 24..35 are the second timed FP64-MG solve, 60..71
    the second timed FP32-MG solve), per iteration and grid size."""
    db = sqlite3.connect(db_path)
    rows = db.execute("select name, duration, grid_x, start, end from kernels order by start").fetchall()
    ux = [i for i, r in enumerate(rows) if "update_xr" in r[0]]
    out = []
    for label, a, b in solves:
        if b >= len(ux):
            continue
        i0, i1 = ux[a], ux[b]
        agg = collections.defaultdict(lambda: [0, 0])
        for n, d, gx, s, e in rows[i0 + 1:i1 + 1]:
            k = (short(n), gx)
            agg[k][0] += 1
            agg[k][1] += d
        its = b - a
        tot = sum(v[1] for v in agg.values())
        span = rows[i1][4] - rows[i0][4]
        out.append(f"{label}: {its} iterations, kernel time {tot / 1e6 / its:.3f} ms/iteration, "
                   f"wall {span / 1e6 / its:.3f} ms/iteration")
        out.append(f"{'us/it':>9} {'calls':>5} {'avg_us':>8} {'grid_x':>9}  kernel")
        for k, v in sorted(agg.items(), key=lambda kv: -kv[1][1])[:top]:
            out.append(f"{v[1] / 1e3 / its:9.1f} {v[0] / its:5.1f} {v[1] / v[0] / 1e3:8.1f} {k[1]:9d}  {k[0]}")
        out.append("")
    return "\n".join(out)


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("db")
    ap.add_argument("--top", type=int, default=30)
    ap.add_argument("--by-grid", default=None)
    ap.add_argument("--per-iteration", action="store_true")
    ap.add_argument("--last", type=int, default=20)
    a = ap.parse_args()
    print(summarize(a.db, a.top, a.by_grid, a.last))
    if a.per_iteration:
        print()
        print(per_iteration(a.db))
