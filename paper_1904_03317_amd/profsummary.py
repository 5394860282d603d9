"""Summarise a rocprofv3 kernel-trace database (rocpd SQLite output): per
kernel total time, dispatch count and average duration, optionally per grid
size, as short text for the profiles/ folder.

python -m paper_1904_03317_amd.profsummary <results.db> [--by-grid PATTERN [--last N]] [--per-iteration]

--last N: beside each grid's average over all its dispatches, the average
of its last N dispatches (bench.py's timed repetitions of one level
operator come last for each precision).

--per-iteration: kernel time per CG iteration inside the last timed solve of
each precision, delimited by the update_xr dispatches (one per iteration).

--small-grid T (with --per-iteration): also the share of that time in
level-kernel dispatches (transfers, level operator passes, coarse solve,
level vector kernels) of fewer than T threads: the coarse levels, since those
kernels launch about one thread per cell, shared node or family, so a
threshold between two levels' sizes splits the V-cycle by level.

--layout W,S,K (with --per-iteration): the bench run had W warm-up and S
timed solves per precision of K iterations each (default 1,2,12); the last
timed solve of each precision is summarised.
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


LEVEL_KERNEL = re.compile(r"(fam_|coarse_solve|seg_residual|seg_restrict_start|cheb_step|fill<)")


def per_iteration(db_path, top=24, solves=(("FP64-MG", 24, 35), ("FP32-MG", 60, 71)), small_grid=None):
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
        if small_grid:
            sm = [v for k, v in agg.items() if k[1] < small_grid and LEVEL_KERNEL.match(k[0])]
            st = sum(v[1] for v in sm)
            out.append(f"  dispatches of fewer than {small_grid} threads: {sum(v[0] for v in sm) / its:.1f} per "
                       f"iteration, {st / 1e6 / its:.3f} ms/iteration, {100 * st / tot:.1f} % of the kernel time")
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
    ap.add_argument("--small-grid", type=int, default=None)
    ap.add_argument("--layout", default="1,2,12")
    a = ap.parse_args()
    print(summarize(a.db, a.top, a.by_grid, a.last))
    if a.per_iteration:
        w, st, k = (int(t) for t in a.layout.split(","))
        n = w + st  # solves per precision; the last one of each is summarised
        solves = (("FP64-MG", (n - 1) * k, n * k - 1), ("FP32-MG", (2 * n - 1) * k, 2 * n * k - 1))
        print()
        print(per_iteration(a.db, a.top, solves, small_grid=a.small_grid))
