"""Summarise a rocprofv3 kernel-trace database (rocpd SQLite output): per
kernel total time, dispatch count and average duration, optionally per grid
size, as short text for the profiles/ folder.

python -m paper_1904_03317_amd.profsummary <results.db> [--by-grid PATTERN]
"""
import argparse
import collections
import re
import sqlite3


def short(name):
    name = re.sub(r"\(.*$", "", name)
    return name.replace("void gmg::dev::", "").replace("gmg::dev::", "")


def summarize(db_path, top=30, by_grid=None):
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
            out.append(f"  grid_x {gx:10d} threads: n={len(v):5d} avg {sum(v) / len(v) / 1e3:9.2f} us "
                       f"min {min(v) / 1e3:9.2f} us")
    return "\n".join(out)


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("db")
    ap.add_argument("--top", type=int, default=30)
    ap.add_argument("--by-grid", default=None)
    a = ap.parse_args()
    print(summarize(a.db, a.top, a.by_grid))
