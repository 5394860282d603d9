"""HBM traffic per kernel from two rocprofv3 counter runs (FETCH_SIZE and
WRITE_SIZE, KiB per dispatch), scaled by what the same counters read for a
plain copy of known size in the same program (the 256 MiB calibration copy
of bench.py).

python -m paper_1904_03317_amd.proftraffic <fetch results.db> <write results.db> [--cal-bytes N]
"""
import argparse
import collections
import re
import sqlite3


def short(name):
    return re.sub(r"\(.*$", "", name).replace("void gmg::dev::", "").replace("gmg::dev::", "")


def per_dispatch(db_path, counter):
    db = sqlite3.connect(db_path)
    rows = db.execute("select name, dispatch_id, counter_name, counter_value from pmc_events").fetchall()
    out = collections.defaultdict(float)
    names = {}
    for name, did, cname, val in rows:
        if cname.startswith(counter):
            out[did] += val
            names[did] = name
    grids = dict(db.execute("select dispatch_id, grid_x from kernels").fetchall())
    return out, names, grids


def summarize(fetch_db, write_db, cal_bytes=2 * (64 << 20) * 4):
    f, names, grids = per_dispatch(fetch_db, "FETCH_SIZE")
    w, _, _ = per_dispatch(write_db, "WRITE_SIZE")
    # calibration: the largest copy kernel (torch elementwise copy of 256 MiB)
    cal = [d for d, n in names.items() if "copy" in n.lower() or "elementwise" in n.lower()]
    cal_d = max(cal, key=lambda d: f.get(d, 0.0)) if cal else None
    lines = []
    if cal_d is not None:
        half = cal_bytes / 2 / 1024.0
        sf, sw = f[cal_d] / half, w.get(cal_d, 0.0) / half
        lines.append(f"calibration copy ({short(names[cal_d])}): FETCH {f[cal_d]:.0f} KiB, "
                     f"WRITE {w.get(cal_d, 0):.0f} KiB for {half:.0f} KiB each way -> factors {sf:.3f}, {sw:.3f}")
    else:
        sf = sw = 1.0
    agg = collections.defaultdict(lambda: [0, 0.0, 0.0])
    for d, n in names.items():
        key = (short(n), grids.get(d))
        a = agg[key]
        a[0] += 1
        a[1] += f.get(d, 0.0) / sf
        a[2] += w.get(d, 0.0) / sw
    lines.append(f"{'kernel':60s} {'grid_x':>9} {'n':>5} {'fetch KiB/disp':>15} {'write KiB/disp':>15}")
    for (n, g), (c, fb, wb) in sorted(agg.items(), key=lambda kv: -(kv[1][1] + kv[1][2])):
        lines.append(f"{n[:60]:60s} {g if g else 0:9d} {c:5d} {fb / c:15.1f} {wb / c:15.1f}")
    return "\n".join(lines)


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("fetch_db")
    ap.add_argument("write_db")
    ap.add_argument("--cal-bytes", type=int, default=2 * (64 << 20) * 4)
    a = ap.parse_args()
    print(summarize(a.fetch_db, a.write_db, a.cal_bytes))
