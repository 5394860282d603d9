"""HBM traffic per kernel dispatch from two rocprofv3 counter runs of the
same command (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch), each scaled by
what the same counter reads for the 256 MiB device-to-device calibration
copy that bench.py performs first (a rocclr copyBuffer dispatch).

python -m paper_1904_03317_amd.proftraffic <fetch results.db> <write results.db> [--json OUT]

With --json, also writes the bytes per launch of the two level-operator
units on the largest level of each precision (the operator apply y = A x and
one Chebyshev step, each pass 1 fam_op + pass 2 fam_sum), keyed by the
SHA-256 of the kernel source they were measured on, and those of the FP64
tiled leaf operator (pass 1 + pass 2, keyed by the SHA-256 of its source).
"""
import argparse
import collections
import hashlib
import json
import os
import re
import sqlite3

CAL_KIB = 256 * 1024  # the calibration copy reads and writes 256 MiB


def short(name):
    return re.sub(r"\(.*$", "", name).replace("void gmg::dev::", "").replace("gmg::dev::", "")


def per_dispatch(db_path, counter):
    db = sqlite3.connect(db_path)
    rows = db.execute("select name, dispatch_id, counter_name, counter_value from pmc_events").fetchall()
    val = collections.defaultdict(float)
    names = {}
    for name, did, cname, v in rows:
        if cname.startswith(counter):
            val[did] += v
            names[did] = name
    grids = dict(db.execute("select dispatch_id, grid_x from kernels").fetchall())
    return val, names, grids


def analyse(fetch_db, write_db):
    f, names, grids = per_dispatch(fetch_db, "FETCH_SIZE")
    w, wnames, wgrids = per_dispatch(write_db, "WRITE_SIZE")
    cal_f = max((d for d, n in names.items() if "copyBuffer" in n), key=lambda d: f[d])
    cal_w = max((d for d, n in wnames.items() if "copyBuffer" in n), key=lambda d: w[d])
    sf, sw = f[cal_f] / CAL_KIB, w[cal_w] / CAL_KIB
    agg = collections.defaultdict(lambda: [0, 0.0, 0, 0.0])
    for d, n in names.items():
        a = agg[(short(n), grids.get(d, 0))]
        a[0] += 1
        a[1] += f[d] / sf * 1024.0
    for d, n in wnames.items():
        a = agg[(short(n), wgrids.get(d, 0))]
        a[2] += 1
        a[3] += w[d] / sw * 1024.0
    table = {k: (v[0], v[1] / max(v[0], 1), v[2], v[3] / max(v[2], 1)) for k, v in agg.items()}
    return (sf, sw, f[cal_f], w[cal_w]), table


def units(table):
    """bytes per launch of apply and Chebyshev step on the largest level, per
    precision: the fam_op / fam_sum grids with the most plain-epilogue
    dispatches (the bench's timing loop) identify the largest level."""
    out = {}
    for tname, key in (("double", "fp64"), ("float", "fp32")):
        def grid_of(kern):
            c = [(v[0], g) for (n, g), v in table.items() if n == kern]
            return max(c)[1] if c else None
        go = grid_of(f"fam_op<3, 2, {tname}, 0>")
        gs = grid_of(f"fam_sum<3, 2, {tname}, 0>")
        if go is None or gs is None:
            continue

        def bytes_of(n, g):
            v = table.get((n, g))
            return None if v is None else v[1] + v[3]

        ap = [bytes_of(f"fam_op<3, 2, {tname}, 0>", go), bytes_of(f"fam_sum<3, 2, {tname}, 0>", gs)]
        ch = [bytes_of(f"fam_op<3, 2, {tname}, 1>", go), bytes_of(f"fam_sum<3, 2, {tname}, 1>", gs)]
        out[key] = {"fam_op_grid": go, "fam_sum_grid": gs,
                    "apply_bytes_per_launch": None if None in ap else sum(ap),
                    "cheb_bytes_per_launch": None if None in ch else sum(ch),
                    "apply_parts": ap, "cheb_parts": ch}
    # the FP64 tiled leaf operator (apply without the dot: the bench's timing
    # loop): pass 1 and pass 2, the grids with the most dispatches
    def most(prefix):
        c = [(v[0], n, g) for (n, g), v in table.items() if n.startswith(prefix)]
        if not c:
            return None
        _, n, g = max(c)
        v = table[(n, g)]
        return v[1] + v[3]
    l1, l2 = most("leaf_tiles<"), most("leaf_pass2<")
    if l1 is not None:
        out["leaf"] = {"bytes_per_launch": l1 + (l2 or 0.0), "parts": [l1, l2]}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("fetch_db")
    ap.add_argument("write_db")
    ap.add_argument("--json", default=None)
    ap.add_argument("--top", type=int, default=24)
    a = ap.parse_args()
    (sf, sw, cf, cw), table = analyse(a.fetch_db, a.write_db)
    print(f"calibration copy 256 MiB: FETCH_SIZE {cf:.0f} KiB, WRITE_SIZE {cw:.0f} KiB -> scale {sf:.3f}, {sw:.3f}")
    print(f"{'kernel':44s} {'grid_x':>9} {'n':>5} {'fetch MB/disp':>14} {'write MB/disp':>14}")
    for (n, g), (nf, fb, nw, wb) in sorted(table.items(), key=lambda kv: -(kv[1][1] + kv[1][3]))[:a.top]:
        print(f"{n[:44]:44s} {g:9d} {nf:5d} {fb / 1e6:14.2f} {wb / 1e6:14.2f}")
    u = units(table)
    for k, v in u.items():
        if k == "leaf":
            print(f"leaf operator: {v['bytes_per_launch'] / 1e6:.1f} MB/launch (pass 1, pass 2: "
                  f"{', '.join('-' if x is None else f'{x / 1e6:.1f}' for x in v['parts'])} MB)")
            continue
        print(f"{k}: apply {v['apply_bytes_per_launch'] / 1e6:.1f} MB/launch, "
              f"Chebyshev step {v['cheb_bytes_per_launch'] / 1e6:.1f} MB/launch "
              f"(fam_op grid {v['fam_op_grid']}, fam_sum grid {v['fam_sum_grid']})")
    if a.json:
        src = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc", "famkernels.hpp")
        u["kernel_source_sha256"] = hashlib.sha256(open(src, "rb").read()).hexdigest()
        lsrc = os.path.join(os.path.dirname(src), "kernels.hpp")
        u["leaf_kernel_source_sha256"] = hashlib.sha256(open(lsrc, "rb").read()).hexdigest()
        u["calibration_scale"] = {"fetch": sf, "write": sw}
        json.dump(u, open(a.json, "w"), indent=1)


if __name__ == "__main__":
    main()
