"""Per-kernel shader counters from rocprofv3 --pmc runs (rocpd SQLite output),
averaged per dispatch for each (kernel, grid size), with the derived rates:

  VALU busy      = SQ_ACTIVE_INST_VALU / (CUs * GRBM_GUI_ACTIVE), GRBM_GUI_ACTIVE
                   the largest of its per-XCD instances
  FP32/FP64 rate = 64 SQ_INSTS_VALU_FLOPS_FP32/64 / kernel duration (the
                   counters add 2 per FMA wave-instruction, 1 per add or
                   multiply: times 64 lanes)
  occupancy      = SQ_WAVE_CYCLES / (CUs * GRBM_GUI_ACTIVE) waves per CU
                   (SQ_WAVE_CYCLES counts in quad-cycles: times 4)
  LDS bank conflict = SQ_LDS_BANK_CONFLICT / (SQ_LDS_IDX_ACTIVE - conflicts)
  LDS busy       = SQ_LDS_IDX_ACTIVE / (CUs * GRBM_GUI_ACTIVE)
  wait / active  = SQ_WAIT_ANY, SQ_ACTIVE_INST_ANY against SQ_WAVE_CYCLES

python -m paper_1904_03317_amd.profcounters <results.db> [<results.db> ...] [--match REGEX] [--cus 256]

Several databases (one per counter pass of the same command) are merged by
kernel name, grid size and dispatch order within that group.
"""
import argparse
import collections
import re
import sqlite3


def short(name):
    name = re.sub(r"\(.*$", "", name)
    return name.replace("void gmg::dev::", "").replace("gmg::dev::", "")


def load(db_path):
    """{(kernel, grid): [ {counter: value, '_dur_ns': d}, ... in dispatch order ]}"""
    db = sqlite3.connect(db_path)
    vals = collections.defaultdict(lambda: collections.defaultdict(float))
    names = {}
    for name, did, cname, v in db.execute(
            "select name, dispatch_id, counter_name, counter_value from pmc_events"):
        # GRBM counters: one instance per XCD, each counting the same
        # dispatch, so the maximum (as the vendor's derived metrics take it);
        # shader counters: summed over their instances
        if cname.startswith("GRBM_"):
            vals[did][cname] = max(vals[did][cname], v)
        else:
            vals[did][cname] += v
        names[did] = name
    kern = {did: (gx, dur) for did, gx, dur in db.execute("select dispatch_id, grid_x, duration from kernels")}
    out = collections.defaultdict(list)
    for did in sorted(vals):
        gx, dur = kern.get(did, (0, 0))
        rec = dict(vals[did])
        rec["_dur_ns"] = dur
        out[(short(names[did]), gx)].append(rec)
    return out


def merge(dbs):
    merged = collections.defaultdict(list)
    for d in dbs:
        for key, recs in d.items():
            m = merged[key]
            for i, r in enumerate(recs):
                if i < len(m):
                    for k, v in r.items():
                        if k == "_dur_ns":
                            m[i].setdefault("_durs", []).append(v)
                        else:
                            m[i][k] = v
                else:
                    r = dict(r)
                    r["_durs"] = [r.pop("_dur_ns")]
                    m.append(r)
    return merged


def derive(recs, cus):
    n = len(recs)
    avg = collections.defaultdict(float)
    for r in recs:
        for k, v in r.items():
            if k != "_durs":
                avg[k] += v / n
    durs = [min(r["_durs"]) for r in recs if r.get("_durs")]
    dur = sum(durs) / len(durs) if durs else 0.0
    g = avg.get("GRBM_GUI_ACTIVE", 0.0)
    d = {"n": n, "dur_us": dur / 1e3}
    if g:
        if "SQ_ACTIVE_INST_VALU" in avg:
            d["valu_busy_pct"] = 100.0 * avg["SQ_ACTIVE_INST_VALU"] / cus / g
        if "SQ_WAVE_CYCLES" in avg:
            d["waves_per_cu"] = 4.0 * avg["SQ_WAVE_CYCLES"] / cus / g
        if "SQ_LDS_IDX_ACTIVE" in avg:
            d["lds_busy_pct"] = 100.0 * avg["SQ_LDS_IDX_ACTIVE"] / cus / g
    if "SQ_LDS_BANK_CONFLICT" in avg and avg.get("SQ_LDS_IDX_ACTIVE", 0) > avg["SQ_LDS_BANK_CONFLICT"]:
        d["lds_conflict_ratio"] = avg["SQ_LDS_BANK_CONFLICT"] / (avg["SQ_LDS_IDX_ACTIVE"] - avg["SQ_LDS_BANK_CONFLICT"])
    if dur:
        for p in ("32", "64"):
            k = f"SQ_INSTS_VALU_FLOPS_FP{p}"
            if k in avg:
                d[f"fp{p}_tflops"] = 64.0 * avg[k] / (dur * 1e-9) / 1e12
    wc = avg.get("SQ_WAVE_CYCLES", 0.0)
    if wc:
        for k, lab in (("SQ_WAIT_ANY", "wait_any_pct"), ("SQ_WAIT_INST_ANY", "wait_issue_pct"),
                       ("SQ_ACTIVE_INST_ANY", "active_any_pct")):
            if k in avg:
                d[lab] = 100.0 * avg[k] / wc
    for k in ("SQ_WAVES", "SQ_INSTS_VALU", "SQ_INSTS_LDS", "SQ_INSTS_VMEM_RD", "SQ_INSTS_VMEM_WR",
              "SQ_INSTS_VALU_FLOPS_FP32", "SQ_INSTS_VALU_FLOPS_FP64"):
        if k in avg:
            d[k] = avg[k]
    return d


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("dbs", nargs="+")
    ap.add_argument("--match", default=".")
    ap.add_argument("--cus", type=int, default=256)
    ap.add_argument("--min-us", type=float, default=50.0, help="only (kernel, grid) groups at least this long")
    a = ap.parse_args()
    merged = merge([load(p) for p in a.dbs])
    rx = re.compile(a.match)
    cols = ["n", "dur_us", "valu_busy_pct", "fp32_tflops", "fp64_tflops", "waves_per_cu", "lds_busy_pct",
            "lds_conflict_ratio", "wait_any_pct", "wait_issue_pct", "active_any_pct"]
    print(f"{'kernel':36s} {'grid_x':>9} " + " ".join(f"{c:>10s}" for c in cols))
    rows = []
    for (k, g), recs in merged.items():
        if not rx.search(k):
            continue
        d = derive(recs, a.cus)
        if d["dur_us"] >= a.min_us:
            rows.append((k, g, d))
    for k, g, d in sorted(rows, key=lambda t: -t[2]["dur_us"]):
        print(f"{k[:36]:36s} {g:9d} " + " ".join(
            f"{d[c]:10.3g}" if isinstance(d.get(c), float) else f"{d.get(c, '-')!s:>10s}" for c in cols))


if __name__ == "__main__":
    main()
