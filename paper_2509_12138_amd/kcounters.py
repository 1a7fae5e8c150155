"""Per-kernel hardware-counter rates from rocprofv3 runs of ``bench.py``.

Each pass is one ``rocprofv3 --kernel-trace --pmc <counters>`` run of the
same bench command, so every counter value belongs to a dispatch whose
duration the same run's kernel trace records (joined on the dispatch id).

    python -m paper_2509_12138_amd.kcounters --run DIR [--run DIR ...] \
        --kernel 'k_raster_bwd_chunked<16, 16>' [--kernel ...] \
        [--copy-fetch CF.csv --copy-write CW.csv] [--out FILE.json] [--plan P]

Rates per kernel (mean over its dispatches, counters summed over the
chip's counter instances, as rocprofv3 reports them):
* VALU busy      = SQ_ACTIVE_INST_VALU / CU count / GRBM_GUI_ACTIVE-per-XCC
                   (the share of the kernel's GPU cycles in which a CU
                   issues vector instructions; the VALUBusy formula);
* VALU lanes     = SQ_THREAD_CYCLES_VALU / (64 SQ_ACTIVE_INST_VALU), the
                   share of lanes active in those instructions;
* LDS bandwidth  = 64 x (SQ_INSTS_LDS_{LOAD,STORE,ATOMIC}_BANDWIDTH) bytes
                   over the dispatch's duration, against 128 B per clock per
                   CU (256 CUs at 2.4 GHz: 78.6 TB/s);
* LDS busy       = SQ_LDS_IDX_ACTIVE / CU count / cycles, and bank-conflict
                   stalls SQ_LDS_BANK_CONFLICT / CU count / cycles;
* HBM            = FETCH_SIZE and WRITE_SIZE (KiB) scaled by a plain copy's
                   readings, over the duration, against 8 TB/s.
"""
from __future__ import annotations

import argparse
import collections
import csv
import glob
import json
import os
import re

CUS, XCDS, CLOCK = 256, 8, 2.4e9
LDS_PEAK = 128.0 * CUS * CLOCK
HBM_PEAK = 8.0e12
COPY_BYTES = 512 * 1024 * 1024


def short(name):
    n = re.sub(r"\(.*", "", name)
    return n.replace("void ", "").replace("gsmi::", "").strip()


def load_run(d):
    """(durations ns by dispatch id, {dispatch id: (kernel, {counter: value})})."""
    trace = glob.glob(os.path.join(d, "**", "*kernel_trace.csv"), recursive=True)
    pmc = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    if not trace or not pmc:
        raise SystemExit(f"{d}: needs a kernel_trace.csv and a counter_collection.csv")
    dur = {}
    for r in csv.DictReader(open(trace[0])):
        dur[r["Dispatch_Id"]] = int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
    ctr = collections.defaultdict(lambda: [None, {}])
    for r in csv.DictReader(open(pmc[0])):
        e = ctr[r["Dispatch_Id"]]
        e[0] = short(r["Kernel_Name"])
        e[1][r["Counter_Name"]] = e[1].get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    return dur, ctr


def copy_factor(path, counter):
    vals = [float(r["Counter_Value"]) for r in csv.DictReader(open(path))
            if "copyBuffer" in r["Kernel_Name"] and r["Counter_Name"] == counter]
    if not vals:
        raise SystemExit(f"no {counter} for the copy kernel in {path}")
    return COPY_BYTES / (sum(vals) / len(vals) * 1024.0)


def summarise(runs, kernels, ff=None, wf=None):
    out = {}
    for k in kernels:
        acc = collections.defaultdict(list)
        durs = []
        for dur, ctr in runs:
            for did, (name, vals) in ctr.items():
                if name.replace(" ", "") != k.replace(" ", ""):
                    continue
                ns = dur.get(did)
                if ns is None:
                    continue
                durs.append(ns)
                for c, v in vals.items():
                    acc[c].append((v, ns))
        if not durs:
            continue
        e = dict(kernel=k, dispatches=len(durs), mean_us=sum(durs) / len(durs) / 1e3)

        def rate(c, f):
            xs = acc.get(c)
            return None if not xs else sum(f(v, ns) for v, ns in xs) / len(xs)

        def mean(c):
            xs = acc.get(c)
            return None if not xs else sum(v for v, _ in xs) / len(xs)

        gui = mean("GRBM_GUI_ACTIVE")
        if mean("SQ_ACTIVE_INST_VALU") is not None and gui:
            e["valu_busy"] = mean("SQ_ACTIVE_INST_VALU") / CUS / (gui / XCDS)
        if mean("SQ_THREAD_CYCLES_VALU") is not None and mean("SQ_ACTIVE_INST_VALU"):
            e["valu_lanes"] = mean("SQ_THREAD_CYCLES_VALU") / (64.0 * mean("SQ_ACTIVE_INST_VALU"))
        for c in ("SQ_INSTS_VALU", "SQ_INSTS_LDS", "SQ_WAVES", "SQ_ACTIVE_INST_LDS"):
            if mean(c) is not None:
                e[c] = mean(c)
        bw = [c for c in ("SQ_INSTS_LDS_LOAD_BANDWIDTH", "SQ_INSTS_LDS_STORE_BANDWIDTH",
                          "SQ_INSTS_LDS_ATOMIC_BANDWIDTH") if c in acc]
        if bw:
            by = sum(mean(c) for c in bw) * 64.0
            e["lds_bytes"] = by
            e["lds_tbps"] = sum(rate(c, lambda v, ns: 64.0 * v / (ns * 1e-9)) for c in bw) / 1e12
            e["lds_frac"] = e["lds_tbps"] * 1e12 / LDS_PEAK
        if mean("SQ_LDS_IDX_ACTIVE") is not None and gui:
            e["lds_busy"] = mean("SQ_LDS_IDX_ACTIVE") / CUS / (gui / XCDS)
        if mean("SQ_LDS_BANK_CONFLICT") is not None and gui:
            e["lds_conflict"] = mean("SQ_LDS_BANK_CONFLICT") / CUS / (gui / XCDS)
        if ff and mean("FETCH_SIZE") is not None and mean("WRITE_SIZE") is not None:
            by = mean("FETCH_SIZE") * 1024.0 * ff + mean("WRITE_SIZE") * 1024.0 * wf
            e["hbm_bytes"] = by
            e["hbm_tbps"] = (rate("FETCH_SIZE", lambda v, ns: v * 1024.0 * ff / (ns * 1e-9)) +
                             rate("WRITE_SIZE", lambda v, ns: v * 1024.0 * wf / (ns * 1e-9))) / 1e12
            e["hbm_frac"] = e["hbm_tbps"] * 1e12 / HBM_PEAK
        out[k] = e
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--run", action="append", required=True)
    ap.add_argument("--kernel", action="append", required=True)
    ap.add_argument("--copy-fetch")
    ap.add_argument("--copy-write")
    ap.add_argument("--out")
    ap.add_argument("--db", help="merge the entries into this JSON table, keyed kernel|plan")
    ap.add_argument("--plan", default="", help="tile,schedule,chunk,fwd_waves,deterministic")
    ap.add_argument("--command", default="", help="the bench command the passes profiled")
    args = ap.parse_args()
    runs = [load_run(d) for d in args.run]
    ff = copy_factor(args.copy_fetch, "FETCH_SIZE") if args.copy_fetch else None
    wf = copy_factor(args.copy_write, "WRITE_SIZE") if args.copy_write else None
    res = summarise(runs, args.kernel, ff, wf)
    keys = ["dispatches", "mean_us", "valu_busy", "valu_lanes", "lds_tbps", "lds_frac",
            "lds_busy", "lds_conflict", "hbm_bytes", "hbm_tbps", "hbm_frac"]
    print("| kernel | " + " | ".join(keys) + " |")
    print("|---|" + "---:|" * len(keys))
    for k, e in res.items():
        cells = []
        for c in keys:
            v = e.get(c)
            cells.append("–" if v is None else (f"{v:.4g}" if isinstance(v, float) else str(v)))
        print(f"| {k} | " + " | ".join(cells) + " |")
    if ff:
        print(f"\ncopy factors: FETCH_SIZE x{ff:.4f}, WRITE_SIZE x{wf:.4f}")
    if args.out:
        with open(args.out, "w") as f:
            json.dump(res, f, indent=1, sort_keys=True)
    if args.db:
        from .traffic import source_hash
        table = {}
        if os.path.exists(args.db):
            with open(args.db) as f:
                table = json.load(f)
        for k, e in res.items():
            table[f"{k}|{args.plan}"] = dict(e, plan=args.plan, command=args.command,
                                             source_sha256_16=source_hash(k))
        with open(args.db, "w") as f:
            json.dump(table, f, indent=1, sort_keys=True)


def lookup(path, kernel, plan):
    """The recorded rates of a kernel under a plan, while its source is unchanged."""
    from .traffic import source_hash
    try:
        with open(path) as f:
            table = json.load(f)
    except (OSError, ValueError):
        return None
    e = table.get(f"{kernel}|{plan}")
    if not e or e.get("source_sha256_16") != source_hash(kernel):
        return None
    return e


if __name__ == "__main__":
    main()
