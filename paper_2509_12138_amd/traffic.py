"""HBM traffic per launch of a kernel from rocprofv3 counter runs.

FETCH_SIZE and WRITE_SIZE (KiB per dispatch) are collected in two separate
``rocprofv3 --pmc`` runs of the same command, and two more runs of
``bench.py --copy-calibration`` (a plain 512 MiB device copy) give the scale
of each counter: factor = bytes the copy moved / bytes the counter reported.

    python -m paper_2509_12138_amd.traffic --kernel k_raster_bwd_chunked \
        --fetch F.csv --write W.csv --copy-fetch CF.csv --copy-write CW.csv \
        --plan 16x16,lpt,64,4,1 --out paper_2509_12138_amd/hbm_traffic.json

The entry records the kernel, the plan and a hash of the kernel's source
file; bench.py reports the traffic only while that hash still matches.
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os

HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCES = {"k_raster_bwd_chunked": "raster.hip", "k_raster_bwd": "raster.hip",
                  "k_raster_fwd": "raster.hip", "k_dup_reduce": "raster.hip",
                  "k_raster_bwd_chunked_q": "raster.hip", "k_raster_fwd_part": "raster.hip",
                  "k_raster_fwd_join": "raster.hip",
                  "k_project_bwd_adam": "project.hip", "k_project": "project.hip",
                  "k_ssim": "loss.hip", "k_adam": "adam.hip", "k_radix_scatter": "binsort.hip",
                  "k_emit": "binsort.hip", "k_depth_keys": "binsort.hip"}
COPY_BYTES = 512 * 1024 * 1024


def source_hash(kernels):
    """Hash of the source files of a '+'-joined list of kernels."""
    h = hashlib.sha256()
    for src in sorted({KERNEL_SOURCES[k.split("<")[0]] for k in kernels.split("+")}):
        with open(os.path.join(HERE, "csrc", src), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def counter_kib(path, kernel, counter):
    """Mean counter value over the dispatches of `kernel`: a plain name
    matches every instantiation, a name with template arguments (e.g.
    "k_raster_fwd<16, 16, 4>") only that one."""
    vals = []
    want = kernel.replace(" ", "")
    with open(path) as f:
        for r in csv.DictReader(f):
            name = r["Kernel_Name"].split("(")[0].replace("void ", "").strip()
            full = name.split("::")[-1].replace(" ", "")
            base = full.split("<")[0]
            if (full == want if "<" in want else base == want) and r["Counter_Name"] == counter:
                vals.append(float(r["Counter_Value"]))
    if not vals:
        raise SystemExit(f"no {counter} samples for {kernel} in {path}")
    return sum(vals) / len(vals), len(vals)


def copy_factor(path, counter):
    kib, _ = counter_kib(path, "__amd_rocclr_copyBuffer", counter)
    return COPY_BYTES / (kib * 1024.0)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--kernel", required=True,
                    help="kernel name, or several joined by '+' (bytes are summed per launch)")
    ap.add_argument("--fetch", required=True)
    ap.add_argument("--write", required=True)
    ap.add_argument("--copy-fetch", required=True)
    ap.add_argument("--copy-write", required=True)
    ap.add_argument("--plan", required=True,
                    help="tile,schedule,chunk,fwd_waves,deterministic e.g. 16x16,lpt,64,4,1")
    ap.add_argument("--command", default="", help="the command the counters were taken on")
    ap.add_argument("--out", required=True)
    a = ap.parse_args(argv)
    f_kib = w_kib = 0.0
    nf = nw = []
    for k in a.kernel.split("+"):
        fk, n1 = counter_kib(a.fetch, k, "FETCH_SIZE")
        wk, n2 = counter_kib(a.write, k, "WRITE_SIZE")
        f_kib += fk
        w_kib += wk
        nf = nf + [n1]
        nw = nw + [n2]
    ff = copy_factor(a.copy_fetch, "FETCH_SIZE")
    fw = copy_factor(a.copy_write, "WRITE_SIZE")
    entry = dict(kernel=a.kernel, plan=a.plan, source_sha256_16=source_hash(a.kernel),
                 fetch_kib=f_kib, write_kib=w_kib, dispatches=[nf, nw],
                 fetch_factor=ff, write_factor=fw,
                 bytes_per_launch=f_kib * 1024.0 * ff + w_kib * 1024.0 * fw,
                 command=a.command)
    table = {}
    if os.path.exists(a.out):
        with open(a.out) as f:
            table = json.load(f)
    table[f"{a.kernel}|{a.plan}"] = entry
    with open(a.out, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)
    print(json.dumps(entry, indent=1))


def lookup(path, kernel, plan):
    """bytes_per_launch of a recorded entry whose source hash still matches."""
    try:
        with open(path) as f:
            table = json.load(f)
    except (OSError, ValueError):
        return None
    e = table.get(f"{kernel}|{plan}")
    if not e or e.get("source_sha256_16") != source_hash(kernel):
        return None
    return e["bytes_per_launch"]


if __name__ == "__main__":
    main()
