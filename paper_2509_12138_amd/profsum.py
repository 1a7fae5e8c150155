"""Summarise a rocprofv3 kernel trace of ``bench.py`` over its timed steps.

    python -m paper_2509_12138_amd.profsum <kernel_trace.csv> --steps K [--pmc <counter.csv> ...]

The timed window is the last K training steps of the run (a step runs from
its k_project to its projection backward + Adam); the renders bench.py runs
afterwards to count the work are left out.  Prints per-kernel
dispatch counts, mean durations and share of the step, as Markdown.  With
--pmc, adds per-dispatch FETCH_SIZE / WRITE_SIZE (KiB, raw counter values) averaged
over the dispatches of each kernel in counter-collection CSVs.
"""
from __future__ import annotations

import argparse
import collections
import csv
import re


def short(name):
    n = re.sub(r"\(.*", "", name)
    n = n.replace("void ", "").replace("gsmi::", "")
    return n


def timed_window(rows, steps):
    """The last `steps` training steps: each ends with the projection
    backward (fused with Adam) and begins at the projection before it;
    renders after training (bench.py's work count) are left out."""
    ends = [i for i, r in enumerate(rows)
            if short(r["Kernel_Name"]).split("<")[0] in ("k_project_bwd_adam", "k_project_bwd")]
    if len(ends) < steps:
        raise SystemExit(f"only {len(ends)} training steps in the trace; need {steps}")
    first = ends[-steps]
    start = max(i for i in range(first) if short(rows[i]["Kernel_Name"]).split("<")[0] ==
                "k_project")
    last = ends[-1]
    # the step's closing kernels (Adam step counter) run right after
    while last + 1 < len(rows) and short(rows[last + 1]["Kernel_Name"]).split("<")[0] in (
            "k_adam_step_inc", "k_adam"):
        last += 1
    return int(rows[start]["Start_Timestamp"]), int(rows[last]["End_Timestamp"]) + 1


def summarise(trace, steps):
    rows = list(csv.DictReader(open(trace)))
    rows.sort(key=lambda r: int(r["Start_Timestamp"]))
    t0, t1 = timed_window(rows, steps)
    dur = collections.defaultdict(list)
    for r in rows:
        s, e = int(r["Start_Timestamp"]), int(r["End_Timestamp"])
        if t0 <= s < t1:
            dur[short(r["Kernel_Name"])].append(e - s)
    total = sum(sum(v) for v in dur.values())
    return dur, total, (t1 - t0) / steps


def counters(paths):
    """Mean value per (kernel, counter) over every dispatch in the
    counter-collection CSVs."""
    acc = collections.defaultdict(list)
    for p in paths:
        for r in csv.DictReader(open(p)):
            acc[(short(r["Kernel_Name"]), r["Counter_Name"])].append(float(r["Counter_Value"]))
    return {k: sum(v) / len(v) for k, v in acc.items()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("trace")
    ap.add_argument("--steps", type=int, required=True)
    ap.add_argument("--pmc", nargs="*", default=[],
                    help="counter-collection CSVs with FETCH_SIZE / WRITE_SIZE")
    args = ap.parse_args()
    dur, total, wall = summarise(args.trace, args.steps)
    pmc = counters(args.pmc)
    print(f"Timed window: {args.steps} steps, {wall / 1e3:.1f} us per step (first k_project to "
          f"the last step's end), kernels busy {total / args.steps / 1e3:.1f} us per step\n")
    head = "| kernel | dispatches/step | mean us | us/step | share |"
    rule = "|---|---:|---:|---:|---:|"
    if pmc:
        head += " FETCH_SIZE KiB | WRITE_SIZE KiB |"
        rule += "---:|---:|"
    print(head)
    print(rule)
    for k, v in sorted(dur.items(), key=lambda kv: -sum(kv[1])):
        line = (f"| {k} | {len(v) / args.steps:.0f} | {sum(v) / len(v) / 1e3:.2f} | "
                f"{sum(v) / args.steps / 1e3:.2f} | {100.0 * sum(v) / total:.1f}% |")
        if pmc:
            f, w = pmc.get((k, "FETCH_SIZE")), pmc.get((k, "WRITE_SIZE"))
            line += (f" {f:.0f} |" if f is not None else " – |") + \
                    (f" {w:.0f} |" if w is not None else " – |")
        print(line)


if __name__ == "__main__":
    main()
