"""Summaries of rocprofv3 output (kernel traces and PMC counter collections).

    python -m paper_2103_10127_amd.profiling trace <kernel_trace.csv> [--match NAME]
    python -m paper_2103_10127_amd.profiling counters <counter_collection.csv> [--match NAME]

A kernel is launched on every level of the hierarchy with a different grid
size, so launches are grouped by (kernel name, grid size): the group with the
largest grid is the finest level.
"""
from __future__ import annotations

import argparse
import csv
import statistics
from collections import defaultdict


def _col(header, *cands):
    low = [h.lower() for h in header]
    for c in cands:
        for i, h in enumerate(low):
            if h == c.lower():
                return i
    for c in cands:
        for i, h in enumerate(low):
            if c.lower() in h:
                return i
    raise KeyError(f"none of {cands} in {header}")


def _short(name: str) -> str:
    name = name.split("(")[0] if "(" in name and "<" not in name.split("(")[0] else name
    return name[:110]


def trace_summary(path: str, match: str | None = None):
    rows = list(csv.reader(open(path)))
    head, data = rows[0], rows[1:]
    kn = _col(head, "Kernel_Name")
    ts = _col(head, "Start_Timestamp")
    te = _col(head, "End_Timestamp")
    gx = _col(head, "Grid_Size_X", "Grid_Size")
    groups = defaultdict(list)
    for r in data:
        name = r[kn]
        if match and match not in name:
            continue
        groups[(name, int(r[gx]))].append((int(r[te]) - int(r[ts])) * 1e-3)   # ns -> us
    out = []
    for (name, grid), d in sorted(groups.items(), key=lambda kv: -sum(kv[1])):
        out.append(dict(kernel=name, grid=grid, calls=len(d), total_us=sum(d), avg_us=statistics.mean(d),
                        median_us=statistics.median(d), min_us=min(d), max_us=max(d)))
    return out


def counter_summary(path: str, match: str | None = None):
    rows = list(csv.reader(open(path)))
    head, data = rows[0], rows[1:]
    kn = _col(head, "Kernel_Name")
    gx = _col(head, "Grid_Size_X", "Grid_Size")
    cn = _col(head, "Counter_Name")
    cv = _col(head, "Counter_Value")
    di = _col(head, "Dispatch_Id", "Correlation_Id")
    per = defaultdict(lambda: defaultdict(float))
    meta = {}
    for r in data:
        if match and match not in r[kn]:
            continue
        key = r[di]
        per[key][r[cn]] += float(r[cv])
        meta[key] = (r[kn], int(r[gx]))
    groups = defaultdict(lambda: defaultdict(list))
    for key, cnts in per.items():
        for c, v in cnts.items():
            groups[meta[key]][c].append(v)
    out = []
    for (name, grid), cnts in groups.items():
        out.append(dict(kernel=name, grid=grid,
                        **{c: statistics.mean(v) for c, v in cnts.items()}, dispatches=len(next(iter(cnts.values())))))
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("mode", choices=["trace", "counters"])
    ap.add_argument("path")
    ap.add_argument("--match", default=None)
    ap.add_argument("--top", type=int, default=25)
    a = ap.parse_args()
    if a.mode == "trace":
        res = trace_summary(a.path, a.match)
        print(f"{'calls':>6} {'grid':>9} {'avg_us':>10} {'median_us':>10} {'total_us':>11}  kernel")
        for r in res[: a.top]:
            print(f"{r['calls']:6d} {r['grid']:9d} {r['avg_us']:10.2f} {r['median_us']:10.2f} "
                  f"{r['total_us']:11.1f}  {_short(r['kernel'])}")
    else:
        for r in counter_summary(a.path, a.match)[: a.top]:
            print(r)


if __name__ == "__main__":
    main()
