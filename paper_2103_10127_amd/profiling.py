"""Summaries of rocprofv3 output (kernel traces and PMC counter collections).

    python -m paper_2103_10127_amd.profiling trace <kernel_trace.csv> [--match NAME]
    python -m paper_2103_10127_amd.profiling counters <counter_collection.csv> [--match NAME]
    python -m paper_2103_10127_amd.profiling traffic <fetch.csv> <write.csv> --match NAME

`traffic` turns one FETCH_SIZE and one WRITE_SIZE collection (separate runs,
both including the 1 GiB copy of `bench.py --copy-calibration`) into HBM bytes
per launch of the largest-grid launch group of the matched kernel: each counter
is scaled by (bytes the copy moves) / (what the counter reads for the copy).
The summary records a hash of the kernel's sources (`--sources apply`: the
uniform-grid apply, `--sources adaptive`: the adaptive-grid kernels);
`bench.py` reports the traffic only while the sources still hash to it.

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
    name = name.replace("(anonymous namespace)::", "")
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


COPY_GRID = 16777216          # launch grid of the 1 GiB calibration copy
COPY_KIB = (1 << 30) / 1024   # bytes the copy reads (and writes), in KiB
TRAFFIC_SOURCES = ("csrc/k_apply.hip", "csrc/rav_internal.h", "csrc/rav_index.h")
ADAPTIVE_SOURCES = ("csrc/k_adapt.hip", "csrc/rav_adapt.h")


def sources_hash(sources=TRAFFIC_SOURCES) -> str:
    import hashlib
    import os
    h = hashlib.sha256()
    here = os.path.dirname(os.path.abspath(__file__))
    for rel in sources:
        with open(os.path.join(here, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def traffic_summary(fetch_csv: str, write_csv: str, match: str, sources=TRAFFIC_SOURCES) -> dict:
    out = {}
    for counter, path in (("FETCH_SIZE", fetch_csv), ("WRITE_SIZE", write_csv)):
        rows = counter_summary(path)
        copy = [r for r in rows if "k_copy" in r["kernel"] and r["grid"] == COPY_GRID]
        kern = [r for r in rows if match in r["kernel"]]
        if not copy or not kern:
            raise SystemExit(f"{path}: calibration copy or kernel '{match}' missing")
        k = max(kern, key=lambda r: r["grid"])
        factor = COPY_KIB / copy[0][counter]
        out[counter] = dict(kernel=k["kernel"], grid=k["grid"], dispatches=k["dispatches"],
                            kib=k[counter], copy_kib=copy[0][counter], factor=factor,
                            bytes=k[counter] * factor * 1024)
    out["traffic_bytes"] = out["FETCH_SIZE"]["bytes"] + out["WRITE_SIZE"]["bytes"]
    out["sources_sha256"] = sources_hash(sources)
    return out


def read_traffic(path: str, sources=TRAFFIC_SOURCES):
    """Traffic per launch from a committed summary, or None when it is missing
    or the kernel sources changed since the counters were taken."""
    import os
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):   # the first kernel of a summary is the one reported
        if ":" in line and line.startswith("    "):
            k, v = line.strip().split(":", 1)
            fields.setdefault(k.strip(), v.strip())
    if fields.get("sources_sha256") != sources_hash(sources):
        return None
    try:
        return float(fields["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("mode", choices=["trace", "counters", "traffic"])
    ap.add_argument("path")
    ap.add_argument("path2", nargs="?")
    ap.add_argument("--match", default=None)
    ap.add_argument("--top", type=int, default=25)
    ap.add_argument("--sources", default="apply", choices=["apply", "adaptive"],
                    help="kernel sources whose hash the traffic summary records")
    a = ap.parse_args()
    if a.mode == "trace":
        res = trace_summary(a.path, a.match)
        print(f"{'calls':>6} {'grid':>9} {'avg_us':>10} {'median_us':>10} {'total_us':>11}  kernel")
        for r in res[: a.top]:
            print(f"{r['calls']:6d} {r['grid']:9d} {r['avg_us']:10.2f} {r['median_us']:10.2f} "
                  f"{r['total_us']:11.1f}  {_short(r['kernel'])}")
    elif a.mode == "counters":
        for r in counter_summary(a.path, a.match)[: a.top]:
            print(r)
    else:
        t = traffic_summary(a.path, a.path2, a.match,
                            ADAPTIVE_SOURCES if a.sources == "adaptive" else TRAFFIC_SOURCES)
        f, w = t["FETCH_SIZE"], t["WRITE_SIZE"]
        print(f"kernel: {f['kernel']} (grid {f['grid']}, {f['dispatches']} dispatches averaged)")
        for c, r in (("FETCH_SIZE", f), ("WRITE_SIZE", w)):
            print(f"{c}: {r['kib']:.1f} KiB per dispatch; copy of 1 GiB reads {r['copy_kib']:.1f} KiB"
                  f" -> factor {r['factor']:.4f} -> {r['bytes'] / 1e6:.2f} MB")
        print()
        print(f"    traffic_bytes_per_launch: {t['traffic_bytes']:.0f}")
        print(f"    sources_sha256: {t['sources_sha256']}")


if __name__ == "__main__":
    main()
