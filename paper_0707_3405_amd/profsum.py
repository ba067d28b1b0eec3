"""Summarise rocprofv3 CSV output (``-f csv``) into a short text table.

    python -m paper_0707_3405_amd.profsum trace <dir>     per-kernel calls / total / mean time
    python -m paper_0707_3405_amd.profsum pmc <dir>       per-kernel mean of each counter (KiB for
                                                          FETCH_SIZE / WRITE_SIZE), per dispatch

<dir> is the rocprofv3 output directory; the kernel-trace or counter CSV is
found below it.  Only the standard library is used.
"""
from __future__ import annotations

import collections
import csv
import glob
import os
import sys


def _find(d, pattern):
    hits = sorted(glob.glob(os.path.join(d, "**", pattern), recursive=True))
    if not hits:
        raise SystemExit(f"no {pattern} under {d}")
    return hits[0]


def _col(header, *keys):
    low = [h.lower() for h in header]
    for k in keys:
        for i, h in enumerate(low):
            if h == k:
                return i
    for k in keys:
        for i, h in enumerate(low):
            if k in h:
                return i
    raise SystemExit(f"no column among {keys} in {header}")


def trace(d, top=30):
    path = _find(d, "*kernel_trace.csv")
    agg = collections.defaultdict(list)
    with open(path) as f:
        rd = csv.reader(f)
        hdr = next(rd)
        ik, i0, i1 = _col(hdr, "kernel_name"), _col(hdr, "start_timestamp"), _col(hdr, "end_timestamp")
        for row in rd:
            agg[row[ik]].append(int(row[i1]) - int(row[i0]))
    tot = sum(sum(v) for v in agg.values())
    lines = [f"{'kernel':72s} {'calls':>7s} {'total_ms':>10s} {'mean_us':>9s} {'pct':>6s}"]
    for k, v in sorted(agg.items(), key=lambda kv: -sum(kv[1]))[:top]:
        lines.append(f"{k[:72]:72s} {len(v):7d} {sum(v) / 1e6:10.2f} {sum(v) / len(v) / 1e3:9.1f} "
                     f"{100 * sum(v) / tot:6.1f}")
    return "\n".join(lines)


def pmc(d):
    path = _find(d, "*counter_collection.csv")
    agg = collections.defaultdict(lambda: collections.defaultdict(list))
    with open(path) as f:
        rd = csv.reader(f)
        hdr = next(rd)
        ik, ic, iv = _col(hdr, "kernel_name"), _col(hdr, "counter_name"), _col(hdr, "counter_value")
        idisp = _col(hdr, "dispatch_id", "correlation_id")
        per = collections.defaultdict(float)
        names = {}
        for row in rd:
            key = (row[idisp], row[ic])
            per[key] += float(row[iv])
            names[row[idisp]] = row[ik]
        for (disp, cn), v in per.items():
            agg[names[disp]][cn].append(v)
    lines = []
    for k, cs in sorted(agg.items()):
        parts = [f"{cn} mean {sum(v) / len(v):.1f} over {len(v)} dispatches" for cn, v in sorted(cs.items())]
        lines.append(f"{k[:90]}: " + "; ".join(parts))
    return "\n".join(lines)


if __name__ == "__main__":
    if len(sys.argv) != 3 or sys.argv[1] not in ("trace", "pmc"):
        raise SystemExit(__doc__)
    print(trace(sys.argv[2]) if sys.argv[1] == "trace" else pmc(sys.argv[2]))
