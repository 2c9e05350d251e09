"""Summarise rocprofv3 CSV output into a short text table (per-kernel counts, durations and
counter averages), so that a profile can be kept as a few KB of text.

    python -m paper_1903_08741_amd.prof_summary DIR [--kernels REGEX] [--by-grid]

DIR is the directory given to rocprofv3 with -d; every *_kernel_stats.csv,
*_kernel_trace.csv and *_counter_collection.csv below it is read.  Output:
  * kernel statistics (calls, total ms, average us, share of GPU time), from the trace
    when present (otherwise from the stats file);
  * for counter runs, per kernel (name up to its template arguments' end) and counter: the
    number of dispatches, the mean and the sum of the counter value.
With --by-grid, both tables are split by launch grid size (threads in x and y), and each
row also reports the launches whose duration (or counter value) is at least half the
row's maximum: in a batched solve the launches after the last sample stopped do no work
and would dilute the mean.
"""
from __future__ import annotations

import argparse
import csv
import glob
import os
import re
import sys
from collections import defaultdict


def _files(root, suffix):
    return sorted(glob.glob(os.path.join(root, "**", f"*{suffix}"), recursive=True))


def _short(name):
    name = name.strip()
    # drop the argument list of the kernel's signature, keep template arguments
    depth, out = 0, []
    for ch in name:
        if ch == "(" and depth == 0:
            break
        depth += ch == "<"
        depth -= ch == ">"
        out.append(ch)
    s = "".join(out)
    return re.sub(r"\s+", " ", s.replace("void ", "").replace("rmg::", "")).strip()


def _full(values):
    """Count and mean of the values at least half the maximum."""
    mx = max(values)
    full = [v for v in values if v >= 0.5 * mx]
    return len(full), sum(full) / len(full)


def grid_kernel_table(root, pattern):
    rows = defaultdict(list)
    for f in _files(root, "kernel_trace.csv"):
        with open(f, newline="") as fh:
            for r in csv.DictReader(fh):
                k = _short(r.get("Kernel_Name", ""))
                if pattern and not re.search(pattern, k):
                    continue
                g = f"{r.get('Grid_Size_X', '?')}x{r.get('Grid_Size_Y', '?')}"
                rows[(k, g)].append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-3)
    out = ["| kernel | grid (threads) | calls | avg us | full calls | full avg us |", "|---|---|---|---|---|---|"]
    for (k, g), v in sorted(rows.items()):
        n, m = _full(v)
        out.append(f"| {k} | {g} | {len(v)} | {sum(v) / len(v):.2f} | {n} | {m:.2f} |")
    return out


def grid_counter_table(root, pattern):
    acc = defaultdict(list)
    for f in _files(root, "counter_collection.csv"):
        with open(f, newline="") as fh:
            for r in csv.DictReader(fh):
                k = _short(r.get("Kernel_Name", ""))
                if pattern and not re.search(pattern, k):
                    continue
                acc[(k, r.get("Grid_Size", "?"), r["Counter_Name"])].append(float(r["Counter_Value"]))
    if not acc:
        return []
    out = ["| kernel | grid (threads) | counter | dispatches | mean | full dispatches | full mean |",
           "|---|---|---|---|---|---|---|"]
    for (k, g, c), v in sorted(acc.items()):
        n, m = _full(v)
        out.append(f"| {k} | {g} | {c} | {len(v)} | {sum(v) / len(v):.6g} | {n} | {m:.6g} |")
    return out


def kernel_table(root, pattern):
    rows = defaultdict(lambda: [0, 0.0])
    traces = _files(root, "kernel_trace.csv")
    if traces:
        for f in traces:
            with open(f, newline="") as fh:
                for r in csv.DictReader(fh):
                    k = _short(r.get("Kernel_Name", ""))
                    d = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-6
                    rows[k][0] += 1
                    rows[k][1] += d
    else:
        for f in _files(root, "kernel_stats.csv"):
            with open(f, newline="") as fh:
                for r in csv.DictReader(fh):
                    k = _short(r["Name"])
                    rows[k][0] += int(r["Calls"])
                    rows[k][1] += float(r["TotalDurationNs"]) * 1e-6
    tot = sum(v[1] for v in rows.values()) or 1.0
    out = ["| kernel | calls | total ms | avg us | % |", "|---|---|---|---|---|"]
    for k, (c, ms) in sorted(rows.items(), key=lambda kv: -kv[1][1]):
        if pattern and not re.search(pattern, k):
            continue
        out.append(f"| {k} | {c} | {ms:.1f} | {1e3 * ms / max(c, 1):.2f} | {100 * ms / tot:.1f} |")
    return out


def counter_table(root, pattern):
    acc = defaultdict(lambda: [0, 0.0])
    for f in _files(root, "counter_collection.csv"):
        with open(f, newline="") as fh:
            for r in csv.DictReader(fh):
                k = _short(r.get("Kernel_Name", ""))
                if pattern and not re.search(pattern, k):
                    continue
                key = (k, r["Counter_Name"])
                acc[key][0] += 1
                acc[key][1] += float(r["Counter_Value"])
    if not acc:
        return []
    out = ["| kernel | counter | dispatches | mean per dispatch | sum |", "|---|---|---|---|---|"]
    for (k, c), (n, v) in sorted(acc.items()):
        out.append(f"| {k} | {c} | {n} | {v / n:.6g} | {v:.6g} |")
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("dir")
    ap.add_argument("--kernels", default="", help="only kernels whose name matches this regex")
    ap.add_argument("--by-grid", action="store_true", help="split by launch grid size")
    a = ap.parse_args(argv)
    lines = []
    if a.by_grid:
        if _files(a.dir, "kernel_trace.csv"):
            lines += grid_kernel_table(a.dir, a.kernels)
        ct = grid_counter_table(a.dir, a.kernels)
    else:
        if _files(a.dir, "kernel_trace.csv") or _files(a.dir, "kernel_stats.csv"):
            lines += kernel_table(a.dir, a.kernels)
        ct = counter_table(a.dir, a.kernels)
    if ct:
        lines += [""] + ct
    if not lines:
        print(f"no rocprofv3 CSV output under {a.dir}", file=sys.stderr)
        return 1
    print("\n".join(lines))
    return 0


if __name__ == "__main__":
    sys.exit(main())
