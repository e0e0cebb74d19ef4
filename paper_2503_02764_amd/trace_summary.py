"""Summaries of rocprofv3 output for the profile records.

    python -m paper_2503_02764_amd.trace_summary trace <kernel_trace.csv>
        [--kernel REGEX] [--after REGEX] [--min-us US] [--min-frac F] [--top N]
    python -m paper_2503_02764_amd.trace_summary pmc <counter_collection.csv>
        [--kernel REGEX] [--scale S] [--min-frac F]

`trace`: per kernel name and grid size, launches, mean / median / min / max
duration.  With --after, only dispatches after the first one whose name
matches that pattern count (e.g. the first step's coefficient kernel, which
leaves out an autotuner's launches before it); with --min-us, dispatches
shorter than that are dropped (launches enqueued after a solve's device stop
flag return at once); with --min-frac, only dispatches lasting at least
that fraction of the longest of their kernel and grid (kernels that run
every multigrid level with one grid size keep their finest level).
`pmc`: per kernel name and grid, the counter's mean value per dispatch
(KiB, as rocprofv3 reports FETCH_SIZE and WRITE_SIZE) over the dispatches
whose value is at least --min-frac of that kernel's largest, times --scale
(the copy-kernel calibration), in MB.
Prints Markdown tables.
"""
from __future__ import annotations

import argparse
import csv
import re
import statistics
from collections import defaultdict


def _col(row, *names):
    for n in names:
        if n in row:
            return row[n]
    raise KeyError(names)


def _grid(row):
    try:
        return int(_col(row, "Grid_Size", "Grid_Size_X")) * \
            int(row.get("Grid_Size_Y", 1) or 1) * int(row.get("Grid_Size_Z", 1) or 1)
    except (KeyError, ValueError):
        return 0


def trace(path, kernel=None, after=None, min_us=0.0, top=25, min_frac=0.0):
    rows = list(csv.DictReader(open(path)))
    rows.sort(key=lambda r: int(_col(r, "Start_Timestamp")))
    started = after is None
    groups = defaultdict(list)
    for r in rows:
        name = _col(r, "Kernel_Name")
        if not started:
            if re.search(after, name):
                started = True
            else:
                continue
        if kernel and not re.search(kernel, name):
            continue
        us = (int(_col(r, "End_Timestamp")) - int(_col(r, "Start_Timestamp"))) / 1e3
        if us < min_us:
            continue
        groups[(name, _grid(r))].append(us)
    if min_frac > 0:
        groups = {k: [x for x in v if x >= min_frac * max(v)]
                  for k, v in groups.items()}
    out = ["| kernel | grid (threads) | launches | mean µs | median µs | min µs | max µs | total ms |",
           "|---|---|---|---|---|---|---|---|"]
    items = sorted(groups.items(), key=lambda kv: -sum(kv[1]))[:top]
    for (name, grid), v in items:
        out.append(f"| `{name[:90]}` | {grid} | {len(v)} | {statistics.mean(v):.2f} | "
                   f"{statistics.median(v):.2f} | {min(v):.2f} | {max(v):.2f} | "
                   f"{sum(v) / 1e3:.3f} |")
    total = sum(sum(v) for v in groups.values())
    out.append("")
    out.append(f"Total over the rows selected: {total / 1e3:.3f} ms in "
               f"{sum(len(v) for v in groups.values())} dispatches.")
    return "\n".join(out)


def pmc(path, kernel=None, scale=1.0, min_frac=0.5):
    rows = list(csv.DictReader(open(path)))
    groups = defaultdict(list)
    counter = None
    for r in rows:
        name = _col(r, "Kernel_Name")
        if kernel and not re.search(kernel, name):
            continue
        counter = _col(r, "Counter_Name")
        groups[(name, _grid(r))].append(float(_col(r, "Counter_Value")))
    out = [f"| kernel | grid | dispatches kept / all | {counter} KiB (raw mean) | calibrated MB |",
           "|---|---|---|---|---|"]
    for (name, grid), v in sorted(groups.items(), key=lambda kv: -max(kv[1])):
        top = max(v)
        keep = [x for x in v if x >= min_frac * top]
        m = statistics.mean(keep)
        out.append(f"| `{name[:90]}` | {grid} | {len(keep)} / {len(v)} | {m:.0f} | "
                   f"{m * 1024 * scale / 1e6:.2f} |")
    return "\n".join(out)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("mode", choices=("trace", "pmc"))
    ap.add_argument("path")
    ap.add_argument("--kernel")
    ap.add_argument("--after")
    ap.add_argument("--min-us", type=float, default=0.0)
    ap.add_argument("--top", type=int, default=25)
    ap.add_argument("--scale", type=float, default=1.0)
    ap.add_argument("--min-frac", type=float, default=None,
                    help="trace: default 0 (keep all); pmc: default 0.5")
    a = ap.parse_args()
    if a.mode == "trace":
        print(trace(a.path, a.kernel, a.after, a.min_us, a.top, a.min_frac or 0.0))
    else:
        print(pmc(a.path, a.kernel, a.scale,
                  0.5 if a.min_frac is None else a.min_frac))


if __name__ == "__main__":
    main()
