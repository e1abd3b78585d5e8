"""Summaries of rocprofv3 output (kernel-trace statistics and PMC counters).

`summarize_stats(dir)` reads a `--kernel-trace --stats --output-format csv`
directory; `kernel_counter(dir, name_part, grid=None, lds=None)` returns the
per-dispatch values of one counter (FETCH_SIZE / WRITE_SIZE are KiB per
dispatch) for the dispatches of one kernel, selected by name and launch shape.
"""
from __future__ import annotations

import csv
import glob
import hashlib
import json
import os
import re


def _rows(directory: str, pattern: str):
    files = glob.glob(os.path.join(directory, "**", pattern), recursive=True)
    out = []
    for f in files:
        with open(f, newline="") as fh:
            out.extend(csv.DictReader(fh))
    return out


def short_name(name: str) -> str:
    name = name.replace("(anonymous namespace)::", "")
    return re.sub(r"\(.*", "", name)[:100]


def summarize_stats(directory: str, top: int = 20):
    rows = _rows(directory, "*kernel_stats.csv")
    out = []
    for r in rows:
        out.append({"kernel": short_name(r.get("Name", r.get("KernelName", ""))),
                    "calls": int(float(r.get("Calls", 0))),
                    "total_ns": float(r.get("TotalDurationNs", 0)),
                    "avg_ns": float(r.get("AverageNs", 0)),
                    "pct": float(r.get("Percentage", 0))})
    out.sort(key=lambda x: -x["total_ns"])
    return out[:top]


def kernel_counter(directory: str, name_part: str, counter: str, grid: int | None = None,
                   lds: int | None = None):
    vals = []
    for r in _rows(directory, "*counter_collection.csv"):
        if name_part not in r.get("Kernel_Name", ""):
            continue
        if r.get("Counter_Name") != counter:
            continue
        if grid is not None and int(float(r.get("Grid_Size", -1))) != grid:
            continue
        if lds is not None and int(float(r.get("LDS_Block_Size", r.get("Lds_Block_Size", -1)))) != lds:
            continue
        vals.append(float(r["Counter_Value"]))
    return vals


def source_digest(paths) -> str:
    h = hashlib.sha256()
    for p in paths:
        with open(p, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def write_stats_markdown(rows, path: str, command: str, note: str = ""):
    with open(path, "w") as fh:
        fh.write("# rocprofv3 kernel statistics\n\n")
        if note:
            fh.write(note.strip() + "\n\n")
        fh.write("Command (repository root, MI355X):\n\n```\n" + command + "\n```\n\n")
        fh.write("| kernel | calls | total us | avg us | % of GPU time |\n|---|---|---|---|---|\n")
        for r in rows:
            fh.write(f"| `{r['kernel']}` | {r['calls']} | {r['total_ns'] / 1e3:.1f} | "
                     f"{r['avg_ns'] / 1e3:.1f} | {r['pct']:.2f} |\n")


def load_traffic(path: str, sources) -> dict | None:
    """Counter-derived traffic recorded for a kernel, or None if its sources changed since."""
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("source_digest") != source_digest(sources):
        return None
    return rec
