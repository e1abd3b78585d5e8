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


# ---------------------------------------------------------------------------
# Command line: summaries under profiles/ from rocprofv3 csv directories
#   python -m paper_1911_02366_amd.profiling stats DIR OUT.md --command "..." [--note "..."]
#   python -m paper_1911_02366_amd.profiling traffic --fetch D --write D --copy-fetch D --copy-write D
#          --workload W --precision P --command "..." (repeatable)
# ---------------------------------------------------------------------------
_COPY_BYTES = 2 << 30     # bench.py --calibrate-copy copies a 2 GiB FP64 buffer


def _by_kernel(directory: str, counter: str):
    """{(short kernel name, grid): [per-dispatch values]} of one counter."""
    out = {}
    for r in _rows(directory, "*counter_collection.csv"):
        if r.get("Counter_Name") != counter:
            continue
        key = (short_name(r.get("Kernel_Name", "")), int(float(r.get("Grid_Size", -1))))
        out.setdefault(key, []).append(float(r["Counter_Value"]))
    return out


def _copy_scale(directory: str, counter: str) -> float:
    vals = [v for (k, _), vs in _by_kernel(directory, counter).items() if "copyBuffer" in k for v in vs]
    if not vals:
        raise RuntimeError(f"no copy kernel in {directory}")
    return _COPY_BYTES / (1024.0 * max(vals))


def traffic_summary(fetch: str, write: str, copy_fetch: str, copy_write: str, workload: str, precision: str,
                    commands, root: str = "."):
    fs, ws = _copy_scale(copy_fetch, "FETCH_SIZE"), _copy_scale(copy_write, "WRITE_SIZE")
    fk, wk = _by_kernel(fetch, "FETCH_SIZE"), _by_kernel(write, "WRITE_SIZE")
    mean = lambda v: sum(v) / len(v)
    rows = []
    for key, fv in fk.items():
        wv = wk.get(key, [0.0])
        rows.append(dict(kernel=key[0], grid=key[1], n=len(fv), fetch=mean(fv), write=mean(wv),
                         bytes=1024.0 * (mean(fv) * fs + mean(wv) * ws)))
    rows.sort(key=lambda r: -r["bytes"] * r["n"])
    csrc = os.path.join(root, "paper_1911_02366_amd", "csrc")
    pick = lambda part: [r for r in rows if part in r["kernel"]]
    recs = {}
    gemv = pick("schur_gemv_rem_kernel")
    if gemv:
        g = gemv[0]
        pulls = sorted(pick("bsr_pull_kernel"), key=lambda r: (abs(r["n"] - g["n"]), -r["n"]))
        b = g["bytes"] + (pulls[0]["bytes"] if pulls else 0.0)
        recs["schur_apply"] = (dict(kernel="schur_apply (schur_gemv_rem_kernel: T_e GEMV tiles and A_bb remainder "
                                           "rows; bsr_pull_kernel)", traffic_bytes_per_launch=b),
                               ["k_vec.hip"])
    inv = pick("gj_resident_kernel") or pick("gj_inverse_kernel")
    if inv:
        recs["inverse"] = (dict(kernel=inv[0]["kernel"], traffic_bytes_per_launch=inv[0]["bytes"]), ["k_inverse.hip"])
    gemms = sorted(pick("gemm_batched_kernel"), key=lambda r: -r["grid"])
    if len(gemms) >= 2:
        recs["gemm_s"] = (dict(kernel=gemms[0]["kernel"] + " (A_bi X_e)",
                               traffic_bytes_per_launch=gemms[0]["bytes"]), ["k_gemm.hip"])
        recs["gemm_x"] = (dict(kernel=gemms[1]["kernel"] + " (A_ii^-1 A_ib)",
                               traffic_bytes_per_launch=gemms[1]["bytes"]), ["k_gemm.hip"])
    md = os.path.join(root, "profiles", f"hbm_counters_{workload}_{precision}.md")
    for name, (rec, srcs) in recs.items():
        rec.update(workload=workload, precision=precision, fetch_scale=fs, write_scale=ws,
                   source_digest=source_digest([os.path.join(csrc, s) for s in srcs]),
                   commands=list(commands), summary=os.path.relpath(md, root))
        with open(os.path.join(root, "profiles", f"traffic_{name}_{workload}_{precision}.json"), "w") as fh:
            json.dump(rec, fh, indent=1)
    with open(md, "w") as fh:
        fh.write(f"# HBM traffic counters, {workload}, {precision.upper()}\n\n")
        fh.write("Commands (repository root, MI355X), one counter per run; the kernel-trace run writes the tile "
                 "choice to the autotune cache first, so the counter runs take the same tiles:\n\n```\n")
        fh.write("\n".join(commands) + "\n```\n\n")
        fh.write(f"Calibration: the {_COPY_BYTES >> 30} GiB device copy of `bench.py --calibrate-copy` gives "
                 f"scale factors fetch x{fs:.3f}, write x{ws:.3f} (bytes = KiB x 1024 x factor).\n\n")
        fh.write("| kernel | grid (threads) | dispatches | FETCH KiB/dispatch | WRITE KiB/dispatch | "
                 "calibrated bytes/dispatch |\n|---|---|---|---|---|---|\n")
        for r in rows[:24]:
            fh.write(f"| `{r['kernel']}` | {r['grid']} | {r['n']} | {r['fetch']:.0f} | {r['write']:.0f} | "
                     f"{r['bytes']:.4g} |\n")
        fh.write("\nTraffic records (read by bench.py while the kernels' sources are unchanged): " +
                 ", ".join(f"`traffic_{k}_{workload}_{precision}.json` {v[0]['traffic_bytes_per_launch']:.4g} B"
                           for k, v in recs.items()) + "\n")
    return recs


def _main(argv=None):
    import argparse
    ap = argparse.ArgumentParser(prog="python -m paper_1911_02366_amd.profiling")
    sub = ap.add_subparsers(dest="what", required=True)
    st = sub.add_parser("stats")
    st.add_argument("directory")
    st.add_argument("out")
    st.add_argument("--command", required=True)
    st.add_argument("--note", default="")
    st.add_argument("--top", type=int, default=24)
    tr = sub.add_parser("traffic")
    for a in ("--fetch", "--write", "--copy-fetch", "--copy-write", "--workload", "--precision"):
        tr.add_argument(a, required=True)
    tr.add_argument("--command", action="append", default=[])
    a = ap.parse_args(argv)
    if a.what == "stats":
        write_stats_markdown(summarize_stats(a.directory, a.top), a.out, a.command, a.note)
    else:
        for k, (rec, _) in traffic_summary(a.fetch, a.write, a.copy_fetch, a.copy_write, a.workload, a.precision,
                                           a.command).items():
            print(k, f"{rec['traffic_bytes_per_launch']:.4g}")


if __name__ == "__main__":
    _main()
