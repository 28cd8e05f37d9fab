"""Summaries of rocprofv3 output for the texsplat kernels (host-side tooling, no GPU work).

* `trace_table(db)` — markdown table of a `rocprofv3 --kernel-trace --stats` database
  (calls, total / average microseconds per kernel).
* `counter_means(csvs, kernel)` — per-dispatch means of the counters of one kernel in
  `rocprofv3 --pmc ... --output-format csv` results.
* `hbm_bytes(fetch_csv, write_csv, kernel, copy_bytes)` — HBM bytes per dispatch of a kernel
  from a FETCH_SIZE pass and a WRITE_SIZE pass (KiB per dispatch), each scaled by what the same
  counter reads for a device copy of known size run in the same program.
* `source_hash(kernel)` — hash of the sources a kernel is compiled from; a counter summary
  records it, and `read_traffic` returns the stored bytes only while the sources are unchanged
  (counters of an older kernel say nothing about the current one).
"""
from __future__ import annotations

import csv
import glob
import hashlib
import os
import re
import sqlite3

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)

# the source files each profiled kernel is built from
KERNEL_SOURCES = {
    "k_raster_fwd": ["csrc/raster.hip", "csrc/eval.h", "csrc/shade.h", "csrc/texture.h",
                     "csrc/ts_internal.h"],
    "k_preprocess": ["csrc/preprocess.hip", "csrc/ts_internal.h"],
    "k_bin_fill": ["csrc/binsort.hip", "csrc/binsort_layout.h", "csrc/ts_internal.h"],
    "k_raster_bwd": ["csrc/raster_bwd.hip", "csrc/eval.h", "csrc/shade.h", "csrc/shade_bwd.h",
                     "csrc/texture.h", "csrc/ts_internal.h"],
    "k_bwd_gather": ["csrc/raster_bwd.hip", "csrc/texture.h", "csrc/ts_internal.h"],
}


def source_hash(kernel: str) -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES[kernel]:
        with open(os.path.join(HERE, rel), "rb") as f:
            h.update(rel.encode() + b"\0" + f.read())
    return h.hexdigest()[:16]


def _short(name: str) -> str:
    s = name.split("(")[0].replace("void ", "")
    return s[:60]


def trace_table(db: str) -> str:
    cur = sqlite3.connect(db).cursor()
    rows = list(cur.execute(
        "select name, total_calls, total_duration, average, percentage from top_kernels"))
    out = ["| kernel | calls | total us | average us | % |", "|---|---:|---:|---:|---:|"]
    for n, c, t, a, p in rows:
        # the top_kernels view reports microseconds
        out.append(f"| `{_short(n)}` | {c} | {t:.1f} | {a:.1f} | {p:.2f} |")
    return "\n".join(out)


def kernel_durations_us(db: str, kernel: str) -> list:
    cur = sqlite3.connect(db).cursor()
    # the kernels table keeps start / end in nanoseconds
    return [(e - s) / 1e3 for n, s, e in cur.execute("select name, start, end from kernels order by start")
            if kernel in n]


def by_grid(db: str, kernel: str) -> str:
    """Dispatches of one kernel grouped by grid size: count and mean duration (us)."""
    cur = sqlite3.connect(db).cursor()
    acc = {}
    for n, gx, gy, gz, s0, e0 in cur.execute(
            "select name, grid_x, grid_y, grid_z, start, end from kernels order by start"):
        if kernel in n:
            acc.setdefault((gx, gy, gz), []).append((e0 - s0) / 1e3)
    out = [f"`{kernel}` by grid size:", "", "| grid (threads) | dispatches | mean us | min us | max us |",
           "|---|---:|---:|---:|---:|"]
    for g, d in sorted(acc.items(), key=lambda kv: -len(kv[1])):
        out.append(f"| {g[0]}x{g[1]}x{g[2]} | {len(d)} | {sum(d) / len(d):.1f} | {min(d):.1f} "
                   f"| {max(d):.1f} |")
    return "\n".join(out)


def first_dispatches(db: str, kernel: str, grid: int, first: int) -> str:
    """Mean duration (us) of the first `first` dispatches of a kernel at one grid size."""
    cur = sqlite3.connect(db).cursor()
    d = [(e0 - s0) / 1e3 for n, gx, s0, e0 in cur.execute(
        "select name, grid_x, start, end from kernels order by start") if kernel in n and gx == grid]
    d = d[:first]
    return (f"First {len(d)} dispatches of `{kernel}` at grid {grid}: mean {sum(d) / len(d):.1f} us "
            f"(min {min(d):.1f}, max {max(d):.1f})")


def _rows(csvs):
    for f in csvs:
        with open(f) as fh:
            yield from csv.DictReader(fh)


def counter_means(csvs, kernel: str) -> dict:
    acc = {}
    for r in _rows(csvs):
        if kernel not in r["Kernel_Name"]:
            continue
        acc.setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
    return {k: sum(v) / len(v) for k, v in acc.items()}


def _copy_counter(csvs, counter: str, copy_bytes: int) -> float:
    """The counter's reading (KiB) for the largest __amd_rocclr_copyBuffer dispatch."""
    best = None
    for r in _rows(csvs):
        if "copyBuffer" in r["Kernel_Name"] and r["Counter_Name"] == counter:
            g = int(r["Grid_Size"])
            if best is None or g > best[0]:
                best = (g, float(r["Counter_Value"]))
    if best is None:
        raise ValueError(f"no copy dispatch with {counter} in {csvs}")
    return best[1]


def hbm_bytes(fetch_csvs, write_csvs, kernel: str, copy_bytes: int) -> dict:
    f_k = counter_means(fetch_csvs, kernel)["FETCH_SIZE"]
    w_k = counter_means(write_csvs, kernel)["WRITE_SIZE"]
    f_c = _copy_counter(fetch_csvs, "FETCH_SIZE", copy_bytes)
    w_c = _copy_counter(write_csvs, "WRITE_SIZE", copy_bytes)
    f_scale = copy_bytes / (f_c * 1024.0)
    w_scale = copy_bytes / (w_c * 1024.0)
    return {"fetch_kib": f_k, "write_kib": w_k, "copy_fetch_kib": f_c, "copy_write_kib": w_c,
            "fetch_scale": f_scale, "write_scale": w_scale,
            "fetch_bytes": f_k * 1024.0 * f_scale, "write_bytes": w_k * 1024.0 * w_scale,
            "bytes": f_k * 1024.0 * f_scale + w_k * 1024.0 * w_scale}


_TRAFFIC = re.compile(r"^traffic_bytes_per_launch:\s*([0-9.eE+]+)\s*$", re.M)
_HASH = re.compile(r"^source_hash:\s*([0-9a-f]+)\s*$", re.M)


def read_traffic(path: str, kernel: str):
    """Bytes per launch recorded in a counter summary, or None if it is missing or was taken
    on other sources than the current ones."""
    if not os.path.exists(path):
        return None
    with open(path) as f:
        text = f.read()
    m, h = _TRAFFIC.search(text), _HASH.search(text)
    if not m or not h or h.group(1) != source_hash(kernel):
        return None
    return float(m.group(1))


def pmc_csvs(directory: str) -> list:
    return sorted(glob.glob(os.path.join(directory, "**", "*_counter_collection.csv"),
                            recursive=True))


def write_counter_summary(out: str, kernel: str, workload: str, fetch_dir: str, write_dir: str,
                          copy_bytes: int, commands: list, notes: str = "") -> dict:
    r = hbm_bytes(pmc_csvs(fetch_dir), pmc_csvs(write_dir), kernel, copy_bytes)
    lines = [
        f"# HBM traffic of `{kernel}`, {workload}",
        "",
        "Commands (run from the repository root on one MI355X; each pass is its own run):",
        "",
        *[f"    {c}" for c in commands],
        "",
        "Per dispatch of the kernel (mean over the dispatches of the run):",
        "",
        "| counter | KiB per dispatch | same counter for the device copy | scale | bytes per dispatch |",
        "|---|---:|---:|---:|---:|",
        f"| FETCH_SIZE | {r['fetch_kib']:.1f} | {r['copy_fetch_kib']:.1f} | {r['fetch_scale']:.4f} "
        f"| {r['fetch_bytes']:.4g} |",
        f"| WRITE_SIZE | {r['write_kib']:.1f} | {r['copy_write_kib']:.1f} | {r['write_scale']:.4f} "
        f"| {r['write_bytes']:.4g} |",
        "",
        f"The device copy moves {copy_bytes} bytes each way; scale = those bytes over the "
        "counter's reading for it.",
        "",
        notes,
        "",
        f"traffic_bytes_per_launch: {r['bytes']:.6g}",
        f"source_hash: {source_hash(kernel)}",
        "",
    ]
    with open(out, "w") as f:
        f.write("\n".join(lines))
    return r


def write_trace_summary(out: str, db: str, title: str, commands: list, notes: str = "",
                        grid_kernels=()):
    parts = [f"# {title}", "", "Command (run from the repository root on one MI355X):",
             "", *[f"    {c}" for c in commands], "",
             "rocprofv3 kernel-trace statistics (microseconds):", "", trace_table(db), ""]
    for k in grid_kernels:
        parts += [by_grid(db, k), ""]
    text = "\n".join(parts + [notes, ""])
    with open(out, "w") as f:
        f.write(text)


if __name__ == "__main__":
    import argparse
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    sub = ap.add_subparsers(dest="what", required=True)
    c = sub.add_parser("counters")
    c.add_argument("--kernel", required=True)
    c.add_argument("--workload", required=True)
    c.add_argument("--fetch", required=True)
    c.add_argument("--write", required=True)
    c.add_argument("--copy-bytes", type=int, default=256 << 20)
    c.add_argument("--command", action="append", default=[])
    c.add_argument("--notes", default="")
    c.add_argument("--out", required=True)
    t = sub.add_parser("trace")
    t.add_argument("--db", required=True)
    t.add_argument("--title", required=True)
    t.add_argument("--command", action="append", default=[])
    t.add_argument("--notes", default="")
    t.add_argument("--grid-kernel", action="append", default=[])
    t.add_argument("--first", nargs=3, metavar=("KERNEL", "GRID", "N"), action="append",
                   default=[])
    t.add_argument("--out", required=True)
    a = ap.parse_args()
    if a.what == "counters":
        print(write_counter_summary(a.out, a.kernel, a.workload, a.fetch, a.write, a.copy_bytes,
                                    a.command, a.notes))
    else:
        extra = [first_dispatches(a.db, k, int(g), int(n)) for k, g, n in a.first]
        notes = "\n\n".join(extra + ([a.notes] if a.notes else []))
        write_trace_summary(a.out, a.db, a.title, a.command, notes, a.grid_kernel)
