"""Summaries of rocprofv3 output for the direction kernels.

    python -m paper_1909_02894_amd.profiling stats <kernel_stats.csv> <out.md> "<command>"
    python -m paper_1909_02894_amd.profiling traffic <fetch.csv> <write.csv> <copy_fetch.csv> \
        <copy_write.csv> <grid | square> <out.json> "<command>"
    python -m paper_1909_02894_amd.profiling trace <kernel_trace.csv> <out.md> "<command>" [filter]

`stats` turns a ``--kernel-trace --stats`` kernel table into a short markdown
summary.  `trace` splits the dispatches of every direction kernel (those whose name
matches the filter regex) in a
``--kernel-trace`` CSV by context: launches between two launches of the same
kernel (a kernel replayed alone, its data still in its XCD's L2) and all the
others (the real alternating x, y order), with the median of each.  `traffic` takes two ``--pmc FETCH_SIZE`` / ``--pmc WRITE_SIZE``
counter-collection CSVs (KiB per dispatch) of a solve, and the same two
counters for a plain 1 GiB device copy, scales each counter by
(bytes the copy moves) / (what the counter reads for the copy), and writes the
median HBM bytes per launch for every direction kernel, keyed by the names
bench.py uses (e.g. ``y_stage_f64_512x512_curved``), and for every batch phase
kernel, keyed by its instantiation (``batch_kernels``), plus a digest of the
kernel sources so that stale numbers are not reported.
"""
from __future__ import annotations

import csv
import hashlib
import json
import os
import re
import statistics
import sys
from collections import defaultdict

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
MODE_NAMES = {0: "flat", 1: "flat_pml", 2: "curved"}
COPY_BYTES = 1 << 30


def kernel_sources_digest() -> str:
    """Digest of the direction-kernel sources (the code the counters measure)."""
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_1909_02894_amd", "csrc")
    for f in sorted(os.listdir(d)):
        if f in ("fft_line.hpp", "stage_kernels.hpp", "batch_kernels.hpp") or \
                (f.startswith(("stages_", "batch_f")) and f.endswith(".hip")):
            h.update(open(os.path.join(d, f), "rb").read())
    return h.hexdigest()[:16]


_STAGE = re.compile(r"(?<![a-z0-9_])stage_kernel<(double|float), (\d+), (\d+), (\d+), (true|false), (\d), (\d)>")


def bench_name(kernel: str, grid: str):
    """Map a stage-kernel instantiation to bench.py's name, e.g.
    'void dirac::stage_kernel<double, 512, 8, 2, true, 2, 1>(...)' ->
    'y_stage_f64_512x512_curved' (template arguments T, N, R, L, COLS, MODE, CPT)."""
    m = _STAGE.search(kernel)
    if not m:
        return None
    t, n, r, lines, cols, mode, cpt = m.groups()
    if grid == "square":                  # every solve in the run is n x n
        grid = f"{n}x{n}"
    return f"{'y' if cols == 'true' else 'x'}_stage_{'f64' if t == 'double' else 'f32'}_{grid}_{MODE_NAMES[int(mode)]}"


def short_name(kernel: str) -> str:
    k = kernel.replace("void dirac::", "").replace("dirac::", "")
    return k.split("(")[0]


def stats(csv_path: str, out_md: str, command: str, top: int = 14):
    rows = list(csv.DictReader(open(csv_path)))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    lines = ["# rocprofv3 kernel statistics", "", "Command (run from the repository root):", "", "```",
             command, "```", "",
             "| kernel | calls | avg (us) | min (us) | max (us) | share |",
             "|---|---:|---:|---:|---:|---:|"]
    for r in rows[:top]:
        lines.append(f"| `{short_name(r['Name'])}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} | "
                     f"{float(r['MinNs']) / 1e3:.2f} | {float(r['MaxNs']) / 1e3:.2f} | {float(r['Percentage']):.1f}% |")
    open(out_md, "w").write("\n".join(lines) + "\n")


def _per_kernel(path, counter):
    d = defaultdict(list)
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] == counter:
            d[r["Kernel_Name"]].append(float(r["Counter_Value"]) * 1024.0)   # KiB -> bytes
    return d


def traffic(fetch_csv, write_csv, copy_fetch_csv, copy_write_csv, grid, out_json, command):
    cf = _per_kernel(copy_fetch_csv, "FETCH_SIZE")
    cw = _per_kernel(copy_write_csv, "WRITE_SIZE")
    copy_k = [k for k in cf if "copyBuffer" in k or "copy" in k.lower()]
    if not copy_k:
        raise SystemExit("no copy kernel in the calibration runs")
    k0 = max(copy_k, key=lambda k: statistics.median(cf[k]))
    f_scale = COPY_BYTES / statistics.median(cf[k0])
    w_scale = COPY_BYTES / statistics.median(cw[k0])
    fe = _per_kernel(fetch_csv, "FETCH_SIZE")
    wr = _per_kernel(write_csv, "WRITE_SIZE")
    out = {"kernel_sources": kernel_sources_digest(), "command": command,
           "calibration": {"copy_kernel": short_name(k0), "copy_bytes_each_way": COPY_BYTES,
                           "fetch_scale": f_scale, "write_scale": w_scale},
           "kernels": {}}
    # several instantiations (schedules) map to one name -- the autotuner runs
    # them all; keep each one, and mark the one dispatched most often
    for k in fe:
        name = bench_name(k, grid)
        if not name or k not in wr:
            continue
        rec = {"fetch_bytes": round(statistics.median(fe[k]) * f_scale),
               "write_bytes": round(statistics.median(wr[k]) * w_scale), "dispatches": len(fe[k])}
        rec["bytes"] = rec["fetch_bytes"] + rec["write_bytes"]
        ent = out["kernels"].setdefault(name, {"by_instantiation": {}})
        ent["by_instantiation"][short_name(k)] = rec
    # batch phase kernels, keyed by instantiation (one per direction, length and schedule)
    out["batch_kernels"] = {}
    for k in fe:
        sk = short_name(k)
        if not sk.startswith(("batch_group_kernel", "batch_multi_kernel")) or k not in wr:
            continue
        rec = {"fetch_bytes": round(statistics.median(fe[k]) * f_scale),
               "write_bytes": round(statistics.median(wr[k]) * w_scale), "dispatches": len(fe[k])}
        rec["bytes"] = rec["fetch_bytes"] + rec["write_bytes"]
        out["batch_kernels"][sk] = rec
    for name, ent in out["kernels"].items():
        top = max(ent["by_instantiation"].items(), key=lambda kv: kv[1]["dispatches"])
        ent.update(top[1])
        ent["instantiation"] = top[0]
    json.dump(out, open(out_json, "w"), indent=1)
    return out


def trace(csv_path: str, out_md: str, command: str, filt: str = r"stage_kernel|batch_group_kernel|batch_multi_kernel"):
    rows = sorted(csv.DictReader(open(csv_path)), key=lambda r: int(r["Start_Timestamp"]))
    seq = [(short_name(r["Kernel_Name"]), int(r["Start_Timestamp"]), int(r["End_Timestamp"])) for r in rows]
    alt, iso = defaultdict(list), defaultdict(list)
    for i in range(1, len(seq) - 1):
        k, t0, t1 = seq[i]
        if not re.search(filt, k):
            continue
        same = seq[i - 1][0] == k and seq[i + 1][0] == k
        (iso if same else alt)[k].append((t1 - t0) / 1e3)
    lines = ["# rocprofv3 kernel trace: direction-kernel durations by context", "", "Command:", "", "```", command,
             "```", "", "| kernel | in sequence: launches | median (us) | replayed alone: launches | median (us) |",
             "|---|---:|---:|---:|---:|"]
    keys = sorted(set(alt) | set(iso), key=lambda k: -len(alt.get(k, [])))
    for k in keys:
        a, b = alt.get(k, []), iso.get(k, [])
        ma = f"{statistics.median(a):.2f}" if a else "-"
        mb = f"{statistics.median(b):.2f}" if b else "-"
        lines.append(f"| `{k}` | {len(a)} | {ma} | {len(b)} | {mb} |")
    open(out_md, "w").write("\n".join(lines) + "\n")


if __name__ == "__main__":
    if sys.argv[1] == "stats":
        stats(sys.argv[2], sys.argv[3], sys.argv[4])
    elif sys.argv[1] == "traffic":
        traffic(*sys.argv[2:9])
    elif sys.argv[1] == "trace":
        trace(*sys.argv[2:6])
    else:
        raise SystemExit(__doc__)
