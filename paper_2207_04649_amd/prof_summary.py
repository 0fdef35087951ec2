"""Summaries of rocprofv3 output, per kernel.

    python -m paper_2207_04649_amd.prof_summary trace RESULTS_DB [command...]
        kernel-trace summary (calls, average / median / min / max microseconds,
        total ms)
        from the rocpd SQLite file of ``rocprofv3 --kernel-trace``;

    python -m paper_2207_04649_amd.prof_summary hbm FETCH_CSV WRITE_CSV MIB [command...]
        HBM bytes per dispatch from two ``rocprofv3 --pmc`` runs (FETCH_SIZE, then
        WRITE_SIZE; KiB per dispatch).  Each counter is scaled by what it reads
        for a plain copy of known size in the same run (``bench.py
        --copy-calibration MIB`` first copies MIB MiB device to device): the
        largest reading of the copy kernels gives each scale (MIB MiB over the
        KiB read).
"""
from __future__ import annotations

import collections
import csv
import re
import sqlite3
import sys


def short_name(name: str) -> str:
    """The library's kernel name (k_* or kb_*, with template arguments), else a short prefix."""
    m = re.search(r"\b(kb?_\w+)(<[^>]*>)?", name)
    return m.group(0) if m else name.split("(")[0][:60]


def summary(db: str) -> list[tuple]:
    """[(kernel, calls, avg, median, min, max microseconds, total milliseconds)], by total."""
    c = sqlite3.connect(db)
    durs = collections.defaultdict(list)
    for name, dur in c.execute("select name, duration from kernels"):
        durs[name].append(dur)
    rows = []
    for name, d in durs.items():
        d = sorted(d)
        med = d[len(d) // 2] if len(d) % 2 else (d[len(d) // 2 - 1] + d[len(d) // 2]) / 2
        rows.append((short_name(name), len(d), sum(d) / len(d) / 1e3, med / 1e3, d[0] / 1e3, d[-1] / 1e3,
                     sum(d) / 1e6))
    rows.sort(key=lambda r: -r[6])
    return rows


def render_trace(db: str, command: str = "") -> str:
    out = []
    if command:
        out.append(f"command: {command}")
    out.append(f"{'kernel':40s} {'calls':>6s} {'avg_us':>10s} {'median_us':>10s} {'min_us':>10s} {'max_us':>10s} "
               f"{'total_ms':>10s}")
    for n, cnt, avg, med, mn, mx, tot in summary(db):
        out.append(f"{n[:40]:40s} {cnt:6d} {avg:10.2f} {med:10.2f} {mn:10.2f} {mx:10.2f} {tot:10.3f}")
    return "\n".join(out)


def _counter_rows(path: str, counter: str):
    """Per-kernel lists of the counter's KiB per dispatch, and the rows of copy kernels in order."""
    per = collections.defaultdict(list)
    copies = []
    with open(path) as fh:
        for r in csv.DictReader(fh):
            if r["Counter_Name"] != counter:
                continue
            name = r["Kernel_Name"]
            value = float(r["Counter_Value"])
            if "copyBuffer" in name or "elementwise_kernel" in name:
                copies.append((name, value))
                continue
            per[short_name(name)].append(value)
    return per, copies


def hbm_table(fetch_csv: str, write_csv: str, calib_mib: float):
    """[(kernel, dispatches, fetch KiB, write KiB, scaled MB per dispatch)], scales."""
    f, fcopy = _counter_rows(fetch_csv, "FETCH_SIZE")
    w, wcopy = _counter_rows(write_csv, "WRITE_SIZE")
    if not fcopy or not wcopy:
        raise SystemExit("no calibration copy found in the counter files")
    want_kib = calib_mib * 1024.0
    fetch_scale = want_kib / max(v for _, v in fcopy)
    write_scale = want_kib / max(v for _, v in wcopy)
    rows = []
    for k, vals in f.items():
        fa = sum(vals) / len(vals)
        wa = sum(w[k]) / len(w[k]) if k in w else 0.0
        rows.append((k, len(vals), fa, wa, (fa * fetch_scale + wa * write_scale) * 1024.0 / 1e6))
    rows.sort(key=lambda t: -t[4])
    return rows, fetch_scale, write_scale


def render_hbm(fetch_csv: str, write_csv: str, calib_mib: float, command: str = "") -> str:
    rows, fs, ws = hbm_table(fetch_csv, write_csv, calib_mib)
    out = []
    if command:
        out.append(f"command: {command}")
    out.append(f"calibration: a {calib_mib:g} MiB device copy; FETCH_SIZE scaled x{fs:.3f}, WRITE_SIZE x{ws:.3f}")
    out.append(f"{'kernel':40s} {'dispatches':>10s} {'FETCH_KiB':>12s} {'WRITE_KiB':>12s} {'HBM_MB':>10s}")
    for k, n, fa, wa, mb in rows:
        out.append(f"{k[:40]:40s} {n:10d} {fa:12.1f} {wa:12.1f} {mb:10.1f}")
    return "\n".join(out)


if __name__ == "__main__":
    if len(sys.argv) >= 3 and sys.argv[1] == "trace":
        print(render_trace(sys.argv[2], " ".join(sys.argv[3:])))
    elif len(sys.argv) >= 5 and sys.argv[1] == "hbm":
        print(render_hbm(sys.argv[2], sys.argv[3], float(sys.argv[4]), " ".join(sys.argv[5:])))
    else:
        raise SystemExit(__doc__)
