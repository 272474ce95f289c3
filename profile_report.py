#!/usr/bin/env python3
"""Text summaries of rocprofv3 results (rocpd SQLite databases).

  python profile_report.py stats RESULTS.db [--top N] [--command "..."]
      per-kernel dispatch count, average and total duration, share of time.

  python profile_report.py traffic --fetch FETCH.db --write WRITE.db --kernel SUBSTRING
                                   --source-hash HASH --out FILE.json [--command "..."]
      HBM bytes per launch of one kernel from a FETCH_SIZE run and a WRITE_SIZE
      run (KiB per dispatch), each scaled by what the same counter reads for a
      plain device copy of known size in the same run: the 1 GiB copy of
      fh_probe_ceilings (k_probe_copy), which bench.py runs first, or else the
      256 MiB torch copy of bench.py --pmc-calib.

  python profile_report.py table --fetch FETCH.db --write WRITE.db [--top N]
      the same calibrated bytes per launch for every kernel of the two runs,
      heaviest first.
"""
from __future__ import annotations

import argparse
import json
import sqlite3
import statistics

COPY_BYTES = 256 * 1024 * 1024


def kernel_stats(db):
    con = sqlite3.connect(db)
    rows = con.execute("select name, count(*), avg(duration), sum(duration) from kernels "
                       "group by name order by sum(duration) desc").fetchall()
    return rows


def cmd_stats(a):
    rows = kernel_stats(a.db)
    tot = sum(r[3] for r in rows)
    print("| calls | avg us | total us | share | kernel |")
    print("|---:|---:|---:|---:|---|")
    for name, n, avg, s in rows[: a.top]:
        print(f"| {n} | {avg / 1e3:.2f} | {s / 1e3:.1f} | {100 * s / tot:.1f}% | `{name[:110]}` |")


def counter_per_dispatch(db, counter, substr):
    con = sqlite3.connect(db)
    rows = con.execute("select kernel_name, value from counters_collection where counter_name = ?",
                       (counter,)).fetchall()
    mine = [v for n, v in rows if substr in n]
    return mine, rows


PROBE_COPY_BYTES = 1024 * 1024 * 1024


def copy_counter(rows):
    """(counter KiB, bytes) of the calibration copy: the probe's plain 1 GiB
    copy when present, else the largest elementwise copy (256 MiB)."""
    probe = [v for n, v in rows if "k_probe_copy(" in n]
    if probe:
        return min(probe), PROBE_COPY_BYTES
    cand = [v for n, v in rows if "copy" in n.lower() or "elementwise" in n.lower()]
    return (max(cand), COPY_BYTES) if cand else (None, None)


def cmd_traffic(a):
    f_mine, f_rows = counter_per_dispatch(a.fetch, "FETCH_SIZE", a.kernel)
    w_mine, w_rows = counter_per_dispatch(a.write, "WRITE_SIZE", a.kernel)
    (f_copy, f_bytes), (w_copy, w_bytes) = copy_counter(f_rows), copy_counter(w_rows)
    if not f_mine or not w_mine or not f_copy or not w_copy:
        raise SystemExit("kernel or calibration copy not found in the counter runs")
    f_scale = f_bytes / (f_copy * 1024.0)
    w_scale = w_bytes / (w_copy * 1024.0)
    fetch = statistics.mean(f_mine) * 1024.0 * f_scale
    write = statistics.mean(w_mine) * 1024.0 * w_scale
    out = {"kernel_substring": a.kernel, "kernel": a.kernel_label or a.kernel, "source_hash": a.source_hash,
           "fetch_bytes_per_launch": fetch, "write_bytes_per_launch": write,
           "bytes_per_launch": fetch + write, "fetch_scale": f_scale, "write_scale": w_scale,
           "dispatches": [len(f_mine), len(w_mine)], "command": a.command}
    with open(a.out, "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out))


def cmd_table(a):
    _, f_rows = counter_per_dispatch(a.fetch, "FETCH_SIZE", "")
    _, w_rows = counter_per_dispatch(a.write, "WRITE_SIZE", "")
    (f_copy, f_bytes), (w_copy, w_bytes) = copy_counter(f_rows), copy_counter(w_rows)
    if not f_copy or not w_copy:
        raise SystemExit("calibration copy not found in the counter runs")
    f_scale = f_bytes / (f_copy * 1024.0)
    w_scale = w_bytes / (w_copy * 1024.0)
    per = {}
    for rows, col, scale in ((f_rows, 0, f_scale), (w_rows, 1, w_scale)):
        for n, v in rows:
            per.setdefault(n, ([], []))[col].append(v * 1024.0 * scale)
    tab = []
    for n, (f, w) in per.items():
        fm = statistics.mean(f) if f else float("nan")
        wm = statistics.mean(w) if w else float("nan")
        tab.append((fm + wm, fm, wm, len(f), len(w), n))
    tab.sort(key=lambda r: -(r[0] if r[0] == r[0] else 0.0))
    print(f"calibration: FETCH_SIZE x {f_scale:.4f}, WRITE_SIZE x {w_scale:.4f} "
          "(bytes of the plain copy over the counter's reading)\n")
    print("| dispatches (fetch, write) | fetch MB/launch | write MB/launch | kernel |")
    print("|---:|---:|---:|---|")
    for tot, fm, wm, nf, nw, n in tab[: a.top]:
        print(f"| {nf}, {nw} | {fm / 1e6:.1f} | {wm / 1e6:.1f} | `{n[:110]}` |")


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("db")
    s.add_argument("--top", type=int, default=30)
    t = sub.add_parser("traffic")
    t.add_argument("--fetch", required=True)
    t.add_argument("--write", required=True)
    t.add_argument("--kernel", required=True)
    t.add_argument("--kernel-label", default=None)
    t.add_argument("--source-hash", required=True)
    t.add_argument("--out", required=True)
    t.add_argument("--command", default="")
    b = sub.add_parser("table")
    b.add_argument("--fetch", required=True)
    b.add_argument("--write", required=True)
    b.add_argument("--top", type=int, default=30)
    a = ap.parse_args()
    {"stats": cmd_stats, "traffic": cmd_traffic, "table": cmd_table}[a.cmd](a)


if __name__ == "__main__":
    main()
