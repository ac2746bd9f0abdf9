"""Per-kernel summary of a rocprofv3 kernel trace, cut to a marked window.

    python -m paper_2005_06104_amd.tracesum <kernel_trace.csv> [--marker NAME]
        [--split-grid SUBSTRING] [--top N]

`bench.py --mark-timed` launches a short marker kernel (torch's sleep
kernel) right before and right after the timed steps of the headline
precision; this tool keeps the dispatches that start between the first and
the last dispatch whose name contains NAME, and prints a markdown table of
kernels by total time (calls, total, average, share of kernel time), the
window length and the fraction of it the device spent in kernels.  With
--split-grid, kernels whose name contains SUBSTRING are listed once per
grid size (the two products of the effective Hamiltonian share a kernel).
With --ranges (the marker_api_trace.csv of the same run, taken with
--marker-trace) the host time of each named range inside the window is
listed too.
"""
from __future__ import annotations

import argparse
import csv
import sys
from collections import defaultdict


def _col(header, *names):
    for n in names:
        if n in header:
            return header.index(n)
    raise SystemExit(f"kernel trace has none of the columns {names}; header: {header}")


def _rows(path):
    with open(path, newline="") as f:
        rows = csv.reader(f)
        header = next(rows)
        i_name = _col(header, "Kernel_Name", "KernelName", "Name")
        i_start = _col(header, "Start_Timestamp", "BeginNs", "Start")
        i_end = _col(header, "End_Timestamp", "EndNs", "End")
        i_grid = [header.index(c) for c in ("Grid_Size_X", "Grid_Size_Y", "Grid_Size_Z") if c in header]
        for r in rows:
            yield r[i_name], int(r[i_start]), int(r[i_end]), tuple(r[i] for i in i_grid)


def _ranges(path):
    with open(path, newline="") as f:
        rows = csv.reader(f)
        header = next(rows)
        i_name = _col(header, "Function", "Message", "Name")
        i_start = _col(header, "Start_Timestamp", "Start")
        i_end = _col(header, "End_Timestamp", "End")
        for r in rows:
            yield r[i_name], int(r[i_start]), int(r[i_end])


def summarize(path, marker="spin_kernel", split_grid=None, top=40, ranges=None):
    # two passes over the file (traces of long runs hold millions of rows)
    marks = sorted(s for n, s, e, g in _rows(path) if marker in n)
    if len(marks) < 2:
        raise SystemExit(f"fewer than two marker dispatches ({marker!r}) in {path}")
    lo, hi = marks[0], marks[-1]
    sel = [r for r in _rows(path) if lo < r[1] < hi and marker not in r[0]]
    by = defaultdict(lambda: [0, 0])
    for n, s, e, g in sel:
        short = n if len(n) <= 100 else n[:97] + "..."
        key = short if not (split_grid and split_grid in n) else f"{short} [grid {'x'.join(g)}]"
        by[key][0] += 1
        by[key][1] += e - s
    total = sum(v[1] for v in by.values())
    # device busy time: union of the dispatch intervals
    busy, cur_s, cur_e = 0, None, None
    for _, s, e, _ in sorted(sel, key=lambda r: r[1]):
        if cur_e is None or s > cur_e:
            if cur_e is not None:
                busy += cur_e - cur_s
            cur_s, cur_e = s, e
        else:
            cur_e = max(cur_e, e)
    if cur_e is not None:
        busy += cur_e - cur_s
    out = [f"window {1e-9 * (hi - lo):.3f} s between the marker dispatches; {len(sel)} dispatches; "
           f"kernel time {1e-9 * total:.3f} s; device busy {100.0 * busy / (hi - lo):.1f}% of the window",
           "",
           "| kernel | calls | total ms | avg us | % of kernel time |",
           "|---|---:|---:|---:|---:|"]
    for key, (c, t) in sorted(by.items(), key=lambda kv: -kv[1][1])[:top]:
        out.append(f"| `{key}` | {c} | {1e-6 * t:.1f} | {1e-3 * t / c:.1f} | {100.0 * t / total:.2f} |")
    if ranges:
        # host time of the named ranges (inclusive of nested ones) in the window
        hr = defaultdict(lambda: [0, 0])
        for n, s, e in _ranges(ranges):
            if lo < s < hi:
                hr[n][0] += 1
                hr[n][1] += e - s
        out += ["", f"host ranges ({ranges.split('/')[-1]}), inclusive:", "",
                "| range | calls | total ms | avg us | % of window |", "|---|---:|---:|---:|---:|"]
        for key, (c, t) in sorted(hr.items(), key=lambda kv: -kv[1][1]):
            out.append(f"| `{key}` | {c} | {1e-6 * t:.1f} | {1e-3 * t / c:.1f} | {100.0 * t / (hi - lo):.2f} |")
    return "\n".join(out)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("trace")
    ap.add_argument("--marker", default="spin_kernel")
    ap.add_argument("--split-grid", default=None)
    ap.add_argument("--top", type=int, default=40)
    ap.add_argument("--ranges", default=None, help="a marker_api_trace.csv of the same run: host time per range")
    a = ap.parse_args(argv)
    print(summarize(a.trace, a.marker, a.split_grid, a.top, a.ranges))


if __name__ == "__main__":
    sys.exit(main())
