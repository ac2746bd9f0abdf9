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
listed too, and the device's idle time (the gaps between the dispatch
intervals) is attributed to the innermost range the host was in at the
middle of each gap, and to the kernel that ran before it.

    python -m paper_2005_06104_amd.tracesum --counters <counter_collection.csv>
        [--kernel SUBSTRING] [--marker NAME] [--calib SUBSTRING --calib-bytes N]

With --counters the file is the counter output of a `rocprofv3 --pmc` run
(one row per dispatch and counter): the dispatches between the first and
the last marker dispatch whose name contains SUBSTRING are averaged per
counter (--marker none: every dispatch of the file); --calib names a plain copy kernel of N bytes read and N written
(anywhere in the file), whose FETCH_SIZE / WRITE_SIZE give the factors that
turn those counters into bytes.
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
        rl = []
        for n, s, e in _ranges(ranges):
            if s < hi and e > lo:
                rl.append((s, e, n))
            if lo < s < hi:
                hr[n][0] += 1
                hr[n][1] += e - s
        out += ["", f"host ranges ({ranges.split('/')[-1]}), inclusive:", "",
                "| range | calls | total ms | avg us | % of window |", "|---|---:|---:|---:|---:|"]
        for key, (c, t) in sorted(hr.items(), key=lambda kv: -kv[1][1]):
            out.append(f"| `{key}` | {c} | {1e-6 * t:.1f} | {1e-3 * t / c:.1f} | {100.0 * t / (hi - lo):.2f} |")
        out += [""] + _gaps(sel, rl, lo, hi)
    return "\n".join(out)


def _gaps(sel, rl, lo, hi):
    """Idle device time between dispatches, by innermost host range and by
    the kernel that ran before the gap (ranges nest on the one host thread)."""
    ev = sorted(sel, key=lambda r: r[1])
    gaps = []   # (start, end, kernel before)
    cur_e, prev = lo, "(window start)"
    for n, s, e, _ in ev:
        if s > cur_e:
            gaps.append((cur_e, s, prev))
        if e > cur_e:
            cur_e, prev = e, n
    if hi > cur_e:
        gaps.append((cur_e, hi, prev))
    rl.sort()
    by_r = defaultdict(lambda: [0, 0])
    by_k = defaultdict(lambda: [0, 0])
    hist = defaultdict(lambda: [0, 0])
    stack, i = [], 0
    for s, e, prev in gaps:
        t = (s + e) // 2
        while i < len(rl) and rl[i][0] <= t:
            while stack and stack[-1][1] < rl[i][0]:
                stack.pop()
            stack.append(rl[i])
            i += 1
        while stack and stack[-1][1] < t:
            stack.pop()
        name = stack[-1][2] if stack else "(no range)"
        d = e - s
        by_r[name][0] += 1
        by_r[name][1] += d
        short = prev if len(prev) <= 80 else prev[:77] + "..."
        by_k[short][0] += 1
        by_k[short][1] += d
        b = "< 5 us" if d < 5000 else "5-20 us" if d < 20000 else "20-100 us" if d < 100000 else ">= 100 us"
        hist[b][0] += 1
        hist[b][1] += d
    tot = sum(g[1] - g[0] for g in gaps)
    out = [f"device idle {1e-6 * tot:.1f} ms ({100.0 * tot / (hi - lo):.1f}% of the window) in {len(gaps)} gaps", "",
           "| gap length | gaps | total ms |", "|---|---:|---:|"]
    for b in ("< 5 us", "5-20 us", "20-100 us", ">= 100 us"):
        if b in hist:
            out.append(f"| {b} | {hist[b][0]} | {1e-6 * hist[b][1]:.1f} |")
    out += ["", "idle time by the innermost host range at the middle of the gap:", "",
            "| range | gaps | idle ms | % of window |", "|---|---:|---:|---:|"]
    for key, (c, d) in sorted(by_r.items(), key=lambda kv: -kv[1][1])[:25]:
        out.append(f"| `{key}` | {c} | {1e-6 * d:.1f} | {100.0 * d / (hi - lo):.2f} |")
    out += ["", "idle time by the kernel before the gap:", "",
            "| kernel | gaps | idle ms | % of window |", "|---|---:|---:|---:|"]
    for key, (c, d) in sorted(by_k.items(), key=lambda kv: -kv[1][1])[:25]:
        out.append(f"| `{key}` | {c} | {1e-6 * d:.1f} | {100.0 * d / (hi - lo):.2f} |")
    return out


def _counter_rows(path):
    """(dispatch id, kernel name, counter name, value) per row of a counter file."""
    with open(path, newline="") as f:
        rows = csv.reader(f)
        header = next(rows)
        i_id = _col(header, "Dispatch_Id", "Correlation_Id", "Index")
        i_name = _col(header, "Kernel_Name", "KernelName", "Name")
        i_cn = _col(header, "Counter_Name")
        i_cv = _col(header, "Counter_Value")
        for r in rows:
            yield int(r[i_id]), r[i_name], r[i_cn], float(r[i_cv])


def counters(path, kernel, marker="spin_kernel", calib=None, calib_bytes=None):
    """Per-dispatch averages of every counter for the kernels containing
    `kernel` inside the marked window, plus the copy calibration."""
    # one dispatch may appear on several rows (one per counter, or per
    # counter dimension): values of one dispatch and counter are summed
    per = defaultdict(lambda: defaultdict(float))
    names = {}
    for d, n, c, v in _counter_rows(path):
        per[d][c] += v
        names[d] = n
    if marker:
        marks = sorted(d for d, n in names.items() if marker in n)
        if len(marks) < 2:
            raise SystemExit(f"fewer than two marker dispatches ({marker!r}) in {path}")
        lo, hi = marks[0], marks[-1]
    else:   # no window: every dispatch of the file
        lo, hi = min(names) - 1, max(names) + 1
    sel = [d for d, n in names.items() if lo < d < hi and kernel in n]
    if not sel:
        raise SystemExit(f"no dispatch of {kernel!r} between the markers in {path}")
    cn = sorted({c for d in sel for c in per[d]})
    avg = {c: sum(per[d].get(c, 0.0) for d in sel) / len(sel) for c in cn}
    out = {"dispatches": len(sel), "avg": avg}
    if calib:
        cal = [d for d, n in names.items() if calib in n]
        if cal and calib_bytes:
            kib = calib_bytes / 1024.0
            fac = {}
            for c in ("FETCH_SIZE", "WRITE_SIZE"):
                vals = [per[d][c] for d in cal if c in per[d]]
                if vals and max(vals) > 0:
                    fac[c] = kib / max(vals)
            out["calib"] = {"dispatches": len(cal), "factors": fac}
            for c, f in fac.items():
                if c in avg:
                    out.setdefault("bytes_per_dispatch", {})[c] = avg[c] * f * 1024.0
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("trace")
    ap.add_argument("--marker", default="spin_kernel")
    ap.add_argument("--split-grid", default=None)
    ap.add_argument("--top", type=int, default=40)
    ap.add_argument("--ranges", default=None, help="a marker_api_trace.csv of the same run: host time per range")
    ap.add_argument("--counters", action="store_true", help="the file is a rocprofv3 --pmc counter file")
    ap.add_argument("--kernel", default="gemm_kernel<float, false, false, false, false, 1>")
    ap.add_argument("--calib", default=None, help="name of a plain copy kernel in the same file")
    ap.add_argument("--calib-bytes", type=float, default=None, help="bytes the copy reads (and writes)")
    a = ap.parse_args(argv)
    if a.counters:
        import json
        marker = None if a.marker.lower() == "none" else a.marker
        print(json.dumps(counters(a.trace, a.kernel, marker, a.calib, a.calib_bytes), indent=1))
        return
    print(summarize(a.trace, a.marker, a.split_grid, a.top, a.ranges))


if __name__ == "__main__":
    sys.exit(main())
