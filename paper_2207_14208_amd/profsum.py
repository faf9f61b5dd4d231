"""Summaries of rocprofv3 output (CSV or rocpd SQLite) for the solver's kernels.

    python -m paper_2207_14208_amd.profsum trace <dir> [--top K] [--last NAME GRID COUNT]
        per (kernel, grid) call count, average and share of the kernel time;
        --last adds the average of the last COUNT dispatches of one kernel at
        one grid (a timed burst at the end of the run)
    python -m paper_2207_14208_amd.profsum traffic <fetch_dir> <write_dir> --kernel NAME --grid G --copy-bytes B
        FETCH_SIZE / WRITE_SIZE per dispatch of one kernel, scaled by what the
        same counters read for the plain copy kernel of B bytes
    python -m paper_2207_14208_amd.profsum markers <dir>
        the library's roctx ranges (rocprofv3 --marker-trace): per range name,
        calls, host time, and the kernel time that fell inside the ranges

Runs on the host; reads only the files rocprofv3 wrote.
"""
from __future__ import annotations

import argparse
import collections
import csv
import glob
import json
import os
import sqlite3


def _short(name: str) -> str:
    n = name.replace("void ", "").replace("bcmg::", "")
    if n.startswith("__amd_rocclr"):
        return n
    # keep template arguments, drop the parameter list
    depth, out = 0, []
    for ch in n:
        if ch == "(" and depth == 0:
            break
        depth += ch == "<"
        depth -= ch == ">"
        out.append(ch)
    return "".join(out).strip()


def _find(d: str, pattern: str) -> list[str]:
    return sorted(glob.glob(os.path.join(d, "**", pattern), recursive=True))


def _col(row: dict, *names, default=None):
    for n in names:
        if n in row and row[n] != "":
            return row[n]
    return default


def kernel_rows(d: str):
    """(short name, grid size in threads, duration ns) per dispatch."""
    csvs = _find(d, "*kernel_trace.csv")
    if csvs:
        for path in csvs:
            with open(path) as fh:
                for r in csv.DictReader(fh):
                    g = int(_col(r, "Grid_Size_X", "Grid_Size", default=0))
                    yield _short(r["Kernel_Name"]), g, int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
        return
    for db in _find(d, "*.db"):
        con = sqlite3.connect(db)
        for name, gx, dur in con.execute("select name, grid_x, duration from kernels"):
            yield _short(name), int(gx), int(dur)


def last_dispatches_us(d: str, kernel: str, grid: int, count: int) -> tuple[float, int]:
    """Average duration (us) of the last `count` dispatches, by start time,
    of one kernel at one grid size in a CSV kernel trace, and how many were
    averaged."""
    found = []
    for path in _find(d, "*kernel_trace.csv"):
        with open(path) as fh:
            for r in csv.DictReader(fh):
                if _short(r["Kernel_Name"]) != kernel or int(_col(r, "Grid_Size_X", "Grid_Size", default=0)) != grid:
                    continue
                t0, t1 = int(r["Start_Timestamp"]), int(r["End_Timestamp"])
                found.append((t0, t1 - t0))
    if not found:
        raise SystemExit(f"no dispatches of {kernel} at grid {grid} in {d}")
    tail = [dur for _, dur in sorted(found)[-count:]]
    return sum(tail) / len(tail) / 1e3, len(tail)


def trace_table(d: str, top: int = 30) -> tuple[list, float]:
    agg = collections.defaultdict(list)
    for name, g, dur in kernel_rows(d):
        agg[(name, g)].append(dur)
    tot = sum(sum(v) for v in agg.values())
    rows = sorted(agg.items(), key=lambda kv: -sum(kv[1]))[:top]
    return [(k, g, len(v), sum(v) / len(v) / 1e3, 100.0 * sum(v) / tot) for (k, g), v in rows], tot / 1e6


def counter_rows(d: str, counter: str):
    """(short name, grid, value, dispatch id) per dispatch of one counter."""
    for path in _find(d, "*counter_collection.csv"):
        with open(path) as fh:
            for r in csv.DictReader(fh):
                if r.get("Counter_Name") != counter:
                    continue
                g = int(_col(r, "Grid_Size", "Grid_Size_X", default=0))
                yield _short(r["Kernel_Name"]), g, float(r["Counter_Value"]), int(_col(r, "Dispatch_Id", default=0))


def traffic(fetch_dir: str, write_dir: str, kernel: str, grid: int, copy_bytes: int) -> dict:
    def per_dispatch(d, counter):
        vals = collections.defaultdict(list)
        copies = []
        for name, g, v, did in counter_rows(d, counter):
            vals[(name, g)].append(v)
            if "copy" in name.lower() and v * 1024.0 > 0.1 * copy_bytes:
                copies.append((did, v))
        g_use = grid if grid else max((g for (n, g) in vals if n == kernel), default=0)
        mine = [v for (n, g), vs in vals.items() if n == kernel and g == g_use for v in vs]
        if not mine:
            raise SystemExit(f"no {counter} rows for {kernel} grid {grid} in {d}")
        # the copy probe: the program's first large copy dispatch (bench.py
        # runs it before anything else; later copies, such as uploads of the
        # inputs, can be larger)
        probe = min(copies)[1] if copies else None
        return sum(mine) / len(mine), probe, len(mine), g_use

    f_k, f_copy, nf, grid = per_dispatch(fetch_dir, "FETCH_SIZE")
    w_k, w_copy, nw, _ = per_dispatch(write_dir, "WRITE_SIZE")
    copy_kib = copy_bytes / 1024.0
    fs = copy_kib / f_copy if f_copy else 1.0
    ws = copy_kib / w_copy if w_copy else 1.0
    return {"kernel": kernel, "grid": grid, "dispatches": [nf, nw],
            "fetch_kib_per_dispatch": f_k, "write_kib_per_dispatch": w_k,
            "copy_probe_bytes": copy_bytes, "copy_fetch_kib": f_copy, "copy_write_kib": w_copy,
            "fetch_scale": fs, "write_scale": ws,
            "bytes_per_launch": (f_k * fs + w_k * ws) * 1024.0}


def _range_key(name: str) -> str:
    # ranges that carry counts (levels, cycle spans) are grouped by their
    # leading words
    if name.startswith("cycles "):
        return "cycles a..b (one host check)"
    if name.startswith("bcmg_batch_step"):
        return "bcmg_batch_step"
    return name


def marker_table(d: str):
    """(range, calls, host ms, kernel ms inside) for the roctx ranges."""
    ranges = []
    for path in _find(d, "*marker_api_trace.csv"):
        with open(path) as fh:
            for r in csv.DictReader(fh):
                ranges.append((r["Function"], int(r["Start_Timestamp"]), int(r["End_Timestamp"])))
    kernels = []
    for path in _find(d, "*kernel_trace.csv"):
        with open(path) as fh:
            for r in csv.DictReader(fh):
                kernels.append((int(r["Start_Timestamp"]), int(r["End_Timestamp"])))
    kernels.sort()
    starts = [k[0] for k in kernels]
    import bisect
    agg = collections.OrderedDict()
    for name, t0, t1 in sorted(ranges, key=lambda x: x[1]):
        k = _range_key(name)
        a = agg.setdefault(k, [0, 0, 0])
        a[0] += 1
        a[1] += t1 - t0
        i = bisect.bisect_left(starts, t0)
        while i < len(kernels) and kernels[i][0] < t1:
            if kernels[i][1] <= t1:
                a[2] += kernels[i][1] - kernels[i][0]
            i += 1
    return [(k, v[0], v[1] / 1e6, v[2] / 1e6) for k, v in agg.items()]


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("trace")
    t.add_argument("dir")
    t.add_argument("--top", type=int, default=30)
    t.add_argument("--last", nargs=3, metavar=("NAME", "GRID", "COUNT"))
    c = sub.add_parser("traffic")
    c.add_argument("fetch_dir")
    c.add_argument("write_dir")
    c.add_argument("--kernel", required=True)
    c.add_argument("--grid", type=int, default=0, help="grid size in threads (0: the kernel's largest)")
    c.add_argument("--copy-bytes", type=int, required=True)
    m = sub.add_parser("markers")
    m.add_argument("dir")
    a = ap.parse_args()
    if a.cmd == "markers":
        print("| range | calls | host ms | kernel ms inside |\n|---|---:|---:|---:|")
        for k, n, host, kern in marker_table(a.dir):
            print(f"| {k} | {n} | {host:.3f} | {kern:.3f} |")
        return
    if a.cmd == "trace":
        rows, tot_ms = trace_table(a.dir, a.top)
        print(f"total kernel time {tot_ms:.3f} ms\n")
        print("| kernel | grid | calls | avg us | share |\n|---|---:|---:|---:|---:|")
        for k, g, n, avg, share in rows:
            print(f"| {k} | {g} | {n} | {avg:.2f} | {share:.1f}% |")
        if a.last:
            avg, n = last_dispatches_us(a.dir, a.last[0], int(a.last[1]), int(a.last[2]))
            print(f"\nlast {n} dispatches of {a.last[0]} at grid {a.last[1]}: {avg:.2f} us on average")
    else:
        print(json.dumps(traffic(a.fetch_dir, a.write_dir, a.kernel, a.grid, a.copy_bytes), indent=1))


if __name__ == "__main__":
    main()
