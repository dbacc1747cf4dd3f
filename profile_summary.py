#!/usr/bin/env python3
"""Short text summaries of rocprofv3 output for profiles/, and the per-kernel
HBM traffic file the benchmark reads.

  python3 profile_summary.py trace OUTDIR --title T --command C > profiles/kernels_X.txt
      per-kernel calls, average / total duration, share and resources from a
      `rocprofv3 --kernel-trace --stats -f csv` output directory;
  python3 profile_summary.py traffic FETCH_DIR WRITE_DIR --workload W --title T
          --command C [--kernel-source K=FILE ...] > profiles/hbm_traffic_X.txt
      FETCH_SIZE and WRITE_SIZE per dispatch (KiB, from two `--pmc` runs, one
      counter each), scaled by what the same counters read for the largest
      device-to-device copy in the run (a plain copy kernel of known size), and
      merges {kernel: bytes per launch, source file and its sha256} for the
      workload W into profiles/traffic.json.

Kernel names are shortened to the kernel and its leading template arguments.
Per kernel, the dispatches averaged are the ones of the largest grid size
(the event-sized launches; small set-up dispatches of the same kernel, e.g.
the response spectrum at plane creation, are left out) unless --all-grids.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import re
import sys
from collections import defaultdict

ROOT = os.path.dirname(os.path.abspath(__file__))


def short_name(full: str) -> str:
    name = re.sub(r"\(anonymous namespace\)::", "", full)
    name = re.sub(r"^void\s+", "", name)
    m = re.match(r"(?:[\w:]+::)?(\w+)(<.*)?\(", name)
    if not m:
        return full[:40]
    base, targs = m.group(1), m.group(2) or ""
    if "FftCt<" in targs:
        sizes = re.findall(r"FftCt<(\d+)", targs)
        flags = re.findall(r">,\s*(true|false)>?$", targs.rstrip())
        return "%s<%s%s>" % (base, "x".join(sizes), (", " + flags[-1]) if flags else "")
    targs = re.sub(r"[\w:]+::", "", targs)
    return base + targs


def _find(d: str, suffix: str) -> list[str]:
    files = sorted(glob.glob(os.path.join(d, "**", "*" + suffix), recursive=True))
    if not files:
        sys.exit("no *%s under %s" % (suffix, d))
    return files


def _col(row: dict, *names, default=None):
    low = {k.lower(): v for k, v in row.items()}
    for n in names:
        if n.lower() in low:
            return low[n.lower()]
    return default


def _rows(files):
    for f in files:
        with open(f, newline="") as fh:
            yield from csv.DictReader(fh)


def _grid(row) -> int:
    g = [int(float(_col(row, a, default=1) or 1)) for a in ("Grid_Size_X", "Grid_Size_Y",
                                                             "Grid_Size_Z")]
    if g == [1, 1, 1]:
        return int(float(_col(row, "Grid_Size", default=0) or 0))
    return g[0] * g[1] * g[2]


def trace(args):
    rows = list(_rows(_find(args.outdir, "kernel_trace.csv")))
    per = defaultdict(list)
    res = {}
    for r in rows:
        n = short_name(_col(r, "Kernel_Name"))
        t = (int(_col(r, "End_Timestamp")) - int(_col(r, "Start_Timestamp"))) / 1e3
        per[n].append(t)
        res[n] = (_col(r, "Arch_VGPR_Count", "VGPR_Count", default="?"),
                  _col(r, "LDS_Block_Size", "LDS_Size", "Group_Segment_Size", default="?"),
                  _col(r, "Scratch_Size", "Private_Segment_Size", default="?"),
                  _col(r, "Workgroup_Size_X", "Workgroup_Size", default="?"))
    total = sum(sum(v) for v in per.values())
    print("# " + args.title)
    print("# command (repository root): " + args.command)
    print("# durations from the kernel trace (end - start per dispatch), all dispatches of the run")
    print()
    print("%-40s %7s %11s %12s %7s %5s %6s %7s %5s" % ("kernel", "calls", "avg_us", "total_us",
                                                       "pct", "vgpr", "lds_B", "scratch", "wg"))
    for n, v in sorted(per.items(), key=lambda kv: -sum(kv[1])):
        vg, lds, scr, wg = res[n]
        print("%-40s %7d %11.1f %12.1f %7.2f %5s %6s %7s %5s" % (
            n[:40], len(v), sum(v) / len(v), sum(v), 100.0 * sum(v) / total, vg, lds, scr, wg))


def _counter(files, counter):
    """{short kernel: [(grid, value) per dispatch]} of one counter."""
    out = defaultdict(list)
    for r in _rows(files):
        if (_col(r, "Counter_Name") or "") != counter:
            continue
        out[short_name(_col(r, "Kernel_Name"))].append((_grid(r),
                                                        float(_col(r, "Counter_Value"))))
    return out


def _largest(v, all_grids=False):
    if all_grids:
        return sum(x for _, x in v) / len(v)
    g = max(gs for gs, _ in v)
    sel = [x for gs, x in v if gs == g]
    return sum(sel) / len(sel)


def traffic(args):
    fetch = _counter(_find(args.fetch_dir, "counter_collection.csv"), "FETCH_SIZE")
    write = _counter(_find(args.write_dir, "counter_collection.csv"), "WRITE_SIZE")
    copy = "__amd_rocclr_copyBuffer"
    keep = (lambda k: k == copy or re.search(args.match, k)) if args.match else (lambda k: True)
    if copy not in fetch or copy not in write:
        sys.exit("no device copy in the runs to calibrate with")
    cal_bytes = args.calibrate_mib * 1024.0  # KiB read and written by the copy
    f_copy = max(x for _, x in fetch[copy])
    w_copy = max(x for _, x in write[copy])
    fs, ws = cal_bytes / f_copy, cal_bytes / w_copy
    print("# " + args.title)
    print("# commands (repository root, one counter per run): " + args.command)
    print("# calibration: the %d MiB device copy reads FETCH_SIZE = %.1f KiB and WRITE_SIZE = "
          "%.1f KiB per dispatch, so FETCH_SIZE is scaled by %.4f and WRITE_SIZE by %.4f"
          % (args.calibrate_mib, f_copy, w_copy, fs, ws))
    print("# per kernel: the mean over its dispatches%s%s" % (
        "" if args.all_grids else " of the largest grid size",
        ("; kernels matching " + args.match) if args.match else ""))
    print()
    print("%-40s %13s %13s %11s %11s %11s" % ("kernel", "FETCH_KiB", "WRITE_KiB", "read_MB",
                                                "write_MB", "total_MB"))
    sources = dict(kv.split("=", 1) for kv in (args.kernel_source or []))
    rec = {}
    for k in sorted((k for k in set(fetch) | set(write) if keep(k)),
                    key=lambda k: -(_largest(fetch.get(k, [(0, 0)])) * fs +
                                    _largest(write.get(k, [(0, 0)])) * ws)):
        fk = _largest(fetch[k], args.all_grids) if k in fetch else 0.0
        wk = _largest(write[k], args.all_grids) if k in write else 0.0
        rb, wb = fk * fs * 1024.0, wk * ws * 1024.0
        print("%-40s %13.1f %13.1f %11.1f %11.1f %11.1f" % (k[:40], fk, wk, rb / 1e6, wb / 1e6,
                                                             (rb + wb) / 1e6))
        base = k.split("<")[0]
        if base in sources:
            src = sources[base]
            digest = hashlib.sha256(open(os.path.join(ROOT, src), "rb").read()).hexdigest()
            prev = rec.get(base)
            if prev is None or rb + wb > prev["bytes_per_launch"]:
                rec[base] = {"name": k, "read_bytes": rb, "write_bytes": wb,
                             "bytes_per_launch": rb + wb, "source": src, "source_sha256": digest}
    path = os.path.join(ROOT, "profiles", "traffic.json")
    table = json.load(open(path)) if os.path.exists(path) else {}
    table[args.workload] = {"title": args.title, "fetch_scale": fs, "write_scale": ws,
                            "kernels": rec}
    with open(path, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="mode", required=True)
    t = sub.add_parser("trace")
    t.add_argument("outdir")
    t.add_argument("--title", required=True)
    t.add_argument("--command", required=True)
    c = sub.add_parser("traffic")
    c.add_argument("fetch_dir")
    c.add_argument("write_dir")
    c.add_argument("--workload", required=True)
    c.add_argument("--title", required=True)
    c.add_argument("--command", required=True)
    c.add_argument("--calibrate-mib", type=int, default=1024)
    c.add_argument("--kernel-source", action="append", metavar="KERNEL=FILE")
    c.add_argument("--all-grids", action="store_true")
    c.add_argument("--match", default=None, help="regex a kernel's short name must match")
    args = ap.parse_args()
    trace(args) if args.mode == "trace" else traffic(args)


if __name__ == "__main__":
    main()
