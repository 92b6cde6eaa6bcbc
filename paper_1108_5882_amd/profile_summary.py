"""Summaries of rocprofv3 CSV output as short markdown (and JSON) files.

Three reports, each from the CSV files one rocprofv3 run writes into a
directory (``-d DIR --output-format csv``):

  trace    per-kernel launch durations from ``*_kernel_trace.csv`` (kernels whose
           name matches a regular expression, optionally only launches longer
           than a minimum), with the top kernels of ``*_kernel_stats.csv``
  counters per-dispatch averages of every counter in ``*_counter_collection.csv``
           for the matching kernels
  traffic  HBM bytes per launch of one kernel from two counter runs (FETCH_SIZE,
           then WRITE_SIZE, in KiB per dispatch), each scaled by what the same
           counter reads for a plain device copy of known size in the same run

Usage (from the repository root):

  python -m paper_1108_5882_amd.profile_summary trace DIR --kernel REGEX [--min-us T]
      --title TEXT --command "CMD" --out profiles/NAME.md
  python -m paper_1108_5882_amd.profile_summary counters DIR --kernel REGEX
      --title TEXT --command "CMD" --out profiles/NAME.md
  python -m paper_1108_5882_amd.profile_summary traffic FETCH_DIR WRITE_DIR --kernel REGEX
      --last N --copy-bytes B --alg-bytes B --units U --config TEXT --source FILE [--source FILE ...]
      --command "CMD1" --command "CMD2" --out profiles/NAME  (writes NAME.md and NAME.json)
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import re
import statistics
import sys

COPY_KERNEL = r"copyBuffer"


def _rows(directory: str, suffix: str):
    files = sorted(glob.glob(os.path.join(directory, "**", f"*{suffix}"), recursive=True))
    if not files:
        raise FileNotFoundError(f"no *{suffix} under {directory}")
    out = []
    for fn in files:
        with open(fn, newline="") as f:
            out.extend(csv.DictReader(f))
    return out


def _name(row) -> str:
    return row.get("Kernel_Name") or row.get("Name") or ""


def _dispatch(row) -> int:
    for key in ("Dispatch_Id", "Correlation_Id"):
        if row.get(key):
            return int(row[key])
    return 0


def trace_table(directory: str, pattern: str, min_us: float = 0.0):
    """Launch statistics (us) per kernel name matching pattern."""
    rx = re.compile(pattern)
    per = {}
    for r in _rows(directory, "_kernel_trace.csv"):
        n = _name(r)
        if not rx.search(n):
            continue
        us = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
        if us >= min_us:
            per.setdefault(n, []).append(us)
    return {n: dict(launches=len(v), mean=statistics.fmean(v), median=statistics.median(v), min=min(v),
                    max=max(v)) for n, v in per.items()}


def stats_top(directory: str, top: int = 10):
    rows = _rows(directory, "_kernel_stats.csv")
    rows.sort(key=lambda r: -float(r.get("TotalDurationNs", 0)))
    return [dict(name=_name(r), calls=int(r["Calls"]), total_ms=float(r["TotalDurationNs"]) / 1e6,
                 avg_us=float(r["AverageNs"]) / 1e3, pct=float(r.get("Percentage", 0.0))) for r in rows[:top]]


def counter_means(directory: str, pattern: str, last: int = 0):
    """{kernel: {counter: mean per dispatch}} over dispatches of matching kernels
    (only the last `last` dispatches of each kernel when last > 0)."""
    rx = re.compile(pattern)
    per = {}
    for r in _rows(directory, "_counter_collection.csv"):
        n = _name(r)
        if not rx.search(n):
            continue
        d = per.setdefault(n, {})
        d.setdefault(_dispatch(r), {})
        c = d[_dispatch(r)]
        c[r["Counter_Name"]] = c.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    out = {}
    for n, disp in per.items():
        ids = sorted(disp)
        if last > 0:
            ids = ids[-last:]
        names = sorted({c for i in ids for c in disp[i]})
        out[n] = {c: statistics.fmean(disp[i].get(c, 0.0) for i in ids) for c in names}
        out[n]["_dispatches"] = len(ids)
    return out


def _header(title: str, commands):
    lines = [f"# {title}", "", "Command(s), from the repository root:", ""]
    lines += [f"    {c}" for c in commands]
    return lines + [""]


def write_trace(args):
    t = trace_table(args.dir, args.kernel, args.min_us)
    lines = _header(args.title, args.command)
    if args.min_us > 0:
        lines.append(f"Launches longer than {args.min_us:g} us.")
        lines.append("")
    lines += ["| Kernel | Launches | Mean us | Median us | Min us | Max us |", "|---|---|---|---|---|---|"]
    for n, s in sorted(t.items(), key=lambda kv: -kv[1]["launches"] * kv[1]["mean"]):
        lines.append(f"| {n[:110]} | {s['launches']} | {s['mean']:.1f} | {s['median']:.1f} | {s['min']:.1f} | "
                     f"{s['max']:.1f} |")
    try:
        top = stats_top(args.dir)
        lines += ["", "Top kernels of the run (kernel stats):", "", "| Kernel | Calls | Total ms | Average us | % |",
                  "|---|---|---|---|---|"]
        lines += [f"| {r['name'][:110]} | {r['calls']} | {r['total_ms']:.2f} | {r['avg_us']:.1f} | {r['pct']:.1f} |"
                  for r in top]
    except FileNotFoundError:
        pass
    for note in args.note:
        lines += ["", note]
    _write(args.out, "\n".join(lines) + "\n")


def write_counters(args):
    m = counter_means(args.dir, args.kernel, args.last)
    lines = _header(args.title, args.command)
    for n, c in m.items():
        lines += [f"`{n[:140]}` ({c['_dispatches']} dispatches, mean per dispatch):", "",
                  "| Counter | Value |", "|---|---|"]
        lines += [f"| {k} | {v:.6g} |" for k, v in c.items() if not k.startswith("_")]
        lines.append("")
    for note in args.note:
        lines += [note, ""]
    _write(args.out, "\n".join(lines))


def write_traffic(args):
    fetch = counter_means(args.fetch_dir, args.kernel, args.last)
    write = counter_means(args.write_dir, args.kernel, args.last)
    cf = counter_means(args.fetch_dir, COPY_KERNEL)
    cw = counter_means(args.write_dir, COPY_KERNEL)
    if len(fetch) != 1 or len(write) != 1 or len(cf) != 1 or len(cw) != 1:
        raise SystemExit(f"expected one matching kernel and one copy kernel per run: {list(fetch)} {list(cf)}")
    kname = next(iter(fetch))
    fk, wk = fetch[kname]["FETCH_SIZE"], next(iter(write.values()))["WRITE_SIZE"]
    cfk, cwk = next(iter(cf.values()))["FETCH_SIZE"], next(iter(cw.values()))["WRITE_SIZE"]
    fscale = args.copy_bytes / (cfk * 1024.0)
    wscale = args.copy_bytes / (cwk * 1024.0)
    hbm = fk * 1024.0 * fscale + wk * 1024.0 * wscale
    h = hashlib.sha256()
    for path in args.source:
        with open(path, "rb") as f:
            h.update(f.read())
    sha = h.hexdigest()[:16]
    rec = {"kernel": args.config, "dispatch_name": kname, "kernel_sha256_16": sha, "units_per_launch": args.units,
           "fetch_size_kib": fk, "write_size_kib": wk, "copy_bytes": args.copy_bytes, "copy_fetch_kib": cfk,
           "copy_write_kib": cwk, "fetch_scale": fscale, "write_scale": wscale, "hbm_bytes_per_launch": hbm,
           "alg_bytes_per_launch": args.alg_bytes, "commands": args.command}
    _write(args.out + ".json", json.dumps(rec, indent=1) + "\n")
    lines = _header(args.title or f"HBM traffic of {args.config}", args.command)
    lines += ["| Dispatch | FETCH_SIZE KiB | WRITE_SIZE KiB |", "|---|---|---|",
              f"| {kname[:100]} (last {args.last}) | {fk:.1f} | {wk:.1f} |",
              f"| plain copy of {args.copy_bytes:,.0f} B | {cfk:.1f} | {cwk:.1f} |", "",
              f"Scale factors from the copy (bytes it reads or writes / counter bytes): FETCH {fscale:.4f}, "
              f"WRITE {wscale:.4f}.",
              f"HBM bytes per launch = {hbm:.4e} against {args.alg_bytes:,.0f} algorithmic bytes: ratio "
              f"{hbm / args.alg_bytes:.4f}.", "",
              f"Launch configuration: {args.config}; kernel source SHA-256 prefix {sha}.", ""]
    _write(args.out + ".md", "\n".join(lines))


def _write(path: str, text: str):
    with open(path, "w") as f:
        f.write(text)
    print(f"wrote {path}")


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="cmd", required=True)
    for name in ("trace", "counters"):
        p = sub.add_parser(name)
        p.add_argument("dir")
        p.add_argument("--kernel", required=True)
        p.add_argument("--min-us", type=float, default=0.0)
        p.add_argument("--last", type=int, default=0)
        p.add_argument("--title", required=True)
        p.add_argument("--command", action="append", default=[])
        p.add_argument("--note", action="append", default=[])
        p.add_argument("--out", required=True)
    p = sub.add_parser("traffic")
    p.add_argument("fetch_dir")
    p.add_argument("write_dir")
    p.add_argument("--kernel", required=True)
    p.add_argument("--last", type=int, default=5)
    p.add_argument("--copy-bytes", type=float, required=True)
    p.add_argument("--alg-bytes", type=float, required=True)
    p.add_argument("--units", type=int, required=True)
    p.add_argument("--config", required=True)
    p.add_argument("--source", action="append", required=True,
                   help="kernel source file; repeat for each file, in the order the bench hashes them")
    p.add_argument("--title", default="")
    p.add_argument("--command", action="append", default=[])
    p.add_argument("--out", required=True)
    a = ap.parse_args(argv)
    {"trace": write_trace, "counters": write_counters, "traffic": write_traffic}[a.cmd](a)
    return 0


if __name__ == "__main__":
    sys.exit(main())
