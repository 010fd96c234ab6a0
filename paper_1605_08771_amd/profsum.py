"""Summaries of rocprofv3 CSV output for this library's kernels.

    python -m paper_1605_08771_amd.profsum stats DIR --title T --cmd C [--top N]
        Markdown table of the kernel statistics (``--kernel-trace --stats --output-format csv``).

    python -m paper_1605_08771_amd.profsum pmc --kernel NAME --fetch DIR --write DIR \
            --cal-fetch DIR --cal-write DIR --cal-bytes B --title T --cmd C ...
        Average FETCH_SIZE / WRITE_SIZE per dispatch (KiB) of the kernels whose name contains
        NAME, scaled by what the same counters read for a plain copy of B bytes (the largest
        dispatch of the calibration runs), i.e. HBM bytes per launch.

DIR is a rocprofv3 output directory (searched recursively for the CSV files).
"""
from __future__ import annotations

import argparse
import csv
import glob
import os
import re
import sys


def _find(d, suffix):
    hits = sorted(glob.glob(os.path.join(d, "**", f"*{suffix}"), recursive=True))
    if not hits:
        raise SystemExit(f"no *{suffix} under {d}")
    return hits


def _short(n: str) -> str:
    if n.startswith("_ZN9rocsolver"):
        return "rocsolver (internal)"
    if re.match(r"(void )?roc(solver|blas)", n):
        return re.sub(r"^void ", "", re.split(r"[<(]", n)[0]).replace("v33001::", "")
    n = re.sub(r"\(anonymous namespace\)::", "", n)
    n = n.replace("feast::", "")
    m = re.match(r"(void )?([\w:<>, ]+?)\(", n)
    s = m.group(2) if m else n
    if s.startswith("Cijk_"):
        s = "rocBLAS " + s[:40] + "..."
    s = re.sub(r"rocsolver::v\d+::", "rocsolver::", s)
    return s.strip()


def stats(args):
    rows = []
    for path in _find(args.dir, "kernel_stats.csv"):
        with open(path, newline="") as fh:
            for r in csv.DictReader(fh):
                rows.append((r["Name"], int(r["Calls"]), float(r["TotalDurationNs"]),
                             float(r["AverageNs"])))
    rows.sort(key=lambda r: -r[2])
    tot = sum(r[2] for r in rows)
    out = [f"# {args.title}\n",
           f"Command (from /tmp with TMPDIR=/tmp):\n\n```\n{args.cmd}\n```\n",
           f"Total kernel time {tot / 1e6:.1f} ms over {sum(r[1] for r in rows)} dispatches.\n",
           "| kernel | calls | total ms | avg us | % |", "|---|---:|---:|---:|---:|"]
    for name, calls, total, avg in rows[: args.top]:
        out.append(f"| `{_short(name)}` | {calls} | {total / 1e6:.1f} | {avg / 1e3:.1f} | "
                   f"{100.0 * total / tot:.1f} |")
    print("\n".join(out))


def _counter(d, counter, kernel=None):
    """Per-dispatch values of `counter` (summed over its instances) for matching kernels."""
    per = {}
    for path in _find(d, "counter_collection.csv"):
        with open(path, newline="") as fh:
            for r in csv.DictReader(fh):
                if r.get("Counter_Name") != counter:
                    continue
                name = r.get("Kernel_Name", "")
                if kernel is not None and kernel not in name:
                    continue
                key = (path, r.get("Dispatch_Id") or r.get("Correlation_Id"))
                per[key] = per.get(key, 0.0) + float(r["Counter_Value"])
    return list(per.values())


def pmc(args):
    f = _counter(args.fetch, "FETCH_SIZE", args.kernel)
    w = _counter(args.write, "WRITE_SIZE", args.kernel)
    cf = _counter(args.cal_fetch, "FETCH_SIZE")
    cw = _counter(args.cal_write, "WRITE_SIZE")
    if not (f and w and cf and cw):
        raise SystemExit("missing counter values")
    kib = args.cal_bytes / 1024.0
    sf, sw = kib / max(cf), kib / max(cw)
    fa, wa = sum(f) / len(f), sum(w) / len(w)
    fetch_b, write_b = fa * sf * 1024.0, wa * sw * 1024.0
    out = [f"# {args.title}\n",
           "Commands (from /tmp with TMPDIR=/tmp):\n",
           "```", *args.cmd, "```\n",
           f"Kernel: names containing `{args.kernel}`; {len(f)} dispatches (FETCH_SIZE run), "
           f"{len(w)} (WRITE_SIZE run).\n",
           f"Calibration: a plain device copy of {args.cal_bytes} bytes reads FETCH_SIZE "
           f"{max(cf):.0f} KiB and WRITE_SIZE {max(cw):.0f} KiB; scale factors "
           f"{sf:.4f} (fetch) and {sw:.4f} (write).\n",
           "| per launch | counter (KiB) | scaled bytes |", "|---|---:|---:|",
           f"| FETCH_SIZE | {fa:.1f} | {fetch_b:.4g} |",
           f"| WRITE_SIZE | {wa:.1f} | {write_b:.4g} |",
           f"| total HBM traffic | | {fetch_b + write_b:.4g} |"]
    if args.alg_bytes:
        out.append(f"\nAlgorithmic bytes per launch: {args.alg_bytes:.4g}; measured / algorithmic "
                   f"= {(fetch_b + write_b) / args.alg_bytes:.2f}.")
    print("\n".join(out))


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__,
                                 formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="mode", required=True)
    s = sub.add_parser("stats")
    s.add_argument("dir")
    s.add_argument("--title", required=True)
    s.add_argument("--cmd", required=True)
    s.add_argument("--top", type=int, default=25)
    p = sub.add_parser("pmc")
    for k in ("--kernel", "--fetch", "--write", "--cal-fetch", "--cal-write", "--title"):
        p.add_argument(k, required=True)
    p.add_argument("--cal-bytes", type=float, required=True)
    p.add_argument("--alg-bytes", type=float, default=0.0)
    p.add_argument("--cmd", action="append", required=True)
    a = ap.parse_args(argv)
    (stats if a.mode == "stats" else pmc)(a)


if __name__ == "__main__":
    sys.exit(main())
