#!/usr/bin/env python3
"""Text summaries of rocprofv3 output for the benchmark's kernels.

Two reports, each printed to stdout:

  stats DIR                 per-kernel launch count and duration from a
                            `rocprofv3 --kernel-trace --stats --output-format csv`
                            run (DIR holds *_kernel_stats.csv)
  traffic FETCH WRITE       HBM bytes per launch of one kernel from two
                            `rocprofv3 --pmc FETCH_SIZE` / `--pmc WRITE_SIZE`
                            runs (each DIR holds *_counter_collection.csv),
                            scaled by what the same counters read for a plain
                            elementwise copy of known size in the same run

The traffic report ends with the SHA-256 of the kernel's sources, so that a
reader can tell whether the kernel has changed since the counters were taken.
Runs without the package being importable (no torch or GPU needed).
"""
from __future__ import annotations

import argparse
import collections
import csv
import glob
import hashlib
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
# sources whose change invalidates a traffic figure of the shift-and-sum
# kernel: the kernel itself, and of the internal header the part before the
# context structure (shape constants, region and window-record layouts)
APPLY_SOURCES = ("csrc/apply.hip", "csrc/soap_internal.hpp")
HEADER_CUT = b"struct soap_ctx {"


def sources_sha256(paths=APPLY_SOURCES) -> str:
    h = hashlib.sha256()
    for rel in paths:
        with open(os.path.join(HERE, rel), "rb") as f:
            data = f.read()
        if rel.endswith(".hpp") and HEADER_CUT in data:
            data = data[: data.index(HEADER_CUT)]
        h.update(data)
    return h.hexdigest()


def _short(name: str) -> str:
    name = name.replace("void ", "")
    return name.split("(")[0]


def stats(d: str) -> str:
    files = glob.glob(os.path.join(d, "**", "*kernel_stats.csv"), recursive=True)
    if not files:
        raise SystemExit(f"no *kernel_stats.csv under {d}")
    rows = []
    with open(files[0]) as f:
        for r in csv.DictReader(f):
            rows.append(
                (
                    _short(r["Name"]),
                    int(r["Calls"]),
                    float(r["TotalDurationNs"]),
                    float(r["AverageNs"]),
                    float(r["MinNs"]),
                    float(r["MaxNs"]),
                    float(r["Percentage"]),
                )
            )
    rows.sort(key=lambda x: -x[2])
    out = [f"{'kernel':64s} {'calls':>6s} {'total_us':>10s} {'avg_us':>9s} {'min_us':>9s} {'max_us':>9s} {'pct':>6s}"]
    for n, c, t, a, lo, hi, p in rows:
        out.append(f"{n[:64]:64s} {c:6d} {t / 1e3:10.1f} {a / 1e3:9.2f} {lo / 1e3:9.2f} {hi / 1e3:9.2f} {p:6.2f}")
    return "\n".join(out)


def _per_dispatch(d: str, counter: str):
    """kernel name -> list of per-dispatch counter totals (summed over
    instances)"""
    files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise SystemExit(f"no *counter_collection.csv under {d}")
    acc = collections.defaultdict(lambda: collections.defaultdict(float))
    with open(files[0]) as f:
        for r in csv.DictReader(f):
            if r["Counter_Name"] != counter:
                continue
            acc[_short(r["Kernel_Name"])][r["Dispatch_Id"]] += float(r["Counter_Value"])
    return {k: list(v.values()) for k, v in acc.items()}


def _find(table, key):
    hits = [k for k in table if key in k]
    if not hits:
        raise SystemExit(f"no kernel matching {key!r}; have {sorted(table)}")
    return hits


def traffic(fetch_dir: str, write_dir: str, kernel: str, calib: str, calib_bytes: int) -> str:
    lines = []
    res = {}
    for counter, d in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        t = _per_dispatch(d, counter)
        ck = _find(t, calib)
        cal = t[ck[0]]
        cal_kib = sum(cal) / len(cal)
        factor = calib_bytes / (cal_kib * 1024.0)
        kk = [k for k in _find(t, kernel)]
        vals = [v for k in kk for v in t[k]]
        kib = sum(vals) / len(vals)
        res[counter] = kib * 1024.0 * factor
        lines.append(
            f"{counter}: {kernel} {kib:.1f} KiB per dispatch (n={len(vals)}); copy calibration {ck[0][:40]} "
            f"{cal_kib:.1f} KiB for {calib_bytes} bytes -> factor {factor:.4f}; scaled {res[counter] / 1e6:.3f} MB"
        )
    total = res["FETCH_SIZE"] + res["WRITE_SIZE"]
    lines.append(f"read_bytes_per_launch: {res['FETCH_SIZE']:.0f}")
    lines.append(f"write_bytes_per_launch: {res['WRITE_SIZE']:.0f}")
    lines.append(f"traffic_bytes_per_launch: {total:.0f}")
    lines.append(f"kernel_source_sha256: {sources_sha256()}")
    return "\n".join(lines)


def read_traffic(path: str):
    """(traffic bytes per launch, sources sha256) from a traffic summary, or
    None when the file is absent"""
    if not os.path.exists(path):
        return None
    val = sha = None
    with open(path) as f:
        for ln in f:
            if ln.startswith("traffic_bytes_per_launch:"):
                val = float(ln.split(":", 1)[1])
            elif ln.startswith("kernel_source_sha256:"):
                sha = ln.split(":", 1)[1].strip()
    if val is None or sha is None:
        return None
    return val, sha


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="cmd", required=True)
    a = sub.add_parser("stats")
    a.add_argument("dir")
    b = sub.add_parser("traffic")
    b.add_argument("fetch_dir")
    b.add_argument("write_dir")
    b.add_argument("--kernel", default="k_apply")
    b.add_argument("--calib", default="neg_kernel")
    b.add_argument("--calib-bytes", type=int, required=True)
    args = ap.parse_args(argv)
    if args.cmd == "stats":
        print(stats(args.dir))
    else:
        print(traffic(args.fetch_dir, args.write_dir, args.kernel, args.calib, args.calib_bytes))


if __name__ == "__main__":
    sys.exit(main())
