"""Summaries of rocprofv3 output (CSV format) for the measurement record.

    python -m paper_2405_00482_amd.profile_summary stats DIR
        per-kernel table from a ``rocprofv3 --kernel-trace --stats
        --output-format csv`` run (reads *_kernel_stats.csv).
    python -m paper_2405_00482_amd.profile_summary traffic --copy-fetch D1
        --copy-write D2 --copy-bytes B --fetch D3 --write D4 --out F.json
        HBM bytes per dispatch of every kernel in D3/D4 (FETCH_SIZE and
        WRITE_SIZE passes, KiB per dispatch), each counter scaled by what it
        reads for a plain copy kernel of B bytes (passes D1/D2).  The JSON
        records a hash of the kernel sources; a reader that finds a different
        hash knows the counters are stale.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import sys
from collections import defaultdict

_CSRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")


def kernel_source_hash() -> str:
    """sha256 over the device-code sources (.hip and .hpp) of the library."""
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(_CSRC, "*.hip")) + glob.glob(os.path.join(_CSRC, "*.hpp"))):
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def _counter_csv(d: str) -> str:
    hits = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    if not hits:
        raise SystemExit(f"no counter_collection.csv under {d}")
    return hits[0]


def per_kernel_counter(d: str, counter: str) -> dict:
    """mean value of `counter` per dispatch, by kernel name"""
    acc = defaultdict(list)
    with open(_counter_csv(d)) as fh:
        for row in csv.DictReader(fh):
            if row["Counter_Name"] == counter:
                acc[row["Kernel_Name"]].append(float(row["Counter_Value"]))
    return {k: (sum(v) / len(v), len(v)) for k, v in acc.items()}


def _short(name: str) -> str:
    s = name.split("(")[0]
    return s.replace("void ", "").replace("pvfl::", "")


def traffic(a) -> dict:
    cf = per_kernel_counter(a.copy_fetch, "FETCH_SIZE")
    cw = per_kernel_counter(a.copy_write, "WRITE_SIZE")
    copy_k = max(cf, key=lambda k: cf[k][0])
    kib = a.copy_bytes / 1024.0
    f_fetch = kib / cf[copy_k][0]
    f_write = kib / cw[copy_k][0]
    fetch = per_kernel_counter(a.fetch, "FETCH_SIZE")
    write = per_kernel_counter(a.write, "WRITE_SIZE")
    out = {"source_hash": kernel_source_hash(), "workload": a.workload,
           "copy_kernel": _short(copy_k), "copy_bytes": a.copy_bytes,
           "copy_fetch_kib": cf[copy_k][0], "copy_write_kib": cw[copy_k][0],
           "fetch_factor": f_fetch, "write_factor": f_write, "kernels": {}}
    for k in sorted(set(fetch) & set(write)):
        fb = fetch[k][0] * 1024.0 * f_fetch
        wb = write[k][0] * 1024.0 * f_write
        out["kernels"][_short(k)] = {"fetch_bytes": fb, "write_bytes": wb, "traffic_bytes": fb + wb,
                                     "dispatches": fetch[k][1]}
    return out


def stats(d: str) -> str:
    hits = glob.glob(os.path.join(d, "**", "*kernel_stats.csv"), recursive=True)
    if not hits:
        raise SystemExit(f"no kernel_stats.csv under {d}")
    rows = list(csv.DictReader(open(hits[0])))
    lines = ["| kernel | calls | total ms | average us | min us | max us | % |", "|---|---|---|---|---|---|---|"]
    for r in rows:
        lines.append(f"| {_short(r['Name'])} | {r['Calls']} | {float(r['TotalDurationNs']) / 1e6:.3f} | "
                     f"{float(r['AverageNs']) / 1e3:.1f} | {float(r['MinNs']) / 1e3:.1f} | "
                     f"{float(r['MaxNs']) / 1e3:.1f} | {float(r['Percentage']):.2f} |")
    return "\n".join(lines)


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("dir")
    t = sub.add_parser("traffic")
    for k in ("copy_fetch", "copy_write", "fetch", "write", "out"):
        t.add_argument("--" + k.replace("_", "-"), required=True)
    t.add_argument("--copy-bytes", type=float, required=True)
    t.add_argument("--workload", default="")
    a = ap.parse_args(argv)
    if a.cmd == "stats":
        print(stats(a.dir))
    else:
        res = traffic(a)
        with open(a.out, "w") as fh:
            json.dump(res, fh, indent=1)
        print(json.dumps(res, indent=1))


if __name__ == "__main__":
    sys.exit(main())
