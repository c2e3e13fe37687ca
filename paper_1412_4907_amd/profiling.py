"""Summaries of rocprofv3 output for the beamform kernels.

``python -m paper_1412_4907_amd.profiling <dir>...`` reads
``*_counter_collection.csv`` (from ``rocprofv3 --pmc``) and
``*_kernel_stats.csv`` (from ``--kernel-trace --stats``) under each
directory and prints, per kernel, the mean of every counter per dispatch
(summed over the dimensions rocprofv3 reports) and the trace statistics.

``traffic_entry`` turns FETCH_SIZE / WRITE_SIZE readings (KiB per dispatch)
into HBM bytes per launch, scaled by what the same counters read for a
plain copy kernel of known size.
"""
from __future__ import annotations

import collections
import csv
import glob
import json
import os
import sys


def counters(path: str) -> dict:
    """{kernel name: {counter: mean per dispatch}} from a counter CSV."""
    per = collections.defaultdict(lambda: collections.defaultdict(float))
    names = {}
    for r in csv.DictReader(open(path)):
        key = r["Dispatch_Id"]
        names[key] = r["Kernel_Name"]
        per[key][r["Counter_Name"]] += float(r["Counter_Value"])
    out = collections.defaultdict(lambda: collections.defaultdict(list))
    for d, vals in per.items():
        for c, v in vals.items():
            out[names[d]][c].append(v)
    return {k: {c: sum(v) / len(v) for c, v in cs.items()} | {"dispatches": len(next(iter(cs.values())))}
            for k, cs in out.items()}


def kernel_stats(path: str) -> dict:
    out = {}
    for r in csv.DictReader(open(path)):
        out[r["Name"]] = {"calls": int(r["Calls"]), "avg_ns": float(r["AverageNs"]),
                          "min_ns": float(r["MinNs"]), "max_ns": float(r["MaxNs"])}
    return out


def copy_scale(fetch_kib: float, write_kib: float, nbytes: int) -> tuple:
    """Factors that turn FETCH_SIZE / WRITE_SIZE KiB into bytes, from a copy
    of ``nbytes`` (which reads and writes ``nbytes``)."""
    return nbytes / (fetch_kib * 1024.0), nbytes / (write_kib * 1024.0)


def traffic_entry(fetch_kib: float, write_kib: float, fscale: float, wscale: float,
                  source_hash: str, command: str) -> dict:
    read = fetch_kib * 1024.0 * fscale
    write = write_kib * 1024.0 * wscale
    return {"read_bytes": read, "write_bytes": write, "bytes_per_launch": read + write,
            "fetch_scale": fscale, "write_scale": wscale, "source_hash": source_hash,
            "command": command}


def main(argv) -> None:
    for d in argv:
        for f in sorted(glob.glob(os.path.join(d, "**", "*_counter_collection.csv"), recursive=True)):
            print(f"== {f}")
            for k, cs in counters(f).items():
                print(f"  {k[:90]}")
                print("    " + json.dumps({c: round(v, 3) for c, v in cs.items()}))
        for f in sorted(glob.glob(os.path.join(d, "**", "*_kernel_stats.csv"), recursive=True)):
            print(f"== {f}")
            for k, st in kernel_stats(f).items():
                print(f"  {k[:90]}: {st}")


if __name__ == "__main__":
    main(sys.argv[1:])
