"""Summaries of rocprofv3 runs of bench.py, for the committed profiles.

Reads the CSV outputs of three rocprofv3 runs of the same bench command
(kernel trace with --stats, --pmc FETCH_SIZE, --pmc WRITE_SIZE) and writes

  profiles/<name>_kernels.md   per-kernel count / total / average duration
  profiles/<name>_traffic.md   HBM bytes per dispatch from the counters,
                               scaled by the same counters read for a
                               device copy of known size
  profiles/<name>_traffic.json the traffic of the dominant kernels with the
                               hash of the source they were measured on
                               (bench.py reports it only while that hash
                               still matches)

Usage (from the repository root, after the three runs):
  python3 -m paper_2403_00306_amd.profile_tools --name NAME \\
      --stats DIR/..._kernel_stats.csv --fetch DIR/..._counter_collection.csv \\
      --write DIR/..._counter_collection.csv --copy-bytes N --command "..."
"""
from __future__ import annotations

import argparse
import collections
import csv
import hashlib
import json
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
KERNEL_SOURCES = {"k_tiled": "csrc/k_tiles.hip", "k_bitset_pass": "csrc/k_tiles.hip",
                  "k_tiled_512": "csrc/k_tiles.hip",
                  "k_tiled_quorum": "csrc/k_tiles.hip",
                  "k_alpha_filter": "csrc/k_alpha.hip",
                  "k_pair_filter": "csrc/k_pair.hip",
                  "k_filter": "csrc/k_filter.hip"}


def _code_text(path: str) -> str:
    """The file without comments and with whitespace collapsed, so that a
    comment edit does not mark a profile as stale."""
    src = open(path, encoding="utf-8").read()
    src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
    src = re.sub(r"//[^\n]*", " ", src)
    return " ".join(src.split())


def source_hash(kernel: str) -> str:
    """Hash of the kernel's source file and the shared device header (the
    constants that shape every kernel), code only."""
    h = hashlib.sha256()
    for rel in (KERNEL_SOURCES[kernel], "csrc/pms_internal.h"):
        h.update(_code_text(os.path.join(HERE, rel)).encode())
    return h.hexdigest()[:16]


def short(name: str) -> str:
    n = name.split("(")[0]
    return n.replace("pms::", "")


def per_dispatch(path: str, counter: str) -> dict:
    vals = collections.defaultdict(list)
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] == counter:
            vals[short(r["Kernel_Name"])].append(float(r["Counter_Value"]))
    return vals


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--name", required=True)
    ap.add_argument("--stats", required=True)
    ap.add_argument("--fetch", required=True)
    ap.add_argument("--write", required=True)
    ap.add_argument("--copy-bytes", type=int, required=True)
    ap.add_argument("--command", required=True)
    ap.add_argument("--out", default=os.path.join(ROOT, "profiles"))
    a = ap.parse_args()
    os.makedirs(a.out, exist_ok=True)

    rows = list(csv.DictReader(open(a.stats)))
    lines = ["# Kernel durations: %s" % a.name, "",
             "Command (repository root, on the MI355X box):", "",
             "    " + a.command, "",
             "| kernel | calls | total ms | average us | % |",
             "|---|---:|---:|---:|---:|"]
    for r in rows:
        lines.append("| %s | %s | %.3f | %.1f | %.2f |" % (
            short(r["Name"]), r["Calls"], float(r["TotalDurationNs"]) / 1e6,
            float(r["AverageNs"]) / 1e3, float(r["Percentage"])))
    open(os.path.join(a.out, "%s_kernels.md" % a.name), "w").write(
        "\n".join(lines) + "\n")

    fetch = per_dispatch(a.fetch, "FETCH_SIZE")
    write = per_dispatch(a.write, "WRITE_SIZE")
    copy = "__amd_rocclr_copyBuffer"
    # the largest copy dispatch is the probe of known size
    cf = max(fetch.get(copy, [0.0])) * 1024.0
    cw = max(write.get(copy, [0.0])) * 1024.0
    kf = a.copy_bytes / cf if cf else None
    kw = a.copy_bytes / cw if cw else None
    lines = ["# HBM traffic per dispatch: %s" % a.name, "",
             "FETCH_SIZE and WRITE_SIZE (KiB per dispatch) from two "
             "rocprofv3 --pmc runs of:", "", "    " + a.command, "",
             "Calibration: a device copy of %d bytes reads FETCH_SIZE %.1f "
             "KiB and WRITE_SIZE %.1f KiB; scale factors %.4f (fetch), "
             "%.4f (write)." % (a.copy_bytes, cf / 1024, cw / 1024,
                                kf or 0, kw or 0), "",
             "| kernel | dispatches | fetch MB (scaled) | write MB (scaled) |",
             "|---|---:|---:|---:|"]
    traffic = {}
    for k in sorted(set(fetch) | set(write)):
        f = fetch.get(k, [0.0])
        w = write.get(k, [0.0])
        fm = sum(f) / len(f) * 1024.0 * (kf or 1.0)
        wm = sum(w) / len(w) * 1024.0 * (kw or 1.0)
        lines.append("| %s | %d | %.3f | %.3f |" % (k, len(f), fm / 1e6,
                                                   wm / 1e6))
        if k in KERNEL_SOURCES:
            # the i-th dispatch of a kernel is the same bench step in both
            # runs; a kernel launched on workloads of different sizes also
            # keeps its smallest and largest dispatch
            per = [a * 1024.0 * (kf or 1.0) + b * 1024.0 * (kw or 1.0)
                   for a, b in zip(f, w)]
            traffic[k] = {"fetch_bytes": fm, "write_bytes": wm,
                          "bytes": fm + wm, "min_bytes": min(per),
                          "max_bytes": max(per), "source_sha": source_hash(k)}
    open(os.path.join(a.out, "%s_traffic.md" % a.name), "w").write(
        "\n".join(lines) + "\n")
    json.dump({"command": a.command, "copy_bytes": a.copy_bytes,
               "fetch_scale": kf, "write_scale": kw, "kernels": traffic},
              open(os.path.join(a.out, "%s_traffic.json" % a.name), "w"),
              indent=1)


if __name__ == "__main__":
    main()
