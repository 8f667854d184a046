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

and, for SQ counter passes (--pmc runs of up to 8 SQ counters each):
  python3 -m paper_2403_00306_amd.profile_tools counters --name NAME \\
      --stats DIR/..._kernel_stats.csv --csv PASS1.csv [PASS2.csv ...] \\
      --kernels k_tiled_512 [...] --command "..."
which writes profiles/<name>_counters.md: per-dispatch averages of every
counter and the derived issue and LDS figures, with the source hash.
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
                  "k_lds_rate": "csrc/k_filter.hip",
                  "k_tiled_512": "csrc/k_tiles.hip",
                  "k_tiled_quorum": "csrc/k_tiles.hip",
                  "k_alpha_filter": "csrc/k_alpha.hip",
                  "k_pair_filter": "csrc/k_pair.hip",
                  "k_filter": "csrc/k_filter.hip",
                  "k_wide_filter": "csrc/k_wide.hip"}


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
    """Kernel name without namespace, return type, template arguments or
    parameter list ("void pms::k_filter<8>(...)" -> "k_filter")."""
    n = name.split("(")[0]
    if n.startswith("void "):
        n = n[len("void "):]
    n = re.sub(r"<[^<>]*>", "", n)
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


# gfx950: 256 CUs at up to 2.4 GHz; SQ cycle counters count quad-cycles
CUS = 256
CLOCK_HZ = 2.4e9


def main_counters(argv):
    ap = argparse.ArgumentParser(prog="profile_tools counters")
    ap.add_argument("--name", required=True)
    ap.add_argument("--stats", required=True)
    ap.add_argument("--csv", nargs="+", required=True)
    ap.add_argument("--kernels", nargs="+", required=True)
    ap.add_argument("--command", required=True)
    ap.add_argument("--out", default=os.path.join(ROOT, "profiles"))
    a = ap.parse_args(argv)
    avg_ns = {short(r["Name"]): float(r["AverageNs"])
              for r in csv.DictReader(open(a.stats))}
    vals = collections.defaultdict(dict)
    for path in a.csv:
        per = collections.defaultdict(lambda: collections.defaultdict(list))
        for r in csv.DictReader(open(path)):
            per[short(r["Kernel_Name"])][r["Counter_Name"]].append(
                float(r["Counter_Value"]))
        for k, cs in per.items():
            for cname, v in cs.items():
                vals[k][cname] = sum(v) / len(v)
    lines = ["# SQ counters per dispatch: %s" % a.name, "",
             "rocprofv3 --pmc passes (at most 8 SQ counters each) of:", "",
             "    " + a.command, "",
             "Kernel durations from the --kernel-trace --stats run of the "
             "same command. Derived figures assume %d CUs at %.1f GHz; "
             "SQ_WAVE_CYCLES and SQ_WAIT_* count quad-cycles; one wave64 "
             "VALU instruction per CU clock is the issue peak (4 SIMDs, "
             "4 clocks each), one SALU instruction per CU clock likewise."
             % (CUS, CLOCK_HZ / 1e9), ""]
    for k in a.kernels:
        v = vals.get(k, {})
        src = source_hash(k) if k in KERNEL_SOURCES else "-"
        ns = avg_ns.get(k)
        lines += ["## %s (source %s)" % (k, src), "",
                  "| counter | per dispatch |", "|---|---:|"]
        for cname in sorted(v):
            lines.append("| %s | %.4g |" % (cname, v[cname]))
        lines.append("")
        if ns:
            cyc = ns * 1e-9 * CLOCK_HZ * CUS      # CU clocks in the dispatch
            lines += ["average duration %.1f us, %.4g CU clocks" %
                      (ns / 1e3, cyc), ""]
            der = []
            for cname, label in (("SQ_INSTS_VALU", "VALU instructions per CU clock"),
                                 ("SQ_INSTS_SALU", "SALU instructions per CU clock"),
                                 ("SQ_INSTS_LDS", "LDS instructions per CU clock")):
                if cname in v:
                    der.append("| %s | %.3f |" % (label, v[cname] / cyc))
            if "SQ_LDS_IDX_ACTIVE" in v:
                der.append("| LDS active share of CU clocks | %.3f |" %
                           (v["SQ_LDS_IDX_ACTIVE"] / cyc))
            if "SQ_LDS_BANK_CONFLICT" in v and v.get("SQ_LDS_IDX_ACTIVE"):
                der.append("| bank-conflict share of LDS active | %.3f |" %
                           (v["SQ_LDS_BANK_CONFLICT"] / v["SQ_LDS_IDX_ACTIVE"]))
            if v.get("SQ_WAVE_CYCLES") and "SQ_WAIT_INST_ANY" in v:
                der.append("| waiting share of wave lifetime | %.3f |" %
                           (v["SQ_WAIT_INST_ANY"] / v["SQ_WAVE_CYCLES"]))
            if der:
                lines += ["| derived | value |", "|---|---:|"] + der + [""]
    open(os.path.join(a.out, "%s_counters.md" % a.name), "w").write(
        "\n".join(lines) + "\n")


if __name__ == "__main__":
    import sys
    if len(sys.argv) > 1 and sys.argv[1] == "counters":
        main_counters(sys.argv[2:])
    else:
        main()
