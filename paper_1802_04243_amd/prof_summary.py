"""Turn rocprofv3 CSV output of bench.py into the committed profile summaries.

Usage (after the rocprofv3 runs listed in the summary files):
  python -m paper_1802_04243_amd.prof_summary <kt_dir> <fetch_dir> <write_dir> \
      <copy_fetch_dir> <copy_write_dir> <out_dir>
  python -m paper_1802_04243_amd.prof_summary sq <sq_dir> [<sq_dir> ...]
  python -m paper_1802_04243_amd.prof_summary trace <kt_dir>

FETCH_SIZE and WRITE_SIZE are reported in KiB per dispatch; each is scaled by
what the same counter reads for a plain 1 GiB device copy (bench.py
--copy-probe), so that the bytes are HBM bytes.
"""
from __future__ import annotations

import csv
import glob
import hashlib
import json
import os
import re
import sys
from collections import defaultdict

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
KERNEL_SOURCES = ["paper_1802_04243_amd/csrc/sts_kernels.hip", "paper_1802_04243_amd/csrc/sts_internal.h"]
def scheme_of(kernel: str):
    """Scheme of a plain (not last, not mixed, no intermediates, no
    slip-jump surfaces) pass kernel k_pass<NTH, IM, TV, RS, MX, IN, SJ>."""
    if not kernel.startswith("k_pass<"):
        return None
    a = [x.strip() for x in kernel[len("k_pass<"):-1].split(",")]
    if len(a) != 7 or any(x != "false" for x in a[3:]):
        return None
    return ("implicit" if a[1] == "true" else "explicit") + ("_tvd" if a[2] == "true" else "_upwind")
NFV = 5120 * 1152


def kernel_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()[:16]


def short(name: str) -> str:
    name = re.sub(r"\b\w+::\(anonymous namespace\)::", "", name).replace("void ", "")
    return name.split("(")[0]


def counters(d: str):
    out = defaultdict(list)
    for f in glob.glob(os.path.join(d, "*counter_collection.csv")):
        for r in csv.DictReader(open(f)):
            out[short(r["Kernel_Name"])].append(float(r["Counter_Value"]))
    return out


def main(kt, fetch, write, cfetch, cwrite, outdir):
    stats = list(csv.DictReader(open(glob.glob(os.path.join(kt, "*kernel_stats.csv"))[0])))
    f, w = counters(fetch), counters(write)
    cf, cw = counters(cfetch), counters(cwrite)
    copy = "__amd_rocclr_copyBuffer"
    fscale = (1 << 30) / (sum(cf[copy]) / len(cf[copy]) * 1024)
    wscale = (1 << 30) / (sum(cw[copy]) / len(cw[copy]) * 1024)
    per = {}
    for k in sorted(f):
        if k not in w or not k.startswith("k_"):
            continue
        rd = sum(f[k]) / len(f[k]) * 1024 * fscale
        wr = sum(w[k]) / len(w[k]) * 1024 * wscale
        per[k] = dict(read_bytes=rd, write_bytes=wr, bytes=rd + wr, bytes_per_fv=(rd + wr) / NFV,
                      dispatches=len(f[k]))
    traffic = {"kernel_hash": kernel_hash(), "workload": "channel_5120x1152",
               "fetch_scale": fscale, "write_scale": wscale,
               "bytes_per_launch": {scheme_of(k): v["bytes"] for k, v in per.items() if scheme_of(k)},
               "per_kernel": per}
    os.makedirs(outdir, exist_ok=True)
    json.dump(traffic, open(os.path.join(outdir, "pass_kernel_hbm_traffic_5120x1152.json"), "w"), indent=1)
    lines = ["| kernel | calls | avg us | min us | max us | HBM read MB | HBM write MB | HBM B/FV |",
             "|---|---|---|---|---|---|---|---|"]
    for r in stats:
        k = short(r["Name"])
        t = per.get(k)
        extra = (f"{t['read_bytes'] / 1e6:.1f} | {t['write_bytes'] / 1e6:.1f} | {t['bytes_per_fv']:.1f}"
                 if t else " | | ")
        lines.append(f"| {k} | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                     f"{float(r['MinNs']) / 1e3:.1f} | {float(r['MaxNs']) / 1e3:.1f} | {extra} |")
    print("\n".join(lines))
    print(f"\nFETCH_SIZE scale {fscale:.4f}, WRITE_SIZE scale {wscale:.4f} (1 GiB copy probe)")
    return lines, fscale, wscale


def sq(dirs):
    """Mean per dispatch of every SQ counter of every k_* kernel over the
    counter runs in dirs, as a markdown table (one column per kernel)."""
    vals = defaultdict(lambda: defaultdict(list))
    for d in dirs:
        for f in glob.glob(os.path.join(d, "*counter_collection.csv")):
            for r in csv.DictReader(open(f)):
                k = short(r["Kernel_Name"])
                if k.startswith("k_"):
                    vals[k][r["Counter_Name"]].append(float(r["Counter_Value"]))
    kernels = sorted(vals)
    names = sorted({c for k in kernels for c in vals[k]})
    lines = ["| counter | " + " | ".join(kernels) + " |", "|---|" + "---|" * len(kernels)]
    for c in names:
        row = [f"{sum(vals[k][c]) / len(vals[k][c]):,.0f}" if vals[k][c] else "" for k in kernels]
        lines.append(f"| {c} | " + " | ".join(row) + " |")
    lines.append("| dispatches | " + " | ".join(
        str(max(len(v) for v in vals[k].values()) // max(1, len(dirs))) for k in kernels) + " |")
    print("\n".join(lines))
    return vals


def trace(kt):
    """Kernel-trace statistics as a markdown table with each kernel's share
    of the summed kernel time."""
    stats = list(csv.DictReader(open(glob.glob(os.path.join(kt, "*kernel_stats.csv"))[0])))
    total = sum(float(r["TotalDurationNs"]) for r in stats)
    lines = ["| kernel | calls | avg us | total ms | share |", "|---|---|---|---|---|"]
    for r in stats:
        lines.append(f"| {short(r['Name'])} | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                     f"{float(r['TotalDurationNs']) / 1e6:.2f} | "
                     f"{100 * float(r['TotalDurationNs']) / total:.1f} % |")
    print("\n".join(lines))
    return stats


if __name__ == "__main__":
    if sys.argv[1] == "sq":
        sq(sys.argv[2:])
    elif sys.argv[1] == "trace":
        trace(sys.argv[2])
    else:
        main(*sys.argv[1:7])
