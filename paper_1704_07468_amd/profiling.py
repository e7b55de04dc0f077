"""Summaries of rocprofv3 output for the kernels of this library.

    python -m paper_1704_07468_amd.profiling stats <kernel_stats.csv> <out.txt> --cmd "<command>"
    python -m paper_1704_07468_amd.profiling traffic <fetch.csv> <write.csv> <out.json> --copy-bytes B --cmd "<command>"

`stats` turns a `rocprofv3 --kernel-trace --stats` kernel-statistics CSV into
a short text table (calls, mean and total duration per kernel).  `traffic`
takes the counter-collection CSVs of two `rocprofv3 --pmc` runs of the same
command -- one with FETCH_SIZE, one with WRITE_SIZE (KiB per dispatch) -- and
records each kernel's mean per dispatch together with the same counters for
a plain copy kernel of known size (the elementwise kernel with the largest
fetch), so that a reader can scale the counters to bytes.  The JSON also
carries a hash of the library sources: the numbers describe the kernels as
they were built from exactly those sources.
"""
from __future__ import annotations

import argparse
import collections
import csv
import hashlib
import json
import os

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)


def source_sha() -> str:
    """SHA-256 over the library's kernel and host sources and its header."""
    h = hashlib.sha256()
    files = []
    for d in (os.path.join(PKG, "csrc"), os.path.join(ROOT, "include")):
        for f in sorted(os.listdir(d)):
            if f.endswith((".hip", ".cpp", ".h")):
                files.append(os.path.join(d, f))
    for f in files:
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def short_name(name: str) -> str:
    """Kernel name without namespace, template arguments or parameters."""
    n = name.split("(")[0]
    for pre in ("void ", "gk::"):
        n = n.replace(pre, "")
    return n.strip()


def stats(csv_path: str, out_path: str, cmd: str, top: int = 20) -> None:
    rows = list(csv.DictReader(open(csv_path)))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    lines = ["# rocprofv3 kernel statistics", "# command: " + cmd,
             "# summarised by: python3 -m paper_1704_07468_amd.profiling stats <dir>/<host>/<pid>/run_kernel_stats.csv "
             "<out> --cmd '<command>'", "",
             "%-44s %7s %12s %12s %7s" % ("kernel", "calls", "mean_us", "total_ms", "pct")]
    for r in rows[:top]:
        lines.append("%-44s %7s %12.1f %12.3f %7.2f" % (
            short_name(r["Name"])[:44], r["Calls"], float(r["AverageNs"]) / 1e3,
            float(r["TotalDurationNs"]) / 1e6, float(r["Percentage"])))
    with open(out_path, "w") as f:
        f.write("\n".join(lines) + "\n")


def _per_dispatch(csv_path: str, counter: str) -> dict:
    acc = collections.defaultdict(list)
    per = collections.defaultdict(float)
    for r in csv.DictReader(open(csv_path)):
        if r["Counter_Name"] != counter:
            continue
        per[(r["Kernel_Name"], r["Dispatch_Id"])] += float(r["Counter_Value"])
    for (k, _d), v in per.items():
        acc[k].append(v)
    return {k: sum(v) / len(v) for k, v in acc.items()}


def traffic(fetch_csv: str, write_csv: str, out_path: str, copy_bytes: int, cmd: str) -> None:
    fetch = _per_dispatch(fetch_csv, "FETCH_SIZE")
    write = _per_dispatch(write_csv, "WRITE_SIZE")
    copies = [k for k in fetch if "elementwise" in k]
    if not copies:
        raise SystemExit("no elementwise copy kernel in the fetch run")
    copy = max(copies, key=lambda k: fetch[k])
    kernels = {}
    for k in fetch:
        if not k.split("(")[0].replace("void ", "").startswith("gk::"):
            continue
        kernels[short_name(k)] = {"fetch_kib": fetch[k], "write_kib": write.get(k)}
    out = {
        "command": cmd,
        "summarised_by": "python3 -m paper_1704_07468_amd.profiling traffic <fetch counter_collection.csv> "
                         "<write counter_collection.csv> <out> --copy-bytes 1073741824 --cmd '<command>'",
        "source_sha": source_sha(),
        "units": "KiB per dispatch, mean over dispatches",
        "copy": {"kernel": short_name(copy), "bytes_read": copy_bytes, "bytes_written": copy_bytes,
                 "fetch_kib": fetch[copy], "write_kib": write.get(copy)},
        "kernels": kernels,
    }
    with open(out_path, "w") as f:
        json.dump(out, f, indent=1, sort_keys=True)
        f.write("\n")


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="what", required=True)
    s = sub.add_parser("stats")
    s.add_argument("csv")
    s.add_argument("out")
    s.add_argument("--cmd", required=True)
    t = sub.add_parser("traffic")
    t.add_argument("fetch_csv")
    t.add_argument("write_csv")
    t.add_argument("out")
    t.add_argument("--copy-bytes", type=int, required=True)
    t.add_argument("--cmd", required=True)
    a = ap.parse_args()
    if a.what == "stats":
        stats(a.csv, a.out, a.cmd)
    else:
        traffic(a.fetch_csv, a.write_csv, a.out, a.copy_bytes, a.cmd)


if __name__ == "__main__":
    main()
