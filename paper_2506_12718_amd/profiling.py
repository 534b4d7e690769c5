"""Summaries of rocprofv3 output for the profiles/ directory.

    python -m paper_2506_12718_amd.profiling stats <kernel_stats.csv> --cmd "<command>"
    python -m paper_2506_12718_amd.profiling traffic --fetch <counter_collection.csv>
        --write <counter_collection.csv> --calib-fetch <csv> --calib-write <csv>
        --kernel <substring> --calib-bytes <bytes> --cmd "<commands>" --out <json>

`stats` turns a --kernel-trace --stats CSV into a short text table.
`traffic` turns two --pmc runs (FETCH_SIZE, then WRITE_SIZE, KiB per
dispatch) into HBM bytes per launch of one kernel, each counter scaled by
what it reads for the plain streaming copy of known size (calibration runs
of ``bench.py --calibrate``), and records the hash of the kernel sources the
counters were taken on.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def kernel_source_hash():
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_2506_12718_amd", "csrc", "*"))):
        if f.endswith((".hip", ".h", ".cpp")):
            with open(f, "rb") as fh:
                h.update(fh.read())
    return h.hexdigest()[:16]


def stats(path, cmd, top=12):
    rows = list(csv.DictReader(open(path)))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    out = ["# rocprofv3 --kernel-trace --stats", "# command: %s" % cmd,
           "# columns: calls, total ms, average us, min us, max us, percent, kernel", ""]
    for r in rows[:top]:
        out.append("%6d %10.3f %10.2f %10.2f %10.2f %6.2f%%  %s" % (
            int(r["Calls"]), float(r["TotalDurationNs"]) / 1e6, float(r["AverageNs"]) / 1e3,
            float(r["MinNs"]) / 1e3, float(r["MaxNs"]) / 1e3, float(r["Percentage"]),
            r["Name"]))
    return "\n".join(out) + "\n"


def _per_kernel(path, counter):
    vals = {}
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] != counter:
            continue
        vals.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
    return vals


def _pick(vals, pattern):
    keys = [k for k in vals if pattern in k]
    if len(keys) != 1:
        raise SystemExit("kernel pattern %r matches %d kernels: %s" % (pattern, len(keys), keys))
    v = vals[keys[0]]
    return keys[0], sum(v) / len(v), len(v)


def traffic(a):
    kf = _per_kernel(a.fetch, "FETCH_SIZE")
    kw = _per_kernel(a.write, "WRITE_SIZE")
    cf = _per_kernel(a.calib_fetch, "FETCH_SIZE")
    cw = _per_kernel(a.calib_write, "WRITE_SIZE")
    name, fetch_kib, nf = _pick(kf, a.kernel)
    _, write_kib, nw = _pick(kw, a.kernel)
    _, cfetch_kib, _ = _pick(cf, "stream_copy")
    _, cwrite_kib, _ = _pick(cw, "stream_copy")
    ffac = a.calib_bytes / (cfetch_kib * 1024.0)
    wfac = a.calib_bytes / (cwrite_kib * 1024.0)
    hbm = fetch_kib * 1024.0 * ffac + write_kib * 1024.0 * wfac
    return {
        "kernel": name, "dispatches": [nf, nw],
        "fetch_kib_per_launch": fetch_kib, "write_kib_per_launch": write_kib,
        "calibration": {"bytes_read_and_written": a.calib_bytes, "fetch_kib": cfetch_kib,
                        "write_kib": cwrite_kib, "fetch_factor": ffac, "write_factor": wfac},
        "hbm_bytes_per_launch": hbm,
        "kernel_source_hash": kernel_source_hash(),
        "commands": a.cmd,
    }


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="what", required=True)
    s = sub.add_parser("stats")
    s.add_argument("csv")
    s.add_argument("--cmd", required=True)
    t = sub.add_parser("traffic")
    for k in ("fetch", "write", "calib_fetch", "calib_write", "kernel", "cmd", "out"):
        t.add_argument("--" + k.replace("_", "-"), required=True)
    t.add_argument("--calib-bytes", type=float, required=True)
    a = ap.parse_args(argv)
    if a.what == "stats":
        sys.stdout.write(stats(a.csv, a.cmd))
    else:
        d = traffic(a)
        with open(a.out, "w") as f:
            json.dump(d, f, indent=1)
        print(json.dumps(d, indent=1))


if __name__ == "__main__":
    main()
