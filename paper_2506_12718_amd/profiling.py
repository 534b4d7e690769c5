"""Summaries of rocprofv3 output for the profiles/ directory.

    python -m paper_2506_12718_amd.profiling stats <kernel_stats.csv> --cmd "<command>"
    python -m paper_2506_12718_amd.profiling traffic --fetch <counter_collection.csv>
        --write <counter_collection.csv> --calib-fetch <csv> --calib-write <csv>
        --kernel <substring> --calib-bytes <bytes> --cmd "<commands>" --out <json>
    python -m paper_2506_12718_amd.profiling calib --fetch <csv> --write <csv>
        --bytes <bytes> --cmd "<commands>" --out <json>
    python -m paper_2506_12718_amd.profiling conv-traffic --fetch <csv> --write <csv>
        --calib-fetch <csv> --calib-write <csv> --calib-bytes <bytes>
        --run <counter-run json> --cmd "<commands>" --out <json>

`stats` turns a --kernel-trace --stats CSV into a short text table.
`traffic` turns two --pmc runs (FETCH_SIZE, then WRITE_SIZE, KiB per
dispatch) into HBM bytes per launch of one kernel, each counter scaled by
what it reads for the plain streaming copy of known size (calibration runs
of ``bench.py --calibrate``), and records the hash of the kernel sources the
counters were taken on.
`calib` reports the scale factors of the three reference kernels of
``bench.py --calibrate`` (copies with 16 and 8 bytes per lane, a read-only
sweep), so that one factor is checked against the others.
`conv-traffic` sums the counters over every kernel of one convolution: the
last K x launches dispatches of library kernels of a ``bench.py
--counter-run K`` run (whose JSON line gives K and the launches).
`sq` tabulates shader counters (SQ_*) per library kernel of such a run,
mean per dispatch, with LDS bank-conflict cycles per LDS instruction.

    python -m paper_2506_12718_amd.profiling sq <counter_collection.csv> --cmd "<command>"
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


def _copy_factors(calib_fetch, calib_write, calib_bytes):
    """FETCH_SIZE and WRITE_SIZE scale factors of the 16-byte streaming copy."""
    cf = _per_kernel(calib_fetch, "FETCH_SIZE")
    cw = _per_kernel(calib_write, "WRITE_SIZE")
    _, cfetch_kib, _ = _pick(cf, "stream_copy_kernel")
    _, cwrite_kib, _ = _pick(cw, "stream_copy_kernel")
    return cfetch_kib, cwrite_kib, calib_bytes / (cfetch_kib * 1024.0), \
        calib_bytes / (cwrite_kib * 1024.0)


def traffic(a):
    kf = _per_kernel(a.fetch, "FETCH_SIZE")
    kw = _per_kernel(a.write, "WRITE_SIZE")
    name, fetch_kib, nf = _pick(kf, a.kernel)
    _, write_kib, nw = _pick(kw, a.kernel)
    cfetch_kib, cwrite_kib, ffac, wfac = _copy_factors(a.calib_fetch, a.calib_write,
                                                       a.calib_bytes)
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


def calib(a):
    """Scale factors (true bytes / counter bytes) of the three reference
    kernels: the 16- and 8-byte copies read and write every byte once, the
    read-only sweep reads every byte once."""
    kf = _per_kernel(a.fetch, "FETCH_SIZE")
    kw = _per_kernel(a.write, "WRITE_SIZE")
    out = {"bytes": a.bytes, "kernels": {}, "commands": a.cmd}
    for label, pat, writes in (("copy16", "stream_copy_kernel", True),
                               ("copy8", "stream_copy8_kernel", True),
                               ("read", "stream_read_kernel", False)):
        _, f_kib, nf = _pick(kf, pat)
        _, w_kib, nw = _pick(kw, pat)
        d = {"dispatches": [nf, nw], "fetch_kib": f_kib, "write_kib": w_kib,
             "fetch_factor": a.bytes / (f_kib * 1024.0)}
        if writes:
            d["write_factor"] = a.bytes / (w_kib * 1024.0)
        out["kernels"][label] = d
    ff = [k["fetch_factor"] for k in out["kernels"].values()]
    out["fetch_factor_spread"] = max(ff) / min(ff) - 1.0
    return out


def _dispatches(path, counter):
    """(dispatch id, kernel, value) of every library kernel dispatch."""
    rows = []
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] != counter or "pafc::" not in r["Kernel_Name"]:
            continue
        rows.append((int(r["Dispatch_Id"]), r["Kernel_Name"], float(r["Counter_Value"])))
    rows.sort()
    return rows


def conv_traffic(a):
    run = json.loads(open(a.run).read().strip().splitlines()[-1])
    K, n = int(run["convs"]), int(run["launches_per_conv"])
    _, _, ffac, wfac = _copy_factors(a.calib_fetch, a.calib_write, a.calib_bytes)
    tot = {}
    per_launch = {}
    for counter, path, fac in (("FETCH_SIZE", a.fetch, ffac), ("WRITE_SIZE", a.write, wfac)):
        rows = _dispatches(path, counter)
        if len(rows) < K * n:
            raise SystemExit("%s: %d library dispatches, fewer than %d" % (path, len(rows), K * n))
        last = rows[-K * n:]
        tot[counter] = sum(v for _, _, v in last) * 1024.0 * fac / K
        for i, (_, name, v) in enumerate(last):
            e = per_launch.setdefault(i % n, {"kernel": name})
            e.setdefault(counter, []).append(v * 1024.0 * fac)
    launches = []
    for i in range(n):
        e = per_launch[i]
        launches.append({"kernel": e["kernel"],
                         "fetch_bytes": sum(e["FETCH_SIZE"]) / len(e["FETCH_SIZE"]),
                         "write_bytes": sum(e["WRITE_SIZE"]) / len(e["WRITE_SIZE"])})
    hbm = tot["FETCH_SIZE"] + tot["WRITE_SIZE"]
    return {"workload": run["workload"], "convs": K, "launches_per_conv": n,
            "fetch_bytes_per_conv": tot["FETCH_SIZE"], "write_bytes_per_conv": tot["WRITE_SIZE"],
            "hbm_bytes_per_conv": hbm, "alg_bytes_per_conv": run["alg_bytes_per_conv"],
            "ratio_to_alg": hbm / run["alg_bytes_per_conv"],
            "fetch_factor": ffac, "write_factor": wfac, "launches": launches,
            "kernel_source_hash": kernel_source_hash(), "commands": a.cmd}


def sq(path, cmd):
    per = {}
    for r in csv.DictReader(open(path)):
        if "pafc::" not in r["Kernel_Name"]:
            continue
        k = per.setdefault(r["Kernel_Name"], {})
        k.setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
    names = sorted({c for k in per.values() for c in k})
    out = ["# rocprofv3 --pmc %s (mean per dispatch)" % " ".join(names), "# command: %s" % cmd, "",
           "| kernel | dispatches | " + " | ".join(names) + " | bank-conflict cycles / LDS instr |",
           "|---|---|" + "---|" * len(names) + "---|"]
    for kname, k in sorted(per.items(), key=lambda kv: -max(len(v) for v in kv[1].values())):
        mean = {c: sum(v) / len(v) for c, v in k.items()}
        n = max(len(v) for v in k.values())
        bc = mean.get("SQ_LDS_BANK_CONFLICT")
        li = mean.get("SQ_INSTS_LDS")
        ratio = "%.3f" % (bc / li) if bc is not None and li else "-"
        short = kname.split("(")[0].replace("void pafc::", "")
        out.append("| %s | %d | %s | %s |" % (short, n, " | ".join("%.4g" % mean.get(c, float("nan"))
                                                              for c in names), ratio))
    return "\n".join(out) + "\n"


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
    c = sub.add_parser("calib")
    for k in ("fetch", "write", "cmd", "out"):
        c.add_argument("--" + k, required=True)
    c.add_argument("--bytes", type=float, required=True)
    v = sub.add_parser("conv-traffic")
    for k in ("fetch", "write", "calib_fetch", "calib_write", "run", "cmd", "out"):
        v.add_argument("--" + k.replace("_", "-"), required=True)
    v.add_argument("--calib-bytes", type=float, required=True)
    q = sub.add_parser("sq")
    q.add_argument("csv")
    q.add_argument("--cmd", required=True)
    a = ap.parse_args(argv)
    if a.what == "stats":
        sys.stdout.write(stats(a.csv, a.cmd))
        return
    if a.what == "sq":
        sys.stdout.write(sq(a.csv, a.cmd))
        return
    d = {"traffic": traffic, "calib": calib, "conv-traffic": conv_traffic}[a.what](a)
    with open(a.out, "w") as f:
        json.dump(d, f, indent=1)
    print(json.dumps(d, indent=1))


if __name__ == "__main__":
    main()
