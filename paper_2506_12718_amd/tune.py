"""Autotuner for the planner's schedule choices.

For every (element type, axis length) it searches, on the GPU, the choices
that change only the schedule -- never the result:

* g3 / g5: how many radix-3 / radix-5 stages are fused into one register
  group (larger groups: fewer LDS round trips, more registers); g3i the same
  for the inner pieces of a cut axis (the middle pass's piece);
* split: the inner length of a 1-D transform cut into an outer (strided) and
  an inner (contiguous) pass;
* W / Wo: the tile widths of the inner and outer pieces.

The search is greedy coordinate descent, started from the better of the
planner's defaults and the existing table's entry: each coordinate in turn
takes the candidate with the lowest measured time (ties within 2 % keep the
current value).  A time is the median wall time of one repetition (all of
its launches and the gaps between them), from HIP events around the
library's own launches (`Batch.profile_levels` for batched size classes,
`Plan.profile_passes` for whole grids).  The result is a table in the format
of `pafc_set_tuning`, written to ``tuning/<device>.txt`` and loaded by the
binding on first use.

    python -m paper_2506_12718_amd.tune [--dtypes c128 c64] [--out PATH]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_TABLE = os.path.join(HERE, "tuning", "mi355x.txt")

BATCH_SIZES = [2 ** e for e in range(8, 17)] + [3 ** e for e in range(6, 11)] + \
              [5 ** e for e in range(4, 8)]
GRIDS = [((2187, 2187), 3), ((5 ** 9,), 5)]
# inner lengths of the prime-length routes' benchmark workloads (Rader at
# n = 995329, Bluestein at n = 995329 and n = 1000003), tuned as 1-D plans
INNER_1D = [995328, 2000000, 2025000]
# the radix-3 and radix-5 axes of the prime-factor route's benchmark
# workload (n = 2^8 3^5 5^3 on the 125 x 243 x 256 grid), each tuned on the
# whole route (register grouping only)
PFA_N = 2 ** 8 * 3 ** 5 * 5 ** 3
PFA_AXES = [243, 125]


def _factors(n):
    f = {}
    for p in (2, 3, 5):
        while n % p == 0:
            f[p] = f.get(p, 0) + 1
            n //= p
    return f


FIELDS = ("split", "W", "Wo", "g3", "g5", "g3i")


def line(dt, n, cfg):
    s = "%s %d %d %d %d %d %d" % (dt, n, cfg["split"], cfg["W"], cfg["Wo"], cfg["g3"], cfg["g5"])
    return s + (" %d" % cfg["g3i"] if cfg.get("g3i") else "")


class Timer:
    def __init__(self, pafc, torch, dt, reps=5, batch_form="auto"):
        self.pafc, self.torch, self.dt, self.reps = pafc, torch, dt, reps
        self.batch_form = batch_form
        self.tdt = torch.complex128 if dt == "c128" else torch.complex64

    def batch(self, n):
        torch = self.torch
        count = max(2, (1 << 24) // n)
        B = self.pafc.Batch([n] * count, [0] * count, 1, self.tdt, form=self.batch_form)
        h = torch.ones(n, dtype=self.tdt, device="cuda")
        B.set_filter(0, h)
        x = torch.ones(n * count, dtype=self.tdt, device="cuda")
        y = torch.empty_like(x)
        B.convolve(x, out=y)
        _, _, per = B.profile_levels(x, y, reps=self.reps)
        B.close()
        return float(np.median(per))

    def grid(self, dims, radix, variant="perm_free"):
        torch = self.torch
        P = self.pafc.Plan(dims, self.tdt, radix=None if radix is None else [radix] * len(dims),
                           variant=variant)
        h = torch.ones(dims, dtype=self.tdt, device="cuda")
        P.set_filter(h)
        x = torch.ones(dims, dtype=self.tdt, device="cuda")
        y = torch.empty_like(x)
        P.convolve(x, out=y)
        _, _, per = P.profile_passes(x, y, reps=self.reps)
        P.close()
        return float(np.median(per))


def candidates(pafc, dt, n, key, cfg):
    f = _factors(n)
    if key in ("g3", "g3i"):
        return [1, 2, 3] if 3 in f else []
    if key == "g5":
        return [1, 2] if 5 in f else []
    d = pafc.describe((n,), dt)
    rho = d["axes"][0]["rho"]
    elem = 16 if dt == "c128" else 8
    fits = lambda L: (L + L // 16 + 1) * elem <= 160 * 1024
    if key == "split":
        out, p = [0], 1
        for r in rho[:-1]:
            p *= r
            if p >= 128 and fits(p) and fits(n // p) and p < n:
                out.append(p)
        return out if len(out) > 1 else []
    pieces = d["axes"][0]["pieces"]
    split = cfg["split"] or (pieces[1]["L"] if len(pieces) == 2 else 0)
    if not split:
        return []
    if key == "W":
        return [w for w in (1, 2, 4, 8) if fits(split * w)]
    if key == "Wo":
        return [w for w in (8, 16, 32, 64, 128) if fits((n // split) * w)]
    return []


def read_table(path, raw=False):
    """(dtype, n) -> config of an existing table (empty if there is none);
    with ``raw`` the table's lines themselves, comments included."""
    out = {}
    if not path or not os.path.exists(path):
        return out
    for text in open(path):
        f = text.split("#")[0].split()
        if len(f) in (7, 8):
            cfg = dict(zip(FIELDS, map(int, f[2:])))
            cfg.setdefault("g3i", 0)
            out[(f[0], int(f[1]))] = text.rstrip("\n") if raw else cfg
    return out


def tune_one(pafc, timer, dt, n, measure, prev=None,
             keys=("g3", "g5", "split", "W", "Wo", "g3i")):
    cfg = {"split": 0, "W": 0, "Wo": 0, "g3": 0, "g5": 0, "g3i": 0}
    pafc.set_tuning(None)
    best = measure()
    log = [("default", best)]
    if prev and any(prev.values()):
        try:
            pafc.set_tuning(line(dt, n, prev))
            t = measure()
            log.append((line(dt, n, prev), t))
            if t < best:
                best, cfg = t, dict(prev)
        except Exception as e:  # the planner no longer accepts it
            log.append((line(dt, n, prev), "rejected: %s" % e))
    for key in keys:
        pafc.set_tuning(line(dt, n, cfg) if any(cfg.values()) else None)
        cands = candidates(pafc, dt, n, key, cfg)
        for v in cands:
            if v == cfg[key]:
                continue
            trial = dict(cfg, **{key: v})
            try:
                pafc.set_tuning(line(dt, n, trial))
                t = measure()
            except Exception as e:  # a candidate the planner rejects
                log.append((line(dt, n, trial), "rejected: %s" % e))
                continue
            log.append((line(dt, n, trial), t))
            if t < best * 0.98:
                best, cfg = t, trial
    pafc.set_tuning(None)
    return cfg, best, log


class TableLib:
    """tune_one's view of the library when one entry of a whole table is
    searched: set_tuning(line) installs the table with that entry replaced
    (None: without it)."""

    def __init__(self, pafc, lines, dt, n):
        self.pafc, self.lines, self.key = pafc, dict(lines), (dt, n)

    def text(self, entry):
        lines = dict(self.lines)
        lines.pop(self.key, None)
        if entry:
            lines[self.key] = entry
        return "\n".join(lines.values()) + "\n"

    def set_tuning(self, entry):
        self.pafc.set_tuning(self.text(entry))

    def describe(self, dims, dt):
        return self.pafc.describe(dims, dt)


class MixedBatch:
    """The benchmark's mixed batch (4096 problems over the 18 size classes)
    timed in one batched form as the benchmark times it: median of graph
    replays, HIP events."""

    def __init__(self, pafc, torch, dt, form, reps):
        from paper_2506_12718_amd import inputs
        self.pafc, self.torch, self.form, self.reps = pafc, torch, form, reps
        self.tdt = torch.complex128 if dt == "c128" else torch.complex64
        psizes, xs, filters = inputs.batched_problems()
        classes = sorted(filters)
        self.sizes = psizes
        self.fids = [classes.index(n) for n in psizes]
        self.nf = len(classes)
        self.x = torch.from_numpy(np.concatenate(xs)).to(self.tdt).cuda()
        self.y = torch.empty_like(self.x)
        self.h = {classes.index(n): torch.from_numpy(h).to(self.tdt).cuda()
                  for n, h in filters.items()}

    def measure(self):
        torch = self.torch
        B = self.pafc.Batch(self.sizes, self.fids, self.nf, self.tdt, form=self.form)
        for f, h in self.h.items():
            B.set_filter(f, h)
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        g = torch.cuda.CUDAGraph()
        with torch.cuda.stream(s):
            B.convolve(self.x, out=self.y, stream=s)
            torch.cuda.synchronize()
            with torch.cuda.graph(g, stream=s):
                B.convolve(self.x, out=self.y, stream=s)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(self.reps + 1)]
        ev[0].record()
        for k in range(self.reps):
            g.replay()
            ev[k + 1].record()
        torch.cuda.synchronize()
        del g
        B.close()
        return float(np.median([ev[k].elapsed_time(ev[k + 1]) for k in range(self.reps)]))


def tune_mixed(pafc, torch, dt, form, lines, reps, sizes):
    """Re-tune the batched size classes' entries against the whole mixed
    batch in `form`, largest classes first, each search starting from the
    table's entry; `lines` ((dtype, n) -> table line) is updated in place."""
    mixed = MixedBatch(pafc, torch, dt, form, reps)
    report = []
    one_d = ("g3", "g5", "split", "W", "Wo", "g3i")
    for n in sorted(sizes, reverse=True):
        lib = TableLib(pafc, lines, dt, n)
        prev = read_table_text(lines.get((dt, n), "")).get((dt, n))
        cfg, t, log = tune_one(lib, None, dt, n, mixed.measure, prev, one_d)
        if any(cfg.values()):
            lines[(dt, n)] = line(dt, n, cfg) + "   # %.4f ms per mixed batch (%s form)" % (t, form)
        else:
            lines.pop((dt, n), None)
        report.append({"dtype": dt, "n": n, "cfg": cfg, "batch_ms": round(t, 5),
                       "start_ms": round(log[0][1], 5) if isinstance(log[0][1], float) else None})
        print(json.dumps(report[-1]), flush=True)
    pafc.set_tuning("\n".join(lines.values()) + "\n")
    return report


def read_table_text(text):
    out = {}
    for t in text.splitlines():
        f = t.split("#")[0].split()
        if len(f) in (7, 8):
            cfg = dict(zip(FIELDS, map(int, f[2:])))
            cfg.setdefault("g3i", 0)
            out[(f[0], int(f[1]))] = cfg
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--dtypes", nargs="+", default=["c128", "c64"])
    ap.add_argument("--out", default=DEFAULT_TABLE)
    ap.add_argument("--reps", type=int, default=7)
    ap.add_argument("--prev", default=DEFAULT_TABLE,
                    help="existing table whose entries are tried as starting points ('' for none)")
    ap.add_argument("--batch-form", default="auto",
                    help="batched form the size classes are timed in (Batch form names)")
    ap.add_argument("--mixed", action="store_true",
                    help="re-tune the batched size classes against the whole mixed batch in "
                         "--batch-form, starting from --prev; other entries are kept")
    ap.add_argument("--sizes", nargs="*", type=int, default=None,
                    help="tune only these axis lengths; the other entries of --prev are kept")
    a = ap.parse_args(argv)
    prev = read_table(a.prev)
    prev_lines = read_table(a.prev, raw=True)
    os.environ["PAFC_NO_TUNING_TABLE"] = "1"
    import torch
    import paper_2506_12718_amd as pafc
    dev = torch.cuda.get_device_properties(0)
    lines = ["# pafc planner tuning table (python -m paper_2506_12718_amd.tune)",
             "# device: %s (%s)" % (dev.name, getattr(dev, "gcnArchName", "?")),
             "# format: dtype n split W Wo g3 g5 [g3i]   (0 = planner default)"]
    if a.mixed:
        table = {k: v.split("#")[0].rstrip() + ("   #" + v.split("#", 1)[1] if "#" in v else "")
                 for k, v in prev_lines.items()}
        sizes = a.sizes if a.sizes is not None else BATCH_SIZES
        for dt in a.dtypes:
            tune_mixed(pafc, torch, dt, a.batch_form, table, a.reps, sizes)
        body = sorted(table.items(), key=lambda kv: (kv[0][0] != "c128", kv[0][1]))
        os.makedirs(os.path.dirname(a.out), exist_ok=True)
        with open(a.out, "w") as f:
            f.write("\n".join(lines + [v for _, v in body]) + "\n")
        print("wrote", a.out, flush=True)
        return
    report = []
    for dt in a.dtypes:
        timer = Timer(pafc, torch, dt, reps=a.reps, batch_form=a.batch_form)
        # whole grids first; a batched size class with the same axis length
        # keeps the grid's entry (the table is keyed by axis length).  The
        # split field acts on 1-D plans only and the width candidates come
        # from the 1-D plan's pieces, so a grid of more than one axis
        # searches the register grouping alone.
        one_d = ("g3", "g5", "split", "W", "Wo", "g3i")
        jobs = [(dims[0], (lambda d=dims, r=radix: timer.grid(d, r)),
                 one_d if len(dims) == 1 else ("g3", "g5", "g3i")) for dims, radix in GRIDS]
        jobs += [(n, (lambda n=n: timer.batch(n)), one_d) for n in BATCH_SIZES
                 if n not in [d[0] for d, _ in GRIDS]]
        jobs += [(n, (lambda n=n: timer.grid((n,), None)), one_d) for n in INNER_1D]
        jobs += [(n, (lambda: timer.grid((PFA_N,), None, "prime_factor")), ("g3", "g5"))
                 for n in PFA_AXES]
        if a.sizes is not None:
            jobs = [j for j in jobs if j[0] in a.sizes]
            for (pdt, pn), pcfg in sorted(prev.items()):
                if pdt == dt and pn not in a.sizes and any(pcfg.values()):
                    lines.append(prev_lines[(pdt, pn)])
        for n, measure, keys in jobs:
            start = prev.get((dt, n))
            if start is not None and keys != one_d:
                start = dict(start, split=0, W=0, Wo=0)
            cfg, t, log = tune_one(pafc, timer, dt, n, measure, start, keys)
            default_t = log[0][1]
            print(json.dumps({"dtype": dt, "n": n, "cfg": cfg, "ms": round(t, 5),
                              "default_ms": round(default_t, 5),
                              "gain": round(default_t / t, 3)}), flush=True)
            report.append((dt, n, cfg))
            if any(cfg.values()):
                lines.append(line(dt, n, cfg) + "   # %.4f ms vs %.4f default" % (t, default_t))
    os.makedirs(os.path.dirname(a.out), exist_ok=True)
    with open(a.out, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("wrote", a.out, flush=True)


if __name__ == "__main__":
    main()
