"""Benchmark of the permutation-avoiding FFT convolution on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

Default workload: 3-D periodic convolution, 256 x 256 x 256 complex128,
radix 4 per axis, input iid N(0,1), filter = unit-sum periodic Gaussian of
width 4 (seeded synthetic data).  A step is one full convolution
y = x (*) h with the filter spectrum resident on the device and the input
already in HBM.  Prints ONE JSON line: conv/s, the roofline of the dominant
kernel (the axis-pass kernel, timed with HIP events on its own stream during
the timed region), the explicit-permutation comparison variant on the same
GPU, per-convolution latency percentiles, the error against the FP64 oracle,
and the oracle itself timed on the host cores.
"""
from __future__ import annotations

import argparse
import glob
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, 8 TB/s


def load_traffic(workload):
    """HBM bytes per launch of the dominant kernel from committed rocprofv3
    counter runs, if they were taken on the current kernel sources."""
    from paper_2506_12718_amd.profiling import kernel_source_hash
    path = os.path.join(ROOT, "profiles", "%s_traffic.json" % workload)
    if not os.path.exists(path):
        return None
    try:
        with open(path) as f:
            d = json.load(f)
        if d.get("kernel_source_hash") != kernel_source_hash():
            return None
        return d.get("hbm_bytes_per_launch")
    except Exception:
        return None


def pct(a, q):
    return float(np.percentile(np.asarray(a), q))


# ----------------------------------------------------------------- workloads

def wl_conv3d(dtype_name):
    from paper_2506_12718_amd import inputs
    x, h = inputs.conv3d_gaussian()
    return dict(name="conv3d_256_%s_r4" % dtype_name, x=x, h=h, radix=[4, 4, 4],
                domain="spatial", rhos=[[4] * 4] * 3,
                config={"workload": "3-D periodic convolution 256x256x256, radix 4 per axis, "
                                    "x iid N(0,1), wrapped Gaussian filter sigma=4",
                        "dims": [256, 256, 256], "radix": 4, "filter": "gaussian_sigma4"})


def wl_conv1d(dtype_name):
    from paper_2506_12718_amd import inputs
    x, h = inputs.conv1d_4096()
    return dict(name="conv1d_4096_%s_r4" % dtype_name, x=x, h=h, radix=[4], domain="spatial",
                rhos=[[4] * 6],
                config={"workload": "1-D circular convolution n=4096, radix 4, single instance",
                        "dims": [4096], "radix": 4})


def wl_conv2d(dtype_name):
    from paper_2506_12718_amd import inputs
    x, hh = inputs.spectral_filter_case(31, (2187, 2187))
    return dict(name="conv2d_2187_%s_r3" % dtype_name, x=x, h=hh, radix=[3, 3],
                domain="spectral_natural", rhos=[[3] * 7] * 2,
                config={"workload": "2-D convolution 2187x2187, radix 3, spectral filter",
                        "dims": [2187, 2187], "radix": 3})


def wl_conv1d5(dtype_name):
    from paper_2506_12718_amd import inputs
    x, hh = inputs.spectral_filter_case(32, (5 ** 9,))
    return dict(name="conv1d_5p9_%s_r5" % dtype_name, x=x, h=hh, radix=[5],
                domain="spectral_natural", rhos=[[5] * 9],
                config={"workload": "1-D convolution n=5^9=1953125, radix 5, spectral filter",
                        "dims": [5 ** 9], "radix": 5})


def wl_batched(dtype_name):
    from paper_2506_12718_amd import inputs
    psizes, xs, filters = inputs.batched_problems()
    classes = sorted(filters)
    return dict(name="batched_4096_%s" % dtype_name, sizes=psizes, xs=xs,
                fids=[classes.index(n) for n in psizes],
                filters={classes.index(n): h for n, h in filters.items()},
                config={"workload": "4096 independent 1-D convolutions, sizes iid uniform over "
                                    "{2^8..2^16, 3^6..3^10, 5^4..5^7}, one filter per size class",
                        "problems": len(psizes), "total_elements": int(sum(psizes))})


def wl_serving(dtype_name):
    return dict(name="serving_%s" % dtype_name,
                config={"workload": "served 2-D/3-D periodic convolutions, Poisson arrivals at 0.7x "
                                    "closed-loop capacity, Gaussian filters sigma~U[1,8] (8 per grid)",
                        "sides_2d": [64, 81, 128, 243, 256, 512, 729, 1024],
                        "sides_3d": [32, 64, 81, 128, 243, 256]})


def wl_aniso2d(dtype_name):
    from paper_2506_12718_amd import inputs
    shape = inputs.ANISO_2D
    x, h = inputs.anisotropic_case(41, shape)
    t = shape[0].bit_length() - 1
    return dict(name="aniso2d_2p%d_%s" % (t, dtype_name), x=x, h=h, radix=[4, 2],
                domain="spatial", rhos=[[4] * (t // 2), [2]],
                config={"workload": "anisotropic 2-D convolution 2^%dx2, radix 4 on the long "
                                    "axis, radix 2 on the short one" % t,
                        "dims": list(shape), "radix": [4, 2]})


def wl_aniso3d(dtype_name):
    from paper_2506_12718_amd import inputs
    shape = inputs.ANISO_3D
    x, h = inputs.anisotropic_case(42, shape)
    t = shape[0].bit_length() - 1
    return dict(name="aniso3d_2p%d_%s" % (t, dtype_name), x=x, h=h, radix=[4, 2, 2],
                domain="spatial", rhos=[[4] * (t // 2), [2], [2]],
                config={"workload": "anisotropic 3-D convolution 2^%dx2x2, radix 4 on the long "
                                    "axis, radix 2 on the short ones" % t,
                        "dims": list(shape), "radix": [4, 2, 2]})


def wl_poisson3d(dtype_name):
    from paper_2506_12718_amd import inputs
    rng = np.random.default_rng(43)
    f = inputs.complex_normal(rng, (256, 256, 256))
    return dict(name="poisson3d_256_%s_r4" % dtype_name, x=f, h=None, radix=[4, 4, 4],
                domain="symbol", symbol=("inv_laplacian_fd", ()), rhos=[[4] * 4] * 3,
                config={"workload": "periodic Poisson solve on 256x256x256 (inverse of the "
                                    "7-point Laplacian as a frequency symbol), radix 4 per axis, "
                                    "right-hand side iid N(0,1)",
                        "dims": [256, 256, 256], "radix": 4, "symbol": "inv_laplacian_fd"})


def wl_pfa1d(dtype_name):
    from paper_2506_12718_amd import inputs
    n = 2 ** 8 * 3 ** 5 * 5 ** 3
    x, h = inputs.anisotropic_case(44, (n,))
    return dict(name="pfa1d_7776000_%s" % dtype_name, x=x, h=h, radix=None, domain="spatial",
                rhos=None, variant="prime_factor",
                compare=["prime_factor_explicit", "perm_free"],
                config={"workload": "1-D convolution n = 2^8 3^5 5^3 = 7776000 by the prime-factor "
                                    "route (Chinese-remainder reindexing onto the 256x243x125 "
                                    "grid), x and h re/im iid U[-1,1]",
                        "dims": [n], "grid": [125, 243, 256]})


def wl_bluestein1d(dtype_name):
    from paper_2506_12718_amd import inputs
    n = 1000003  # prime
    x, h = inputs.anisotropic_case(45, (n,))
    return dict(name="bluestein1d_1000003_%s" % dtype_name, x=x, h=h, radix=None,
                domain="spatial", rhos=None, oracle="direct_sampled",
                compare=["explicit_perm", "perm_free_unfused"],
                config={"workload": "1-D convolution of prime length n = 1000003 by Bluestein's "
                                    "method (inner convolution of length 2025000 = 2^3 3^4 5^5), "
                                    "x and h re/im iid U[-1,1]",
                        "dims": [n], "inner_length": 2025000})


def wl_rader1d(dtype_name):
    from paper_2506_12718_amd import inputs
    n = 995329  # prime, n - 1 = 2^12 3^5
    x, h = inputs.anisotropic_case(47, (n,))
    return dict(name="rader1d_995329_%s" % dtype_name, x=x, h=h, radix=None,
                domain="spatial", rhos=None, oracle="direct_sampled",
                compare=["explicit_perm", "perm_free_unfused", "bluestein"],
                config={"workload": "1-D convolution of prime length n = 995329 by Rader's "
                                    "method (inner convolution of length n - 1 = 2^12 3^5), "
                                    "x and h re/im iid U[-1,1]",
                        "dims": [n], "inner_length": n - 1})


WORKLOADS = {"conv3d": wl_conv3d, "poisson3d": wl_poisson3d, "pfa1d": wl_pfa1d,
             "bluestein1d": wl_bluestein1d, "rader1d": wl_rader1d, "conv1d": wl_conv1d, "conv2d": wl_conv2d,
             "conv1d5": wl_conv1d5, "batched": wl_batched, "serving": wl_serving,
             "aniso2d": wl_aniso2d, "aniso3d": wl_aniso3d}


def bench_serving(pafc, torch, wl, tdtype, args):
    """Warm-up + calibration (closed loop, twice over the first 200 requests),
    then 2000 requests with Poisson arrivals at 0.7 x the calibrated capacity."""
    from paper_2506_12718_amd import inputs
    from paper_2506_12718_amd.serve import (GpuExecutor, Request, Server, latency_stats,
                                            run_closed_loop, run_open_loop)
    raw = inputs.serving_requests(seed=5, count=2200)
    pool = {}

    def make_input(req):
        key = (tuple(req.dims), req.meta["x_seed"] % 2)
        if key not in pool:
            x = inputs.serving_input({"dims": req.dims, "x_seed": key[1] + 1000 * req.dims[0]},
                                     dtype=np.complex64 if tdtype == torch.complex64 else np.complex128)
            pool[key] = torch.from_numpy(x).cuda()
            torch.cuda.synchronize()
        return pool[key]

    def reqs(lo, hi):
        return [Request(rid=r["id"], dims=r["dims"], fid=r["filter"], meta={"x_seed": r["x_seed"]})
                for r in raw[lo:hi]]

    slots = 4
    ex = GpuExecutor(dtype=tdtype, sigma_of=inputs.serving_sigma, slots=slots)
    budget = 64 << 30
    srv = Server(ex, budget_bytes=budget, slots=slots)
    print("bench: serving warm-up", file=sys.stderr, flush=True)
    for r in reqs(0, 200):
        make_input(r)
    run_closed_loop(srv, reqs(0, 200), make_input=make_input)
    srv.completed = []
    t0 = time.perf_counter()
    run_closed_loop(srv, reqs(0, 200), make_input=make_input)
    cap = 200 / (time.perf_counter() - t0)
    rate = 0.7 * cap
    srv.completed = []
    meas = reqs(200, 2200)
    for r in meas:
        make_input(r)
    print("bench: serving 2000 requests at %.1f/s (capacity %.1f/s)" % (rate, cap),
          file=sys.stderr, flush=True)
    keep = {r.rid for r in meas[::50]}
    done = run_open_loop(srv, meas, rate, make_input=make_input)
    torch.cuda.synchronize()
    st = latency_stats(done)
    kept = {r.rid: (r, r.out.cpu().numpy()) for r in done if r.rid in keep}
    for r in done:
        r.out = None
    elems = sum(int(np.prod(r.dims)) for r in done)
    elem = 8 if tdtype == torch.complex64 else 16
    out = {
        "metric": "convolutions/s + HBM GB/s (% roofline), perm-free vs explicit-perm; p99 latency",
        "value": round(st["throughput_per_s"], 2), "unit": "conv/s", "n_gpus": 1,
        "steps": len(done), "warmup": 200, "ms_per_step": round(1e3 / st["throughput_per_s"], 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if tdtype == torch.complex64 else "f64", "data": "synthetic",
        "config": dict(wl["config"], slots=slots, hbm_budget_bytes=budget),
        "latency_ms": {"p50": round(st["p50_ms"], 4), "p99": round(st["p99_ms"], 4),
                       "mean": round(st["mean_ms"], 4)},
        "offered_rate_per_s": round(rate, 2), "closed_loop_capacity_per_s": round(cap, 2),
        "max_inflight": srv.max_inflight,
        "cache": {"plans_prepared": ex.prepared, "hits": srv.cache.hits,
                  "evictions": srv.cache.evictions, "bytes": srv.cache.bytes},
        "elements_served": elems,
        "roofline": None,
    }
    if not args.no_cpu:
        import oracle
        errs = []
        t0 = time.perf_counter()
        for rid, (r, y) in sorted(kept.items()):
            x = make_input(r).cpu().numpy().astype(np.complex128)
            h = inputs.wrapped_gaussian(r.dims, inputs.serving_sigma(r.dims, r.fid))
            if tdtype == torch.complex64:
                h = h.astype(np.complex64)
            ref = oracle.conv_fft(x, h.astype(np.complex128))
            errs.append(float(np.linalg.norm(y - ref) / np.linalg.norm(ref)))
        t_cpu = time.perf_counter() - t0
        out["rel_l2_vs_fp64_oracle_max_sampled"] = max(errs)
        out["oracle_checked_requests"] = len(errs)
        out["cpu_baseline"] = {"value": round(len(errs) / t_cpu, 3), "unit": "conv/s",
                               "cores": oracle.num_threads(), "kind": "oracle",
                               "sample": "1 in 50 of the measured requests (%d), FP64 explicit "
                                         "route; %.2f s" % (len(errs), t_cpu)}
    print(json.dumps(out), flush=True)


def bench_batched(pafc, torch, wl, tdtype, args):
    B = pafc.Batch(wl["sizes"], wl["fids"], len(wl["filters"]), tdtype)
    for f, h in wl["filters"].items():
        B.set_filter(f, torch.from_numpy(h).to(tdtype).cuda())
    x = torch.from_numpy(np.concatenate(wl["xs"])).to(tdtype).cuda()
    y = torch.empty_like(x)
    for _ in range(args.warmup):
        B.convolve(x, out=y)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ms_lv, by_lv, ms_rep = B.profile_levels(x, y, reps=args.steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    nprob = len(wl["sizes"])
    value = nprob * args.steps / wall
    dom = max(range(len(ms_lv)), key=lambda i: ms_lv[i])
    ach = by_lv[dom] / (ms_lv[dom] * 1e-3) / 1e9
    alg = sum(by_lv)
    out = {
        "metric": "convolutions/s + HBM GB/s (% roofline), perm-free vs explicit-perm; p99 latency",
        "value": round(value, 1), "unit": "conv/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(wall * 1e3 / args.steps, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if tdtype == torch.complex128 else "f32", "data": "synthetic",
        "config": dict(wl["config"], variant="perm_free", levels=len(ms_lv)),
        "hbm_gbps_alg": round(alg / (sum(ms_lv) * 1e-3) / 1e9, 1),
        "alg_bytes_per_batch": alg,
        "latency_ms": {"p50": round(pct(ms_rep, 50), 5), "p99": round(pct(ms_rep, 99), 5)},
        "ms_per_level": [round(v, 5) for v in ms_lv],
        "roofline": {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4),
                     "traffic": load_traffic(wl["name"]),
                     "kernel": "batch_kernel level %d" % dom, "alg_bytes_per_launch": by_lv[dom],
                     "avg_launch_ms": round(ms_lv[dom], 5)},
    }
    yh = y.cpu().numpy().astype(np.complex128)
    B.close()
    if not args.no_cpu:
        import oracle
        offs = np.concatenate([[0], np.cumsum(wl["sizes"])])
        # bounded sample: the first 512 problems in order (about 1/8 of the batch)
        sample = list(range(512))
        errs = []
        t0 = time.perf_counter()
        for i in sample:
            xi = wl["xs"][i]
            hi = wl["filters"][wl["fids"][i]]
            if tdtype == torch.complex64:
                xi = xi.astype(np.complex64).astype(np.complex128)
                hi = hi.astype(np.complex64).astype(np.complex128)
            ref = oracle.conv_fft(xi, hi)
            got = yh[offs[i]:offs[i + 1]]
            errs.append(float(np.linalg.norm(got - ref) / np.linalg.norm(ref)))
        t_cpu = time.perf_counter() - t0
        out["rel_l2_vs_fp64_oracle_max_sampled"] = max(errs)
        out["cpu_baseline"] = {
            "value": round(len(sample) / t_cpu, 3), "unit": "conv/s",
            "cores": oracle.num_threads(), "kind": "oracle",
            "sample": "the first %d of the 4096 problems (%d elements), FP64 explicit route; "
                      "%.2f s" % (len(sample), int(sum(wl["sizes"][:len(sample)])), t_cpu)}
    print(json.dumps(out), flush=True)


def conv_bytes(desc, filter_per_call):
    """Algorithmic HBM bytes of one convolution; with the filter transformed
    in the call, its forward passes (and, for the explicit variant, its
    reversal) count too."""
    b = desc["hbm_bytes_conv"]
    if filter_per_call:
        b += desc["hbm_bytes_forward"]
        if desc.get("variant") == 1:  # explicit: the filter's reversal pass
            b += 2 * desc["N"] * (16 if desc["dtype"] == "c128" else 8)
    return b


def measure(pafc, torch, wl, tdtype, variant, steps, warmup, filter_per_call=False):
    """Plan, set the filter, warm up (with a HIP event around every launch,
    which names the dominant launch), then time `steps` convolutions with
    HIP events at the start of each and around the dominant launch only
    (pafc_profile_launch); the per-launch breakdown of all launches comes
    from a further, untimed run.  With `filter_per_call` the timed
    calls are pafc_convolve_with_filter (the filter transformed in every
    call, wall clock over the stream), and the per-launch events come from a
    second run of the convolution passes alone.  Variant "bluestein" is the
    permutation-avoiding variant with a prime length planned by Bluestein's
    method (PAFC_BLUESTEIN=1) where Rader's would apply.  Returns a dict of
    results."""
    force_bluestein = variant == "bluestein"
    if force_bluestein:
        os.environ["PAFC_BLUESTEIN"] = "1"
        variant = "perm_free"
    plan = pafc.Plan(wl["x"].shape, tdtype, radix=wl["radix"], variant=variant)
    xd = torch.from_numpy(wl["x"]).to(tdtype).cuda()
    yd = torch.empty_like(xd)
    if wl["domain"] == "symbol":
        plan.set_symbol(wl["symbol"][0], *wl["symbol"][1])
        hd = None
    else:
        hd = torch.from_numpy(wl["h"]).to(tdtype).cuda()
        plan.set_filter(hd, domain=wl["domain"])
    if filter_per_call:
        for _ in range(warmup):
            plan.convolve_with_filter(xd, hd, out=yd)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        starts = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
        starts[0].record()
        for k in range(steps):
            plan.convolve_with_filter(xd, hd, out=yd)
            starts[k + 1].record()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        fpc_rep = [starts[k].elapsed_time(starts[k + 1]) for k in range(steps)]
        ms_pass, bytes_pass, _ = plan.profile_passes(xd, yd, reps=max(5, steps // 2))
        ms_rep = fpc_rep
        dom = max(range(len(ms_pass)), key=lambda i: ms_pass[i])
        dom_ms = ms_pass[dom]
        plan.convolve_with_filter(xd, hd, out=yd)
    else:
        # warm-up: `warmup` convolutions with an event around every launch,
        # which names the dominant launch (the most expensive one)
        ms_pass, _, _ = plan.profile_passes(xd, yd, reps=max(1, warmup))
        dom = max(range(len(ms_pass)), key=lambda i: ms_pass[i])
        torch.cuda.synchronize()
        # timed region: `steps` convolutions, events at the start of every
        # one and around the dominant launch only
        t0 = time.perf_counter()
        dom_ms, ms_rep = plan.profile_launch(xd, yd, dom, reps=steps)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        # untimed: the per-launch breakdown of every launch
        ms_pass, bytes_pass, _ = plan.profile_passes(xd, yd, reps=max(5, steps // 2))
    del hd
    desc = pafc.describe(wl["x"].shape, "c128" if tdtype == torch.complex128 else "c64",
                         wl["radix"], variant)
    if force_bluestein:
        del os.environ["PAFC_BLUESTEIN"]
    y = yd.cpu().numpy()
    plan.close()
    del xd, yd
    torch.cuda.empty_cache()
    return dict(wall=wall, ms_pass=ms_pass, bytes_pass=bytes_pass, ms_rep=ms_rep, desc=desc, y=y,
                labels=desc["conv_passes"], dom=dom, dom_ms=dom_ms)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="conv3d", choices=sorted(WORKLOADS))
    ap.add_argument("--dtype", default="c128", choices=["c128", "c64"])
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle timing and error check")
    ap.add_argument("--no-compare", action="store_true", help="skip the comparison variants")
    ap.add_argument("--filter-per-call", action="store_true",
                    help="transform the filter inside every timed call (three transforms per "
                         "convolution, as the paper times it)")
    ap.add_argument("--calibrate", action="store_true",
                    help="run only the plain streaming copy of 256 MiB (counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(each convolution runs on a single MI355X); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2506_12718_amd as pafc
    pafc.lib()
    torch.cuda.set_device(0)
    if args.calibrate:
        nbytes = 256 << 20
        a = torch.zeros(nbytes // 16, dtype=torch.complex128, device="cuda")
        b = torch.empty_like(a)
        pafc.stream_copy(a, b)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(10):
            pafc.stream_copy(a, b)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / 10
        print(json.dumps({"calibration_copy_bytes": nbytes, "ms": dt * 1e3,
                          "GBps_read_plus_write": 2 * nbytes / dt / 1e9}))
        return
    tdtype = torch.complex128 if args.dtype == "c128" else torch.complex64
    wl = WORKLOADS[args.workload](args.dtype)
    if args.workload == "batched":
        print("bench: %s steps=%d warmup=%d" % (wl["name"], args.steps, args.warmup),
              file=sys.stderr, flush=True)
        bench_batched(pafc, torch, wl, tdtype, args)
        return
    if args.workload == "serving":
        bench_serving(pafc, torch, wl, tdtype, args)
        return
    N = wl["x"].size
    elem = 16 if args.dtype == "c128" else 8

    print("bench: %s steps=%d warmup=%d" % (wl["name"], args.steps, args.warmup),
          file=sys.stderr, flush=True)
    fpc = args.filter_per_call
    if fpc and wl["domain"] != "spatial":
        print("--filter-per-call needs a workload with a spatial filter", file=sys.stderr)
        sys.exit(2)
    main_variant = wl.get("variant", "perm_free")
    main_r = measure(pafc, torch, wl, tdtype, main_variant, args.steps, args.warmup, fpc)
    total_s = sum(main_r["ms_rep"]) / 1e3
    value = args.steps / main_r["wall"]
    ms_step = main_r["wall"] * 1e3 / args.steps

    # dominant kernel: the single most expensive launch of a convolution (for
    # multi-pass plans the fused middle pass, which also reads the spectrum),
    # its mean duration from the events of the timed region
    dom = main_r["dom"]
    dom_ms = main_r["dom_ms"]
    dom_bytes = main_r["bytes_pass"][dom]
    achieved = dom_bytes / (dom_ms * 1e-3) / 1e9
    traffic = load_traffic(wl["name"])
    kern = [i for i, l in enumerate(main_r["labels"]) if not l.startswith(("mul", "permute"))]
    all_ms = sum(main_r["ms_pass"][i] for i in kern)
    all_bytes = sum(main_r["bytes_pass"][i] for i in kern)
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "kernel": main_r["labels"][dom], "alg_bytes_per_launch": dom_bytes,
            "avg_launch_ms": round(dom_ms, 5),
            "all_passes": {"source": "per-launch breakdown run after the timed region",
                           "launches": len(kern), "alg_bytes": all_bytes,
                           "ms": round(all_ms, 5),
                           "achieved": round(all_bytes / (all_ms * 1e-3) / 1e9, 1)}}
    alg_bytes = conv_bytes(main_r["desc"], fpc)
    out = {
        "metric": "convolutions/s + HBM GB/s (% roofline), perm-free vs explicit-perm; p99 latency",
        "value": round(value, 3),
        "unit": "conv/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.dtype == "c128" else "f32",
        "data": "synthetic",
        "config": dict(wl["config"], variant=main_variant, dtype=args.dtype,
                       passes=main_r["labels"], filter_per_call=fpc),
        "hbm_gbps_alg": round(alg_bytes * value / 1e9, 1),
        "hbm_frac_alg": round(alg_bytes * value / 1e9 / HBM_PEAK_GBS, 4),
        "alg_bytes_per_conv": alg_bytes,
        "latency_ms": {"p50": round(pct(main_r["ms_rep"], 50), 5),
                       "p99": round(pct(main_r["ms_rep"], 99), 5),
                       "mean": round(total_s * 1e3 / args.steps, 5)},
        "ms_per_pass": [round(v, 5) for v in main_r["ms_pass"]],
        "roofline": roof,
    }
    if not args.no_compare:
        comp = {}
        compare = wl.get("compare", ["explicit_perm", "perm_free_unfused"])
        for variant in compare:
            print("bench: comparison variant %s" % variant, file=sys.stderr, flush=True)
            r = measure(pafc, torch, wl, tdtype, variant, max(5, args.steps // 2), 2, fpc)
            v = len(r["ms_rep"]) / r["wall"]
            comp[variant] = {
                "conv_per_s": round(v, 3),
                "ms_per_conv": round(1e3 / v, 5),
                "p99_ms": round(pct(r["ms_rep"], 99), 5),
                "alg_bytes_per_conv": conv_bytes(r["desc"], fpc),
                "hbm_gbps_alg": round(conv_bytes(r["desc"], fpc) * v / 1e9, 1),
                "ms_per_pass": [round(t, 5) for t in r["ms_pass"]],
                "passes": r["labels"],
                "max_abs_diff_vs_perm_free": float(np.abs(r["y"] - main_r["y"]).max()),
            }
        comp["speedup_perm_free_over_explicit"] = round(
            value / comp[compare[0]]["conv_per_s"], 3)
        out["compare"] = comp
    if not args.no_cpu:
        import oracle
        print("bench: oracle on host cores", file=sys.stderr, flush=True)
        x = wl["x"]
        h = wl["h"]
        if args.dtype == "c64":
            x = x.astype(np.complex64).astype(np.complex128)
            if h is not None:
                h = h.astype(np.complex64).astype(np.complex128)
        t0 = time.perf_counter()
        if wl.get("oracle") == "direct_sampled":
            # the oracle's FFT has no route for a prime length: the direct
            # sum at a bounded sample of outputs, scaled to whole convolutions
            idx = np.random.default_rng(46).integers(0, N, 81920)
            ref = oracle.conv_direct_at(x, h, idx)
            t_cpu = time.perf_counter() - t0
            got = main_r["y"].reshape(-1)[idx]
            out["rel_l2_vs_fp64_oracle_sampled"] = float(
                np.linalg.norm(got - ref) / np.linalg.norm(ref))
            out["cpu_baseline"] = {
                "value": round(idx.size / N / t_cpu, 8), "unit": "conv/s",
                "cores": oracle.num_threads(), "kind": "oracle",
                "sample": "%d of the %d outputs by the direct sum (long double, OpenMP over "
                          "outputs), scaled to one convolution; %.2f s" % (idx.size, N, t_cpu)}
            print(json.dumps(out), flush=True)
            return
        # whole convolutions of the same workload, repeated until about 10 s
        # of host time have passed
        runs = 0
        while True:
            if wl["domain"] == "spatial":
                ref = oracle.conv_fft(x, h, wl["rhos"])
            elif wl["domain"] == "symbol":
                from oracle import symbols
                kind, params = wl["symbol"]
                sym = getattr(symbols, kind)(x.shape, *params)
                ref = symbols.apply(x, sym)
            else:
                ref = oracle.fft(h * oracle.fft(x, wl["rhos"]), wl["rhos"], inverse=True)
            runs += 1
            t_cpu = time.perf_counter() - t0
            if t_cpu >= 10.0 or runs >= 10000:
                break
        err = float(np.linalg.norm(main_r["y"] - ref) / np.linalg.norm(ref))
        out["rel_l2_vs_fp64_oracle"] = err
        out["cpu_baseline"] = {
            "value": round(runs / t_cpu, 5), "unit": "conv/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": "%d full convolution(s) of the same workload (standard FFT route with "
                      "explicit index reversal, FP64, OpenMP over pencils); %.2f s" % (runs, t_cpu)}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
