"""Benchmark of the permutation-avoiding FFT convolution on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

Default (``--workload all``): the headline workload -- 3-D periodic
convolution, 256 x 256 x 256 complex128, radix 4 per axis, input iid N(0,1),
filter = unit-sum periodic Gaussian of width 4 (seeded synthetic data) -- and,
in the same JSON line under ``configs``, every other workload of the
benchmark set measured in the same run:

* the single 4096-point 1-D convolution, radix-2 and radix-4 plans;
* 256^3 in complex64;
* 2187 x 2187 radix 3 with a spectral filter;
* n = 5^9 radix 5, complex128 and complex64;
* 4096 independent 1-D convolutions of mixed sizes, one hipGraph replay per
  batch, complex128 and complex64, beside the same problems run one plan at
  a time;
* served 2-D/3-D requests with Poisson arrivals (p50/p99 latency), beside the
  same requests served one at a time.

A step is one full convolution y = x (*) h with the filter spectrum resident
on the device and the input already in HBM.  For each workload: conv/s, the
algorithmic HBM bytes of one convolution and their rate against 8 TB/s, the
dominant launch timed with HIP events, the explicit-permutation variant of
the same plan, the error against the FP64 oracle (rel-L2 and the largest
entry error over the RMS of the reference), and the oracle itself timed on
the host cores (all of them, and one thread).
"""
from __future__ import annotations

import argparse
import json
import os
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0     # MI355X HBM3E, 8 TB/s
LDS_BYTES = 160 * 1024    # LDS of one compute unit
METRIC = "convolutions/s + HBM GB/s (% roofline), perm-free vs explicit-perm; p99 latency"


def load_traffic(workload, launch=None, whole=False):
    """HBM bytes per launch of the dominant kernel from committed rocprofv3
    counter runs, if they were taken on the current kernel sources: the
    kernel's own summary (<workload>_traffic.json), else its launch in the
    per-convolution breakdown (<workload>_conv_traffic.json, launch index
    `launch` of one convolution), or with `whole` that breakdown's total over
    one convolution (one batch)."""
    from paper_2506_12718_amd.profiling import kernel_source_hash
    try:
        h = kernel_source_hash()
        if whole:
            path = os.path.join(ROOT, "profiles", "%s_conv_traffic.json" % workload)
            with open(path) as f:
                d = json.load(f)
            return d["hbm_bytes_per_conv"] if d.get("kernel_source_hash") == h else None
        path = os.path.join(ROOT, "profiles", "%s_traffic.json" % workload)
        if os.path.exists(path):
            with open(path) as f:
                d = json.load(f)
            if d.get("kernel_source_hash") == h:
                return d.get("hbm_bytes_per_launch")
        path = os.path.join(ROOT, "profiles", "%s_conv_traffic.json" % workload)
        if launch is None or not os.path.exists(path):
            return None
        with open(path) as f:
            d = json.load(f)
        if d.get("kernel_source_hash") != h or launch >= len(d["launches"]):
            return None
        e = d["launches"][launch]
        return e["fetch_bytes"] + e["write_bytes"]
    except Exception:
        return None


def pct(a, q):
    return float(np.percentile(np.asarray(a), q))


def minimal_passes(dims, elem):
    """HBM passes of the minimal pass structure: a 1-D transform whose array
    fits one compute unit's LDS runs in 1 pass; other 1-D lengths and 2-D
    grids in 3 (forward outer, fused middle, inverse outer); 3-D grids in 5."""
    n = int(np.prod(dims))
    if len(dims) == 1:
        return 1 if n * elem <= LDS_BYTES else 3
    return 3 if len(dims) == 2 else 5


def alg_bytes(dims, elem):
    """Algorithmic HBM bytes of one convolution: one read and one write of
    the array per pass of the minimal pass structure, plus one read of the
    filter spectrum (3, 7 or 11 N elem)."""
    n = int(np.prod(dims))
    return (2 * minimal_passes(dims, elem) + 1) * n * elem


def errors(got, ref):
    """rel-L2 error and the largest entry error over the RMS of the reference."""
    a = np.asarray(got, dtype=np.complex128).ravel()
    b = np.asarray(ref, dtype=np.complex128).ravel()
    nb = float(np.linalg.norm(b))
    d = np.abs(a - b)
    return float(np.linalg.norm(a - b)) / nb, float(d.max()) / (nb / np.sqrt(b.size))


def roofline_obj(nbytes, ms, **extra):
    ach = nbytes / (ms * 1e-3) / 1e9
    d = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
         "frac": round(ach / HBM_PEAK_GBS, 4)}
    d.update(extra)
    return d


# ----------------------------------------------------------------- workloads

def wl_conv3d(dtype_name):
    from paper_2506_12718_amd import inputs
    x, h = inputs.conv3d_gaussian()
    return dict(name="conv3d_256_%s_r4" % dtype_name, x=x, h=h, radix=[4, 4, 4],
                domain="spatial", rhos=[[4] * 4] * 3,
                config={"workload": "3-D periodic convolution 256x256x256, radix 4 per axis, "
                                    "x iid N(0,1), wrapped Gaussian filter sigma=4",
                        "dims": [256, 256, 256], "radix": 4, "filter": "gaussian_sigma4"})


def wl_conv1d(dtype_name, radix=4):
    from paper_2506_12718_amd import inputs
    x, h = inputs.conv1d_4096()
    t = 12 if radix == 2 else 6
    return dict(name="conv1d_4096_%s_r%d" % (dtype_name, radix), x=x, h=h, radix=[radix],
                domain="spatial", rhos=[[radix] * t], oracle="direct",
                config={"workload": "1-D circular convolution n=4096, radix %d, single instance"
                                    % radix, "dims": [4096], "radix": radix})


def wl_conv1d_r2(dtype_name):
    return wl_conv1d(dtype_name, radix=2)


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
             "bluestein1d": wl_bluestein1d, "rader1d": wl_rader1d, "conv1d": wl_conv1d,
             "conv1d_r2": wl_conv1d_r2, "conv2d": wl_conv2d,
             "conv1d5": wl_conv1d5, "batched": wl_batched, "serving": wl_serving,
             "aniso2d": wl_aniso2d, "aniso3d": wl_aniso3d}


# ------------------------------------------------------------- oracle timing

def oracle_reference(wl, tdtype_is_c64):
    """The FP64 oracle's result for a plain workload (inputs rounded to the
    plan's precision first), and the function that recomputes it."""
    import oracle
    x, h = wl["x"], wl["h"]
    if tdtype_is_c64:
        x = x.astype(np.complex64).astype(np.complex128)
        if h is not None:
            h = h.astype(np.complex64).astype(np.complex128)
    if wl.get("oracle") == "direct":
        def run():
            return oracle.conv_direct(x, h)
    elif wl["domain"] == "spatial":
        def run():
            return oracle.conv_fft(x, h, wl["rhos"])
    elif wl["domain"] == "symbol":
        from oracle import symbols
        kind, params = wl["symbol"]

        def run():
            return symbols.apply(x, getattr(symbols, kind)(x.shape, *params))
    else:
        def run():
            return oracle.fft(h * oracle.fft(x, wl["rhos"]), wl["rhos"], inverse=True)
    return run


def time_oracle(run, min_s):
    """Run the oracle until min_s seconds have passed (at least once)."""
    runs, t0 = 0, time.perf_counter()
    ref = None
    while True:
        ref = run()
        runs += 1
        t = time.perf_counter() - t0
        if t >= min_s or runs >= 10000:
            return ref, runs, t


def oracle_samples(min_s):
    """The oracle's bounded samples of every workload of the default run:
    name -> (prepare, text); prepare() makes the inputs and returns run(),
    which does the timed oracle work and returns (convolutions, seconds)."""
    import oracle
    from paper_2506_12718_amd import inputs
    out = {}

    def timed(run):
        t0 = time.perf_counter()
        k = time_oracle(run, min_s)[1]
        return k, time.perf_counter() - t0

    for name, fn in (("conv1d_4096_r2", wl_conv1d_r2), ("conv1d_4096_r4", wl_conv1d),
                     ("conv3d_256", wl_conv3d), ("conv2d_2187_r3", wl_conv2d),
                     ("conv1d_5p9_r5", wl_conv1d5)):
        def prep(fn=fn):
            run = oracle_reference(dict(fn("c128"), oracle=None), False)  # the FFT route
            return lambda: timed(run)
        out[name] = (prep, "whole convolutions, standard FFT route with explicit index "
                           "reversal, FP64")

    def prep_direct():
        wl = wl_conv1d("c128")
        return lambda: timed(lambda: oracle.conv_direct(wl["x"], wl["h"]))
    out["conv1d_4096_direct"] = (prep_direct, "whole convolutions by the direct O(n^2) sum "
                                              "in long double")

    def prep_batched():
        psizes, xs, filters = inputs.batched_problems()

        def run():
            k, t = 0, 0.0
            while t < min_s and k < len(psizes):
                t0 = time.perf_counter()
                oracle.conv_fft(xs[k], filters[psizes[k]])
                t += time.perf_counter() - t0
                k += 1
            return k, t
        return run
    out["batched_4096"] = (prep_batched, "the first problems of the 4096 in order, standard "
                                         "FFT route, FP64")

    def prep_served():
        raw = inputs.serving_requests(seed=5, count=2200)[200:]

        def run():
            k, t = 0, 0.0
            while t < min_s and k < len(raw):
                r = raw[k]
                x = inputs.serving_input(r).astype(np.complex128)
                h = inputs.wrapped_gaussian(r["dims"],
                                            inputs.serving_sigma(r["dims"], r["filter"]))
                t0 = time.perf_counter()
                oracle.conv_fft(x, h)
                t += time.perf_counter() - t0
                k += 1
            return k, t
        return run
    out["serving"] = (prep_served, "the first measured requests in order, standard FFT "
                                   "route, FP64")
    return out


def oracle_worker(min_s):
    """Time every sample with the threads this process was started with and
    print one JSON line (the bench runs this at one thread, in a process of
    its own, while the GPU is measured)."""
    import oracle
    res = {}
    for name, (prep, text) in oracle_samples(min_s).items():
        k, t = prep()()
        res[name] = {"value": round(k / t, 6), "unit": "conv/s",
                     "cores": oracle.num_threads(), "sample": "%d %s; %.2f s" % (k, text, t)}
    print(json.dumps(res), flush=True)


def start_one_thread_oracle(min_s):
    env = dict(os.environ, OMP_NUM_THREADS="1")
    return subprocess.Popen([sys.executable, os.path.abspath(__file__), "--oracle-worker",
                             "--oracle-min-s", str(min_s)], env=env, stdout=subprocess.PIPE,
                            stderr=subprocess.DEVNULL, text=True)


def collect_one_thread_oracle(proc):
    try:
        out, _ = proc.communicate(timeout=300)
        return json.loads(out.strip().splitlines()[-1])
    except Exception as e:  # reported, never fatal for the GPU figures
        proc.kill()
        return {"error": str(e)}


# ------------------------------------------------------------ plain workloads

def measure(pafc, torch, wl, tdtype, variant, steps, warmup, filter_per_call=False):
    """Plan, set the filter, warm up (with a HIP event around every launch,
    which names the dominant launch), then time `steps` convolutions with
    HIP events around the dominant launch only (pafc_profile_launch); the
    latency of each convolution and the per-launch breakdown of all
    launches come from further, untimed runs.  With `filter_per_call` the timed
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
        # timed region: `steps` convolutions with events around the dominant
        # launch only (a pipelined launch carries them itself, so no marker
        # packet enters the stream)
        t0 = time.perf_counter()
        dom_ms, _ = plan.profile_launch(xd, yd, dom, reps=steps, per_rep=False)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        # untimed: latency of every convolution (an event at the start of
        # each), then the per-launch breakdown of every launch
        _, ms_rep = plan.profile_launch(xd, yd, dom, reps=steps)
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


def conv_bytes(desc, filter_per_call):
    """HBM bytes the plan moves in one convolution; with the filter
    transformed in the call, its forward passes (and, for the explicit
    variant, its reversal) count too."""
    b = desc["hbm_bytes_conv"]
    if filter_per_call:
        b += desc["hbm_bytes_forward"]
        if desc.get("variant") == 1:  # explicit: the filter's reversal pass
            b += 2 * desc["N"] * (16 if desc["dtype"] == "c128" else 8)
    return b


def bench_plain(pafc, torch, wl, tdtype, args, cpu_min_s=10.0, steps=None):
    """One plain workload: the JSON object of its measurement."""
    steps = steps or args.steps
    dname = "c128" if tdtype == torch.complex128 else "c64"
    elem = 16 if dname == "c128" else 8
    N = wl["x"].size
    print("bench: %s steps=%d warmup=%d" % (wl["name"], steps, args.warmup),
          file=sys.stderr, flush=True)
    fpc = args.filter_per_call
    main_variant = wl.get("variant", "perm_free")
    main_r = measure(pafc, torch, wl, tdtype, main_variant, steps, args.warmup, fpc)
    total_s = sum(main_r["ms_rep"]) / 1e3
    value = steps / main_r["wall"]
    ms_step = main_r["wall"] * 1e3 / steps

    # dominant kernel: the single most expensive launch of a convolution (for
    # multi-pass plans the fused middle pass, which also reads the spectrum),
    # its mean duration from the events of the timed region
    dom = main_r["dom"]
    dom_ms = main_r["dom_ms"]
    dom_bytes = main_r["bytes_pass"][dom]
    kern = [i for i, l in enumerate(main_r["labels"]) if not l.startswith(("mul", "permute"))]
    all_ms = sum(main_r["ms_pass"][i] for i in kern)
    all_bytes = sum(main_r["bytes_pass"][i] for i in kern)
    # (a plan of one launch is timed by one event pair over the whole timed
    # sequence: its mean launch time includes the gaps between launches)
    timing = ("one event pair over the timed sequence, span / steps"
              if len(main_r["labels"]) == 1 and not fpc and steps > 1
              else "an event pair around the dominant launch of every timed convolution")
    roof = roofline_obj(dom_bytes, dom_ms, traffic=load_traffic(wl["name"], dom),
                        kernel=main_r["labels"][dom], alg_bytes_per_launch=dom_bytes,
                        avg_launch_ms=round(dom_ms, 5), launch_timing=timing,
                        all_passes={"source": "per-launch breakdown run after the timed region",
                                    "launches": len(kern), "alg_bytes": all_bytes,
                                    "ms": round(all_ms, 5),
                                    "achieved": round(all_bytes / (all_ms * 1e-3) / 1e9, 1)})
    plan_bytes = conv_bytes(main_r["desc"], fpc)
    minimal = alg_bytes(wl["x"].shape, elem) if wl.get("variant") is None else plan_bytes
    if fpc:
        minimal = plan_bytes
    out = {
        "metric": METRIC, "value": round(value, 3), "unit": "conv/s", "n_gpus": 1,
        "steps": steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if dname == "c128" else "f32", "data": "synthetic",
        "config": dict(wl["config"], variant=main_variant, dtype=dname,
                       passes=main_r["labels"], filter_per_call=fpc),
        "alg_bytes_per_conv": minimal,
        "hbm_gbps_alg": round(minimal * value / 1e9, 1),
        "hbm_frac_alg": round(minimal * value / 1e9 / HBM_PEAK_GBS, 4),
        "plan_bytes_per_conv": plan_bytes,
        "latency_ms": {"p50": round(pct(main_r["ms_rep"], 50), 5),
                       "p99": round(pct(main_r["ms_rep"], 99), 5),
                       "mean": round(total_s * 1e3 / steps, 5)},
        "ms_per_pass": [round(v, 5) for v in main_r["ms_pass"]],
        "roofline": roof,
    }
    if not args.no_compare:
        comp = {}
        compare = wl.get("compare", ["explicit_perm", "perm_free_unfused"])
        for variant in compare:
            print("bench: comparison variant %s" % variant, file=sys.stderr, flush=True)
            r = measure(pafc, torch, wl, tdtype, variant, max(5, steps // 2), 2, fpc)
            v = len(r["ms_rep"]) / r["wall"]
            comp[variant] = {
                "conv_per_s": round(v, 3),
                "ms_per_conv": round(1e3 / v, 5),
                "p99_ms": round(pct(r["ms_rep"], 99), 5),
                "plan_bytes_per_conv": conv_bytes(r["desc"], fpc),
                "hbm_gbps_plan_bytes": round(conv_bytes(r["desc"], fpc) * v / 1e9, 1),
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
        x, h = wl["x"], wl["h"]
        if dname == "c64":
            x = x.astype(np.complex64).astype(np.complex128)
            if h is not None:
                h = h.astype(np.complex64).astype(np.complex128)
        if wl.get("oracle") == "direct_sampled":
            # the oracle's FFT has no route for a prime length: the direct
            # sum at a bounded sample of outputs, scaled to whole convolutions
            t0 = time.perf_counter()
            idx = np.random.default_rng(46).integers(0, N, 81920)
            ref = oracle.conv_direct_at(x, h, idx)
            t_cpu = time.perf_counter() - t0
            e2, emax = errors(main_r["y"].reshape(-1)[idx], ref)
            out["rel_l2_vs_fp64_oracle_sampled"] = e2
            out["max_entry_err_over_rms_sampled"] = emax
            out["cpu_baseline"] = {
                "value": round(idx.size / N / t_cpu, 8), "unit": "conv/s",
                "cores": oracle.num_threads(), "kind": "oracle",
                "sample": "%d of the %d outputs by the direct sum (long double, OpenMP over "
                          "outputs), scaled to one convolution; %.2f s" % (idx.size, N, t_cpu)}
            return out, main_r["y"]
        # whole convolutions of the same workload, repeated until cpu_min_s
        # of host time have passed
        ref, runs, t_cpu = time_oracle(oracle_reference(wl, dname == "c64"), cpu_min_s)
        e2, emax = errors(main_r["y"], ref)
        out["rel_l2_vs_fp64_oracle"] = e2
        out["max_entry_err_over_rms"] = emax
        route = ("direct O(n^2) sum in long double" if wl.get("oracle") == "direct" else
                 "standard FFT route with explicit index reversal, FP64, OpenMP over pencils")
        out["cpu_baseline"] = {
            "value": round(runs / t_cpu, 5), "unit": "conv/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": "%d full convolution(s) of the same workload (%s); %.2f s"
                      % (runs, route, t_cpu)}
    return out, main_r["y"]


# -------------------------------------------------------------------- batched

def graph_of(torch, fn):
    """Capture fn(stream) in a CUDA/HIP graph on a side stream."""
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        fn(s)  # warm-up outside the graph
        torch.cuda.synchronize()
        with torch.cuda.graph(g, stream=s):
            fn(s)
    torch.cuda.synchronize()
    return g


def batch_alg_bytes(sizes, filters, elem):
    """Algorithmic bytes of one batch: per problem one read and one write per
    pass of its minimal pass structure, plus one read of each size class's
    spectrum."""
    b = sum(2 * minimal_passes((n,), elem) * n * elem for n in sizes)
    return b + sum(int(np.asarray(h).size) * elem for h in filters.values())


def time_batch_form(pafc, torch, wl, tdtype, form, steps, warmup):
    """One batch form timed as one graph replay per batch: median and p99 ms
    per replay, the per-launch breakdown of an eager run (mean ms and
    algorithmic bytes per launch), the plan description and the output."""
    B = pafc.Batch(wl["sizes"], wl["fids"], len(wl["filters"]), tdtype, form=form)
    for f, h in wl["filters"].items():
        B.set_filter(f, torch.from_numpy(h).to(tdtype).cuda())
    x = torch.from_numpy(np.concatenate(wl["xs"])).to(tdtype).cuda()
    y = torch.empty_like(x)
    g = graph_of(torch, lambda s: B.convolve(x, out=y, stream=s))
    for _ in range(warmup):
        g.replay()
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    t0 = time.perf_counter()
    ev[0].record()
    for k in range(steps):
        g.replay()
        ev[k + 1].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_rep = [ev[k].elapsed_time(ev[k + 1]) for k in range(steps)]
    ms_lv, by_lv, _ = B.profile_levels(x, y, reps=max(5, steps // 2))
    desc = B.describe()
    yh = y.cpu().numpy().astype(np.complex128)
    B.close()
    del x, y, g
    torch.cuda.empty_cache()
    return {"ms_rep": ms_rep, "wall": wall, "ms_lv": ms_lv, "by_lv": by_lv, "desc": desc,
            "y": yh}


BATCH_FORMS = {"persistent": "one persistent launch: resident blocks claim whole problems "
                             "(largest first) and run all of a problem's passes",
               "levels": "one launch per pass level, register class and LDS occupancy",
               "classes": "per pass level, one pipelined launch per size class whose plan "
                          "runs that pass on the pipelined kernel, the rest as in levels"}


def bench_batched(pafc, torch, wl, tdtype, args, cpu_min_s=10.0):
    """The batch timed as one graph replay per batch (conv/s = problems /
    median replay) in the form args.batch_form, the other forms timed the
    same way beside it, and the same problems run one plan at a time (the
    plain form)."""
    elem = 16 if tdtype == torch.complex128 else 8
    nprob = len(wl["sizes"])
    steps = args.steps
    r = time_batch_form(pafc, torch, wl, tdtype, args.batch_form, steps, args.warmup)
    form = r["desc"]["form"]  # "auto" resolved by the library
    med = pct(r["ms_rep"], 50)
    value = nprob / (med * 1e-3)
    ms_lv, by_lv = r["ms_lv"], r["by_lv"]
    dom = max(range(len(ms_lv)), key=lambda i: ms_lv[i])
    alg = batch_alg_bytes(wl["sizes"], wl["filters"], elem)
    out = {
        "metric": METRIC, "value": round(value, 1), "unit": "conv/s", "n_gpus": 1,
        "steps": steps, "warmup": args.warmup, "ms_per_step": round(med, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if elem == 16 else "f32", "data": "synthetic",
        "config": dict(wl["config"], variant="perm_free", form=form, launches=len(ms_lv),
                       timing="one graph replay per batch (median)"),
        "form": BATCH_FORMS[form],
        "alg_bytes_per_batch": alg,
        "hbm_gbps_alg": round(alg / (med * 1e-3) / 1e9, 1),
        "hbm_frac_alg": round(alg / (med * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "wall_conv_per_s": round(nprob * steps / r["wall"], 1),
        "latency_ms": {"p50": round(med, 5), "p99": round(pct(r["ms_rep"], 99), 5)},
        "ms_per_launch": [round(v, 5) for v in ms_lv],
        # the batch's unit of work is one graph launch: its launches overlap
        # on several streams (classes form), and one kernel instance serves
        # several size classes, so no single kernel's duration stands for it
        "roofline": roofline_obj(alg, med, traffic=load_traffic(wl["name"], whole=True),
                                 kernel="one hipGraph launch of the batch (%d launches, %d "
                                        "stream(s), form %s)" % (len(ms_lv),
                                                                 r["desc"].get("streams", 1), form),
                                 alg_bytes_per_launch=alg, avg_launch_ms=round(med, 5)),
        "longest_launch": {"index": dom, "ms_alone": round(ms_lv[dom], 5),
                           "alg_bytes": by_lv[dom],
                           "achieved_gbs": round(by_lv[dom] / (ms_lv[dom] * 1e-3) / 1e9, 1),
                           "desc": (r["desc"].get("levels") or [None] * (dom + 1))[dom]},
        "launch_desc": r["desc"].get("levels"),
    }
    yh = r["y"]
    if not args.no_compare:
        out["other_forms"] = []
        for other in sorted(BATCH_FORMS):
            if other == form:
                continue
            o = time_batch_form(pafc, torch, wl, tdtype, other, steps, args.warmup)
            omed = pct(o["ms_rep"], 50)
            out["other_forms"].append({
                "form": other, "what": BATCH_FORMS[other],
                "conv_per_s": round(nprob / (omed * 1e-3), 1),
                "ms_per_batch": round(omed, 5), "launches": len(o["ms_lv"]),
                "hbm_gbps_alg": round(alg / (omed * 1e-3) / 1e9, 1),
                "max_abs_diff": float(np.abs(o["y"] - yh).max()),
                "speedup_of_%s" % form: round(omed / med, 3)})
        out["plain"] = bench_batched_plain(pafc, torch, wl, tdtype, yh)
        out["plain"]["speedup_batched_over_plain"] = round(
            value / out["plain"]["conv_per_s"], 3)
    if not args.no_cpu:
        batched_oracle(out, wl, yh, elem, cpu_min_s)
    return out, yh


def batched_oracle(out, wl, yh, elem, cpu_min_s):
    """Check the first problems in order against the FP64 oracle (inputs
    rounded to the plan's precision) until cpu_min_s of host time have
    passed, and report that rate as the CPU baseline."""
    import oracle
    nprob = len(wl["sizes"])
    offs = np.concatenate([[0], np.cumsum(wl["sizes"])])
    errs, emaxs = [], []
    k = 0
    t0 = time.perf_counter()
    while True:
        xi = wl["xs"][k]
        hi = wl["filters"][wl["fids"][k]]
        if elem == 8:
            xi = xi.astype(np.complex64).astype(np.complex128)
            hi = hi.astype(np.complex64).astype(np.complex128)
        ref = oracle.conv_fft(xi, hi)
        e2, em = errors(yh[offs[k]:offs[k + 1]], ref)
        errs.append(e2)
        emaxs.append(em)
        k += 1
        if time.perf_counter() - t0 >= cpu_min_s or k == nprob:
            break
    t_cpu = time.perf_counter() - t0
    out["rel_l2_vs_fp64_oracle_max_sampled"] = max(errs)
    out["max_entry_err_over_rms_sampled"] = max(emaxs)
    out["cpu_baseline"] = {
        "value": round(k / t_cpu, 3), "unit": "conv/s",
        "cores": oracle.num_threads(), "kind": "oracle",
        "sample": "the first %d of the 4096 problems (%d elements), FP64 standard route; "
                  "%.2f s" % (k, int(sum(wl["sizes"][:k])), t_cpu)}


def bench_batched_plain(pafc, torch, wl, tdtype, y_batched):
    """The same problems, one pafc_convolve per problem on one plan per size
    class (views into the packed arrays), timed by wall clock over the
    stream."""
    sizes = wl["sizes"]
    plans = {}
    for f, h in wl["filters"].items():
        n = int(np.asarray(h).size)
        p = pafc.Plan((n,), tdtype)
        p.set_filter(torch.from_numpy(h).to(tdtype).cuda())
        plans[f] = p
    x = torch.from_numpy(np.concatenate(wl["xs"])).to(tdtype).cuda()
    y = torch.empty_like(x)
    offs = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    views = [(plans[wl["fids"][i]], x[offs[i]:offs[i + 1]], y[offs[i]:offs[i + 1]])
             for i in range(len(sizes))]

    def run():
        for p, xi, yi in views:
            p.convolve(xi, out=yi)
    run()
    torch.cuda.synchronize()
    reps = 3
    t0 = time.perf_counter()
    for _ in range(reps):
        run()
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / reps
    yh = y.cpu().numpy().astype(np.complex128)
    for p in plans.values():
        p.close()
    del x, y, views
    torch.cuda.empty_cache()
    return {"conv_per_s": round(len(sizes) / wall, 1), "ms_per_batch": round(wall * 1e3, 4),
            "form": "one pafc_convolve per problem, one plan per size class",
            "max_abs_diff_vs_batched": float(np.abs(yh - y_batched).max())}


# -------------------------------------------------------------------- serving

def bench_serving(pafc, torch, wl, tdtype, args):
    """Warm-up + calibration (closed loop, twice over the first 200 requests),
    then 2000 requests with Poisson arrivals at 0.7 x the calibrated capacity;
    the plain form serves the calibration requests one at a time."""
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
    # the plain form: the same 200 requests served one at a time (one slot,
    # plans already cached)
    one = Server(ex, budget_bytes=budget, slots=1)
    one.cache = srv.cache
    t0 = time.perf_counter()
    run_closed_loop(one, reqs(0, 200), make_input=make_input)
    plain = 200 / (time.perf_counter() - t0)
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
    abytes = sum(alg_bytes(r.dims, elem) for r in done)
    span = st["n"] / st["throughput_per_s"]
    out = {
        "metric": METRIC,
        "value": round(st["throughput_per_s"], 2), "unit": "conv/s", "n_gpus": 1,
        "steps": len(done), "warmup": 200, "ms_per_step": round(1e3 / st["throughput_per_s"], 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if tdtype == torch.complex64 else "f64", "data": "synthetic",
        "config": dict(wl["config"], slots=slots, hbm_budget_bytes=budget),
        "latency_ms": {"p50": round(st["p50_ms"], 4), "p99": round(st["p99_ms"], 4),
                       "mean": round(st["mean_ms"], 4)},
        "offered_rate_per_s": round(rate, 2), "closed_loop_capacity_per_s": round(cap, 2),
        "plain_one_at_a_time_per_s": round(plain, 2),
        "speedup_served_over_plain": round(cap / plain, 3),
        "max_inflight": srv.max_inflight,
        "cache": {"plans_prepared": ex.prepared, "hits": srv.cache.hits,
                  "evictions": srv.cache.evictions, "bytes": srv.cache.bytes},
        "elements_served": elems,
        "alg_bytes_served": abytes,
        "hbm_gbps_alg_at_offered_rate": round(abytes / span / 1e9, 1),
        "roofline": None,
    }
    checked = [(r.dims, r.fid, make_input(r).cpu().numpy(), y)
               for rid, (r, y) in sorted(kept.items())]
    pool.clear()
    torch.cuda.empty_cache()
    if not args.no_cpu:
        serving_oracle(out, checked)
    return out, checked


def serving_oracle(out, checked):
    """Check the kept requests (1 in 50) against the FP64 oracle: the served
    input with the unit-sum wrapped Gaussian formed in space."""
    import oracle
    from paper_2506_12718_amd import inputs
    errs, emaxs = [], []
    t0 = time.perf_counter()
    for dims, fid, x, y in checked:
        h = inputs.wrapped_gaussian(dims, inputs.serving_sigma(dims, fid))
        ref = oracle.conv_fft(x.astype(np.complex128), h)
        e2, em = errors(y, ref)
        errs.append(e2)
        emaxs.append(em)
    t_cpu = time.perf_counter() - t0
    out["rel_l2_vs_fp64_oracle_max_sampled"] = max(errs)
    out["max_entry_err_over_rms_sampled"] = max(emaxs)
    out["oracle_checked_requests"] = len(errs)
    out["cpu_baseline"] = {"value": round(len(errs) / t_cpu, 3), "unit": "conv/s",
                           "cores": oracle.num_threads(), "kind": "oracle",
                           "sample": "1 in 50 of the measured requests (%d), FP64 standard "
                                     "route; %.2f s" % (len(errs), t_cpu)}


# ----------------------------------------------------------------------- main

def brief(o):
    """The compact form of one workload's measurement under `configs`."""
    keys = ("value", "unit", "dtype", "ms_per_step", "latency_ms", "alg_bytes_per_conv",
            "alg_bytes_per_batch", "plan_bytes_per_conv", "hbm_gbps_alg", "hbm_frac_alg",
            "rel_l2_vs_fp64_oracle", "max_entry_err_over_rms",
            "rel_l2_vs_fp64_oracle_max_sampled", "max_entry_err_over_rms_sampled",
            "cpu_baseline", "offered_rate_per_s", "closed_loop_capacity_per_s",
            "plain_one_at_a_time_per_s", "speedup_served_over_plain", "max_inflight",
            "hbm_gbps_alg_at_offered_rate", "wall_conv_per_s", "plain", "form", "other_forms")
    d = {k: o[k] for k in keys if k in o}
    d["workload"] = o["config"]["workload"]
    if o.get("roofline"):
        r = o["roofline"]
        d["roofline_dominant_launch"] = {k: r[k] for k in ("achieved", "frac", "kernel",
                                                           "avg_launch_ms", "launch_timing",
                                                           "traffic")
                                         if k in r}
    if "compare" in o:
        c = o["compare"]
        d["explicit_perm_conv_per_s"] = c.get("explicit_perm", {}).get("conv_per_s")
        d["speedup_perm_free_over_explicit"] = c.get("speedup_perm_free_over_explicit")
        if "perm_free_unfused" in c:
            d["unfused_conv_per_s"] = c["perm_free_unfused"]["conv_per_s"]
    return d


def run_all(pafc, torch, args):
    """The headline workload with every other workload of the set under
    `configs`; the one-thread oracle runs in a process of its own meanwhile,
    and the all-core oracle timings run after it has finished."""
    worker = None if args.no_cpu else start_one_thread_oracle(0.5 * args.oracle_min_s)
    gpu_args = argparse.Namespace(**dict(vars(args), no_cpu=True))
    results = {}
    head, y_head = bench_plain(pafc, torch, wl_conv3d("c128"), torch.complex128, gpu_args)
    plain_runs = [("conv1d_4096_c128_r2", wl_conv1d_r2, torch.complex128, 200),
                  ("conv1d_4096_c128_r4", wl_conv1d, torch.complex128, 200),
                  ("conv3d_256_c64_r4", wl_conv3d, torch.complex64, None),
                  ("conv2d_2187_c128_r3", wl_conv2d, torch.complex128, None),
                  ("conv1d_5p9_c128_r5", wl_conv1d5, torch.complex128, None),
                  ("conv1d_5p9_c64_r5", wl_conv1d5, torch.complex64, None)]
    ys = {}
    for name, fn, dt, steps in plain_runs:
        wl = fn("c128" if dt == torch.complex128 else "c64")
        results[name], ys[name] = bench_plain(pafc, torch, wl, dt, gpu_args, steps=steps)
    kept = {}
    for dname, dt in (("c128", torch.complex128), ("c64", torch.complex64)):
        print("bench: batched %s" % dname, file=sys.stderr, flush=True)
        wl = wl_batched(dname)
        results["batched_4096_%s" % dname], yb = bench_batched(
            pafc, torch, wl, dt, argparse.Namespace(**dict(vars(gpu_args), steps=10)))
        kept["batched_4096_%s" % dname] = (wl, yb)
    print("bench: serving c64", file=sys.stderr, flush=True)
    results["serving_c64"], kept["serving_c64"] = bench_serving(
        pafc, torch, wl_serving("c64"), torch.complex64, gpu_args)
    if not args.no_cpu:
        import oracle
        print("bench: waiting for the one-thread oracle", file=sys.stderr, flush=True)
        one = collect_one_thread_oracle(worker)
        print("bench: oracle on all host cores", file=sys.stderr, flush=True)
        cores = oracle.num_threads()
        # headline: whole FP64 convolutions of the same workload
        wl = wl_conv3d("c128")
        ref, runs, t = time_oracle(oracle_reference(wl, False), args.oracle_min_s)
        e2, em = errors(y_head, ref)
        head["rel_l2_vs_fp64_oracle"] = e2
        head["max_entry_err_over_rms"] = em
        head["cpu_baseline"] = {
            "value": round(runs / t, 5), "unit": "conv/s", "cores": cores, "kind": "oracle",
            "sample": "%d full convolution(s) of the same workload (standard FFT route with "
                      "explicit index reversal, FP64, OpenMP over pencils); %.2f s" % (runs, t),
            "one_thread": one.get("conv3d_256")}
        del ref
        for name, fn, dt, steps in plain_runs:
            wl = fn("c128" if dt == torch.complex128 else "c64")
            ref, runs, t = time_oracle(oracle_reference(wl, dt == torch.complex64),
                                       0.25 * args.oracle_min_s)
            e2, em = errors(ys[name], ref)
            results[name]["rel_l2_vs_fp64_oracle"] = e2
            results[name]["max_entry_err_over_rms"] = em
            key = {"conv1d_4096_c128_r2": "conv1d_4096_r2", "conv1d_4096_c128_r4": "conv1d_4096_r4",
                   "conv3d_256_c64_r4": "conv3d_256", "conv2d_2187_c128_r3": "conv2d_2187_r3",
                   "conv1d_5p9_c128_r5": "conv1d_5p9_r5",
                   "conv1d_5p9_c64_r5": "conv1d_5p9_r5"}[name]
            route = ("direct O(n^2) sum in long double" if wl.get("oracle") == "direct" else
                     "standard FFT route with explicit index reversal, FP64")
            results[name]["cpu_baseline"] = {
                "value": round(runs / t, 5), "unit": "conv/s", "cores": cores, "kind": "oracle",
                "sample": "%d full convolution(s) (%s); %.2f s" % (runs, route, t),
                "one_thread": one.get(key)}
            if name == "conv1d_4096_c128_r4":
                results[name]["cpu_baseline"]["one_thread_direct"] = one.get("conv1d_4096_direct")
            del ref
        for name in ("batched_4096_c128", "batched_4096_c64"):
            wl, yb = kept.pop(name)
            batched_oracle(results[name], wl, yb, 16 if name.endswith("c128") else 8,
                           0.25 * args.oracle_min_s)
            results[name]["cpu_baseline"]["one_thread"] = one.get("batched_4096")
            del wl, yb
        serving_oracle(results["serving_c64"], kept.pop("serving_c64"))
        results["serving_c64"]["cpu_baseline"]["one_thread"] = one.get("serving")
    head["configs"] = {k: brief(v) for k, v in results.items()}
    return head


def stream_probe(pafc, torch, args):
    """The strided middle pass's access pattern with no arithmetic, beside a
    plain copy: 256 MiB arrays, 256-byte row segments (pafc_stream_copy kinds
    tile_copy / tile_mul); GB/s of the bytes each kernel moves."""
    nbytes = 256 << 20
    n16 = nbytes // 16
    src = torch.zeros(2 * n16, dtype=torch.complex128, device="cuda")
    dst = torch.zeros(n16, dtype=torch.complex128, device="cuda")
    out = {"bytes_per_array": nbytes}
    for kind, moved, s_view in (("copy16", 2, src[:n16]), ("tile_copy", 2, src[:n16]),
                                ("tile_mul", 3, src)):
        for _ in range(3):
            pafc.stream_copy(s_view, dst, kind=kind)
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(21)]
        ev[0].record()
        for k in range(20):
            pafc.stream_copy(s_view, dst, kind=kind)
            ev[k + 1].record()
        torch.cuda.synchronize()
        ms = sorted(ev[k].elapsed_time(ev[k + 1]) for k in range(20))[10]
        out[kind] = {"ms": round(ms, 5), "gbs": round(moved * nbytes / (ms * 1e-3) / 1e9, 1)}
    return out


def counter_run(pafc, torch, args):
    """K convolutions of one workload after its set-up, for rocprofv3 counter
    runs: the last K x launches_per_conv dispatches of library kernels are
    the convolutions."""
    tdtype = torch.complex128 if args.dtype == "c128" else torch.complex64
    elem = 16 if args.dtype == "c128" else 8
    wl = WORKLOADS[args.workload](args.dtype)
    K = args.counter_run
    if args.workload == "batched":
        B = pafc.Batch(wl["sizes"], wl["fids"], len(wl["filters"]), tdtype, form=args.batch_form)
        for f, h in wl["filters"].items():
            B.set_filter(f, torch.from_numpy(h).to(tdtype).cuda())
        x = torch.from_numpy(np.concatenate(wl["xs"])).to(tdtype).cuda()
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        for _ in range(K):
            B.convolve(x, out=y)
        torch.cuda.synchronize()
        out = {"workload": wl["name"], "form": B.describe()["form"], "convs": K,
               "launches_per_conv": len(B.describe()["levels"]),
               "alg_bytes_per_conv": batch_alg_bytes(wl["sizes"], wl["filters"], elem)}
        B.close()
        return out
    plan = pafc.Plan(wl["x"].shape, tdtype, radix=wl["radix"])
    x = torch.from_numpy(wl["x"]).to(tdtype).cuda()
    y = torch.empty_like(x)
    if wl["domain"] == "symbol":
        plan.set_symbol(wl["symbol"][0], *wl["symbol"][1])
    else:
        plan.set_filter(torch.from_numpy(wl["h"]).to(tdtype).cuda(), domain=wl["domain"])
    torch.cuda.synchronize()
    for _ in range(K):
        plan.convolve(x, out=y)
    torch.cuda.synchronize()
    d = plan.describe()
    out = {"workload": wl["name"], "convs": K, "launches_per_conv": len(d["conv_passes"]),
           "conv_passes": d["conv_passes"], "alg_bytes_per_conv": alg_bytes(wl["x"].shape, elem),
           "plan_bytes_per_conv": d["hbm_bytes_conv"]}
    plan.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="all", choices=["all"] + sorted(WORKLOADS))
    ap.add_argument("--dtype", default="c128", choices=["c128", "c64"])
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle timing and error check")
    ap.add_argument("--no-compare", action="store_true", help="skip the comparison variants")
    ap.add_argument("--counter-run", type=int, default=0, metavar="K",
                    help="plan, set the filter, then run exactly K convolutions of --workload "
                         "and nothing else (for hardware counter runs); prints the launches "
                         "of one convolution and its algorithmic bytes")
    ap.add_argument("--batch-form", default="auto", choices=sorted(BATCH_FORMS) + ["auto"],
                    help="form of the batched workload that `value` reports (auto: the "
                         "library's choice for the dtype)")
    ap.add_argument("--probe", action="store_true",
                    help="streaming probes of the strided middle pass's access pattern")
    ap.add_argument("--filter-per-call", action="store_true",
                    help="transform the filter inside every timed call (three transforms per "
                         "convolution, as the paper times it)")
    ap.add_argument("--calibrate", action="store_true",
                    help="run only the plain streaming copy of 256 MiB (counter calibration)")
    ap.add_argument("--oracle-min-s", type=float, default=8.0,
                    help="host seconds of oracle work per timed sample")
    ap.add_argument("--oracle-worker", action="store_true", help=argparse.SUPPRESS)
    args = ap.parse_args()

    if args.oracle_worker:
        oracle_worker(args.oracle_min_s)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(each convolution runs on a single MI355X); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2506_12718_amd as pafc
    pafc.lib()
    torch.cuda.set_device(0)
    if args.probe:
        print(json.dumps(stream_probe(pafc, torch, args)))
        return
    if args.calibrate:
        nbytes = 256 << 20
        a = torch.zeros(nbytes // 16, dtype=torch.complex128, device="cuda")
        b = torch.empty_like(a)
        out = {"calibration_bytes": nbytes}
        for kind in ("copy16", "copy8", "read"):
            pafc.stream_copy(a, b, kind=kind)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(10):
                pafc.stream_copy(a, b, kind=kind)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / 10
            moved = nbytes if kind == "read" else 2 * nbytes
            out[kind] = {"ms": round(dt * 1e3, 5), "GBps": round(moved / dt / 1e9, 1)}
        print(json.dumps(out))
        return
    if args.counter_run:
        print(json.dumps(counter_run(pafc, torch, args)), flush=True)
        return
    if args.workload == "all":
        if args.filter_per_call:
            print("--filter-per-call needs a single --workload", file=sys.stderr)
            sys.exit(2)
        out = run_all(pafc, torch, args)
        print(json.dumps(out), flush=True)
        return
    tdtype = torch.complex128 if args.dtype == "c128" else torch.complex64
    wl = WORKLOADS[args.workload](args.dtype)
    if args.workload == "batched":
        out, _ = bench_batched(pafc, torch, wl, tdtype, args)
    elif args.workload == "serving":
        out, _ = bench_serving(pafc, torch, wl, tdtype, args)
    else:
        if args.filter_per_call and wl["domain"] != "spatial":
            print("--filter-per-call needs a workload with a spatial filter", file=sys.stderr)
            sys.exit(2)
        out, _ = bench_plain(pafc, torch, wl, tdtype, args)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
