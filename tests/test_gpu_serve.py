"""GPU tests of the serving loop: a request gives the same result alone and
in a mix of concurrent requests; served results match the FP64 oracle; an
HBM budget small enough to force evictions changes nothing in the results."""
import sys

import numpy as np
import pytest

import oracle
from paper_2506_12718_amd import inputs
from gpu_util import check_close, rel_l2, torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def make_requests(seed, count, sides2=(64, 81, 128, 243), sides3=(32, 64, 81)):
    from paper_2506_12718_amd.serve import Request
    reqs = inputs.serving_requests(seed=seed, count=count, sides_2d=sides2, sides_3d=sides3)
    return [Request(rid=r["id"], dims=r["dims"], fid=r["filter"], meta={"x_seed": r["x_seed"]})
            for r in reqs]


def device_input(req):
    x = inputs.serving_input({"dims": req.dims, "x_seed": req.meta["x_seed"]})
    return torch.from_numpy(x).cuda()


def serve(reqs, slots, budget=8 << 30, rate=None):
    from paper_2506_12718_amd.serve import GpuExecutor, Server, run_closed_loop, run_open_loop
    ex = GpuExecutor(dtype=torch.complex64, sigma_of=inputs.serving_sigma, slots=slots)
    srv = Server(ex, budget_bytes=budget, slots=slots)
    if rate is None:
        done = run_closed_loop(srv, reqs, make_input=device_input)
    else:
        done = run_open_loop(srv, reqs, rate, make_input=device_input)
    torch.cuda.synchronize()
    outs = {r.rid: r.out.cpu().numpy() for r in done}
    return outs, srv


def test_alone_equals_mix():
    mix = make_requests(11, 40)
    target = mix[17]
    from paper_2506_12718_amd.serve import Request
    alone = [Request(rid=target.rid, dims=target.dims, fid=target.fid, meta=dict(target.meta))]
    say("alone", target.dims)
    outs_alone, _ = serve(alone, slots=1)
    say("mix of", len(mix))
    outs_mix, srv = serve(mix, slots=4, rate=4000.0)
    assert srv.max_inflight > 1  # the target really overlapped with others
    assert np.array_equal(outs_alone[target.rid], outs_mix[target.rid])


def served_reference(dims, x_seed, sigma):
    """The oracle's FP64 convolution of the FP32 input the server was given
    with the unit-sum wrapped Gaussian of width sigma (formed in space)."""
    x = inputs.serving_input({"dims": dims, "x_seed": x_seed}).astype(np.complex128)
    h = inputs.wrapped_gaussian(dims, sigma)
    return oracle.conv_fft(x, h)


def test_served_results_match_oracle():
    reqs = make_requests(12, 12)
    outs, _ = serve(reqs, slots=4)
    for r in reqs[:8]:
        ref = served_reference(r.dims, r.meta["x_seed"], inputs.serving_sigma(r.dims, r.fid))
        check_close(outs[r.rid], ref, 1e-5, what=str(r.dims))


SERVED_GRIDS = ([(s, s) for s in inputs.SERVE_SIDES_2D] +
                [(s, s, s) for s in inputs.SERVE_SIDES_3D])


@pytest.mark.parametrize("dims", SERVED_GRIDS, ids=lambda d: "x".join(map(str, d)))
def test_every_served_grid_fp32(dims):
    """Every grid the served workload draws, through the server's own plan
    path (FP32 plan, Gaussian filter installed as its closed-form spectrum),
    at the widest and narrowest filter widths of the pool of that grid,
    against the FP64 oracle element by element; and the plan's device
    memory stays within what admission charged for it beforehand."""
    from paper_2506_12718_amd.serve import GpuExecutor, Request
    ex = GpuExecutor(dtype=torch.complex64, sigma_of=inputs.serving_sigma, slots=1)
    sig = {f: inputs.serving_sigma(dims, f) for f in range(8)}
    for fid in (min(sig, key=sig.get), max(sig, key=sig.get)):
        req = Request(rid=fid, dims=dims, fid=fid, meta={"x_seed": 7000 + fid})
        say("served grid", dims, "sigma %.3f" % sig[fid])
        req.x = device_input(req)
        obj = ex.prepare(req, 0)
        assert ex.held_bytes(obj) <= ex.plan_bytes(req), (ex.held_bytes(obj), ex.plan_bytes(req))
        ex.launch(req, obj, 0)
        torch.cuda.synchronize()
        y = req.out.cpu().numpy()
        ex.release_plan(obj)
        check_close(y, served_reference(dims, req.meta["x_seed"], sig[fid]), 1e-5,
                    what=str(dims))


def test_tight_budget_evicts_and_agrees():
    reqs = make_requests(13, 30, sides2=(64, 128), sides3=(32,))
    outs_free, srv_free = serve(reqs, slots=4)
    reqs2 = make_requests(13, 30, sides2=(64, 128), sides3=(32,))
    # room for the largest request with its plan (as charged before
    # planning) plus one more output: far less than the ~24 plans the mix
    # uses, so plans are evicted and prepared again
    from paper_2506_12718_amd.serve import GpuExecutor, Request
    ex = GpuExecutor(dtype=torch.complex64, slots=1)
    worst = max(ex.request_bytes(r) + ex.plan_bytes(r) for r in reqs2)
    budget = worst + max(ex.request_bytes(r) for r in reqs2)
    outs_tight, srv_tight = serve(reqs2, slots=4, budget=budget)
    assert not srv_tight.failed
    assert srv_tight.cache.evictions > 0
    for rid in outs_free:
        assert np.array_equal(outs_free[rid], outs_tight[rid])


def test_injected_failures_fail_one_request_each(monkeypatch):
    """PAFC_FAULT_INJECT makes one preparation and one launch fail: those two
    requests fail with the error, every other request is served with the
    same bits as an undisturbed run, and the server ends with nothing held."""
    reqs = make_requests(15, 24)
    outs_ok, _ = serve(reqs, slots=3)
    for spec in ("prepare:2", "launch:7"):
        monkeypatch.setenv("PAFC_FAULT_INJECT", spec)
        reqs2 = make_requests(15, 24)
        from paper_2506_12718_amd.serve import GpuExecutor, Server, run_closed_loop
        ex = GpuExecutor(dtype=torch.complex64, sigma_of=inputs.serving_sigma, slots=3)
        srv = Server(ex, budget_bytes=8 << 30, slots=3)
        done = run_closed_loop(srv, reqs2, make_input=device_input)
        torch.cuda.synchronize()
        say(spec, "failed", [(r.rid, r.error) for r in srv.failed])
        assert len(srv.failed) == 1 and "injected" in srv.failed[0].error
        assert len(done) == len(reqs2) - 1
        for r in done:
            assert np.array_equal(r.out.cpu().numpy(), outs_ok[r.rid])
        assert srv.reserved == 0 and not srv.inflight
        assert all(e[2] == 0 for e in srv.cache.entries.values())


def test_injected_out_of_memory_leaks_nothing(monkeypatch):
    """PAFC_FAULT_INJECT=oom: pafc_plan reports OUT_OF_MEMORY after its first
    allocations and frees them; the device's free memory is unchanged after
    many such failures of a 256^3 plan (about 300 MB each)."""
    import paper_2506_12718_amd as pafc
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    monkeypatch.setenv("PAFC_FAULT_INJECT", "oom")
    for _ in range(20):
        with pytest.raises(pafc.PafcError) as e:
            pafc.Plan((256, 256, 256), torch.complex128)
        assert e.value.status == 3
    monkeypatch.delenv("PAFC_FAULT_INJECT")
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    assert abs(free1 - free0) < (64 << 20), (free0, free1)
    P = pafc.Plan((64, 64), torch.complex128)  # planning works again
    P.close()
