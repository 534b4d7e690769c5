"""GPU tests of the serving loop: a request gives the same result alone and
in a mix of concurrent requests; served results match the FP64 oracle; an
HBM budget small enough to force evictions changes nothing in the results."""
import sys

import numpy as np
import pytest

import oracle
from paper_2506_12718_amd import inputs
from gpu_util import rel_l2, torch

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


def test_served_results_match_oracle():
    reqs = make_requests(12, 12)
    outs, _ = serve(reqs, slots=4)
    for r in reqs[:8]:
        x = inputs.serving_input({"dims": r.dims, "x_seed": r.meta["x_seed"]}).astype(np.complex128)
        h = inputs.wrapped_gaussian(r.dims, inputs.serving_sigma(r.dims, r.fid))
        h = h.astype(np.complex64).astype(np.complex128)
        ref = oracle.conv_fft(x, h)
        assert rel_l2(outs[r.rid], ref) < 1e-5, r.dims


def test_tight_budget_evicts_and_agrees():
    reqs = make_requests(13, 30, sides2=(64, 128), sides3=(32,))
    outs_free, srv_free = serve(reqs, slots=4)
    reqs2 = make_requests(13, 30, sides2=(64, 128), sides3=(32,))
    outs_tight, srv_tight = serve(reqs2, slots=4, budget=3 * 128 * 128 * 8 + 4 * 128 * 128 * 8)
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
