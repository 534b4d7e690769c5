"""GPU test of pafc_convolve_with_filter_noalloc, called through the C ABI:
its output against pafc_convolve_with_filter's on the same inputs (same
kernels, so the same bits), and against the FP64 oracle, on two calls in a
row with the second input smaller; the plan's own filter is left in effect;
spectra beyond the library's fixed array and unsupported plans are refused.
"""
import ctypes
import sys

import numpy as np
import pytest

import oracle
from paper_2506_12718_amd import inputs
from gpu_util import TOL, check_close, rounded, to_dev, to_host, torch

pytestmark = pytest.mark.gpu

C128, C64 = torch.complex128, torch.complex64


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2506_12718_amd as pafc
    pafc.lib()  # fail loudly if the library is missing
    yield


def _abi_call(fn, plan, x, h, y):
    import paper_2506_12718_amd as pafc
    L = pafc.lib()
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return getattr(L, fn)(plan.handle, ctypes.c_void_p(x.data_ptr()),
                          ctypes.c_void_p(h.data_ptr()), ctypes.c_void_p(y.data_ptr()), stream)


# (first shape, second smaller shape): 2-D grids whose strided middle pass
# stores the spectrum tile-major, 3-D, a single-pass 1-D length, mixed radix
SEQUENCES = [
    ((256, 256), (4096,)),
    ((128, 128, 128), (60, 45)),
    ((5 ** 7,), (2187,)),
    ((96, 80, 64), (1000,)),
]


@pytest.mark.parametrize("dtype", [C128, C64], ids=["c128", "c64"])
@pytest.mark.parametrize("shapes", SEQUENCES, ids=lambda s: "%s_then_%s" % s)
def test_noalloc_matches_convolve_with_filter(shapes, dtype):
    import paper_2506_12718_amd as pafc
    if dtype == C128 and shapes[0] == (128, 128, 128):
        shapes = ((128, 128, 64), shapes[1])  # 2^20 complex128 elements
    rng = np.random.default_rng(7)
    for k, shape in enumerate(shapes):
        say("noalloc call %d shape=%s dtype=%s" % (k, shape, dtype))
        x = inputs.complex_uniform(rng, shape)
        h_set = inputs.complex_uniform(rng, shape)
        h = inputs.complex_uniform(rng, shape)
        plan = pafc.Plan(shape, dtype)
        try:
            plan.set_filter(to_dev(h_set, dtype))
            xd, hd = to_dev(x, dtype), to_dev(h, dtype)
            y_na = torch.empty_like(xd)
            st = _abi_call("pafc_convolve_with_filter_noalloc", plan, xd, hd, y_na)
            assert st == 0, st
            # the plan's own filter is untouched by the no-alloc call
            y_set = to_host(plan.convolve(xd))
            ref_set = oracle.conv_fft(rounded(x, dtype), rounded(h_set, dtype))
            check_close(y_set, ref_set, TOL[dtype], "plan filter after noalloc %s" % (shape,))
            # the existing entry point on the same inputs (it replaces the
            # plan's filter, so it runs second)
            y_wf = torch.empty_like(xd)
            st = _abi_call("pafc_convolve_with_filter", plan, xd, hd, y_wf)
            assert st == 0, st
            a, b = to_host(y_na), to_host(y_wf)
            assert np.array_equal(a, b), ("noalloc differs from convolve_with_filter",
                                          shape, float(np.abs(a - b).max()))
            ref = oracle.conv_fft(rounded(x, dtype), rounded(h, dtype))
            check_close(a, ref, TOL[dtype], "noalloc %s" % (shape,))
        finally:
            plan.close()


def test_noalloc_refuses_spectra_beyond_the_array():
    import paper_2506_12718_amd as pafc
    n = 1 << 22  # 64 MiB of complex128 spectrum > 32 MiB
    assert n * 16 > pafc.NOALLOC_MAX_BYTES
    plan = pafc.Plan((n,), C128)
    try:
        x = torch.zeros(n, dtype=C128, device="cuda")
        y = torch.empty_like(x)
        say("noalloc refusal n=%d" % n)
        st = _abi_call("pafc_convolve_with_filter_noalloc", plan, x, x, y)
        assert st == 2, st  # PAFC_ERROR_UNSUPPORTED_SIZE
        with pytest.raises(pafc.PafcError):
            plan.convolve_with_filter_noalloc(x, x, y)
    finally:
        plan.close()
    # the same length in complex64 (32 MiB) is at the limit and runs
    plan = pafc.Plan((n,), C64)
    try:
        rng = np.random.default_rng(11)
        x = inputs.complex_uniform(rng, (n,))
        h = inputs.complex_uniform(rng, (n,))
        xd, hd = to_dev(x, C64), to_dev(h, C64)
        y = torch.empty_like(xd)
        plan.convolve_with_filter_noalloc(xd, hd, y)
        y2 = plan.convolve_with_filter(xd, hd)
        assert np.array_equal(to_host(y), to_host(y2))
    finally:
        plan.close()


@pytest.mark.parametrize("shape,variant", [((4096,), "explicit_perm"),
                                           ((4096,), "perm_free_unfused"),
                                           ((97,), "perm_free"),
                                           ((7776,), "prime_factor")])
def test_noalloc_refuses_other_routes(shape, variant):
    import paper_2506_12718_amd as pafc
    plan = pafc.Plan(shape, C128, variant=variant)
    try:
        x = torch.zeros(shape, dtype=C128, device="cuda")
        y = torch.empty_like(x)
        say("noalloc refusal %s %s" % (shape, variant))
        assert _abi_call("pafc_convolve_with_filter_noalloc", plan, x, x, y) == 1
    finally:
        plan.close()
