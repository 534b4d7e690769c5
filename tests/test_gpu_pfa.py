"""GPU parity of the prime-factor route (variants PAFC_PRIME_FACTOR and
PAFC_PRIME_FACTOR_EXPLICIT): a 1-D length with pairwise coprime factors
reindexed onto the factor grid by the Chinese-remainder map, convolved there,
mapped back.  Checked against the 1-D oracle.  Tolerances: relative L2 <=
1e-12 (complex128), <= 1e-5 (complex64, oracle on the same rounded inputs)."""
import sys

import numpy as np
import pytest

import oracle
from paper_2506_12718_amd import inputs
from gpu_util import TOL, check_close, rel_l2, rounded, to_dev, to_host, torch

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
    pafc.lib()
    yield


def pafc():
    import paper_2506_12718_amd as m
    return m


SIZES = [6, 10, 15, 30, 60, 360, 720, 2 ** 6 * 3 ** 3 * 5 ** 2, 2 ** 10 * 3 ** 5,
         2 ** 8 * 3 ** 5 * 5 ** 3]


@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("variant", ["prime_factor", "prime_factor_explicit"])
@pytest.mark.parametrize("dtype", [C128, C64])
def test_prime_factor_matches_oracle(n, variant, dtype):
    say("pfa", n, variant, dtype)
    rng = np.random.default_rng([n, 7])
    x = inputs.complex_uniform(rng, (n,))
    h = inputs.complex_uniform(rng, (n,))
    P = pafc().Plan((n,), dtype, variant=variant)
    P.set_filter(to_dev(h, dtype))
    y = to_host(P.convolve(to_dev(x, dtype)))
    P.close()
    ref = oracle.conv_fft(rounded(x, dtype), rounded(h, dtype))
    check_close(y, ref, TOL[dtype])


@pytest.mark.parametrize("dtype", [C128, C64])
def test_prime_factor_spectral_filter_in_place_and_filter_per_call(dtype):
    n = 2 ** 5 * 3 ** 4 * 5 ** 2
    rng = np.random.default_rng(8)
    x = inputs.complex_uniform(rng, (n,))
    h = inputs.complex_uniform(rng, (n,))
    ref = oracle.conv_fft(rounded(x, dtype), rounded(h, dtype))
    P = pafc().Plan((n,), dtype, variant="prime_factor")
    # natural-order spectrum of h (the oracle's DFT)
    P.set_filter(to_dev(oracle.fft(rounded(h, dtype)), dtype), domain="spectral_natural")
    xd = to_dev(x, dtype)
    P.convolve(xd, out=xd)  # in place
    check_close(to_host(xd), ref, TOL[dtype])
    y = to_host(P.convolve_with_filter(to_dev(x, dtype), to_dev(h, dtype)))
    check_close(y, ref, TOL[dtype])
    ms, by, rep = P.profile_passes(to_dev(x, dtype), torch.empty(n, dtype=dtype, device="cuda"),
                                   reps=2)
    d = P.describe()
    assert len(ms) == len(d["conv_passes"]) and by[0] == by[-1] == 2 * n * (16 if dtype == C128 else 8)
    P.close()


def test_prime_factor_rejections():
    P = pafc().Plan((60,), C128, variant="prime_factor")
    a = torch.zeros(60, dtype=C128, device="cuda")
    for call in (lambda: P.forward(a), lambda: P.inverse(a), lambda: P.set_symbol("heat", 1.0),
                 lambda: P.radices(0)):
        with pytest.raises(pafc().PafcError):
            call()
    P.close()
    for dims in ((1024,), (2187,), (30, 2)):
        with pytest.raises(pafc().PafcError):
            pafc().Plan(dims, C128, variant="prime_factor")
