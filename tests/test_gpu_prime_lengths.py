"""GPU parity of the routes for 1-D lengths with a prime factor above 5
(Sec. "Rader's and Bluestein's frameworks"), both on a permutation-avoiding
inner plan:
* Bluestein: the length-n DFT as a length-m convolution (m >= 2n - 1,
  {2,3,5}-smooth), for any such n;
* Rader: for a prime p with p - 1 {2,3,5}-smooth, the DFT at the nonzero
  frequencies as a length p - 1 convolution after reindexing by powers of a
  generator (the planner's choice for such primes).
Checked against the oracle's direct sum (long double), whole arrays up to
n = 6007 and sampled outputs at n ~ 10^6.  Tolerances: relative L2 <= 1e-12
(complex128), <= 1e-5 (complex64, oracle on the rounded inputs)."""
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


SIZES = [7, 11, 13, 14, 97, 127, 1001, 1009, 4099, 6007]


@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("variant", ["perm_free", "explicit_perm", "perm_free_unfused"])
@pytest.mark.parametrize("dtype", [C128, C64])
def test_bluestein_matches_direct_sum(n, variant, dtype, monkeypatch):
    monkeypatch.setenv("PAFC_BLUESTEIN", "1")  # also for the primes Rader's method takes
    say("bluestein", n, variant, dtype)
    rng = np.random.default_rng([n, 9])
    x = inputs.complex_uniform(rng, (n,))
    h = inputs.complex_uniform(rng, (n,))
    P = pafc().Plan((n,), dtype, variant=variant)
    d = P.describe()
    assert d["bluestein_m"] >= 2 * n - 1
    P.set_filter(to_dev(h, dtype))
    y = to_host(P.convolve(to_dev(x, dtype)))
    P.close()
    ref = oracle.conv_direct(rounded(x, dtype), rounded(h, dtype))
    check_close(y, ref, TOL[dtype], what="bluestein m=%d" % d["bluestein_m"])


def dft_definition(h):
    n = h.size
    jk = np.outer(np.arange(n), np.arange(n)) % n
    return np.exp(-2j * np.pi * jk / n) @ h


@pytest.mark.parametrize("dtype", [C128, C64])
def test_bluestein_spectral_filter_filter_per_call_and_profile(dtype):
    n = 1013
    rng = np.random.default_rng(10)
    x = inputs.complex_uniform(rng, (n,))
    h = inputs.complex_uniform(rng, (n,))
    ref = oracle.conv_direct(rounded(x, dtype), rounded(h, dtype))
    P = pafc().Plan((n,), dtype)
    P.set_filter(to_dev(dft_definition(rounded(h, dtype)), dtype), domain="spectral_natural")
    xd = to_dev(x, dtype)
    P.convolve(xd, out=xd)  # in place
    check_close(to_host(xd), ref, TOL[dtype])
    y = to_host(P.convolve_with_filter(to_dev(x, dtype), to_dev(h, dtype)))
    check_close(y, ref, TOL[dtype])
    ms, by, rep = P.profile_passes(to_dev(x, dtype), torch.empty(n, dtype=dtype, device="cuda"),
                                   reps=2)
    assert len(ms) == len(P.describe()["conv_passes"]) and min(by) > 0
    P.close()


def test_bluestein_large_prime_sampled():
    n = 1000003
    rng = np.random.default_rng(11)
    x = inputs.complex_uniform(rng, (n,))
    h = inputs.complex_uniform(rng, (n,))
    P = pafc().Plan((n,), C128)
    P.set_filter(to_dev(h, C128))
    y = to_host(P.convolve(to_dev(x, C128)))
    P.close()
    idx = rng.integers(0, n, 64)
    ref = oracle.conv_direct_at(x, h, idx)
    check_close(y[idx], ref, 1e-12, what="1000003 sampled")


def test_bluestein_rejections():
    P = pafc().Plan((1009,), C128)
    a = torch.zeros(1009, dtype=C128, device="cuda")
    for call in (lambda: P.forward(a), lambda: P.inverse(a), lambda: P.set_symbol("heat", 1.0),
                 lambda: P.radices(0)):
        with pytest.raises(pafc().PafcError):
            call()
    P.close()
    for dims, radix in (((7, 7), None), ((97,), [4])):
        with pytest.raises(pafc().PafcError):
            pafc().Plan(dims, C128, radix=radix)


RADER = [7, 11, 13, 17, 19, 31, 97, 257, 769, 3457]


@pytest.mark.parametrize("n", RADER)
@pytest.mark.parametrize("variant", ["perm_free", "explicit_perm", "perm_free_unfused"])
@pytest.mark.parametrize("dtype", [C128, C64])
def test_rader_matches_direct_sum(n, variant, dtype):
    say("rader", n, variant, dtype)
    rng = np.random.default_rng([n, 12])
    x = inputs.complex_uniform(rng, (n,))
    h = inputs.complex_uniform(rng, (n,))
    P = pafc().Plan((n,), dtype, variant=variant)
    d = P.describe()
    assert d["rader_inner"] == n - 1
    P.set_filter(to_dev(h, dtype))
    y = to_host(P.convolve(to_dev(x, dtype)))
    P.close()
    ref = oracle.conv_direct(rounded(x, dtype), rounded(h, dtype))
    check_close(y, ref, TOL[dtype], what="rader g=%d" % d["rader_generator"])


@pytest.mark.parametrize("dtype", [C128, C64])
def test_rader_spectral_filter_in_place_filter_per_call_and_profile(dtype):
    n = 1153  # 2^7 3^2 + 1
    rng = np.random.default_rng(13)
    x = inputs.complex_uniform(rng, (n,))
    h = inputs.complex_uniform(rng, (n,))
    ref = oracle.conv_direct(rounded(x, dtype), rounded(h, dtype))
    P = pafc().Plan((n,), dtype)
    assert "rader_generator" in P.describe()
    P.set_filter(to_dev(dft_definition(rounded(h, dtype)), dtype), domain="spectral_natural")
    xd = to_dev(x, dtype)
    P.convolve(xd, out=xd)  # in place: x_0 is read before y is written
    check_close(to_host(xd), ref, TOL[dtype])
    y = to_host(P.convolve_with_filter(to_dev(x, dtype), to_dev(h, dtype)))
    check_close(y, ref, TOL[dtype])
    ms, by, rep = P.profile_passes(to_dev(x, dtype), torch.empty(n, dtype=dtype, device="cuda"),
                                   reps=2)
    assert len(ms) == len(P.describe()["conv_passes"]) and min(by) > 0
    P.close()


@pytest.mark.parametrize("n", [97, 65537])
def test_rader_and_bluestein_agree(n, monkeypatch):
    """The two routes for the same prime length (Bluestein forced by
    PAFC_BLUESTEIN=1) give the same convolution to rounding."""
    rng = np.random.default_rng([n, 14])
    x = inputs.complex_uniform(rng, (n,))
    h = inputs.complex_uniform(rng, (n,))
    out = {}
    for route in ("rader", "bluestein"):
        monkeypatch.setenv("PAFC_BLUESTEIN", "1" if route == "bluestein" else "0")
        P = pafc().Plan((n,), C128)
        assert ("rader_generator" in P.describe()) == (route == "rader")
        P.set_filter(to_dev(h, C128))
        out[route] = to_host(P.convolve(to_dev(x, C128)))
        P.close()
    check_close(out["rader"], out["bluestein"], 1e-12)
    idx = rng.integers(0, n, 32)
    ref = oracle.conv_direct_at(x, h, idx)
    check_close(out["rader"][idx], ref, 1e-12, what="rader sampled")


@pytest.mark.parametrize("dtype", [C128, C64])
def test_rader_large_prime_sampled(dtype):
    n = 995329  # 2^12 3^5 + 1
    rng = np.random.default_rng(15)
    x = inputs.complex_uniform(rng, (n,))
    h = inputs.complex_uniform(rng, (n,))
    P = pafc().Plan((n,), dtype)
    assert P.describe()["rader_inner"] == n - 1
    P.set_filter(to_dev(h, dtype))
    y = to_host(P.convolve(to_dev(x, dtype)))
    P.close()
    idx = rng.integers(0, n, 64)
    idx[0] = 0  # the DC output has its own formula
    ref = oracle.conv_direct_at(rounded(x, dtype), rounded(h, dtype), idx)
    check_close(y[idx], ref, TOL[dtype], what="995329 %s sampled" % dtype)


def test_rader_rejections():
    P = pafc().Plan((97,), C128)
    assert "rader_generator" in P.describe()
    a = torch.zeros(97, dtype=C128, device="cuda")
    for call in (lambda: P.forward(a), lambda: P.inverse(a), lambda: P.set_symbol("heat", 1.0),
                 lambda: P.radices(0)):
        with pytest.raises(pafc().PafcError):
            call()
    P.close()
