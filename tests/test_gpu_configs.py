"""GPU parity at the full sizes of the benchmark workloads, in the launch
configuration the benchmark times."""
import sys

import numpy as np
import pytest

import oracle
from paper_2506_12718_amd import inputs
from gpu_util import TOL, check_close, rel_l2, rounded, to_dev, to_host, torch

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def pafc():
    import paper_2506_12718_amd as m
    return m


@pytest.fixture(scope="module")
def conv3d():
    x, h = inputs.conv3d_gaussian()
    say("oracle 256^3 ...")
    ref = oracle.conv_fft(x, h, [[4] * 4] * 3)
    return x, h, ref


@pytest.mark.parametrize("variant", ["perm_free", "explicit_perm"])
def test_conv3d_256_fp64(conv3d, variant):
    x, h, ref = conv3d
    say("256^3 fp64", variant)
    P = pafc().Plan(x.shape, torch.complex128, radix=[4, 4, 4], variant=variant)
    P.set_filter(to_dev(h, torch.complex128))
    y = to_host(P.convolve(to_dev(x, torch.complex128)))
    P.close()
    check_close(y, ref, 1e-12)
    # direct-sum spot checks at sampled entries (the definition, O(N) each)
    idx = np.random.default_rng(0).integers(0, x.size, 32)
    direct = oracle.conv_direct_at(x, h, idx)
    check_close(y.ravel()[idx], direct, 1e-12, what="direct-sum spot checks")


def test_conv3d_256_fp32(conv3d):
    x, h, _ = conv3d
    xr, hr = rounded(x, torch.complex64), rounded(h, torch.complex64)
    say("256^3 fp32")
    ref = oracle.conv_fft(xr, hr, [[4] * 4] * 3)
    P = pafc().Plan(x.shape, torch.complex64, radix=[4, 4, 4])
    P.set_filter(to_dev(h, torch.complex64))
    y = to_host(P.convolve(to_dev(x, torch.complex64)))
    P.close()
    check_close(y, ref, 1e-5)


def test_conv2d_2187_radix3_spectral():
    x, hhat = inputs.spectral_filter_case(31, (2187, 2187))
    say("2187^2")
    ref = oracle.fft(hhat * oracle.fft(x), inverse=True)
    P = pafc().Plan(x.shape, torch.complex128, radix=[3, 3])
    P.set_filter(to_dev(hhat, torch.complex128), domain="spectral_natural")
    y = to_host(P.convolve(to_dev(x, torch.complex128)))
    P.close()
    check_close(y, ref, 1e-12)


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
def test_conv1d_5pow9_radix5(dtype):
    x, hhat = inputs.spectral_filter_case(32, (5 ** 9,))
    xr, hr = rounded(x, dtype), rounded(hhat, dtype)
    say("5^9", dtype)
    ref = oracle.fft(hr * oracle.fft(xr), inverse=True)
    P = pafc().Plan(x.shape, dtype, radix=[5])
    P.set_filter(to_dev(hhat, dtype), domain="spectral_natural")
    y = to_host(P.convolve(to_dev(x, dtype)))
    P.close()
    check_close(y, ref, TOL[dtype])


def test_maximum_size_64bit_offsets():
    """16384 x 16384 complex128: 4 GiB per array, beyond the pipelined
    kernels' 32-bit byte offsets, so every pass runs on the general engine
    with 64-bit offsets.  Sampled outputs (first, last, random) against the
    oracle's direct sum."""
    shape = (2 ** 14, 2 ** 14)
    d = pafc().describe(shape, "c128")
    assert not any("pipe_kernel" in l for l in d["conv_passes"])
    rng = np.random.default_rng(77)
    x = inputs.complex_uniform(rng, shape)
    h = inputs.complex_uniform(rng, shape)
    P = pafc().Plan(shape, torch.complex128)
    hd = to_dev(h, torch.complex128)
    P.set_filter(hd)
    del hd
    xd = to_dev(x, torch.complex128)
    P.convolve(xd, out=xd)  # in place
    y = to_host(xd).reshape(-1)
    del xd
    P.close()
    torch.cuda.empty_cache()
    idx = rng.integers(0, y.size, 8)
    idx[0], idx[1] = 0, y.size - 1
    ref = oracle.conv_direct_at(x, h, idx)
    check_close(y[idx], ref, TOL[torch.complex128], what="16384^2 c128 sampled")
