"""GPU parity at the full sizes and in the plans the benchmark times for the
workloads beyond the headline configurations: the anisotropic grids
2^24 x 2 and 2^22 x 2 x 2 (radix 4 on the long axis, 2 on the short ones)
and the 256^3 periodic Poisson solve.  The convolutions are checked on
sampled outputs against the oracle's long-double direct sum (O(N) per
output), the Poisson solve against the oracle's symbol route on the whole
array and against the 7-point stencil itself.  Tolerances: relative L2
<= 1e-12 (complex128), <= 1e-5 (complex64, oracle on the rounded inputs)."""
import sys

import numpy as np
import pytest

import oracle
from oracle import symbols
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


@pytest.mark.parametrize("shape,radix,seed", [(inputs.ANISO_2D, [4, 2], 41),
                                              (inputs.ANISO_3D, [4, 2, 2], 42)])
@pytest.mark.parametrize("dtype", [C128, C64])
def test_anisotropic_full_size_sampled(shape, radix, seed, dtype):
    say("aniso full", shape, dtype)
    x, h = inputs.anisotropic_case(seed, shape)
    P = pafc().Plan(shape, dtype, radix=radix)
    P.set_filter(to_dev(h, dtype))
    y = to_host(P.convolve(to_dev(x, dtype))).reshape(-1)
    P.close()
    idx = np.random.default_rng(seed + 100).integers(0, y.size, 24)
    idx[0] = 0
    idx[1] = y.size - 1
    ref = oracle.conv_direct_at(rounded(x, dtype), rounded(h, dtype), idx)
    check_close(y[idx], ref, TOL[dtype], what="sampled")


@pytest.mark.parametrize("dtype", [C128, C64])
def test_poisson_full_size(dtype):
    shape = (256, 256, 256)
    f = inputs.complex_normal(np.random.default_rng(43), shape)
    P = pafc().Plan(shape, dtype, radix=[4, 4, 4])
    P.set_symbol("inv_laplacian_fd")
    y = to_host(P.convolve(to_dev(f, dtype)))
    P.close()
    fr = rounded(f, dtype)
    ref = symbols.apply(fr, symbols.inv_laplacian_fd(shape))
    check_close(y, ref, TOL[dtype], what="poisson 256^3 %s" % dtype)
    if dtype == C128:
        lap = -6.0 * y
        for ax in range(3):
            lap = lap + np.roll(y, 1, axis=ax) + np.roll(y, -1, axis=ax)
        check_close(lap, fr - fr.mean(), 1e-11)
