"""GPU parity of pafc_set_symbol: diagonal operators applied between the
unordered transforms, the spectrum written on the device in the plan's
digit-reversed layout, checked against the oracle's symbols applied by the
standard route (oracle/symbols.py).  Tolerances: relative L2 <= 1e-12
(complex128), <= 1e-5 (complex64, oracle on the same rounded input)."""
import sys

import numpy as np
import pytest

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


def ref_symbol(shape, kind, params):
    if kind == "inv_laplacian":
        return symbols.inv_laplacian(shape)
    if kind == "inv_laplacian_fd":
        return symbols.inv_laplacian_fd(shape)
    if kind == "heat":
        return symbols.heat(shape, params[0])
    return symbols.derivative(shape, int(params[0]))


SHAPES = [((64,), [4]), ((27, 32), None), ((16, 12, 10), None), ((8, 9, 10), None),
          ((2 ** 12, 2), [4, 2]), ((125,), [5])]


def kinds(ndim):
    out = [("inv_laplacian", ()), ("inv_laplacian_fd", ()), ("heat", (0.37,))]
    out += [("derivative", (float(a),)) for a in range(ndim)]
    return out


@pytest.mark.parametrize("shape,radix", SHAPES)
@pytest.mark.parametrize("variant", ["perm_free", "explicit_perm", "perm_free_unfused"])
@pytest.mark.parametrize("dtype", [C128, C64])
def test_symbols_match_oracle(shape, radix, variant, dtype):
    say("symbols", shape, variant, dtype)
    rng = np.random.default_rng(21)
    x = inputs.complex_uniform(rng, shape)
    P = pafc().Plan(shape, dtype, radix=radix, variant=variant)
    xd = to_dev(x, dtype)
    for kind, params in kinds(len(shape)):
        P.set_symbol(kind, *params)
        y = to_host(P.convolve(xd))
        ref = symbols.apply(rounded(x, dtype), ref_symbol(shape, kind, params))
        if not np.any(ref_symbol(shape, kind, params)):
            # e.g. the derivative along a length-2 axis: only k = 0 and the
            # dropped Nyquist frequency -- the zero operator
            say("  ", kind, params, "zero operator")
            assert not np.any(y)
            continue
        check_close(y, ref, TOL[dtype], what="%s %s" % (kind, params))
    P.close()


@pytest.mark.parametrize("shape,radix", SHAPES)
@pytest.mark.parametrize("variant", ["perm_free", "explicit_perm", "perm_free_unfused"])
@pytest.mark.parametrize("dtype", [C128, C64])
def test_gaussian_symbol_is_the_wrapped_gaussian_filter(shape, radix, variant, dtype):
    """The GAUSSIAN symbol (closed-form spectrum by Poisson summation) gives
    the convolution with the unit-sum periodic Gaussian formed in space and
    transformed by the oracle's standard route, at narrow, medium and wide
    filters."""
    import oracle
    rng = np.random.default_rng(23)
    x = inputs.complex_uniform(rng, shape)
    P = pafc().Plan(shape, dtype, radix=radix, variant=variant)
    xd = to_dev(x, dtype)
    for sigma in (0.3, 1.7, 8.0):
        P.set_symbol("gaussian", sigma)
        y = to_host(P.convolve(xd))
        ref = oracle.conv_fft(rounded(x, dtype), inputs.wrapped_gaussian(shape, sigma))
        check_close(y, ref, TOL[dtype], what="gaussian sigma=%g" % sigma)
    for bad in (0.0, 0.01, -1.0, float("nan"), 2e6):
        with pytest.raises(pafc().PafcError):
            P.set_symbol("gaussian", bad)
    P.close()


def test_poisson_solve_inverts_the_stencil():
    """64^3 FP64: y = inverse FD Laplacian of f; the (2d+1)-point stencil of
    y gives back f minus its mean."""
    shape = (64, 64, 64)
    rng = np.random.default_rng(22)
    f = inputs.complex_normal(rng, shape)
    P = pafc().Plan(shape, C128, radix=[4, 4, 4])
    P.set_symbol("inv_laplacian_fd")
    y = to_host(P.convolve(to_dev(f, C128)))
    P.close()
    lap = -6.0 * y
    for ax in range(3):
        lap = lap + np.roll(y, 1, axis=ax) + np.roll(y, -1, axis=ax)
    check_close(lap, f - f.mean(), 1e-12)


def test_symbol_errors_and_replacement():
    P = pafc().Plan((16, 12), C128)
    with pytest.raises(pafc().PafcError):
        P.set_symbol("heat", -1.0)
    with pytest.raises(pafc().PafcError):
        P.set_symbol("heat")
    with pytest.raises(pafc().PafcError):
        P.set_symbol("derivative", 2.0)
    with pytest.raises(pafc().PafcError):
        P.set_symbol("derivative", 0.5)
    with pytest.raises(pafc().PafcError):
        P.set_symbol("inv_laplacian", 1.0)
    # a filter after a symbol replaces it
    rng = np.random.default_rng(23)
    x = inputs.complex_uniform(rng, (16, 12))
    h = np.zeros((16, 12), dtype=np.complex128)
    h[0, 0] = 1.0
    P.set_symbol("heat", 2.0)
    P.set_filter(to_dev(h, C128))
    y = to_host(P.convolve(to_dev(x, C128)))
    P.close()
    check_close(y, x, 1e-13)
