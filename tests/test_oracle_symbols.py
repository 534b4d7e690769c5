"""Pins of the oracle's diagonal-operator symbols (CPU): each symbol against
a closed form that does not use it -- the finite-difference stencil applied
with array shifts, plane waves (eigenfunctions of every symbol), the heat
semigroup, and derivatives of trigonometric functions."""
import numpy as np
import pytest

import oracle
from oracle import symbols
from paper_2506_12718_amd import inputs

SHAPES = [(16,), (27,), (12, 10), (8, 9, 10), (5, 4, 6)]


def plane_wave(shape, k):
    grids = np.meshgrid(*[np.arange(n) for n in shape], indexing="ij")
    return np.exp(2j * np.pi * sum(ki * g / n for ki, g, n in zip(k, grids, shape)))


def laplacian_fd(u):
    out = -2.0 * u.ndim * u
    for ax in range(u.ndim):
        out = out + np.roll(u, 1, axis=ax) + np.roll(u, -1, axis=ax)
    return out


@pytest.mark.parametrize("shape", SHAPES)
def test_inverse_fd_laplacian_undoes_the_stencil(shape):
    rng = np.random.default_rng(1)
    u = inputs.complex_uniform(rng, shape)
    u = u - u.mean()
    f = laplacian_fd(u)
    assert abs(f.sum()) < 1e-9 * np.abs(f).sum()
    v = symbols.apply(f, symbols.inv_laplacian_fd(shape))
    assert np.abs(v - u).max() < 1e-12 * np.abs(u).max() * np.prod(shape)
    # and the stencil of the solution gives back the right-hand side
    assert np.allclose(laplacian_fd(v), f, atol=1e-11)


@pytest.mark.parametrize("shape", SHAPES)
def test_plane_waves_are_eigenfunctions(shape):
    rng = np.random.default_rng(2)
    for _ in range(4):
        k = [int(rng.integers(0, n)) for n in shape]
        u = plane_wave(shape, k)
        kt = [ki if 2 * ki <= n else ki - n for ki, n in zip(k, shape)]
        w2 = sum((2 * np.pi * t / n) ** 2 for t, n in zip(kt, shape))
        s2 = sum(4 * np.sin(np.pi * ki / n) ** 2 for ki, n in zip(k, shape))
        lam = -1.0 / w2 if w2 else 0.0
        assert np.allclose(symbols.apply(u, symbols.inv_laplacian(shape)), lam * u, atol=1e-11)
        lam = -1.0 / s2 if s2 else 0.0
        assert np.allclose(symbols.apply(u, symbols.inv_laplacian_fd(shape)), lam * u, atol=1e-11)
        assert np.allclose(symbols.apply(u, symbols.heat(shape, 0.7)), np.exp(-0.7 * w2) * u,
                           atol=1e-12)
        for ax in range(len(shape)):
            n = shape[ax]
            wa = 0.0 if 2 * k[ax] == n else 2 * np.pi * kt[ax] / n
            assert np.allclose(symbols.apply(u, symbols.derivative(shape, ax)), 1j * wa * u,
                               atol=1e-11)


def test_heat_semigroup_and_zero_time():
    shape = (8, 9, 10)
    rng = np.random.default_rng(3)
    x = inputs.complex_uniform(rng, shape)
    a = symbols.apply(symbols.apply(x, symbols.heat(shape, 0.3)), symbols.heat(shape, 0.5))
    b = symbols.apply(x, symbols.heat(shape, 0.8))
    assert np.allclose(a, b, atol=1e-13)
    assert np.allclose(symbols.apply(x, symbols.heat(shape, 0.0)), x, atol=1e-13)


def test_derivative_of_sine_and_real_input():
    n = 32
    j = np.arange(n)
    u = np.sin(2 * np.pi * 3 * j / n) + 0.5 * np.cos(2 * np.pi * 5 * j / n)
    du = (2 * np.pi * 3 / n) * np.cos(2 * np.pi * 3 * j / n) \
        - 0.5 * (2 * np.pi * 5 / n) * np.sin(2 * np.pi * 5 * j / n)
    got = symbols.apply(u, symbols.derivative((n,), 0))
    assert np.allclose(got, du, atol=1e-12)
    # a real input has a real derivative (the Nyquist term is dropped)
    rng = np.random.default_rng(4)
    r = rng.standard_normal(n)
    assert np.abs(symbols.apply(r, symbols.derivative((n,), 0)).imag).max() < 1e-12


def test_inverse_laplacian_removes_the_mean():
    shape = (12, 10)
    rng = np.random.default_rng(5)
    x = inputs.complex_uniform(rng, shape) + 3.0
    for sym in (symbols.inv_laplacian(shape), symbols.inv_laplacian_fd(shape)):
        y = symbols.apply(x, sym)
        assert abs(y.mean()) < 1e-13
