"""Diagonal operators of the DFT by their symbols (test infrastructure).

TEST INFRASTRUCTURE ONLY, like the rest of this package: the definitions the
GPU library's pafc_set_symbol is checked against, written from the
mathematics in FP64 numpy on the natural frequency grid, and their
application y = DFT^{-1}(S o DFT(x)) through the oracle's standard FFT route.

The permutation-avoiding scheme (Sec. "Permutation-avoiding convolution")
only needs the operation between the forward and inverse transforms to be
elementwise in the frequency basis, with both operands in the same
digit-reversed order; convolution is the case S = DFT(h), and fast Poisson
solvers are among the applications the Introduction names.  Frequencies are
signed, kt = k for 2k <= n and k - n otherwise, and w = 2 pi kt / n (unit
grid spacing, period n):

* ``inv_laplacian``     -1 / sum_i w_i^2, 0 at k = 0
* ``inv_laplacian_fd``  -1 / sum_i 4 sin^2(pi k_i / n_i), 0 at k = 0: the
                        eigenvalues of the (2d+1)-point Laplacian
                        u(j+e_i) - 2 u(j) + u(j-e_i) are -4 sin^2(pi k_i/n_i)
* ``heat``              exp(-t sum_i w_i^2)
* ``derivative``        i w_a along axis a, 0 at the Nyquist frequency of an
                        even axis
"""
from __future__ import annotations

import numpy as np

from . import fft


def signed_freq(n):
    k = np.arange(n)
    return np.where(2 * k <= n, k, k - n)


def _axis_grid(shape, i, values):
    s = [1] * len(shape)
    s[i] = shape[i]
    return np.asarray(values).reshape(s)


def _w2(shape):
    tot = np.zeros(shape)
    for i, n in enumerate(shape):
        w = 2 * np.pi * signed_freq(n) / n
        tot = tot + _axis_grid(shape, i, w * w)
    return tot


def _inv_neg(s):
    out = np.zeros(s.shape)
    nz = s != 0
    out[nz] = -1.0 / s[nz]
    return out


def inv_laplacian(shape):
    return _inv_neg(_w2(shape)).astype(np.complex128)


def inv_laplacian_fd(shape):
    tot = np.zeros(shape)
    for i, n in enumerate(shape):
        tot = tot + _axis_grid(shape, i, 4 * np.sin(np.pi * np.arange(n) / n) ** 2)
    return _inv_neg(tot).astype(np.complex128)


def heat(shape, t):
    return np.exp(-t * _w2(shape)).astype(np.complex128)


def derivative(shape, axis):
    n = shape[axis]
    w = 2 * np.pi * signed_freq(n) / n
    if n % 2 == 0:
        w[n // 2] = 0.0
    return np.broadcast_to(_axis_grid(shape, axis, 1j * w), shape).astype(np.complex128)


def apply(x, symbol):
    """y = DFT^{-1}(S o DFT(x)), the standard route (explicit index reversal)."""
    return fft(symbol * fft(x), inverse=True)
