"""Seeded synthetic inputs for the convolution workloads.

This module holds random-number draws and input construction only: no step
of the convolution method, no FFT, no twiddle.  It imports nothing from the
rest of this package nor from the oracle, so the GPU path and the CPU oracle
can both be fed the very same arrays.

Generator: numpy PCG64 via ``default_rng(seed)``, in FP64 on the host.  A
complex array of shape s is drawn as its real part (shape s), then its
imaginary part (shape s).  Where a workload has both an input and a filter,
the input is drawn first.  FP32 runs use the FP64 draws rounded to nearest.
"""
from __future__ import annotations

import math

import numpy as np


def complex_uniform(rng, shape):
    """Real and imaginary parts iid Uniform[-1, 1]."""
    re = rng.uniform(-1.0, 1.0, size=shape)
    im = rng.uniform(-1.0, 1.0, size=shape)
    return re + 1j * im


def complex_normal(rng, shape):
    """Real and imaginary parts iid N(0, 1)."""
    re = rng.standard_normal(size=shape)
    im = rng.standard_normal(size=shape)
    return re + 1j * im


def wrapped_gaussian_1d(n, sigma):
    """exp(-j^2 / (2 sigma^2)) summed over all periodic images j + p n.

    The images are summed until their terms underflow relative to the
    central one (|j + p n| > 40 sigma is below 1e-340).
    """
    j = np.arange(n, dtype=np.float64)
    g = np.zeros(n)
    reach = int(math.ceil(40.0 * sigma / n)) + 1
    for p in range(-reach, reach + 1):
        g += np.exp(-((j + p * n) ** 2) / (2.0 * sigma * sigma))
    return g


def wrapped_gaussian(dims, sigma):
    """Separable periodic Gaussian on the torus, normalised to unit sum, im = 0."""
    out = np.ones((), dtype=np.float64)
    for n in dims:
        g = wrapped_gaussian_1d(int(n), sigma)
        out = np.multiply.outer(out, g / g.sum())
    return out.astype(np.complex128)


# ---------------------------------------------------------------- workloads

def conv1d_4096(seed=1, n=4096):
    """1-D, n = 2^12: x and h with re/im iid U[-1, 1] (x first)."""
    rng = np.random.default_rng(seed)
    x = complex_uniform(rng, (n,))
    h = complex_uniform(rng, (n,))
    return x, h


def conv3d_gaussian(seed=2, n=256, sigma=4.0):
    """3-D n^3 grid: x re/im iid N(0, 1); h = unit-sum wrapped Gaussian."""
    rng = np.random.default_rng(seed)
    x = complex_normal(rng, (n, n, n))
    h = wrapped_gaussian((n, n, n), sigma)
    return x, h


def spectral_filter_case(seed, shape):
    """x re/im iid U[-1, 1]; the filter is given as its natural-order
    spectrum with re/im iid N(0, 1) (x first)."""
    rng = np.random.default_rng(seed)
    x = complex_uniform(rng, shape)
    hhat = complex_normal(rng, shape)
    return x, hhat


ANISO_2D = (2 ** 24, 2)
ANISO_3D = (2 ** 22, 2, 2)
"""Anisotropic grids of the paper's n_1 >> n_2 (= n_3) tables, at the sizes
measured here: one long axis that does not fit any cache level, and short
axes of length 2."""


def anisotropic_case(seed, shape):
    """x and h re/im iid U[-1, 1] (x first)."""
    rng = np.random.default_rng(seed)
    x = complex_uniform(rng, shape)
    h = complex_uniform(rng, shape)
    return x, h


BATCH_SIZES = tuple([2 ** e for e in range(8, 17)]
                    + [3 ** e for e in range(6, 11)]
                    + [5 ** e for e in range(4, 8)])


def batched_problems(seed=4, count=4096, sizes=BATCH_SIZES):
    """Mixed-size 1-D batch.

    Sizes iid uniform over ``sizes``; then every input (problem order,
    re/im iid U[-1, 1]); then one filter per size class in ``sizes`` order
    (re/im iid U[-1, 1]).  Returns (size_of_problem, inputs, filters) where
    filters maps size -> array.
    """
    rng = np.random.default_rng(seed)
    which = rng.integers(0, len(sizes), size=count)
    psizes = [int(sizes[i]) for i in which]
    xs = [complex_uniform(rng, (n,)) for n in psizes]
    filters = {int(n): complex_uniform(rng, (int(n),)) for n in sizes}
    return psizes, xs, filters


SERVE_SIDES_2D = (64, 81, 128, 243, 256, 512, 729, 1024)
SERVE_SIDES_3D = (32, 64, 81, 128, 243, 256)
"""Isotropic grid sides of the served workload (radix-2 and radix-3 sides).

A 3-D grid of side 243 or 256 in FP32 is 115-128 MiB per array."""


def serving_requests(seed=5, count=2200, sides_2d=SERVE_SIDES_2D,
                     sides_3d=SERVE_SIDES_3D, filters_per_grid=8):
    """Request mix of the served workload.

    Each request: ndim 2 or 3 with p = 1/2, an isotropic side drawn uniformly
    from the list of that ndim, a filter id drawn uniformly from a pool of
    ``filters_per_grid`` per grid, and an input seed.  Filter widths are
    sigma ~ U[1, 8], drawn per (grid, filter id) from a separate stream so
    that they do not depend on the request order.
    """
    rng = np.random.default_rng(seed)
    reqs = []
    for i in range(count):
        nd = 2 if rng.uniform() < 0.5 else 3
        sides = sides_2d if nd == 2 else sides_3d
        side = int(sides[rng.integers(0, len(sides))])
        fid = int(rng.integers(0, filters_per_grid))
        reqs.append({"id": i, "dims": (side,) * nd, "filter": fid,
                     "x_seed": int(rng.integers(0, 2 ** 31 - 1))})
    return reqs


def serving_sigma(dims, fid, seed=5):
    """sigma ~ U[1, 8] of filter ``fid`` on grid ``dims``."""
    key = [seed, len(dims), int(dims[0]), int(fid)]
    return float(np.random.default_rng(key).uniform(1.0, 8.0))


def serving_input(req, dtype=np.complex64):
    rng = np.random.default_rng(req["x_seed"])
    return complex_uniform(rng, req["dims"]).astype(dtype)
