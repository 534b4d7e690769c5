"""Pins for the CPU oracle against what the paper and mathematics fix.

None of these checks compares the oracle with itself: each side is either a
value the paper prints (tests/golden), a closed form, an invariant, a
brute-force evaluation of a definition on tiny inputs, or an independent
library routine (numpy.fft, corroboration only).
"""
import itertools
import os

import numpy as np
import pytest

import oracle
from oracle import dense as D
from paper_2506_12718_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
RNG = np.random.default_rng(12345)


def crand(shape, rng=RNG):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def smooth_sizes(limit):
    return [n for n in range(2, limit + 1)
            if all(p in (2, 3, 5) for p in _factors(n))]


def _factors(n):
    out, p = [], 2
    while n > 1:
        while n % p == 0:
            out.append(p)
            n //= p
        p += 1
    return out


def brute_dft(x, inverse=False):
    """sum_k x_k w^{jk} per axis, straight from the definition (tiny sizes)."""
    y = np.asarray(x, dtype=complex)
    for ax in range(y.ndim):
        n = y.shape[ax]
        j = np.arange(n)
        e = np.outer(j, j) % n
        mat = np.exp((2j if inverse else -2j) * np.pi * e / n)
        if inverse:
            mat = mat / n
        y = np.moveaxis(np.tensordot(mat, np.moveaxis(y, ax, 0), axes=(1, 0)), 0, ax)
    return y


def brute_conv(x, h):
    """y_j = sum_k x_k h_{(j-k) mod n}, pure Python loops (tiny sizes)."""
    shape = x.shape
    y = np.zeros(shape, dtype=complex)
    for j in itertools.product(*[range(n) for n in shape]):
        s = 0j
        for k in itertools.product(*[range(n) for n in shape]):
            hk = tuple((a - b) % n for a, b, n in zip(j, k, shape))
            s += x[k] * h[hk]
        y[j] = s
    return y


def rel_l2(a, b):
    return np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel())


# ------------------------------------------------------------ printed values

def _golden_matrices():
    a = (1 - 1j) / np.sqrt(2)
    b = -(1 + 1j) / np.sqrt(2)
    tok = {"1": 1, "-1": -1, "i": 1j, "-i": -1j, "a": a, "-a": -a, "b": b, "-b": -b}
    mats, cur = {}, None
    with open(os.path.join(GOLDEN, "fourier_small.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            if line in ("F4", "F8"):
                cur = line
                mats[cur] = []
                continue
            mats[cur].append([tok[t] for t in line.split()])
    return {k: np.array(v, dtype=complex) for k, v in mats.items()}


def test_printed_fourier_matrices_match_definition():
    g = _golden_matrices()
    assert np.abs(D.fourier(4) - g["F4"]).max() < 1e-15
    assert np.abs(D.fourier(8) - g["F8"]).max() < 1e-15


@pytest.mark.parametrize("n,rho", [(4, [4]), (4, [2, 2]), (8, [8]), (8, [2, 2, 2]),
                                   (8, [2, 4]), (8, [4, 2])])
def test_oracle_fft_of_unit_vectors_gives_printed_columns(n, rho):
    """FFT(e_k) must be column k of the printed F_n: pins the sign of w_n,
    the twiddles and the permutation of the oracle's standard route."""
    g = _golden_matrices()["F%d" % n]
    for k in range(n):
        e = np.zeros(n, complex)
        e[k] = 1
        assert np.abs(oracle.fft(e, [rho]) - g[:, k]).max() < 1e-15


def test_radix2_and_radix4_block_forms():
    """B_{2,k} = [[I, W], [I, -W]] and the radix-4 block rows (App. A)."""
    for k in (2, 4, 8, 16):
        m = k // 2
        W = np.diag(D.w(k, np.arange(m)))
        I = np.eye(m)
        assert np.abs(D.butterfly(2, k) - np.block([[I, W], [I, -W]])).max() < 1e-15
    k = 16
    m = k // 4
    W = np.diag(D.w(k, np.arange(m)))
    I = np.eye(m)
    W2, W3 = W @ W, W @ W @ W
    ref = np.block([[I, W, W2, W3],
                    [I, -1j * W, -W2, 1j * W3],
                    [I, -W, W2, -W3],
                    [I, 1j * W, -W2, -1j * W3]])
    assert np.abs(D.butterfly(4, k) - ref).max() < 1e-14


# ---------------------------------------------------- factorization identities

RHOS = [[2] * 4, [4] * 3, [8, 8], [3] * 4, [5] * 3, [2, 3, 4], [5, 2, 3], [4, 4, 2], [2, 8]]


@pytest.mark.parametrize("rho", RHOS)
def test_dense_factorization_identities(rho):
    n = int(np.prod(rho))
    F, A, P = D.fourier(n), D.a_rho(rho), D.p_rho(rho)
    assert np.abs(F - A @ P.T).max() < 1e-13            # F = A P^T
    assert np.abs(F - P @ A.T).max() < 1e-13            # F = P A^T
    assert np.abs(np.linalg.inv(F) - np.conj(A) @ P.T / n).max() < 1e-13
    if len(set(rho)) == 1:                               # uniform radix: P symmetric
        Pu = D.p_uniform(rho[0], len(rho))
        assert np.array_equal(P, Pu) and np.array_equal(P, P.T)


@pytest.mark.parametrize("rho", RHOS)
def test_convolution_without_permutation_dense(rho):
    """conj(A)((A^T h) o (A^T x))/n equals the convolution (eq. 35 and its
    mixed-radix form), checked against the direct sum."""
    n = int(np.prod(rho))
    A = D.a_rho(rho)
    x, h = crand(n), crand(n)
    y = np.conj(A) @ ((A.T @ h) * (A.T @ x)) / n
    assert rel_l2(y, brute_conv(x, h)) < 1e-13


@pytest.mark.parametrize("rho", RHOS)
def test_layout_law_pos(rho):
    """(A^T x)[pos(k)] = (F x)[k], and pos agrees with P_rho."""
    n = int(np.prod(rho))
    A = D.a_rho(rho)
    x = crand(n)
    pt = D.pos_table(rho)
    assert np.abs((A.T @ x)[pt] - brute_dft(x)).max() < 1e-12
    assert sorted(pt.tolist()) == list(range(n))
    # delta_0 -> all ones; delta_1 -> entry at pos(k) is w_n^k
    d0 = np.zeros(n, complex); d0[0] = 1
    assert np.abs(A.T @ d0 - 1).max() < 1e-13
    d1 = np.zeros(n, complex); d1[1] = 1
    assert np.abs((A.T @ d1)[pt] - D.w(n, np.arange(n))).max() < 1e-13


# ------------------------------------------------------- the C oracle, pinned

@pytest.mark.parametrize("rho", RHOS)
def test_perm_index_matches_dense_definition(rho):
    perm = oracle.perm_index(rho)
    P = D.p_rho(rho)
    n = len(perm)
    assert np.array_equal(P, np.eye(n)[perm])
    # (P z)[i] = z[perm[i]] and F = P A^T give (F x)[k] = (A^T x)[perm[k]],
    # so perm is the layout law pos
    assert np.array_equal(perm, D.pos_table(rho))


@pytest.mark.parametrize("n", smooth_sizes(64))
def test_oracle_fft_equals_definition_all_small_sizes(n):
    x = crand(n)
    rho = oracle.default_rho(n)
    for r in (rho, rho[::-1]):
        assert np.abs(oracle.fft(x, [r]) - brute_dft(x)).max() < 1e-12 * n
        assert np.abs(oracle.fft(x, [r], inverse=True) - brute_dft(x, True)).max() < 1e-13


@pytest.mark.parametrize("shape", [(4, 6), (3, 5), (8, 9), (2, 3, 4), (4, 4, 5), (5, 2, 8)])
def test_oracle_fft_equals_definition_multid(shape):
    x = crand(shape)
    assert np.abs(oracle.fft(x) - brute_dft(x)).max() < 1e-12
    assert np.abs(oracle.fft(x, inverse=True) - brute_dft(x, True)).max() < 1e-13
    np.testing.assert_allclose(oracle.fft(x), np.fft.fftn(x), atol=1e-12)


@pytest.mark.parametrize("shape", [(1,), (2,), (5,), (12,), (3, 4), (2, 2, 3), (4, 1, 3)])
def test_conv_direct_equals_python_definition(shape):
    x, h = crand(shape), crand(shape)
    assert np.abs(oracle.conv_direct(x, h) - brute_conv(x, h)).max() < 1e-13


@pytest.mark.parametrize("n", smooth_sizes(64))
def test_conv_fft_equals_direct_all_small_1d(n):
    x, h = crand(n), crand(n)
    ref = oracle.conv_direct(x, h)
    assert rel_l2(oracle.conv_fft(x, h), ref) < 1e-14
    assert rel_l2(oracle.conv_fft(x, h, [oracle.default_rho(n)[::-1]]), ref) < 1e-14


@pytest.mark.parametrize("shape", [(4, 4), (8, 6), (9, 5), (16, 12), (2, 4, 8), (4, 3, 5), (6, 6, 6)])
def test_conv_fft_equals_direct_small_multid(shape):
    x, h = crand(shape), crand(shape)
    assert rel_l2(oracle.conv_fft(x, h), oracle.conv_direct(x, h)) < 1e-14


def test_conv_direct_at_matches_full():
    x, h = crand((6, 10)), crand((6, 10))
    full = oracle.conv_direct(x, h).ravel()
    idx = np.array([0, 7, 33, 59])
    assert np.array_equal(oracle.conv_direct_at(x, h, idx), full[idx])


# --------------------------------------------------------------- invariants

def test_delta_identity_and_shift():
    x = crand((8, 9, 5))
    d = np.zeros_like(x); d[0, 0, 0] = 1
    assert np.abs(oracle.conv_fft(x, d) - x).max() < 1e-14
    s = (3, 4, 2)
    ds = np.zeros_like(x); ds[s] = 1
    assert np.abs(oracle.conv_fft(x, ds) - np.roll(x, s, axis=(0, 1, 2))).max() < 1e-14
    assert np.abs(oracle.conv_direct(x, ds) - np.roll(x, s, axis=(0, 1, 2))).max() == 0


def test_linearity_commutativity_shift_equivariance_dc():
    shape = (16, 27)
    x1, x2, h = crand(shape), crand(shape), crand(shape)
    a, b = 0.3 - 1.1j, 2.0 + 0.5j
    y = oracle.conv_fft(a * x1 + b * x2, h)
    assert rel_l2(y, a * oracle.conv_fft(x1, h) + b * oracle.conv_fft(x2, h)) < 1e-14
    assert rel_l2(oracle.conv_fft(h, x1), oracle.conv_fft(x1, h)) < 1e-14
    sh = np.roll(x1, (5, 7), axis=(0, 1))
    assert rel_l2(oracle.conv_fft(sh, h), np.roll(oracle.conv_fft(x1, h), (5, 7), axis=(0, 1))) < 1e-14
    y = oracle.conv_direct(x1, h)
    assert abs(y.sum() - x1.sum() * h.sum()) < 1e-11


def test_parseval_and_real_even_filter():
    x = crand((32, 24))
    X = oracle.fft(x)
    assert abs(np.vdot(X, X).real / x.size - np.vdot(x, x).real) < 1e-10
    g = inputs.wrapped_gaussian((32, 24), 3.0)
    G = oracle.fft(g)
    assert np.abs(G.imag).max() < 1e-15


# ---------------------------------------------------------------- closed forms

def theta(k, n, sigma, reach=60):
    m = np.arange(-reach, reach + 1)
    return np.exp(-2 * np.pi ** 2 * sigma ** 2 * (k / n + m) ** 2).sum()


@pytest.mark.parametrize("n,sigma", [(256, 4.0), (32, 8.0), (81, 1.0), (64, 2.5)])
def test_wrapped_gaussian_spectrum_closed_form(n, sigma):
    """Poisson summation: the DFT of the image-sum Gaussian is
    sum_m exp(-2 pi^2 sigma^2 (k/n + m)^2) up to a constant factor; the unit-sum
    normalisation makes entry 0 equal to 1."""
    g = inputs.wrapped_gaussian((n,), sigma)
    G = oracle.fft(g)
    ref = np.array([theta(k, n, sigma) for k in range(n)])
    ref = ref / ref[0]
    assert np.abs(G - ref).max() < 1e-14


def test_separable_gaussian_3d_equals_axis_by_axis():
    """A 3-D convolution with a separable filter equals three 1-D circular
    convolutions along the axes."""
    n, sigma = 16, 2.0
    x = crand((n, n, n))
    h = inputs.wrapped_gaussian((n, n, n), sigma)
    g = inputs.wrapped_gaussian((n,), sigma)
    y = x.copy()
    for ax in range(3):
        y = np.apply_along_axis(lambda v: oracle.conv_direct(v, g), ax, y)
    assert rel_l2(oracle.conv_fft(x, h), y) < 1e-14


def test_unordered_spectrum_is_dense_transposed_product():
    for rhos in ([[4, 4], [2, 3]], [[3, 3], [5]], [[2, 2, 2], [4], [3]]):
        shape = tuple(int(np.prod(r)) for r in rhos)
        x = crand(shape)
        mat = np.ones((1, 1))
        for r in rhos:
            mat = np.kron(mat, D.a_rho(r).T)
        ref = (mat @ x.ravel()).reshape(shape)
        assert np.abs(oracle.unordered_spectrum(x, rhos) - ref).max() < 1e-12


def test_numpy_fft_corroboration_medium():
    x = crand((64, 45))
    np.testing.assert_allclose(oracle.fft(x), np.fft.fftn(x), atol=1e-11)
    x, h = crand(4096), crand(4096)
    y = oracle.conv_fft(x, h, [[4] * 6])
    assert rel_l2(y, np.fft.ifft(np.fft.fft(x) * np.fft.fft(h))) < 1e-14


@pytest.mark.parametrize("factors", [(2, 3), (4, 5), (3, 8), (2, 3, 5), (4, 9, 5)])
def test_prime_factor_reindexing_is_an_isomorphism_of_convolutions(factors):
    """Sec. "Prime factor framework": for pairwise coprime N_q and n = prod
    N_q, j -> (j mod N_q)_q maps the length-n circular convolution onto the
    grid convolution (Chinese remainder theorem), so the prime-factor route
    reindexes x and h, convolves on the grid and maps back.  Checked with the
    direct sum on both sides."""
    n = int(np.prod(factors))
    rng = np.random.default_rng(n)
    x = inputs.complex_uniform(rng, (n,))
    h = inputs.complex_uniform(rng, (n,))
    j = np.arange(n)
    grid_index = tuple(j % N for N in factors)
    xg = np.zeros(factors, dtype=np.complex128)
    hg = np.zeros(factors, dtype=np.complex128)
    xg[grid_index] = x
    hg[grid_index] = h
    yg = oracle.conv_direct(xg, hg)
    y = yg[grid_index]
    assert np.allclose(y, oracle.conv_direct(x, h), atol=1e-12 * n)
