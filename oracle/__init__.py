"""CPU oracle for FFT-based circular convolution (arXiv 2506.12718).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark may import this package; the GPU library and its Python
binding never do, and this package imports nothing from them.

Two independent routes to the same exact result, both in FP64 (the paper's
precision, complex double):

* ``conv_direct`` / ``conv_direct_at`` -- the definition of circular
  convolution, y_j = sum_k x_k h_{(j-k) mod n} per axis, summed directly in
  long double (Sec. "1D problem", eq. convolution, and its d-way form
  eq. convolution-multi-dimensional).  That this sum equals
  DFT^{-1}(DFT(h) o DFT(x)) is the circular-convolution theorem with the
  paper's sign convention w_n = exp(-2 pi i / n) and the 1/n on the inverse.
* ``conv_fft`` -- the paper's *standard* route with explicit index reversal,
  F = A_rho P_rho^T and F^{-1} = conj(A_rho) P_rho^T / n, per axis
  (Alg. alg:fft-based-convolution, Sec. "Mixed-radix framework").

``perm_index`` builds P_rho from its definition as a product of perfect
shuffles, and ``unordered_spectrum`` gives (A^T (x) ... (x) A^T) x = P^T F x,
the digit-reversed spectrum that the permutation-avoiding forward transform
leaves behind.  ``dense`` builds the same matrices densely for tiny n.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc (-O2, OpenMP, no fast-math)."""
    if (not force and os.path.exists(_LIB)
            and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC)):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
           "-fno-fast-math", "-o", tmp, _SRC, "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, _LIB)
    return _LIB


def _bind(path):
    lib = ctypes.CDLL(path)
    i64p = ctypes.POINTER(ctypes.c_int64)
    dp = ctypes.POINTER(ctypes.c_double)
    ip = ctypes.POINTER(ctypes.c_int)
    lib.orc_conv_direct.argtypes = [ctypes.c_int, i64p, dp, dp, dp]
    lib.orc_conv_direct_at.argtypes = [ctypes.c_int, i64p, dp, dp,
                                       ctypes.c_int64, i64p, dp]
    lib.orc_perm_index.argtypes = [ctypes.c_int64, ctypes.c_int, ip, i64p]
    lib.orc_fft.argtypes = [ctypes.c_int, i64p, ip, ip, ctypes.c_int, dp]
    lib.orc_conv_fft.argtypes = [ctypes.c_int, i64p, ip, ip, dp, dp, dp]
    lib.orc_num_threads.argtypes = []
    for f in (lib.orc_conv_direct, lib.orc_conv_direct_at,
              lib.orc_perm_index, lib.orc_fft, lib.orc_conv_fft,
              lib.orc_num_threads):
        f.restype = ctypes.c_int
    return lib


def _load():
    global _lib
    with _lock:
        if _lib is None:
            build()
            _lib = _bind(_LIB)
    return _lib


class use_library:
    """Context manager that points this module at another build of oracle.c
    (used by the tests that plant mistakes in a copy of the source)."""

    def __init__(self, path):
        self.path = path

    def __enter__(self):
        global _lib
        _load()
        self.saved = _lib
        _lib = _bind(self.path)
        return self

    def __exit__(self, *exc):
        global _lib
        _lib = self.saved
        return False


def compile_variant(source_text, out_path):
    """Compile a (modified) copy of oracle.c to ``out_path``."""
    src = out_path + ".c"
    with open(src, "w") as f:
        f.write(source_text)
    subprocess.check_call(["gcc", "-O1", "-fopenmp", "-fPIC", "-shared",
                           "-std=c11", "-o", out_path, src, "-lm"])
    return out_path


def source_text():
    with open(_SRC) as f:
        return f.read()


def num_threads() -> int:
    """Threads the oracle's OpenMP loops use."""
    return int(_load().orc_num_threads())


def _c128(a):
    a = np.ascontiguousarray(a, dtype=np.complex128)
    return a


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _dims(shape):
    d = np.ascontiguousarray(shape, dtype=np.int64)
    return d, d.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))


def conv_direct(x, h):
    """Direct circular convolution of two equal-shape complex arrays (1-3 D)."""
    x = _c128(x)
    h = _c128(h)
    assert x.shape == h.shape and 1 <= x.ndim <= 3
    y = np.empty_like(x)
    d, dp = _dims(x.shape)
    rc = _load().orc_conv_direct(x.ndim, dp, _dp(x), _dp(h), _dp(y))
    if rc != 0:
        raise RuntimeError("orc_conv_direct failed: %d" % rc)
    return y


def conv_direct_at(x, h, flat_idx):
    """Selected entries (row-major flat indices) of the direct convolution."""
    x = _c128(x)
    h = _c128(h)
    idx = np.ascontiguousarray(flat_idx, dtype=np.int64)
    out = np.empty(idx.size, dtype=np.complex128)
    d, dp = _dims(x.shape)
    rc = _load().orc_conv_direct_at(
        x.ndim, dp, _dp(x), _dp(h), idx.size,
        idx.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), _dp(out))
    if rc != 0:
        raise RuntimeError("orc_conv_direct_at failed: %d" % rc)
    return out


def perm_index(rho):
    """perm with (P_rho z)[i] = z[perm[i]], rho listed r_1 first."""
    rho_a = np.ascontiguousarray(rho, dtype=np.int32)
    n = int(np.prod(rho_a, dtype=np.int64))
    perm = np.empty(n, dtype=np.int64)
    rc = _load().orc_perm_index(
        n, rho_a.size, rho_a.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
        perm.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
    if rc != 0:
        raise RuntimeError("orc_perm_index failed: %d" % rc)
    return perm


def _rho_args(shape, rhos):
    if rhos is None:
        rhos = [default_rho(n) for n in shape]
    rhos = [list(r) for r in rhos]
    assert len(rhos) == len(shape)
    for n, r in zip(shape, rhos):
        assert int(np.prod(r)) == n, (n, r)
    flat = np.ascontiguousarray([v for r in rhos for v in r], dtype=np.int32)
    lens = np.ascontiguousarray([len(r) for r in rhos], dtype=np.int32)
    return (flat, lens, flat.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
            lens.ctypes.data_as(ctypes.POINTER(ctypes.c_int)))


def default_rho(n):
    """A radix sequence of n over {2, 3, 5} (the oracle's own choice)."""
    rho = []
    for p in (2, 3, 5):
        while n % p == 0:
            rho.append(p)
            n //= p
    if n != 1:
        raise ValueError("size has a prime factor outside {2, 3, 5}")
    return rho


def fft(x, rhos=None, inverse=False):
    """Ordered DFT (or inverse DFT) along every axis, standard route."""
    y = _c128(x).copy()
    d, dp = _dims(y.shape)
    flat, lens, fp, lp = _rho_args(y.shape, rhos)
    rc = _load().orc_fft(y.ndim, dp, fp, lp, 1 if inverse else -1, _dp(y))
    if rc != 0:
        raise RuntimeError("orc_fft failed: %d" % rc)
    return y


def conv_fft(x, h, rhos=None):
    """Standard FFT-based convolution with explicit index reversal."""
    x = _c128(x)
    h = _c128(h)
    assert x.shape == h.shape
    y = np.empty_like(x)
    d, dp = _dims(x.shape)
    flat, lens, fp, lp = _rho_args(x.shape, rhos)
    rc = _load().orc_conv_fft(x.ndim, dp, fp, lp, _dp(x), _dp(h), _dp(y))
    if rc != 0:
        raise RuntimeError("orc_conv_fft failed: %d" % rc)
    return y


def unordered_spectrum(x, rhos):
    """(A_rho1^T (x) ... (x) A_rhod^T) vec(x) = P^T F x per axis.

    Since F = P_rho A_rho^T (Sec. "Mixed-radix framework"), A^T = P^T F; with
    (P z)[i] = z[perm[i]], entry perm[k] of A^T x is entry k of F x.
    """
    spec = fft(x, rhos)
    out = np.empty_like(spec)
    out[...] = spec
    for ax, rho in enumerate(rhos):
        perm = perm_index(rho)
        src = np.moveaxis(out, ax, -1).copy()
        dst = np.empty_like(src)
        dst[..., perm] = src
        out = np.moveaxis(dst, -1, ax)
    return np.ascontiguousarray(out)
