"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every symbol the header declares, and the planner's host-only entry point
reports the expected plans and errors."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2506_12718_amd as pafc
from oracle import dense

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_symbols():
    src = open(os.path.join(ROOT, "include", "pafc.h")).read()
    return sorted(set(re.findall(r"\b(pafc_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = pafc.lib()
    syms = header_symbols()
    assert len(syms) >= 17
    for s in syms:
        assert hasattr(L, s), s
    assert sorted(pafc.EXPORTS) == syms


def test_status_strings():
    L = pafc.lib()
    for st in range(6):
        assert L.pafc_status_string(st)


@pytest.mark.parametrize("dims,dtype,radix,passes,hbm_factor", [
    ((4096,), "c128", 2, 1, 3),
    ((4096,), "c128", 4, 1, 3),
    ((256, 256, 256), "c128", 4, 5, 11),
    ((256, 256, 256), "c64", 4, 5, 11),
    ((2187, 2187), "c128", 3, 5, 11),  # strided axis cut into two pieces
    ((5 ** 9,), "c128", 5, 3, 7),
    ((5 ** 9,), "c64", 5, 3, 7),
])
def test_describe_pass_structure(dims, dtype, radix, passes, hbm_factor):
    d = pafc.describe(dims, dtype, radix)
    N = int(np.prod(dims))
    elem = 16 if dtype == "c128" else 8
    assert len(d["conv_passes"]) == passes
    assert d["hbm_bytes_conv"] == hbm_factor * N * elem
    for ax in d["axes"]:
        assert all(r == radix for r in ax["rho"])
    # the product with the spectrum sits in exactly one pass
    assert sum("MID" in p for p in d["conv_passes"]) == 1


def test_describe_explicit_and_unfused():
    N = 256 ** 3
    d = pafc.describe((256, 256, 256), "c128", 4, "explicit_perm")
    assert d["hbm_bytes_conv"] == 17 * 16 * N
    assert sum("permute" in p for p in d["conv_passes"]) == 2
    d = pafc.describe((256, 256, 256), "c128", 4, "perm_free_unfused")
    assert d["hbm_bytes_conv"] == 15 * 16 * N


@pytest.mark.parametrize("n", [2, 6, 64, 96, 729, 1000, 3125, 4096, 65536, 78125, 59049])
def test_auto_radix_factorizes(n):
    d = pafc.describe((n,), "c128")
    rho = d["axes"][0]["rho"]
    assert int(np.prod(rho)) == n
    assert all(r in (2, 3, 4, 5, 8) for r in rho)


def test_describe_errors():
    with pytest.raises(pafc.PafcError) as e:  # Bluestein is 1-D only
        pafc.describe((7, 4), "c128")
    assert e.value.status == 2
    with pytest.raises(pafc.PafcError) as e:
        pafc.describe((1,), "c128")
    assert e.value.status == 1
    with pytest.raises(pafc.PafcError) as e:
        pafc.describe((32,), "c128", 4)
    assert e.value.status == 2
    with pytest.raises(pafc.PafcError) as e:
        pafc.describe((2, 2, 2, 2), "c128")
    assert e.value.status == 1
    # a long strided axis is cut into as many pieces as its tiles need
    d = pafc.describe((5 ** 9, 2), "c128")
    assert len(d["axes"][0]["pieces"]) == 3
    L = 1
    for p in d["axes"][0]["pieces"]:
        L *= p["L"]
    assert L == 5 ** 9


def test_tuning_override_changes_split():
    try:
        pafc.set_tuning("c128 65536 1024 0\n")
        d = pafc.describe((65536,), "c128")
        assert [p["L"] for p in d["axes"][0]["pieces"]] == [64, 1024]
    finally:
        pafc.set_tuning(None)
    d = pafc.describe((65536,), "c128")
    assert [p["L"] for p in d["axes"][0]["pieces"]] == [16, 4096]
    with pytest.raises(pafc.PafcError):
        pafc.set_tuning("garbage line")


def test_infeasible_tuning_entry_falls_back_to_defaults():
    # single radix-3 groups suit the 2187 axis of a 2187 x 2187 grid (cut
    # into pieces) but would give a 2187-point 1-D middle pass 13 ops
    try:
        pafc.set_tuning("c128 2187 0 0 0 1 0\n")
        grid = pafc.describe((2187, 2187), "c128")
        assert any("DIF3,DIF3" in s for s in grid["conv_passes"])
        one = pafc.describe((2187,), "c128")
        assert not any("DIF3," in s for s in one["conv_passes"])
    finally:
        pafc.set_tuning(None)
    assert pafc.describe((2187,), "c128")["conv_passes"] == one["conv_passes"]


def test_inner_piece_grouping_and_radix9_pieces():
    # g3 = 2 with g3i = 1: the 2187 x 2187 grid's contiguous axis runs
    # radix-9 groups ending in a radix-3 one (9 x 9 x 9 x 3), its strided
    # axis's 9-long outer piece one radix-9 group, and the inner 243-long
    # piece (the middle pass) single radix-3 stages -- all pipelined
    try:
        pafc.set_tuning("c128 2187 0 0 0 2 0 1\n")
        grid = pafc.describe((2187, 2187), "c128")["conv_passes"]
        assert "[DIF9,DIF9,DIF9,DIF3] pipe_kernel<double,3,2,4,0,0,1,0>" in grid[0], grid
        assert "[DIF9] pipe_kernel<double,3,2,1,0,2>" in grid[1], grid
        assert "[DIF3,DIF3,DIF3,DIF3,MID3,DIT3,DIT3,DIT3,DIT3] pipe_kernel<double,3,1,5,2,1>" in grid[2], grid
        assert "[DIT3,DIT9,DIT9,DIT9] pipe_kernel<double,3,2,4,1,0,1,0>" in grid[4], grid
        # g3i = 2 puts radix-9 groups in the inner piece too
        pafc.set_tuning("c128 2187 0 0 0 2 0 2\n")
        grid = pafc.describe((2187, 2187), "c128")["conv_passes"]
        assert "[DIF9,DIF9,MID3,DIT9,DIT9] pipe_kernel<double,3,2,3,2,1,1,0>" in grid[2], grid
    finally:
        pafc.set_tuning(None)
    with pytest.raises(pafc.PafcError):
        pafc.set_tuning("c128 2187 0 0 0 2 0 4\n")


def test_outer_pieces_take_the_pipelined_kernel(monkeypatch):
    # one-stage radix-5 groups: 5^9 is cut into 625 x 3125, and the 625-long
    # outer pieces run the pipelined kernel in its outer-piece mode, one
    # thread per item (125 items x 8 columns); the 2187^2 grid's 9-long
    # outer pieces too; PAFC_PIPE_OUTER=0 keeps them on the general engine
    try:
        pafc.set_tuning("c128 1953125 0 0 0 0 1\nc128 2187 0 0 0 1 0\n")
        one = pafc.describe((5 ** 9,), "c128")["conv_passes"]
        outer = [l for l in one if l.endswith(",2>")]
        assert len(outer) == 2 and all("L=625 W=8" in l and "thr=1000" in l for l in outer), one
        grid = pafc.describe((2187, 2187), "c128")["conv_passes"]
        assert sum(l.endswith(",2>") and "L=9 " in l for l in grid) == 2, grid
        monkeypatch.setenv("PAFC_PIPE_OUTER", "0")
        assert not any(l.endswith(",2>") for l in pafc.describe((5 ** 9,), "c128")["conv_passes"])
        assert not any(l.endswith(",2>") for l in pafc.describe((2187, 2187), "c128")["conv_passes"])
    finally:
        pafc.set_tuning(None)


def _smooth(n):
    for q in (2, 3, 5):
        while n % q == 0:
            n //= q
    return n == 1


def test_every_descriptor_passes_the_host_bounds_check():
    """pafc_describe runs the planner's bounds check (the kernels' own index
    formulas) on every pass; any shape it accepts is in bounds."""
    import itertools
    for dt in ("c128", "c64"):
        for n in [n for n in range(2, 100000) if _smooth(n)][::7] + [5 ** 9, 2 ** 20, 3 ** 12]:
            pafc.describe((n,), dt)
        for a, b in itertools.product([2, 3, 81, 100, 2187], [2, 9, 125, 729, 4096]):
            pafc.describe((a, b), dt)
        for a, b, c in itertools.product([2, 32, 81, 256], [3, 48, 256], [2, 100, 256]):
            pafc.describe((a, b, c), dt)


def _exact_omega(n, e, digits=40):
    """cos/sin of 2 pi e / n to `digits` digits with the decimal module."""
    from decimal import Decimal, getcontext
    getcontext().prec = digits + 10
    pi = Decimal(0)
    # Machin's formula
    def atan_inv(x):
        x = Decimal(x)
        t, k, s = 1 / x, 0, Decimal(0)
        while True:
            term = t / (2 * k + 1) * (-1) ** k
            if abs(term) < Decimal(10) ** -(digits + 5):
                break
            s += term
            t /= x * x
            k += 1
        return s
    pi = 16 * atan_inv(5) - 4 * atan_inv(239)
    a = 2 * pi * (e % n) / n
    c, s_, term, k = Decimal(0), Decimal(0), Decimal(1), 0
    while abs(term) > Decimal(10) ** -(digits + 5) or k < 4:
        c += term
        k += 2
        term = -term * a * a / (k * (k - 1))
    term, k = a, 1
    while abs(term) > Decimal(10) ** -(digits + 5):
        s_ += term
        k += 2
        term = -term * a * a / (k * (k - 1))
    return float(c), float(-s_)


def test_twiddles_exact_points_and_rounding():
    """Twiddle generation: exact at multiples of pi/4, correctly rounded (to
    within 1 ulp) elsewhere, conjugate-symmetric."""
    import math
    for n in (8, 16, 256, 4096, 2187, 3125, 1953125, 65536 * 3):
        for k in range(8):
            if (k * n) % 8:
                continue
            w = pafc.twiddle(n, k * n // 8)
            h = math.sqrt(0.5)
            ref = [(1, 0), (h, -h), (0, -1), (-h, -h), (-1, 0), (-h, h), (0, 1), (h, h)][k]
            assert w.real == ref[0] and w.imag == ref[1], (n, k, w)
    rng = np.random.default_rng(0)
    for n in (3, 5, 27, 2187, 3125, 78125, 1953125):
        for e in rng.integers(0, n, 12):
            w = pafc.twiddle(n, int(e))
            c, s = _exact_omega(n, int(e))
            assert abs(w.real - c) <= math.ulp(max(abs(c), 1e-300)) and \
                abs(w.imag - s) <= math.ulp(max(abs(s), 1e-300)), (n, e)
            wc = pafc.twiddle(n, n - int(e))
            assert wc.real == w.real and wc.imag == -w.imag or e == 0


def test_anisotropic_plans():
    """Host-only plans of the GPU anisotropic cases: the long axis is cut
    into the expected number of pieces, and the short faster axes fold into
    the fused middle pass (2 passes fewer per folded grid)."""
    import importlib.util, os
    spec = importlib.util.spec_from_file_location(
        "gpu_aniso_cases", os.path.join(os.path.dirname(__file__), "test_gpu_aniso.py"))
    # the case lists only; importing the module needs torch, which is present
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    for dims, radix, dtype, npieces in mod.ANISO:
        dt = "c128" if dtype == mod.C128 else "c64"
        d = pafc.describe(dims, dt, radix=radix)
        assert len(d["axes"][0]["pieces"]) == npieces, (dims, dt)
        if len(dims) > 1:
            assert any("XDIF" in l for l in d["conv_passes"]), (dims, dt)
            assert len(d["conv_passes"]) == 2 * npieces - 1, (dims, dt)
    for dims, radix, dtype in mod.FOLD:
        dt = "c128" if dtype == mod.C128 else "c64"
        d = pafc.describe(dims, dt, radix=radix)
        assert any("XDIF" in l for l in d["conv_passes"]), (dims, dt)


def test_bluestein_plans():
    """A 1-D length with a prime factor above 5 (other than a prime that
    Rader's method takes) runs by Bluestein's method on an inner convolution
    of the smallest {2,3,5}-smooth length >= 2n - 1."""
    for n in (23, 1009, 4099, 1000003, 1001, 14):
        d = pafc.describe((n,), "c128")
        m = d["bluestein_m"]
        assert m >= 2 * n - 1
        k = m
        for p in (2, 3, 5):
            while k % p == 0:
                k //= p
        assert k == 1
        for c in range(2 * n - 1, m):  # m is the smallest such length
            for p in (2, 3, 5):
                while c % p == 0:
                    c //= p
            assert c != 1
        inner = len(d["inner"]["conv_passes"])
        assert len(d["conv_passes"]) == 2 * inner + 3
    with pytest.raises(pafc.PafcError):
        pafc.describe((7, 7), "c128")


def test_rader_plans(monkeypatch):
    """A prime p with p - 1 {2,3,5}-smooth runs by Rader's method: the
    reported generator generates the multiplicative group mod p, the inner
    convolution has length p - 1; PAFC_BLUESTEIN=1 switches to Bluestein."""
    for n in (7, 11, 13, 17, 97, 257, 769, 65537, 786433, 995329):
        d = pafc.describe((n,), "c128")
        g = d["rader_generator"]
        assert d["rader_inner"] == n - 1
        for q in (2, 3, 5):
            if (n - 1) % q == 0:
                assert pow(g, (n - 1) // q, n) != 1
        # the smallest generator: every smaller candidate has a proper order
        for c in range(2, g):
            assert any(pow(c, (n - 1) // q, n) == 1 for q in (2, 3, 5) if (n - 1) % q == 0)
        k = len(d["inner"]["conv_passes"])
        assert len(d["conv_passes"]) == 2 * k + 4
    for n in (23, 1009, 1000003):  # p - 1 not smooth
        assert "bluestein_m" in pafc.describe((n,), "c128")
    monkeypatch.setenv("PAFC_BLUESTEIN", "1")
    assert "bluestein_m" in pafc.describe((97,), "c128")


def test_size_limits_and_batch_argument_errors():
    """The planner's bounds on the host: up to 2^34 elements per array (the
    pass kernels switch from 32-bit to 64-bit offsets above 4 GiB), and the
    batched form's argument checks, which run before any device call."""
    d = pafc.describe((2 ** 14, 2 ** 14), "c128")  # 4 GiB per array
    assert not any("pipe_kernel" in l for l in d["conv_passes"])  # 64-bit engine
    d = pafc.describe((2 ** 13, 2 ** 14), "c128")  # 2 GiB: 32-bit offsets suffice
    assert any("pipe_kernel" in l for l in d["conv_passes"])
    for dims in [(2 ** 18, 2 ** 17), (2 ** 12, 2 ** 12, 2 ** 11)]:
        with pytest.raises(pafc.PafcError) as e:
            pafc.describe(dims, "c128")
        assert e.value.status == 2
    L = pafc.lib()
    h = ctypes.c_void_p()
    I64, I32 = ctypes.c_int64, ctypes.c_int
    cases = [
        (0, [], [], 1),                    # no problems
        (2, [64, 1], [0, 0], 1),           # a length below 2
        (2, [64, 128], [0, 0], 1),         # one filter, two lengths
        (2, [64, 64], [0, 1], 1),          # filter id out of range
        (1, [64], [0], 0),                 # no filters
    ]
    for count, sizes, fids, nf in cases:
        for form in (0, 1, 2, 3):
            st = L.pafc_batch_plan(ctypes.byref(h), count, (I64 * max(1, count))(*sizes),
                                   (I32 * max(1, count))(*fids), nf, 2, form, None)
            assert st == 1, (count, sizes, fids, nf, form)
            assert not h.value
    # a form that does not exist
    st = L.pafc_batch_plan(ctypes.byref(h), 1, (I64 * 1)(64), (I32 * 1)(0), 1, 2, 4, None)
    assert st == 1 and not h.value
    # a length with a prime factor above 5 (no pass plan), after a valid one
    for form in (0, 1, 3):
        st = L.pafc_batch_plan(ctypes.byref(h), 2, (I64 * 2)(64, 97), (I32 * 2)(0, 1), 2, 2, form,
                               None)
        assert st == 2 and not h.value


def test_stream_probe_argument_checks():
    """pafc_stream_copy rejects unknown kinds and, for the tile probes, sizes
    that are not whole 256-row x 16-column tiles -- before any device call."""
    L = pafc.lib()
    a, b = ctypes.c_void_p(1 << 20), ctypes.c_void_p(2 << 20)  # aligned, never dereferenced
    assert L.pafc_stream_copy(a, b, 1 << 16, 5, None) == 1
    assert L.pafc_stream_copy(a, b, 1 << 16, -1, None) == 1
    for kind in (3, 4):
        assert L.pafc_stream_copy(a, b, (1 << 16) + 16, kind, None) == 1
        assert L.pafc_stream_copy(a, b, 4096, kind, None) == 1
