"""GPU parity for the anisotropic grids of the paper's n_1 >> n_2 tables, for
axes cut into three or more pieces, for twiddles read from the global table,
and for the filter-per-call entry point (pafc_convolve_with_filter).

Tolerances as everywhere: relative L2 <= 1e-12 (complex128), <= 1e-5
(complex64, oracle on the same rounded inputs).
"""
import os
import sys

import numpy as np
import pytest

import oracle
from paper_2506_12718_amd import inputs
from gpu_util import AGREE_C, TOL, check_close, rel_l2, rounded, to_dev, to_host, torch

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


def conv_gpu(x, h, dtype, radix):
    P = pafc().Plan(x.shape, dtype, radix=radix)
    P.set_filter(to_dev(h, dtype))
    y = to_host(P.convolve(to_dev(x, dtype)))
    P.close()
    return y


def ref_conv(x, h, dtype):
    return oracle.conv_fft(rounded(x, dtype), rounded(h, dtype))


def pieces(dims, dt, radix):
    d = pafc().describe(dims, dt, radix=radix)
    return [len(a["pieces"]) for a in d["axes"]], d["conv_passes"]


# shapes of the paper's anisotropic tables at sizes the oracle handles in
# seconds, and long axes cut into three pieces (checked below)
ANISO = [
    ((2 ** 20, 2), [4, 2], C128, 3),
    ((2 ** 20, 4), [4, 4], C128, 3),
    ((2 ** 16, 2, 2), [4, 2, 2], C128, 2),
    ((2 ** 18, 2), [2, 2], C64, 2),
    ((3 ** 12, 2), [3, 2], C128, 3),
    ((5 ** 8, 2), [5, 2], C64, 2),
    ((2 ** 22,), [4], C128, 2),
]


@pytest.mark.parametrize("dims,radix,dtype,npieces", ANISO)
def test_anisotropic_and_multilevel(dims, radix, dtype, npieces):
    dt = "c128" if dtype == C128 else "c64"
    got_pieces, labels = pieces(dims, dt, radix)
    say("aniso", dims, radix, dt, got_pieces, len(labels), "passes")
    rng = np.random.default_rng([len(dims), dims[0] % 100003, 1 if dt == "c128" else 2])
    x = inputs.complex_uniform(rng, dims)
    h = inputs.complex_uniform(rng, dims)
    y = conv_gpu(x, h, dtype, radix)
    check_close(y, ref_conv(x, h, dtype), TOL[dtype])


GLOBAL_TW = [
    ((4096, 64), [4, 4]),
    ((2187, 12), None),
    ((5 ** 6,), None),
    ((729, 100), None),
    ((2 ** 18, 2), [2, 2]),
]


@pytest.mark.parametrize("dims,radix", GLOBAL_TW)
@pytest.mark.parametrize("dtype", [C128, C64])
def test_global_table_twiddles(dims, radix, dtype, monkeypatch):
    """Every pass reading its twiddles from the global table instead of an
    LDS copy (the planner's fallback for very long axes, forced here)."""
    monkeypatch.setenv("PAFC_TUNE_TWG", "1")
    dt = "c128" if dtype == C128 else "c64"
    _, labels = pieces(dims, dt, radix)
    assert all(" twg" in l for l in labels), labels
    say("twg", dims, dt, len(labels), "passes")
    rng = np.random.default_rng(7)
    x = inputs.complex_uniform(rng, dims)
    h = inputs.complex_uniform(rng, dims)
    y = conv_gpu(x, h, dtype, radix)
    check_close(y, ref_conv(x, h, dtype), TOL[dtype])


FPC = [((32, 27, 20), None), ((4096,), [4]), ((729, 100), None), ((64, 64, 64), [4, 4, 4])]


@pytest.mark.parametrize("dims,radix", FPC)
@pytest.mark.parametrize("variant", ["perm_free", "explicit_perm", "perm_free_unfused"])
@pytest.mark.parametrize("dtype", [C128, C64])
def test_filter_per_call(dims, radix, variant, dtype):
    """pafc_convolve_with_filter equals pafc_set_filter + pafc_convolve bit
    for bit, matches the oracle, and leaves h as the plan's filter."""
    say("fpc", dims, variant, dtype)
    rng = np.random.default_rng(11)
    x = inputs.complex_uniform(rng, dims)
    h = inputs.complex_uniform(rng, dims)
    x2 = inputs.complex_uniform(rng, dims)
    h0 = inputs.complex_uniform(rng, dims)
    P = pafc().Plan(dims, dtype, radix=radix, variant=variant)
    xd, hd, x2d = to_dev(x, dtype), to_dev(h, dtype), to_dev(x2, dtype)
    P.set_filter(to_dev(h0, dtype))  # a different filter first
    y_fpc = to_host(P.convolve_with_filter(xd, hd))
    y_after = to_host(P.convolve(x2d))  # h is now the plan's filter
    P.set_filter(hd)
    y_set = to_host(P.convolve(xd))
    P.close()
    assert np.array_equal(y_fpc, y_set)
    check_close(y_fpc, ref_conv(x, h, dtype), TOL[dtype])
    check_close(y_after, ref_conv(x2, h, dtype), TOL[dtype])


def test_filter_per_call_rejects_aliasing():
    P = pafc().Plan((64,), C128)
    a = torch.zeros(64, dtype=C128, device="cuda")
    with pytest.raises(ValueError):
        P.convolve_with_filter(a, a, out=a)
    P.close()


FOLD = [
    ((64, 16), None, C128),
    ((4096, 8, 4), None, C128),
    ((1000, 2), None, C64),
    ((2 ** 16, 2), [4, 2], C128),
    ((2 ** 14, 2, 2), [4, 2, 2], C64),
    ((81, 8, 8), None, C128),
]


@pytest.mark.parametrize("dims,radix,dtype", FOLD)
def test_short_axes_folded_into_middle_pass(dims, radix, dtype, monkeypatch):
    """Short faster axes run as column ops inside the fused middle pass (one
    pass fewer each way per axis); same result as the plan that keeps them in
    passes of their own, and as the oracle."""
    dt = "c128" if dtype == C128 else "c64"
    _, labels = pieces(dims, dt, radix)
    say("fold", dims, dt, labels)
    assert any("XDIF" in l for l in labels)
    assert len(labels) == 2 * len(pafc().describe(dims, dt, radix=radix)["axes"][0]["pieces"]) - 1
    rng = np.random.default_rng([len(dims), dims[0], 3])
    x = inputs.complex_uniform(rng, dims)
    h = inputs.complex_uniform(rng, dims)
    y = conv_gpu(x, h, dtype, radix)
    ref = ref_conv(x, h, dtype)
    check_close(y, ref, TOL[dtype])
    monkeypatch.setenv("PAFC_FOLD", "0")
    _, labels0 = pieces(dims, dt, radix)
    assert not any("XDIF" in l for l in labels0)
    y0 = conv_gpu(x, h, dtype, radix)
    check_close(y, y0, TOL[dtype])


@pytest.mark.parametrize("dims,radix,dtype", FOLD)
@pytest.mark.parametrize("variant", ["explicit_perm", "perm_free_unfused"])
def test_folded_transforms_in_comparison_variants(dims, radix, dtype, variant, monkeypatch):
    """The comparison variants run the transforms alone, whose innermost
    forward and inverse passes of the slowest axis carry the folded short
    axes; same result as without folding, and as the oracle."""
    dt = "c128" if dtype == C128 else "c64"
    labels = pafc().describe(dims, dt, radix, variant)["conv_passes"]
    say("fold", variant, dims, dt, labels)
    assert any("XDIF" in l for l in labels) and any("XDIT" in l for l in labels)
    rng = np.random.default_rng([len(dims), dims[0], 4])
    x = inputs.complex_uniform(rng, dims)
    h = inputs.complex_uniform(rng, dims)
    P = pafc().Plan(dims, dtype, radix=radix, variant=variant)
    P.set_filter(to_dev(h, dtype))
    y = to_host(P.convolve(to_dev(x, dtype)))
    P.close()
    check_close(y, ref_conv(x, h, dtype), TOL[dtype])
    monkeypatch.setenv("PAFC_FOLD", "0")
    assert not any("XDIF" in l for l in pafc().describe(dims, dt, radix, variant)["conv_passes"])
    P = pafc().Plan(dims, dtype, radix=radix, variant=variant)
    P.set_filter(to_dev(h, dtype))
    y0 = to_host(P.convolve(to_dev(x, dtype)))
    P.close()
    check_close(y, y0, TOL[dtype])


@pytest.mark.parametrize("dims,radix", [((64, 16), None), ((4096, 8, 4), None), ((2 ** 14, 2, 2), [4, 2, 2])])
def test_folded_forward_layout(dims, radix, monkeypatch):
    """pafc_forward with folded short axes writes the same digit-reversed
    spectrum as the unfolded plan (to rounding: the same register groups per
    axis, in other kernels), and pafc_inverse undoes it."""
    rng = np.random.default_rng(5)
    x = inputs.complex_uniform(rng, dims)
    assert any("XDIF" in l for l in pafc().describe(dims, "c128", radix)["conv_passes"])
    P = pafc().Plan(dims, C128, radix=radix)
    z = to_host(P.forward(to_dev(x, C128)))
    back = to_host(P.inverse(to_dev(z, C128)))
    P.close()
    check_close(back, x, 1e-13)
    monkeypatch.setenv("PAFC_FOLD", "0")
    P = pafc().Plan(dims, C128, radix=radix)
    z0 = to_host(P.forward(to_dev(x, C128)))
    P.close()
    check_close(z, z0, 1e-14)


# middle passes on the pipelined kernel with folded length-2 columns
# (exchanged across lanes) and/or a shorter innermost group (16 x 16 x 4)
MIDX = [
    ((1024, 2, 2), None, C128),
    ((1024, 2, 2), None, C64),
    ((1024, 2), None, C128),
    ((4096, 2), None, C128),
    ((256, 2, 2), None, C64),
    ((2 ** 14, 2, 2), [4, 2, 2], C64),
    ((2 ** 16, 2), [4, 2], C128),
    ((2 ** 16, 2, 2), [4, 2, 2], C128),
    ((4096, 2), None, C64),
    ((2 ** 16, 2), [4, 2], C64),
]


@pytest.mark.parametrize("dims,radix,dtype", MIDX)
def test_folded_middle_pass_pipelined(dims, radix, dtype, monkeypatch):
    """The fused middle pass of an anisotropic grid runs on the pipelined
    kernel: against the oracle, against the general engine (PAFC_PIPE_MIDX=0)
    to a few ulps, and unchanged with its LDS poisoned."""
    dt = "c128" if dtype == C128 else "c64"
    _, labels = pieces(dims, dt, radix)
    mid = [l for l in labels if "MID" in l]
    say("midx", dims, dt, mid)
    assert len(mid) == 1 and "pipe_kernel" in mid[0] and "XDIF2" in mid[0]
    rng = np.random.default_rng([dims[0], len(dims), 17])
    x = inputs.complex_uniform(rng, dims)
    h = inputs.complex_uniform(rng, dims)
    y = conv_gpu(x, h, dtype, radix)
    check_close(y, ref_conv(x, h, dtype), TOL[dtype], "midx %s" % (dims,))
    monkeypatch.setenv("PAFC_LDS_POISON", "1")
    yp = conv_gpu(x, h, dtype, radix)
    assert np.array_equal(y, yp)
    monkeypatch.delenv("PAFC_LDS_POISON")
    monkeypatch.setenv("PAFC_PIPE_MIDX", "0")
    _, labels0 = pieces(dims, dt, radix)
    assert not any("pipe_kernel" in l and "MID" in l for l in labels0)
    y0 = conv_gpu(x, h, dtype, radix)
    check_close(y, y0, 2e-15 if dtype == C128 else 2e-6, "midx vs engine", elem_c=AGREE_C)


# forward and inverse passes with a short innermost group and/or folded
# columns (the comparison variants' and the transforms' passes of the
# anisotropic grids, and 1024-long contiguous axes)
EXT_ALL = [
    ((1024, 2, 2), None, C128),
    ((4096, 2), None, C64),
    ((2 ** 14, 2, 2), [4, 2, 2], C64),
    ((2 ** 16, 2), [4, 2], C128),
    ((64, 1024), None, C128),
    ((96, 1024), None, C64),
]


@pytest.mark.parametrize("dims,radix,dtype", EXT_ALL)
@pytest.mark.parametrize("variant", ["explicit_perm", "perm_free_unfused", "perm_free"])
def test_pipelined_short_and_folded_passes_every_kind(dims, radix, dtype, variant, monkeypatch):
    """Forward and inverse passes on the pipelined kernel with a shorter
    innermost group or folded length-2 columns: the convolution of every
    variant against the oracle, and the unordered forward transform against
    the general engine's (PAFC_PIPE_MIDX=0) to a few ulps."""
    dt = "c128" if dtype == C128 else "c64"
    labels = pafc().describe(dims, dt, radix=radix, variant=variant)["conv_passes"]
    ext = [l for l in labels if "pipe_kernel" in l and l.count(",") >= 7]
    say("ext", dims, dt, variant, ext)
    assert ext
    rng = np.random.default_rng([dims[0], len(dims), 23])
    x = inputs.complex_uniform(rng, dims)
    h = inputs.complex_uniform(rng, dims)
    P = pafc().Plan(dims, dtype, radix=radix, variant=variant)
    P.set_filter(to_dev(h, dtype))
    y = to_host(P.convolve(to_dev(x, dtype)))
    z = to_host(P.forward(to_dev(x, dtype))) if variant == "perm_free" else None
    P.close()
    check_close(y, ref_conv(x, h, dtype), TOL[dtype], "ext %s %s" % (dims, variant))
    if z is not None:
        monkeypatch.setenv("PAFC_PIPE_MIDX", "0")
        P = pafc().Plan(dims, dtype, radix=radix)
        z0 = to_host(P.forward(to_dev(x, dtype)))
        P.close()
        check_close(z, z0, 2e-15 if dtype == C128 else 2e-6, "forward vs engine", elem_c=AGREE_C)


# radix-16 outer pieces of cut axes on the pipelined kernel, with the axis's
# twiddles from the LDS copy or (forced: PAFC_TUNE_TWG) the global table
OUTER16 = [
    ((2 ** 20, 2), [4, 2], C128),
    ((2 ** 18, 2, 2), None, C64),
    ((2 ** 20, 4), [4, 4], C64),
]


@pytest.mark.parametrize("twg", [False, True])
@pytest.mark.parametrize("dims,radix,dtype", OUTER16)
def test_radix16_outer_pieces_pipelined(dims, radix, dtype, twg, monkeypatch):
    """Outer pieces of 256 positions (two radix-16 groups) with the whole
    axis's twiddles: against the oracle, and against the general engine
    (PAFC_PIPE_OUTER=0) to a few ulps."""
    if twg:
        monkeypatch.setenv("PAFC_TUNE_TWG", "1")
    dt = "c128" if dtype == C128 else "c64"
    labels = pafc().describe(dims, dt, radix=radix)["conv_passes"]
    outer = [l for l in labels if "L=256 W=16" in l and "pipe_kernel" in l]
    say("outer16", dims, dt, twg, outer)
    assert outer and all((" twg" in l) == twg for l in outer)
    rng = np.random.default_rng([dims[0], len(dims), 29])
    x = inputs.complex_uniform(rng, dims)
    h = inputs.complex_uniform(rng, dims)
    y = conv_gpu(x, h, dtype, radix)
    check_close(y, ref_conv(x, h, dtype), TOL[dtype], "outer16 %s" % (dims,))
    monkeypatch.setenv("PAFC_PIPE_OUTER", "0")
    assert not any("L=256 W=16" in l and "pipe_kernel" in l
                   for l in pafc().describe(dims, dt, radix=radix)["conv_passes"])
    y0 = conv_gpu(x, h, dtype, radix)
    check_close(y, y0, 4e-15 if dtype == C128 else 4e-6, "outer16 vs engine", elem_c=AGREE_C)
