"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Tolerances: relative L2 error <= 1e-12 for complex128 and <= 1e-5 for
complex64 (the oracle consumes the same FP32-rounded inputs, upcast), with the
error metric ||y - y_ref||_2 / ||y_ref||_2 over all entries.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2506_12718_amd import inputs
from gpu_util import AGREE_C, TOL, check_close, rel_l2, rounded, to_dev, to_host, torch

pytestmark = pytest.mark.gpu

C128, C64 = torch.complex128, torch.complex64
DTYPES = [C128, C64]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2506_12718_amd as pafc
    pafc.lib()  # fail loudly if the library is missing
    yield


def pafc():
    import paper_2506_12718_amd as m
    return m


def crand(rng, shape):
    return inputs.complex_uniform(rng, shape)


def run_conv(x, h, dtype, radix=None, variant="perm_free", domain="spatial"):
    P = pafc().Plan(x.shape, dtype, radix=radix, variant=variant)
    P.set_filter(to_dev(h, dtype), domain=domain)
    y = P.convolve(to_dev(x, dtype))
    out = to_host(y)
    rhos = [P.radices(a) for a in range(x.ndim)]
    P.close()
    return out, rhos


def smooth(limit):
    out = []
    for n in range(2, limit + 1):
        m = n
        for p in (2, 3, 5):
            while m % p == 0:
                m //= p
        if m == 1:
            out.append(n)
    return out


# ----------------------------------------------------------- brute force

@pytest.mark.parametrize("dtype", DTYPES)
def test_all_small_1d_sizes_against_direct(dtype):
    rng = np.random.default_rng(101)
    for n in smooth(64):
        x, h = crand(rng, (n,)), crand(rng, (n,))
        say("1d n=%d %s" % (n, dtype))
        y, _ = run_conv(x, h, dtype)
        ref = oracle.conv_direct(rounded(x, dtype), rounded(h, dtype))
        check_close(y, ref, TOL[dtype], what=str(n))


@pytest.mark.parametrize("shape", [(2, 2), (4, 6), (8, 9), (16, 25), (27, 12), (64, 64),
                                   (2, 3, 4), (4, 4, 4), (5, 8, 9), (16, 12, 10), (32, 9, 8)])
@pytest.mark.parametrize("dtype", DTYPES)
def test_small_multid_against_direct(shape, dtype):
    rng = np.random.default_rng(sum(shape))
    x, h = crand(rng, shape), crand(rng, shape)
    say("nd", shape, dtype)
    y, _ = run_conv(x, h, dtype)
    ref = oracle.conv_direct(rounded(x, dtype), rounded(h, dtype))
    check_close(y, ref, TOL[dtype])


@pytest.mark.parametrize("n,radix", [(64, 2), (64, 4), (64, 8), (81, 3), (125, 5), (256, 2),
                                     (256, 4), (512, 8), (729, 3), (625, 5), (4096, 8)])
def test_uniform_radix_plans(n, radix):
    rng = np.random.default_rng(n + radix)
    x, h = crand(rng, (n,)), crand(rng, (n,))
    say("radix", n, radix)
    y, rhos = run_conv(x, h, C128, radix=[radix])
    assert rhos == [[radix] * len(rhos[0])]
    check_close(y, oracle.conv_direct(x, h), 1e-12)


# --------------------------------------------------- config 1: 1-D n = 4096

@pytest.mark.parametrize("dtype", DTYPES)
def test_radix4_4096_in_groups_of_four(dtype, monkeypatch):
    """A 1-D 4096-point radix-4 transform in six 4-point groups runs the
    pipelined kernel in one 1024-thread block (the FP32 default; FP64 asks
    for it through PAFC_TUNE_GMAX4_4096); the result is the convolution."""
    monkeypatch.setenv("PAFC_TUNE_GMAX4_4096", "1")
    m = pafc()
    d = m.describe((4096,), "c128" if dtype == C128 else "c64", [4])
    assert d["conv_passes"][0].startswith("contig L=4096 W=1 tiles=1 thr=1024 [DIF4,")
    assert "pipe_kernel<" in d["conv_passes"][0]
    rng = np.random.default_rng(4444)
    x, h = crand(rng, (4096,)), crand(rng, (4096,))
    say("radix-4 4096 in groups of four", dtype)
    y, rhos = run_conv(x, h, dtype, radix=[4])
    assert rhos[0] == [4] * 6
    ref = oracle.conv_fft(rounded(x, dtype), rounded(h, dtype))
    check_close(y, ref, TOL[dtype])


@pytest.mark.parametrize("shape,radix", [((4096,), [8]), ((4096,), [2]), ((3, 4096), [3, 8]),
                                         ((2, 5, 4096), [2, 5, 8]), ((8, 4096), [8, 8])])
@pytest.mark.parametrize("dtype", DTYPES)
def test_radix8_4096_axis_pipelined(shape, radix, dtype):
    """A 4096-long contiguous axis in four 8-point groups (radix-8 stages,
    or a 1-D transform of radix-2 stages grouped by three) runs the
    pipelined kernel in 512-thread blocks (one tile as the middle pass, and
    persistent blocks over several tiles as forward and inverse passes); the
    result is the convolution."""
    m = pafc()
    d = m.describe(shape, "c128" if dtype == C128 else "c64", radix)
    assert any("pipe_kernel<" in lbl and "thr=512" in lbl and "L=4096" in lbl
               for lbl in d["conv_passes"])
    rng = np.random.default_rng(4096 + len(shape))
    x, h = crand(rng, shape), crand(rng, shape)
    say("radix-8 4096 axis", shape, dtype)
    y, _ = run_conv(x, h, dtype, radix=radix)
    ref = oracle.conv_fft(rounded(x, dtype), rounded(h, dtype))
    check_close(y, ref, TOL[dtype])


@pytest.mark.parametrize("radix", [2, 4])
def test_conv1d_4096_radix_plans(radix):
    x, h = inputs.conv1d_4096()
    say("conv1d 4096 radix", radix)
    y, rhos = run_conv(x, h, C128, radix=[radix])
    assert rhos[0] == [radix] * (12 if radix == 2 else 6)
    check_close(y, oracle.conv_direct(x, h), 1e-12)


# ------------------------------------------------ forward-only layout law

@pytest.mark.parametrize("shape,radix", [((64,), [2]), ((64,), [4]), ((64,), [8]), ((243,), [3]),
                                         ((4096,), [4]), ((4096,), [2]), ((24, 45), None),
                                         ((16, 27, 25), None), ((3125 * 5,), None),
                                         ((2 ** 14,), None)])
@pytest.mark.parametrize("dtype", DTYPES)
def test_forward_is_digit_reversed_spectrum(shape, radix, dtype):
    rng = np.random.default_rng(7)
    x = crand(rng, shape)
    P = pafc().Plan(shape, dtype, radix=radix)
    say("forward", shape, radix, dtype)
    z = to_host(P.forward(to_dev(x, dtype)))
    rhos = [P.radices(a) for a in range(len(shape))]
    ref = oracle.unordered_spectrum(rounded(x, dtype), rhos)
    check_close(z, ref, TOL[dtype] * 10)
    # and back: inverse(forward(x)) = x
    xb = to_host(P.inverse(to_dev(ref, dtype)))
    check_close(xb, rounded(x, dtype), TOL[dtype])
    P.close()


def test_forward_delta_layout():
    """x = delta_0 gives all ones; x = delta_1 gives w_n^k at pos(k)."""
    n = 256
    P = pafc().Plan((n,), C128, radix=[4])
    d0 = np.zeros(n, complex); d0[0] = 1
    z0 = to_host(P.forward(to_dev(d0, C128)))
    assert np.abs(z0 - 1).max() < 1e-15
    d1 = np.zeros(n, complex); d1[1] = 1
    z1 = to_host(P.forward(to_dev(d1, C128)))
    from oracle import dense
    pt = dense.pos_table(P.radices(0))
    assert np.abs(z1[pt] - np.exp(-2j * np.pi * np.arange(n) / n)).max() < 1e-14
    P.close()


# ------------------------------------------------------------ invariants

def test_delta_filter_identity_and_shift():
    rng = np.random.default_rng(3)
    shape = (32, 27, 20)
    x = crand(rng, shape)
    d = np.zeros(shape, complex); d[0, 0, 0] = 1
    y, _ = run_conv(x, d, C128)
    check_close(y, x, 1e-14)
    s = (5, 7, 11)
    ds = np.zeros(shape, complex); ds[s] = 1
    y, _ = run_conv(x, ds, C128)
    check_close(y, np.roll(x, s, axis=(0, 1, 2)), 1e-14)


def test_linearity_and_commutativity():
    rng = np.random.default_rng(4)
    shape = (48, 64)
    x1, x2, h = crand(rng, shape), crand(rng, shape), crand(rng, shape)
    a, b = 0.7 - 0.2j, -1.3 + 0.4j
    P = pafc().Plan(shape, C128)
    P.set_filter(to_dev(h, C128))
    y1 = to_host(P.convolve(to_dev(x1, C128)))
    y2 = to_host(P.convolve(to_dev(x2, C128)))
    y12 = to_host(P.convolve(to_dev(a * x1 + b * x2, C128)))
    check_close(y12, a * y1 + b * y2, 1e-13)
    P.set_filter(to_dev(x1, C128))
    yc = to_host(P.convolve(to_dev(h, C128)))
    check_close(yc, y1, 1e-13)
    P.close()


# -------------------------------------------------------------- variants

@pytest.mark.parametrize("variant", ["perm_free", "explicit_perm", "perm_free_unfused"])
@pytest.mark.parametrize("shape", [(4096,), (64, 81), (16, 32, 24), (5 ** 7,)])
def test_variants_agree_with_oracle(variant, shape):
    rng = np.random.default_rng(11)
    x, h = crand(rng, shape), crand(rng, shape)
    say("variant", variant, shape)
    y, _ = run_conv(x, h, C128, variant=variant)
    ref = oracle.conv_fft(x, h)
    check_close(y, ref, 1e-12)


def test_in_place():
    rng = np.random.default_rng(12)
    shape = (81, 64)
    x, h = crand(rng, shape), crand(rng, shape)
    P = pafc().Plan(shape, C128)
    P.set_filter(to_dev(h, C128))
    xd = to_dev(x, C128)
    P.convolve(xd, out=xd)
    check_close(to_host(xd), oracle.conv_fft(x, h), 1e-12)
    P.close()


@pytest.mark.parametrize("variant", ["perm_free", "explicit_perm"])
@pytest.mark.parametrize("shape", [(243, 81), (3125,), (16, 9, 25)])
def test_spectral_filter_domain(variant, shape):
    x, hhat = inputs.spectral_filter_case(31, shape)
    say("spectral", variant, shape)
    y, _ = run_conv(x, hhat, C128, variant=variant, domain="spectral_natural")
    ref = oracle.fft(hhat * oracle.fft(x), inverse=True)
    check_close(y, ref, 1e-12)


# ----------------------------------------------- medium sizes, ragged tails

@pytest.mark.parametrize("shape", [(2 ** 14,), (3 ** 9,), (5 ** 6,), (2 ** 15 * 3,),
                                   (1000, 36), (100, 243), (24, 50, 36), (9, 10, 12),
                                   (512, 40, 3), (2, 2, 4096)])
@pytest.mark.parametrize("dtype", DTYPES)
def test_medium_and_ragged(shape, dtype):
    rng = np.random.default_rng(int(np.prod(shape)) % 1000)
    x, h = crand(rng, shape), crand(rng, shape)
    say("medium", shape, dtype)
    y, _ = run_conv(x, h, dtype)
    ref = oracle.conv_fft(rounded(x, dtype), rounded(h, dtype))
    check_close(y, ref, TOL[dtype])


# --------------------------------------------------------- error handling

def test_errors():
    m = pafc()
    P = m.Plan((64,), C128)
    x = to_dev(np.ones(64, complex), C128)
    with pytest.raises(m.PafcError) as e:
        P.convolve(x)
    assert e.value.status == 5  # filter not set
    import ctypes
    st = m.lib().pafc_convolve(P.handle, ctypes.c_void_p(x.data_ptr() + 8),
                               ctypes.c_void_p(x.data_ptr()), None)
    assert st == 1  # misaligned for complex128
    P.close()
    with pytest.raises(m.PafcError) as e:  # 1-D lengths 7, 11, ... have their own routes
        m.Plan((7, 4), C128)
    assert e.value.status == 2
    with pytest.raises(m.PafcError) as e:
        m.Plan((48,), C128, radix=[4])
    assert e.value.status == 2


@pytest.mark.parametrize("shape", [(64, 64, 64), (4096,), (97,), (1009,), (2 ** 6 * 3 ** 3,)])
def test_profile_launch(shape):
    """pafc_profile_launch times one launch position with fewer events: its
    mean agrees with the full per-launch profile, every repetition is
    timed, the result is the convolution, and positions out of range are
    rejected."""
    m = pafc()
    rng = np.random.default_rng(21)
    x = inputs.complex_uniform(rng, shape)
    h = inputs.complex_uniform(rng, shape)
    P = m.Plan(shape, C128)
    P.set_filter(to_dev(h, C128))
    xd = to_dev(x, C128)
    yd = torch.empty_like(xd)
    ms, by, _ = P.profile_passes(xd, yd, reps=5)
    for k in (0, len(ms) - 1, max(range(len(ms)), key=lambda i: ms[i])):
        t, per = P.profile_launch(xd, yd, k, reps=6)
        assert len(per) == 6 and min(per) > 0 and t > 0
        assert t <= max(per)
        # without per-repetition events: only the pair around the launch (a
        # pipelined launch carries them itself), the same order of duration
        t1, none = P.profile_launch(xd, yd, k, reps=6, per_rep=False)
        assert none is None and t1 > 0
        assert t1 <= 2.0 * max(per) + 0.05
        if len(ms) == 1:
            # one launch: one pair spans the sequence, at least the launch
            # itself on average
            assert t1 >= 0.5 * ms[0]
        say("launch", k, "of", len(ms), t, t1, ms[k])
    ref = oracle.conv_fft(x, h) if len(shape) > 1 or shape[0] in (4096, 1728) else \
        oracle.conv_direct(x, h)
    check_close(to_host(yd), ref, TOL[C128])
    for bad in (-1, len(ms)):
        with pytest.raises(m.PafcError):
            P.profile_launch(xd, yd, bad, reps=2)
    P.close()


@pytest.mark.parametrize("shape", [(729, 100), (2187, 12), (512, 20, 6), (81, 729, 8), (1024, 3)])
@pytest.mark.parametrize("dtype", DTYPES)
def test_split_strided_axes(shape, dtype):
    """Strided axes too long for a 16-column tile are cut into an outer and an
    inner pass (twiddles of the outer piece depend on the inner position)."""
    rng = np.random.default_rng(int(np.prod(shape)) % 977)
    x, h = crand(rng, shape), crand(rng, shape)
    say("split strided", shape, dtype)
    m = pafc()
    d = m.describe(shape, "c128" if dtype == C128 else "c64")
    y, _ = run_conv(x, h, dtype)
    ref = oracle.conv_fft(rounded(x, dtype), rounded(h, dtype))
    check_close(y, ref, TOL[dtype], what=str(d["conv_passes"]))


HTM_SHAPES = [((64, 64, 64), [4, 4, 4]), ((256, 256), [4, 4]), ((4096, 48), [4, 0]), ((256, 64), [2, 2]),
              ((512, 40), [8, 0])]


@pytest.mark.parametrize("shape,radix", HTM_SHAPES)
@pytest.mark.parametrize("dtype", DTYPES)
def test_tile_major_spectrum(shape, radix, dtype, monkeypatch):
    """Plans whose strided middle pass reads the spectrum tile-major (the
    filter's last forward pass writes that order; natural-order spectra and
    symbols are reordered into it) give the same bits as plans that keep the
    plan layout (PAFC_HTM=0), for spatial, natural-spectral, per-call and
    symbol filters, and match the oracle."""
    rng = np.random.default_rng([len(shape), shape[0], 9])
    x = inputs.complex_uniform(rng, shape)
    h = inputs.complex_uniform(rng, shape)
    hn = inputs.complex_normal(rng, shape)
    out = {}
    for htm in ("1", "0"):
        monkeypatch.setenv("PAFC_HTM", htm)
        P = pafc().Plan(shape, dtype, radix=radix)
        xd = to_dev(x, dtype)
        P.set_filter(to_dev(h, dtype))
        a = to_host(P.convolve(xd))
        P.set_filter(to_dev(hn, dtype), domain="spectral_natural")
        b = to_host(P.convolve(xd))
        c = to_host(P.convolve_with_filter(xd, to_dev(h, dtype)))
        P.set_symbol("heat", 0.5)
        d = to_host(P.convolve(xd))
        P.close()
        out[htm] = (a, b, c, d)
    for u, v in zip(out["1"], out["0"]):
        assert np.array_equal(u, v)
    xr, hr = rounded(x, dtype), rounded(h, dtype)
    check_close(out["1"][0], oracle.conv_fft(xr, hr), TOL[dtype])
    assert rel_l2(out["1"][2], out["1"][0]) == 0.0
    ref_b = oracle.fft(rounded(hn, dtype) * oracle.fft(xr), inverse=True)
    check_close(out["1"][1], ref_b, TOL[dtype])


STREAM_CASES = [((256, 256), [4, 4]), ((64, 64, 64), [4, 4, 4]), ((4096, 48), [4, 0]),
                ((2048, 2, 2), None), ((1 << 14, 2), None), ((243, 243), None), ((4096,), [4])]


@pytest.mark.parametrize("shape,radix", STREAM_CASES)
@pytest.mark.parametrize("dtype", DTYPES)
def test_streamed_loads_leave_results_unchanged(shape, radix, dtype, monkeypatch):
    """Plans read the spectrum and the first pass's input with non-temporal
    loads when the arrays exceed the last-level cache (PAFC_LLC_MB, default
    256).  With the bound at 0 every plan takes them wherever its layout
    allows (tile-major spectra, contiguous and 64-byte-or-longer strided
    segments, folded columns): bit-identical to ordinary loads (bound out of
    reach), for the convolution, the filter's forward transform and the
    per-call filter, and in the comparison variants (their product kernels
    stream the spectrum too), matching the oracle."""
    rng = np.random.default_rng([len(shape), shape[0], 17])
    x = inputs.complex_uniform(rng, shape)
    h = inputs.complex_uniform(rng, shape)
    out = {}
    for mb in ("0", "1048576"):
        monkeypatch.setenv("PAFC_LLC_MB", mb)
        P = pafc().Plan(shape, dtype, radix=radix)
        xd = to_dev(x, dtype)
        P.set_filter(to_dev(h, dtype))
        a = to_host(P.convolve(xd))
        b = to_host(P.forward(xd))
        c = to_host(P.convolve_with_filter(xd, to_dev(h, dtype)))
        P.close()
        ys = []
        for variant in ("explicit_perm", "perm_free_unfused"):
            Q = pafc().Plan(shape, dtype, radix=radix, variant=variant)
            Q.set_filter(to_dev(h, dtype))
            ys.append(to_host(Q.convolve(xd)))
            Q.close()
        out[mb] = (a, b, c, *ys)
    for u, v in zip(out["0"], out["1048576"]):
        assert np.array_equal(u, v), shape
    ref = oracle.conv_fft(rounded(x, dtype), rounded(h, dtype))
    for y in (out["0"][0], out["0"][3], out["0"][4]):
        check_close(y, ref, TOL[dtype])


POISON_CASES = [((256, 256), [4, 4]), ((4096,), [4]), ((4096, 48), [4, 0]), ((512, 40), [8, 0]),
                ((2187, 12), None), ((5 ** 6,), None), ((81, 8, 8), None), ((729, 100), None),
                ((1000, 2), None), ((2 ** 15 * 3,), None), ((97,), None), ((1001,), None),
                ((360,), None)]


@pytest.mark.parametrize("shape,radix", POISON_CASES)
@pytest.mark.parametrize("dtype", DTYPES)
def test_lds_poison_leaves_results_unchanged(shape, radix, dtype, monkeypatch):
    """LDS race guard: with PAFC_LDS_POISON=1 every pass fills its LDS tile
    with NaN before each tile, so an op that read LDS no earlier op wrote (a
    missing barrier, a wrong index) would turn results into NaN or change
    them.  Every variant, pipelined and general passes, folded column ops,
    split axes, partial tiles, the prime routes: bit-identical to the normal
    run."""
    rng = np.random.default_rng([len(shape), shape[0], 13])
    x = inputs.complex_uniform(rng, shape)
    h = inputs.complex_uniform(rng, shape)
    variants = ["perm_free", "explicit_perm", "perm_free_unfused"]
    if shape == (360,):
        variants = ["prime_factor", "prime_factor_explicit"]
    for variant in variants:
        out = {}
        for flag in ("0", "1"):
            monkeypatch.setenv("PAFC_LDS_POISON", flag)
            P = pafc().Plan(shape, dtype, radix=radix, variant=variant)
            xd = to_dev(x, dtype)
            P.set_filter(to_dev(h, dtype))
            y = to_host(P.convolve(xd))
            z = to_host(P.forward(xd)) if not P.describe().get("rader_inner") and \
                "bluestein_m" not in P.describe() and not variant.startswith("prime") else None
            P.close()
            out[flag] = (y, z)
        assert not np.isnan(out["1"][0]).any(), (shape, variant)
        assert np.array_equal(out["0"][0], out["1"][0]), (shape, variant)
        if out["0"][1] is not None:
            assert np.array_equal(out["0"][1], out["1"][1]), (shape, variant)


@pytest.mark.parametrize("form", ["persistent", "levels", "classes"])
def test_lds_poison_batched(monkeypatch, form):
    sizes = [256, 729, 625, 4096, 8192, 6561, 3125, 256, 15625, 2048]
    classes = sorted(set(sizes))
    fids = [classes.index(n) for n in sizes]
    rng = np.random.default_rng(14)
    xs = np.concatenate([inputs.complex_uniform(rng, (n,)) for n in sizes])
    hs = {n: inputs.complex_uniform(rng, (n,)) for n in classes}
    out = {}
    for flag in ("0", "1"):
        monkeypatch.setenv("PAFC_LDS_POISON", flag)
        B = pafc().Batch(sizes, fids, len(classes), C128, form=form)
        for n in classes:
            B.set_filter(classes.index(n), to_dev(hs[n], C128))
        out[flag] = to_host(B.convolve(to_dev(xs, C128)))
        B.close()
    assert not np.isnan(out["1"]).any()
    assert np.array_equal(out["0"], out["1"])


SHAPE_CASES = [((256, 256), [4, 4]), ((2187, 12), None), ((5 ** 6,), None), ((64, 64, 64), [4, 4, 4]),
               ((4096, 48), [4, 0])]
KNOBS = [{"PAFC_TUNE_WS": "8"}, {"PAFC_TUNE_WS": "32"}, {"PAFC_TUNE_WC": "2"},
         {"PAFC_TUNE_WC": "4"}, {"PAFC_PIPE": "0"}]


@pytest.mark.parametrize("shape,radix", SHAPE_CASES)
def test_tile_shapes_and_kernels_agree(shape, radix, monkeypatch):
    """The same convolution planned with other tile widths, or with the
    general pass engine instead of the pipelined kernel, agrees with the
    default plan to a few ulps (the same arithmetic per column; kernels may
    contract multiply-adds differently); walking every pass's tiles in one
    direction (PAFC_SNAKE=0) gives the same bits."""
    rng = np.random.default_rng([len(shape), shape[0], 17])
    x = inputs.complex_uniform(rng, shape)
    h = inputs.complex_uniform(rng, shape)

    def run():
        P = pafc().Plan(shape, C128, radix=radix)
        P.set_filter(to_dev(h, C128))
        y = to_host(P.convolve(to_dev(x, C128)))
        labels = P.describe()["conv_passes"]
        P.close()
        return y, labels

    y0, l0 = run()
    check_close(y0, oracle.conv_fft(x, h), TOL[C128])
    monkeypatch.setenv("PAFC_SNAKE", "0")
    y1, _ = run()
    monkeypatch.delenv("PAFC_SNAKE")
    assert np.array_equal(y0, y1)
    for knob in KNOBS:
        for k, v in knob.items():
            monkeypatch.setenv(k, v)
        y, labels = run()
        for k in knob:
            monkeypatch.delenv(k)
        say(shape, knob, labels != l0)
        check_close(y, y0, 2e-15, what=str((shape, knob)), elem_c=AGREE_C)


# (a length-2187 axis as the fused middle pass would need 15 single-stage
# ops, more than a pass holds: those plans keep larger groups)
SMALL_RADIX = [((3125,), None), ((243, 20), None), ((729, 12), None), ((625, 36), None),
               ((24, 2187), None), ((4, 2187), None), ((10, 3125), None), ((81, 243), None),
               ((5 ** 7,), None), ((2187, 2187), [3, 3])]


@pytest.mark.parametrize("shape,radix", SMALL_RADIX)
@pytest.mark.parametrize("dtype", DTYPES)
def test_small_radix_pipelined_passes(shape, radix, dtype, monkeypatch):
    """Single radix-3 / radix-5 stages per op (PAFC_TUNE_GMAX3/5=1) make the
    uniform pieces run on the pipelined kernel with up to 1024 threads, one
    item per thread, the tile narrowed to fit; against the oracle, in every
    variant, and against the general engine (PAFC_PIPE=0)."""
    monkeypatch.setenv("PAFC_NO_TUNING_TABLE", "1")
    monkeypatch.setenv("PAFC_TUNE_GMAX3", "1")
    monkeypatch.setenv("PAFC_TUNE_GMAX5", "1")
    import paper_2506_12718_amd as m
    m.set_tuning(None)
    try:
        dt = "c128" if dtype == C128 else "c64"
        labels = m.describe(shape, dt, radix)["conv_passes"]
        say("small radix", shape, dt, labels)
        assert any(("<double,3,1," in l or "<double,5,1," in l or "<float,3,1," in l or
                    "<float,5,1," in l) for l in labels), labels
        rng = np.random.default_rng([len(shape), shape[0], 19])
        x = inputs.complex_uniform(rng, shape)
        h = inputs.complex_uniform(rng, shape)
        ref = oracle.conv_fft(rounded(x, dtype), rounded(h, dtype))
        ys = {}
        for variant in ("perm_free", "explicit_perm", "perm_free_unfused"):
            P = m.Plan(shape, dtype, radix=radix, variant=variant)
            P.set_filter(to_dev(h, dtype))
            ys[variant] = to_host(P.convolve(to_dev(x, dtype)))
            P.close()
            check_close(ys[variant], ref, TOL[dtype], what=str(variant))
        monkeypatch.setenv("PAFC_PIPE", "0")
        P = m.Plan(shape, dtype, radix=radix)
        P.set_filter(to_dev(h, dtype))
        y0 = to_host(P.convolve(to_dev(x, dtype)))
        P.close()
        check_close(ys["perm_free"], y0, (2e-15 if dtype == C128 else 1e-6), elem_c=AGREE_C)
    finally:
        monkeypatch.delenv("PAFC_NO_TUNING_TABLE")
        m._load_tuning_table(m.lib())  # the table the other tests plan with


# radix-9 groups of radix-3 axes on the pipelined kernel: uniform (729 =
# 9^3), ending in a radix-3 group (2187 = 9 x 9 x 9 x 3, 243 = 9 x 9 x 3),
# one group (9-long outer pieces), with the inner pieces' grouping (g3i)
# single-stage or radix-9
RADIX9 = [((2187, 2187), "2 0 1"), ((2187, 2187), "2 0 2"), ((243, 2187), "2 0 2"),
          ((2187,), "2 0 2"), ((729,), "2 0 2"), ((81, 729), "2 0 2"), ((59049,), "2 0 2")]


@pytest.mark.parametrize("shape,g", RADIX9)
@pytest.mark.parametrize("dtype", DTYPES)
def test_radix9_pipelined_passes(shape, g, dtype):
    """Planner entries with radix-9 groups (g3 = 2) put radix-3 axes on the
    pipelined kernel's radix-9 instances; against the oracle and against the
    general engine's result of the same plan (PAFC_PIPE=0 is not needed: the
    single-stage plan is the reference)."""
    import paper_2506_12718_amd as m
    dt = "c128" if dtype == C128 else "c64"
    table = "".join("%s %d 0 0 0 %s\n" % (dt, n, g) for n in sorted(set(shape)))
    try:
        m.set_tuning(table)
        labels = m.describe(shape, dt)["conv_passes"]
        say("radix-9", shape, dt, g, labels)
        assert any(",3,2," in l for l in labels), labels
        rng = np.random.default_rng([len(shape), shape[0], 23])
        x = inputs.complex_uniform(rng, shape)
        h = inputs.complex_uniform(rng, shape)
        P = m.Plan(shape, dtype)
        P.set_filter(to_dev(h, dtype))
        y = to_host(P.convolve(to_dev(x, dtype)))
        P.close()
        check_close(y, oracle.conv_fft(rounded(x, dtype), rounded(h, dtype)), TOL[dtype])
    finally:
        m.set_tuning(None)
        m._load_tuning_table(m.lib())  # the table the other tests plan with


# (shape, dtype, table): outer pieces of cut axes on the pipelined kernel
# (MODE_OUTER): the tuned 1-D plans' 625- and 243-long outer pieces (tuning
# table), and the 9- and 125-long outer pieces of cut grid axes, whose
# column's inner position is the column divided by the axis stride
OUTER_PIECES = [((5 ** 9,), C128, True), ((995328,), C128, True), ((995328,), C64, True),
                ((2187, 2187), C128, True), ((2187, 2187), C64, True),
                ((2025000,), C128, True), ((390625, 2), C128, False), ((390625, 2), C64, False),
                ((78125, 8), C128, False)]


@pytest.mark.parametrize("shape,dtype,table", OUTER_PIECES)
def test_outer_pieces_pipelined(shape, dtype, table, monkeypatch):
    """Outer pieces of a cut axis run on the pipelined kernel with the whole
    axis's twiddles (two-level LDS table, exponent j*jmul + inner position);
    against the oracle and against the general engine (PAFC_PIPE_OUTER=0)."""
    import paper_2506_12718_amd as m
    if not table:
        monkeypatch.setenv("PAFC_NO_TUNING_TABLE", "1")
        monkeypatch.setenv("PAFC_TUNE_GMAX3", "1")
        monkeypatch.setenv("PAFC_TUNE_GMAX5", "1")
        m.set_tuning(None)
    try:
        dt = "c128" if dtype == C128 else "c64"
        labels = m.describe(shape, dt)["conv_passes"]
        say("outer pieces", shape, dt, labels)
        assert sum(l.endswith(",2>") for l in labels) == 2, labels
        rng = np.random.default_rng([len(shape), shape[0], 23])
        x = inputs.complex_uniform(rng, shape)
        h = inputs.complex_uniform(rng, shape)
        ref = oracle.conv_fft(rounded(x, dtype), rounded(h, dtype))
        ys = {}
        for flag in ("1", "0"):
            monkeypatch.setenv("PAFC_PIPE_OUTER", flag)
            P = m.Plan(shape, dtype)
            if flag == "0":
                assert not any(l.endswith(",2>") for l in m.describe(shape, dt)["conv_passes"])
            P.set_filter(to_dev(h, dtype))
            ys[flag] = to_host(P.convolve(to_dev(x, dtype)))
            P.close()
            check_close(ys[flag], ref, TOL[dtype], what="PAFC_PIPE_OUTER=%s" % flag)
        check_close(ys["1"], ys["0"], (2e-15 if dtype == C128 else 1e-6), elem_c=AGREE_C)
    finally:
        if not table:
            monkeypatch.delenv("PAFC_NO_TUNING_TABLE")
            m._load_tuning_table(m.lib())
