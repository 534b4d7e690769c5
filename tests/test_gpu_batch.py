"""GPU parity of the batched form (many independent 1-D convolutions of
uneven, mixed-radix sizes) against the CPU oracle, and of its hipGraph replay
against eager execution, in every form: one persistent launch; one launch
per pass level and kernel class; and the same with one pipelined launch per
size class for the passes whose plan runs on the pipelined kernel."""
import sys

import numpy as np
import pytest

import oracle
from paper_2506_12718_amd import inputs
from gpu_util import AGREE_C, TOL, check_close, rel_l2, rounded, to_dev, to_host, torch

pytestmark = pytest.mark.gpu
FORMS = ["persistent", "levels", "classes"]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def pafc():
    import paper_2506_12718_amd as m
    return m


def pack(xs):
    return np.concatenate([np.asarray(x).ravel() for x in xs])


def unpack(y, sizes):
    out, o = [], 0
    for n in sizes:
        out.append(y[o:o + n])
        o += n
    return out


def check_batch(sizes, fids, filters, xs, dtype, spectral=False, sample=None, form="persistent"):
    m = pafc()
    B = m.Batch(sizes, fids, len(filters), dtype, form=form)
    levels = B.describe()["levels"]
    say("batch form", form, levels)
    if form == "classes" and any(n >= 4096 and n % 4 == 0 for n in sizes):
        # a 4096-long class runs its middle pass on the pipelined kernel
        assert any(L.get("pipe") for L in levels), levels
    for f, h in filters.items():
        B.set_filter(f, to_dev(h, dtype), domain="spectral_natural" if spectral else "spatial")
    y = to_host(B.convolve(to_dev(pack(xs), dtype)))
    ys = unpack(y, sizes)
    idx = range(len(sizes)) if sample is None else sample
    for i in idx:
        x = rounded(xs[i], dtype)
        h = rounded(filters[fids[i]], dtype)
        if spectral:
            ref = oracle.fft(h * oracle.fft(x), inverse=True)
        else:
            ref = oracle.conv_fft(x, h)
        check_close(ys[i], ref, TOL[dtype], what=str((i, sizes[i])))
    B.close()
    return ys


@pytest.mark.parametrize("form", FORMS)
@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
def test_small_mixed_batch(dtype, form):
    rng = np.random.default_rng(5)
    classes = [16, 27, 64, 81, 125, 243, 256, 625, 1024, 4096, 3 ** 8, 2 ** 14, 5 ** 6, 3 ** 9]
    sizes = [classes[i] for i in rng.integers(0, len(classes), 60)] + classes
    filters = {k: inputs.complex_uniform(rng, (n,)) for k, n in enumerate(classes)}
    fids = [classes.index(n) for n in sizes]
    xs = [inputs.complex_uniform(rng, (n,)) for n in sizes]
    say("small batch", dtype, len(sizes), form)
    check_batch(sizes, fids, filters, xs, dtype, form=form)


@pytest.mark.parametrize("form", FORMS)
def test_two_filters_per_size_class_and_spectral(form):
    rng = np.random.default_rng(6)
    sizes = [256, 256, 243, 243, 256]
    fids = [0, 1, 2, 3, 1]
    filters = {0: inputs.complex_normal(rng, (256,)), 1: inputs.complex_normal(rng, (256,)),
               2: inputs.complex_normal(rng, (243,)), 3: inputs.complex_normal(rng, (243,))}
    xs = [inputs.complex_uniform(rng, (n,)) for n in sizes]
    check_batch(sizes, fids, filters, xs, torch.complex128, spectral=True, form=form)


@pytest.mark.parametrize("form", FORMS)
@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
def test_full_batched_workload_sampled(dtype, form):
    """The 4096-problem batched workload in the launch configuration the
    benchmark times; 48 problems (the largest of every size class first)
    checked against the oracle."""
    psizes, xs, filters = inputs.batched_problems()
    classes = sorted(filters)
    fids = [classes.index(n) for n in psizes]
    filt = {classes.index(n): h for n, h in filters.items()}
    first_of = {}
    for i, n in enumerate(psizes):
        first_of.setdefault(n, i)
    sample = sorted(set(list(first_of.values()) + list(np.random.default_rng(0).integers(0, 4096, 30))))
    say("full batch", dtype, sum(psizes), form)
    check_batch(psizes, fids, filt, xs, dtype, sample=sample, form=form)


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
def test_forms_agree(dtype):
    """The two forms plan the size classes under different limits (other
    register groups and tiles), so they agree to rounding, entry by entry,
    on every problem of a mixed batch."""
    rng = np.random.default_rng(12)
    classes = [256, 729, 4096, 6561, 3125, 2 ** 15, 3 ** 10, 5 ** 7]
    sizes = [classes[i] for i in rng.integers(0, len(classes), 50)] + classes
    filters = {k: inputs.complex_uniform(rng, (n,)) for k, n in enumerate(classes)}
    fids = [classes.index(n) for n in sizes]
    x = to_dev(pack([inputs.complex_uniform(rng, (n,)) for n in sizes]), dtype)
    out = {}
    for form in FORMS:
        B = pafc().Batch(sizes, fids, len(classes), dtype, form=form)
        for f, h in filters.items():
            B.set_filter(f, to_dev(h, dtype))
        say("forms agree", dtype, form, B.describe()["levels"])
        out[form] = to_host(B.convolve(x))
        B.close()
    yb = unpack(out["levels"], sizes)
    for form in ("persistent", "classes"):
        ya = unpack(out[form], sizes)
        for i in range(len(sizes)):
            # two roundings of the same sums: a few ulps in rel-L2
            check_close(ya[i], yb[i], 2e-6 if dtype == torch.complex64 else 2e-15,
                        what="%s vs levels %d" % (form, sizes[i]), elem_c=AGREE_C)


@pytest.mark.parametrize("form", FORMS)
def test_batch_graph_replays_match_eager(form):
    rng = np.random.default_rng(8)
    classes = [64, 243, 3125, 2 ** 14]
    sizes = [classes[i] for i in rng.integers(0, 4, 40)]
    filters = {k: inputs.complex_uniform(rng, (n,)) for k, n in enumerate(classes)}
    fids = [classes.index(n) for n in sizes]
    xs = [inputs.complex_uniform(rng, (n,)) for n in sizes]
    m = pafc()
    B = m.Batch(sizes, fids, len(classes), torch.complex128, form=form)
    for f, h in filters.items():
        B.set_filter(f, to_dev(h, torch.complex128))
    x = to_dev(pack(xs), torch.complex128)
    say("graph replays", form, B.describe()["levels"])
    eager = to_host(B.convolve(x))
    for i, n in enumerate(sizes[:6]):
        check_close(unpack(eager, sizes)[i], oracle.conv_fft(xs[i], filters[fids[i]]), 1e-12,
                    what="eager %d" % n)
    y = torch.empty_like(x)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        B.convolve(x, out=y, stream=s)  # warm-up outside the graph
        torch.cuda.synchronize()
        with torch.cuda.graph(g, stream=s):
            B.convolve(x, out=y, stream=s)
    torch.cuda.synchronize()
    for rep in range(4):
        y.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(to_host(y), eager), rep
        # eager work between replays
        _ = B.convolve(x)
        torch.cuda.synchronize()
    B.close()


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
def test_classes_form_on_several_streams(dtype, monkeypatch):
    """The classes form's size-class chains forked onto four streams and
    joined back into the caller's: the same result, bit for bit, as on one
    stream (the same kernels on the same tiles), eager and replayed from a
    captured hipGraph with eager work between the replays."""
    m = pafc()
    rng = np.random.default_rng(17)
    classes = [256, 729, 3125, 4096, 2 ** 14, 3 ** 9, 5 ** 6, 2 ** 16]
    sizes = [classes[i] for i in rng.integers(0, len(classes), 60)] + classes
    filters = {k: inputs.complex_uniform(rng, (n,)) for k, n in enumerate(classes)}
    fids = [classes.index(n) for n in sizes]
    x = to_dev(pack([inputs.complex_uniform(rng, (n,)) for n in sizes]), dtype)
    out = {}
    for k in ("1", "4"):
        monkeypatch.setenv("PAFC_BATCH_STREAMS", k)
        B = m.Batch(sizes, fids, len(classes), dtype, form="classes")
        d = B.describe()
        assert d["streams"] == int(k), d["streams"]
        if k == "4":
            assert len({L["stream"] for L in d["levels"]}) == 4, d["levels"]
        for f, h in filters.items():
            B.set_filter(f, to_dev(h, dtype))
        say("streams", k, dtype, d["levels"])
        out[k] = to_host(B.convolve(x))
        if k == "4":
            y = torch.empty_like(x)
            s = torch.cuda.Stream()
            s.wait_stream(torch.cuda.current_stream())
            g = torch.cuda.CUDAGraph()
            with torch.cuda.stream(s):
                B.convolve(x, out=y, stream=s)
                torch.cuda.synchronize()
                with torch.cuda.graph(g, stream=s):
                    B.convolve(x, out=y, stream=s)
            torch.cuda.synchronize()
            for rep in range(3):
                y.zero_()
                torch.cuda.synchronize()
                g.replay()
                torch.cuda.synchronize()
                assert np.array_equal(to_host(y), out["1"]), rep
                _ = B.convolve(x)
                torch.cuda.synchronize()
        B.close()
    assert np.array_equal(out["4"], out["1"])
    ys = unpack(out["4"], sizes)
    for i in range(len(sizes) - len(classes), len(sizes)):
        check_close(ys[i], oracle.conv_fft(rounded(unpack(to_host(x), sizes)[i], dtype),
                                           rounded(filters[fids[i]], dtype)),
                    TOL[dtype], what="streams %d" % sizes[i])


def test_profile_reports_every_launch():
    """32 size classes of three passes each: the classes form makes one
    launch per class and pass on its streams (more than the 72 the binding
    once assumed); the profile reports every one of them, timed in order
    on one stream, and leaves the same result as a convolution."""
    m = pafc()
    sizes = [8192, 9216, 10000, 10800, 11664, 12500, 13500, 15000, 16000, 17280, 18432, 19683,
             20736, 23040, 24576, 26244, 28800, 30720, 32400, 34560, 36864, 39366, 41472, 46080,
             48600, 51200, 54675, 58320, 61440, 64800, 69120, 73728]
    rng = np.random.default_rng(21)
    xs = [inputs.complex_uniform(rng, (n,)) for n in sizes]
    hs = [inputs.complex_uniform(rng, (n,)) for n in sizes]
    B = m.Batch(sizes, list(range(len(sizes))), len(sizes), torch.complex128, form="classes")
    for f, h in enumerate(hs):
        B.set_filter(f, to_dev(h, torch.complex128))
    levels = B.describe()["levels"]
    assert len(levels) > 72, len(levels)
    x = to_dev(pack(xs), torch.complex128)
    y = torch.empty_like(x)
    ms, by, per = B.profile_levels(x, y, reps=2)
    assert len(ms) == len(by) == len(levels) and len(per) == 2
    assert all(t > 0 for t in ms) and all(b > 0 for b in by)
    ys = unpack(to_host(y), sizes)
    for i in (0, 11, 31):
        check_close(ys[i], oracle.conv_fft(xs[i], hs[i]), 1e-12, what=str(sizes[i]))
    B.close()


@pytest.mark.parametrize("form", FORMS)
def test_batch_errors(form):
    m = pafc()
    with pytest.raises(m.PafcError):
        m.Batch([256, 128], [0, 0], 1, torch.complex128, form=form)  # one filter, two sizes
    B = m.Batch([64, 64], [0, 0], 1, torch.complex128, form=form)
    with pytest.raises(m.PafcError) as e:
        B.convolve(to_dev(np.zeros(128, complex), torch.complex128))
    assert e.value.status == 5
    B.close()


@pytest.mark.parametrize("form", FORMS)
def test_batch_with_five_pass_size(form):
    """A length whose 1-D plan runs five passes (2^23 complex128: the axis is
    cut twice) in a batch with one- and three-pass lengths: every pass level
    runs.  The long problem is checked at sampled outputs (first, last,
    random) against the oracle's direct sum, the short ones whole."""
    m = pafc()
    n = 2 ** 23
    assert len(m.describe((n,), "c128")["conv_passes"]) == 5
    rng = np.random.default_rng(9)
    sizes = [256, n, 4096, 3 ** 9]
    filters = {k: inputs.complex_uniform(rng, (s,)) for k, s in enumerate(sizes)}
    xs = [inputs.complex_uniform(rng, (s,)) for s in sizes]
    B = m.Batch(sizes, [0, 1, 2, 3], 4, torch.complex128, form=form)
    for f, h in filters.items():
        B.set_filter(f, to_dev(h, torch.complex128))
    say("batch with a five-pass length", B.describe()["levels"])
    ys = unpack(to_host(B.convolve(to_dev(pack(xs), torch.complex128))), sizes)
    B.close()
    for i in (0, 2, 3):
        check_close(ys[i], oracle.conv_fft(xs[i], filters[i]), 1e-12, what=str(sizes[i]))
    idx = rng.integers(0, n, 8)
    idx[0], idx[1] = 0, n - 1
    check_close(ys[1][idx], oracle.conv_direct_at(xs[1], filters[1], idx), 1e-12,
                what="2^23 sampled")


def test_auto_form_is_the_fastest():
    """PAFC_BATCH_AUTO picks the form measured fastest on the mixed
    workload: the classes form, in both element types."""
    m = pafc()
    for dtype, want in ((torch.complex128, "classes"), (torch.complex64, "classes")):
        B = m.Batch([256, 729, 4096], [0, 1, 2], 3, dtype)
        assert B.describe()["form"] == want, (dtype, B.describe()["form"])
        B.close()
