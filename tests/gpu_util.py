"""Helpers shared by the GPU tests (no method arithmetic here)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")


def have_gpu():
    return torch.cuda.is_available()


def to_dev(a, dtype):
    t = torch.from_numpy(np.ascontiguousarray(a))
    return t.to(dtype).cuda()


def to_host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy().astype(np.complex128)


def rounded(a, dtype):
    """The values a device tensor of `dtype` holds for host array `a`."""
    if dtype == torch.complex64:
        return a.astype(np.complex64).astype(np.complex128)
    return a.astype(np.complex128)


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.complex128).ravel()
    b = np.asarray(b, dtype=np.complex128).ravel()
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


TOL = {torch.complex128: 1e-12, torch.complex64: 1e-5}

# Entry-wise factor of every parity check.  A norm bound alone lets a few
# entries be far off (one entry of 256^3 may be off by 4 % of the RMS under
# rel-L2 <= 1e-5); so, beside the relative L2 error over all compared
# entries, every single entry must satisfy |y_j - ref_j| <= ELEM_C * tol *
# rms(ref).  FFT rounding errors spread evenly over the outputs (each output
# is a sum over all inputs), so the largest entry error is a small multiple
# (about sqrt(2 ln N) < 6) of the RMS error, itself <= 5e-7 * rms(ref) in
# FP32 and <= 2e-15 * rms(ref) in FP64 here: with ELEM_C = 1 the entry-wise
# bound keeps a margin of about 3x (FP32) and 100x (FP64) over rounding while
# catching any single entry wrong by more than tol times the typical size.
ELEM_C = 1.0
# Two kernel schedules of the same convolution (other tile widths, engines,
# outer-piece kernels) are compared at a few ulps in rel-L2 (2e-15 FP64);
# there the entry-wise bound is the largest-of-N multiple of that RMS
# agreement, sqrt(2 ln N) <= 6 for N <= 2^26, rounded up to 8.
AGREE_C = 8.0


def check_close(got, ref, tol, what="", elem_c=ELEM_C):
    """Assert rel-L2(got, ref) <= tol and max_j |got_j - ref_j| <=
    elem_c * tol * rms(ref); returns the rel-L2 error."""
    a = np.asarray(got, dtype=np.complex128).ravel()
    b = np.asarray(ref, dtype=np.complex128).ravel()
    assert a.shape == b.shape, (what, a.shape, b.shape)
    assert np.all(np.isfinite(a)), ("non-finite output", what)
    d = np.abs(a - b)
    nb = float(np.linalg.norm(b))
    if nb == 0.0:
        assert float(d.max(initial=0.0)) <= tol, (what, "reference is zero")
        return 0.0
    l2 = float(np.linalg.norm(a - b)) / nb
    rms = nb / np.sqrt(b.size)
    emax = float(d.max(initial=0.0))
    print("  check %s rel_l2=%.3e max_entry_err/rms=%.3e (tol %.1e)"
          % (what, l2, emax / rms, tol), flush=True)
    assert l2 <= tol, ("rel-L2", what, l2, tol)
    assert emax <= elem_c * tol * rms, ("entry-wise", what, int(d.argmax()), emax / rms, tol)
    return l2
