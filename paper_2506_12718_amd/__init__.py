"""Permutation-avoiding FFT-based circular convolution on AMD MI355X (gfx950).

Thin Python binding over the C ABI of ``include/pafc.h`` (``libpafc.so``).
Every step of the computation runs in the library's HIP kernels; this module
only marshals arguments.  PyTorch supplies device memory and streams: tensors
are passed by ``data_ptr()`` and work is enqueued on
``torch.cuda.current_stream()``.

    >>> import torch, paper_2506_12718_amd as pafc
    >>> plan = pafc.Plan((256, 256, 256), torch.complex128)
    >>> plan.set_filter(h)            # h: complex128 CUDA tensor, same shape
    >>> y = plan.convolve(x)          # y = x (*) h, circular, per axis

The method (Venkovic & Anzt, arXiv 2506.12718): forward decimation-in-
frequency transforms leave the spectrum digit-reversed, the filter spectrum
is kept in that same order, and decimation-in-time inverses return natural
order, so no index reversal is ever executed (eq. 35 and its d-way form).
"""
from __future__ import annotations

import ctypes
import json
import os

__all__ = ["Plan", "Batch", "describe", "lib", "set_tuning", "PafcError",
           "PERM_FREE", "EXPLICIT_PERM", "PERM_FREE_UNFUSED"]

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpafc.so")

PERM_FREE, EXPLICIT_PERM, PERM_FREE_UNFUSED = 0, 1, 2
_VARIANTS = {"perm_free": PERM_FREE, "explicit_perm": EXPLICIT_PERM,
             "perm_free_unfused": PERM_FREE_UNFUSED, "prime_factor": 3,
             "prime_factor_explicit": 4}
_C64, _C128 = 1, 2
# PAFC_NOALLOC_MAX_BYTES of include/pafc.h
NOALLOC_MAX_BYTES = 32 << 20
_DOMAINS = {"spatial": 0, "spectral_natural": 1}

# every symbol include/pafc.h declares
EXPORTS = ("pafc_plan", "pafc_set_filter", "pafc_convolve", "pafc_forward",
           "pafc_inverse", "pafc_destroy", "pafc_status_string",
           "pafc_plan_device_bytes", "pafc_plan_radices", "pafc_describe",
           "pafc_batch_plan", "pafc_batch_set_filter", "pafc_batch_convolve",
           "pafc_batch_destroy", "pafc_batch_device_bytes",
           "pafc_batch_describe", "pafc_set_tuning", "pafc_profile_passes",
           "pafc_stream_copy", "pafc_batch_profile", "pafc_twiddle",
           "pafc_convolve_with_filter", "pafc_set_symbol", "pafc_profile_launch",
           "pafc_convolve_with_filter_noalloc")


class PafcError(RuntimeError):
    def __init__(self, status, what):
        self.status = status
        super().__init__("%s: %s (status %d)" % (what, _status_string(status), status))


_lib = None


def lib():
    """The loaded libpafc.so.  Raises if it has not been built: there is no
    fallback path."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                "libpafc.so not found at %s; build it with "
                "`python -m paper_2506_12718_amd.build`" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        vp, i64p, ip = ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int)
        sz = ctypes.c_size_t
        sig = {
            "pafc_plan": [ctypes.POINTER(vp), ctypes.c_int, i64p, ip, ctypes.c_int, ctypes.c_int, vp],
            "pafc_set_filter": [vp, vp, ctypes.c_int, vp],
            "pafc_convolve": [vp, vp, vp, vp],
            "pafc_convolve_with_filter": [vp, vp, vp, vp, vp],
            "pafc_convolve_with_filter_noalloc": [vp, vp, vp, vp, vp],
            "pafc_set_symbol": [vp, ctypes.c_int, ctypes.POINTER(ctypes.c_double), ctypes.c_int,
                                vp],
            "pafc_forward": [vp, vp, vp, vp],
            "pafc_inverse": [vp, vp, vp, vp],
            "pafc_destroy": [vp],
            "pafc_plan_device_bytes": [vp, ctypes.POINTER(sz)],
            "pafc_plan_radices": [vp, ctypes.c_int, ip, ip],
            "pafc_describe": [ctypes.c_int, i64p, ip, ctypes.c_int, ctypes.c_int,
                              ctypes.c_char_p, sz, ctypes.POINTER(sz)],
            "pafc_batch_plan": [ctypes.POINTER(vp), ctypes.c_int, i64p, ip, ctypes.c_int,
                                ctypes.c_int, ctypes.c_int, vp],
            "pafc_batch_set_filter": [vp, ctypes.c_int, vp, ctypes.c_int, vp],
            "pafc_batch_convolve": [vp, vp, vp, vp],
            "pafc_batch_destroy": [vp],
            "pafc_batch_device_bytes": [vp, ctypes.POINTER(sz)],
            "pafc_batch_describe": [vp, ctypes.c_char_p, sz, ctypes.POINTER(sz)],
            "pafc_set_tuning": [ctypes.c_char_p],
            "pafc_stream_copy": [vp, vp, sz, ctypes.c_int, vp],
            "pafc_twiddle": [ctypes.c_int64, ctypes.c_int64, ctypes.POINTER(ctypes.c_double),
                             ctypes.POINTER(ctypes.c_double)],
            "pafc_batch_profile": [vp, vp, vp, vp, ctypes.c_int, ctypes.POINTER(ctypes.c_double),
                                   ctypes.POINTER(ctypes.c_int64),
                                   ctypes.POINTER(ctypes.c_double), ip],
            "pafc_profile_passes": [vp, vp, vp, vp, ctypes.c_int, ctypes.POINTER(ctypes.c_double),
                                    ctypes.POINTER(ctypes.c_int64),
                                    ctypes.POINTER(ctypes.c_double), ip],
            "pafc_profile_launch": [vp, vp, vp, vp, ctypes.c_int, ctypes.c_int,
                                    ctypes.POINTER(ctypes.c_double),
                                    ctypes.POINTER(ctypes.c_double)],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = ctypes.c_int
        L.pafc_status_string.argtypes = [ctypes.c_int]
        L.pafc_status_string.restype = ctypes.c_char_p
        _lib = L
        _load_tuning_table(L)
    return _lib


TUNING_TABLE = os.path.join(_HERE, "tuning", "mi355x.txt")


def _load_tuning_table(L):
    """Install the autotuner's table (schedule choices only; results do not
    depend on it) unless PAFC_NO_TUNING_TABLE is set; PAFC_TUNING_TABLE names
    another table file."""
    path = os.environ.get("PAFC_TUNING_TABLE") or TUNING_TABLE
    if os.environ.get("PAFC_NO_TUNING_TABLE") or not os.path.exists(path):
        return
    with open(path) as f:
        text = f.read()
    st = L.pafc_set_tuning(text.encode())
    if st != 0:
        raise PafcError(st, "loading %s" % path)


def _status_string(st):
    try:
        return lib().pafc_status_string(st).decode()
    except Exception:
        return "status"


def _check(st, what):
    if st != 0:
        raise PafcError(st, what)


def _dims_arr(dims):
    arr = (ctypes.c_int64 * len(dims))(*[int(d) for d in dims])
    return arr


def _radix_arr(radix, ndim):
    if radix is None:
        return None
    if isinstance(radix, int):
        radix = [radix] * ndim
    assert len(radix) == ndim
    return (ctypes.c_int * ndim)(*[int(r) for r in radix])


def _dtype_code(dtype):
    import torch
    if dtype in (torch.complex128, "c128", "complex128"):
        return _C128
    if dtype in (torch.complex64, "c64", "complex64"):
        return _C64
    raise ValueError("dtype must be complex64 or complex128")


def _variant_code(variant):
    if isinstance(variant, int):
        return variant
    return _VARIANTS[variant]


def _stream(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def describe(dims, dtype="c128", radix=None, variant="perm_free"):
    """Plan on the host only (no GPU needed) and return the planner's JSON."""
    code = _C128 if dtype in ("c128", "complex128") else _C64 if dtype in ("c64", "complex64") \
        else _dtype_code(dtype)
    need = ctypes.c_size_t(0)
    d = _dims_arr(dims)
    r = _radix_arr(radix, len(dims))
    st = lib().pafc_describe(len(dims), d, r, code, _variant_code(variant), None, 0,
                             ctypes.byref(need))
    _check(st, "pafc_describe")
    buf = ctypes.create_string_buffer(need.value)
    st = lib().pafc_describe(len(dims), d, r, code, _variant_code(variant), buf, need.value,
                             ctypes.byref(need))
    _check(st, "pafc_describe")
    return json.loads(buf.value.decode())


def twiddle(n, e):
    """The FP64 twiddle w_n^e the planner generates (host only)."""
    re, im = ctypes.c_double(), ctypes.c_double()
    _check(lib().pafc_twiddle(int(n), int(e), ctypes.byref(re), ctypes.byref(im)), "pafc_twiddle")
    return complex(re.value, im.value)


STREAM_KINDS = {"copy16": 0, "copy8": 1, "read": 2, "tile_copy": 3, "tile_mul": 4}


def stream_copy(src, dst, stream=None, kind="copy16"):
    """Reference kernels of known traffic (pafc_stream_copy): a streaming
    copy with 16 or 8 bytes per lane or a read-only sweep of src (counter
    calibration), and the strided middle pass's access pattern without its
    arithmetic ("tile_copy"; "tile_mul": src holds x then h, dst gets x*h)."""
    nbytes = dst.numel() * dst.element_size()
    want = 2 * nbytes if kind == "tile_mul" else nbytes
    assert src.numel() * src.element_size() == want
    _check(lib().pafc_stream_copy(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()),
                                  nbytes, STREAM_KINDS[kind], _stream(stream)), "pafc_stream_copy")


def set_tuning(text):
    """Install planner overrides (lines "<c64|c128> <n> <split> <W>"); None clears."""
    _check(lib().pafc_set_tuning(None if text is None else text.encode()), "pafc_set_tuning")


class Plan:
    """A convolution plan for one grid shape, dtype and variant (pafc_plan)."""

    def __init__(self, dims, dtype=None, radix=None, variant="perm_free", stream=None):
        import torch
        self.dims = tuple(int(d) for d in dims)
        self.dtype = dtype if dtype is not None else torch.complex128
        self._code = _dtype_code(self.dtype)
        self.variant = _variant_code(variant)
        self._h = ctypes.c_void_p()
        self._radix = radix
        self.device = torch.device("cuda", torch.cuda.current_device())
        st = lib().pafc_plan(ctypes.byref(self._h), len(self.dims), _dims_arr(self.dims),
                             _radix_arr(radix, len(self.dims)), self._code, self.variant,
                             _stream(stream))
        _check(st, "pafc_plan")

    # -- helpers
    def _check_tensor(self, t, name):
        if not t.is_cuda or t.dtype != self.dtype or tuple(t.shape) != self.dims:
            raise ValueError("%s must be a %s CUDA tensor of shape %s" % (name, self.dtype, self.dims))
        if not t.is_contiguous():
            raise ValueError("%s must be contiguous" % name)

    @property
    def handle(self):
        return self._h

    def radices(self, axis):
        n = ctypes.c_int(64)
        rho = (ctypes.c_int * 64)()
        _check(lib().pafc_plan_radices(self._h, axis, rho, ctypes.byref(n)), "pafc_plan_radices")
        return [rho[i] for i in range(n.value)]

    @property
    def device_bytes(self):
        b = ctypes.c_size_t(0)
        _check(lib().pafc_plan_device_bytes(self._h, ctypes.byref(b)), "pafc_plan_device_bytes")
        return b.value

    def set_filter(self, h, domain="spatial", stream=None):
        self._check_tensor(h, "h")
        _check(lib().pafc_set_filter(self._h, ctypes.c_void_p(h.data_ptr()), _DOMAINS[domain],
                                     _stream(stream)), "pafc_set_filter")

    def _run(self, fn, x, out, stream, what):
        import torch
        self._check_tensor(x, "x")
        if out is None:
            out = torch.empty_like(x)
        else:
            self._check_tensor(out, "out")
        _check(fn(self._h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                  _stream(stream)), what)
        return out

    def convolve(self, x, out=None, stream=None):
        """y = x (*) h; ``out`` may be ``x`` (in place)."""
        return self._run(lib().pafc_convolve, x, out, stream, "pafc_convolve")

    SYMBOLS = {"inv_laplacian": 0, "inv_laplacian_fd": 1, "heat": 2, "derivative": 3,
               "gaussian": 4}

    def set_symbol(self, kind, *params, stream=None):
        """Make the plan's operator the diagonal symbol `kind` (see
        pafc_set_symbol): 'inv_laplacian', 'inv_laplacian_fd', 'heat' (t),
        'derivative' (axis), 'gaussian' (sigma: the spectrum of the unit-sum
        periodic Gaussian filter).  convolve() then applies it."""
        arr = (ctypes.c_double * max(1, len(params)))(*[float(v) for v in params])
        _check(lib().pafc_set_symbol(self._h, self.SYMBOLS[kind], arr if params else None,
                                     len(params), _stream(stream)), "pafc_set_symbol")

    def convolve_with_filter(self, x, h, out=None, stream=None):
        """y = x (*) h with h transformed inside the call (three transforms
        per call); h becomes the plan's filter."""
        import torch
        self._check_tensor(x, "x")
        self._check_tensor(h, "h")
        if out is None:
            out = torch.empty_like(x)
        else:
            self._check_tensor(out, "out")
        if out.data_ptr() == h.data_ptr():
            raise ValueError("out may not alias h")
        _check(lib().pafc_convolve_with_filter(self._h, ctypes.c_void_p(x.data_ptr()),
                                               ctypes.c_void_p(h.data_ptr()),
                                               ctypes.c_void_p(out.data_ptr()), _stream(stream)),
               "pafc_convolve_with_filter")
        return out

    def convolve_with_filter_noalloc(self, x, h, out, stream=None):
        """As convolve_with_filter, allocating nothing: the per-call spectrum
        goes to the library's fixed per-device array (PAFC_NOALLOC_MAX_BYTES)
        and the plan's own filter is left as it is.  `out` is required.
        Calls that overlap on one device race on that array."""
        self._check_tensor(x, "x")
        self._check_tensor(h, "h")
        self._check_tensor(out, "out")
        if out.data_ptr() == h.data_ptr():
            raise ValueError("out may not alias h")
        _check(lib().pafc_convolve_with_filter_noalloc(
            self._h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(h.data_ptr()),
            ctypes.c_void_p(out.data_ptr()), _stream(stream)),
            "pafc_convolve_with_filter_noalloc (device array of %d bytes)" % NOALLOC_MAX_BYTES)
        return out

    def profile_passes(self, x, out, reps=10, stream=None):
        """Run `reps` convolutions with a HIP event around every kernel launch
        (on the plan's stream).  Returns (mean ms per launch position,
        algorithmic HBM bytes per launch position, ms of every repetition)."""
        self._check_tensor(x, "x")
        self._check_tensor(out, "out")
        n = ctypes.c_int(64)
        ms = (ctypes.c_double * 64)()
        by = (ctypes.c_int64 * 64)()
        per = (ctypes.c_double * int(reps))()
        _check(lib().pafc_profile_passes(self._h, ctypes.c_void_p(x.data_ptr()),
                                         ctypes.c_void_p(out.data_ptr()), _stream(stream),
                                         int(reps), ms, by, per, ctypes.byref(n)),
               "pafc_profile_passes")
        return ([ms[i] for i in range(n.value)], [by[i] for i in range(n.value)],
                [per[i] for i in range(int(reps))])

    def profile_launch(self, x, out, launch, reps=10, stream=None, per_rep=True):
        """Run `reps` convolutions with HIP events around launch `launch`
        and, with `per_rep`, at the start of every repetition.  Returns (mean
        ms of that launch, ms of every repetition, or None without
        `per_rep`)."""
        self._check_tensor(x, "x")
        self._check_tensor(out, "out")
        ms = ctypes.c_double(0.0)
        per = (ctypes.c_double * int(reps))() if per_rep else None
        _check(lib().pafc_profile_launch(self._h, ctypes.c_void_p(x.data_ptr()),
                                         ctypes.c_void_p(out.data_ptr()), _stream(stream),
                                         int(reps), int(launch), ctypes.byref(ms), per),
               "pafc_profile_launch")
        return ms.value, ([per[i] for i in range(int(reps))] if per_rep else None)

    def describe(self):
        """The planner's JSON for this plan's problem (host only)."""
        code = {1: "c64", 2: "c128"}[self._code]
        return describe(self.dims, code, None if not hasattr(self, "_radix") else self._radix,
                        self.variant)

    def forward(self, x, out=None, stream=None):
        """Unscaled forward DFT left in digit-reversed order along every axis."""
        return self._run(lib().pafc_forward, x, out, stream, "pafc_forward")

    def inverse(self, z, out=None, stream=None):
        """Inverse DFT from digit-reversed order to natural order, scaled by 1/N."""
        return self._run(lib().pafc_inverse, z, out, stream, "pafc_inverse")

    def close(self):
        if self._h:
            lib().pafc_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Many independent 1-D convolutions of uneven sizes (pafc_batch_*).

    ``sizes[i]`` is the length of problem i and ``filter_ids[i]`` the filter it
    uses; inputs and outputs are packed 1-D tensors of ``sum(sizes)`` elements.
    """

    FORMS = {"persistent": 0, "levels": 1, "auto": 2, "classes": 3}

    def __init__(self, sizes, filter_ids, nfilters, dtype=None, stream=None, form="auto"):
        import torch
        self.form = form
        self.sizes = [int(n) for n in sizes]
        self.filter_ids = [int(f) for f in filter_ids]
        self.dtype = dtype if dtype is not None else torch.complex128
        self._code = _dtype_code(self.dtype)
        self.total = sum(self.sizes)
        self._h = ctypes.c_void_p()
        n = len(self.sizes)
        st = lib().pafc_batch_plan(ctypes.byref(self._h), n, (ctypes.c_int64 * n)(*self.sizes),
                                   (ctypes.c_int * n)(*self.filter_ids), int(nfilters),
                                   self._code, self.FORMS[form], _stream(stream))
        _check(st, "pafc_batch_plan")

    def set_filter(self, fid, h, domain="spatial", stream=None):
        if not h.is_cuda or h.dtype != self.dtype or not h.is_contiguous():
            raise ValueError("h must be a contiguous %s CUDA tensor" % self.dtype)
        _check(lib().pafc_batch_set_filter(self._h, int(fid), ctypes.c_void_p(h.data_ptr()),
                                           _DOMAINS[domain], _stream(stream)),
               "pafc_batch_set_filter")

    def convolve(self, x, out=None, stream=None):
        import torch
        if not x.is_cuda or x.dtype != self.dtype or x.numel() != self.total or not x.is_contiguous():
            raise ValueError("x must be a packed contiguous %s CUDA tensor of %d elements"
                             % (self.dtype, self.total))
        if out is None:
            out = torch.empty_like(x)
        _check(lib().pafc_batch_convolve(self._h, ctypes.c_void_p(x.data_ptr()),
                                         ctypes.c_void_p(out.data_ptr()), _stream(stream)),
               "pafc_batch_convolve")
        return out

    def profile_levels(self, x, out, reps=10, stream=None):
        """Run `reps` batched convolutions with a HIP event around every
        launch.  Returns (mean ms per level, algorithmic bytes per level, ms of
        every repetition)."""
        n = ctypes.c_int(0)  # first ask for the number of launches
        st = lib().pafc_batch_profile(self._h, ctypes.c_void_p(x.data_ptr()),
                                      ctypes.c_void_p(out.data_ptr()), _stream(stream),
                                      int(reps), (ctypes.c_double * 1)(), None, None,
                                      ctypes.byref(n))
        if st not in (0, 1):
            _check(st, "pafc_batch_profile")
        cap = max(1, n.value)
        n = ctypes.c_int(cap)
        ms = (ctypes.c_double * cap)()
        by = (ctypes.c_int64 * cap)()
        per = (ctypes.c_double * int(reps))()
        _check(lib().pafc_batch_profile(self._h, ctypes.c_void_p(x.data_ptr()),
                                        ctypes.c_void_p(out.data_ptr()), _stream(stream),
                                        int(reps), ms, by, per, ctypes.byref(n)),
               "pafc_batch_profile")
        return ([ms[i] for i in range(n.value)], [by[i] for i in range(n.value)],
                [per[i] for i in range(int(reps))])

    def describe(self):
        need = ctypes.c_size_t(0)
        _check(lib().pafc_batch_describe(self._h, None, 0, ctypes.byref(need)), "describe")
        buf = ctypes.create_string_buffer(need.value)
        _check(lib().pafc_batch_describe(self._h, buf, need.value, ctypes.byref(need)), "describe")
        return json.loads(buf.value.decode())

    @property
    def device_bytes(self):
        b = ctypes.c_size_t(0)
        _check(lib().pafc_batch_device_bytes(self._h, ctypes.byref(b)), "bytes")
        return b.value

    def close(self):
        if self._h:
            lib().pafc_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
