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
