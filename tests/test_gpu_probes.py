"""The streaming probes behind the middle pass's bandwidth ceiling
(pafc_stream_copy kinds tile_copy / tile_mul): they move exactly the data
their definition says, on a small array of 256 rows x 64 columns."""
import numpy as np
import pytest

from gpu_util import to_host, torch

pytestmark = pytest.mark.gpu


def test_tile_probes_move_what_they_say():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2506_12718_amd as m
    rows, cols = 256, 64
    n = rows * cols
    rng = np.random.default_rng(2)
    src = rng.standard_normal(2 * n) + 1j * rng.standard_normal(2 * n)
    s = torch.from_numpy(src).cuda()
    y = torch.zeros(n, dtype=torch.complex128, device="cuda")
    m.stream_copy(s[:n], y, kind="tile_copy")
    assert np.array_equal(to_host(y), src[:n])
    y.zero_()
    m.stream_copy(s, y, kind="tile_mul")
    x = src[:n].reshape(rows, cols)
    h = src[n:]
    want = np.empty((rows, cols), complex)
    for t in range(cols // 16):  # tile t: all rows x columns 16t..16t+15, h in tile order
        want[:, 16 * t:16 * t + 16] = x[:, 16 * t:16 * t + 16] * \
            h[4096 * t:4096 * (t + 1)].reshape(rows, 16)
    got = to_host(y).reshape(rows, cols)
    assert np.abs(got - want).max() <= 4e-16 * np.abs(want).max()
