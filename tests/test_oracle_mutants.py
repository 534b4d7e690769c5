"""Plant plausible mistakes in a copy of the oracle's C source and check that
the pins catch every one of them (the mutants are compiled and run on the
CPU only, each in a child process since a mutant may corrupt memory; the real
oracle is untouched)."""
import os
import subprocess
import sys

import numpy as np
import pytest

import oracle
from oracle import dense as D
from test_oracle import brute_conv, brute_dft, crand, rel_l2

MUTANTS = {
    "twiddle_sign": ("long double a = -2.0L * ORC_PI", "long double a = 2.0L * ORC_PI"),
    "no_inverse_scale": ("double s = dir > 0 ? 1.0 / (double)n : 1.0;", "double s = 1.0;"),
    "conv_index_swapped": ("int64_t d = jd[a] - kd[a];", "int64_t d = kd[a] - jd[a];"),
    "perm_gather_not_scatter": ("u[2 * perm[i]] = v[2 * i];\n        u[2 * perm[i] + 1] = v[2 * i + 1];",
                                "u[2 * i] = v[2 * perm[i]];\n        u[2 * i + 1] = v[2 * perm[i] + 1];"),
    "shuffle_is_sort": ("tmp[blk + b * r + a] = z[blk + a * mr + b];",
                        "tmp[blk + a * mr + b] = z[blk + b * r + a];"),
    "conj_ignored": ("butterflies(n, t, rho, dir > 0, u, tmp, tw);",
                     "butterflies(n, t, rho, 0, u, tmp, tw);"),
    "stage_twiddle_index": ("orc_omega(k, p * j, &tw", "orc_omega(k, p * (j + 1), &tw"),
    "dropped_term_fft": ("sr += wr * xr - wi * xi;", "sr += wr * xr;"),
    "dropped_term_conv": ("si += xr * hm + xi * hr;", "si += xr * hm;"),
    "hadamard_sign": ("y[2 * i + 1] = ar * bi + ai * br;", "y[2 * i + 1] = ar * bi - ai * br;"),
    "wrong_axis_stride": ("for (int b = a + 1; b < ndim; ++b) stride *= dims[b];",
                          "for (int b = a + 1; b < ndim; ++b) stride *= dims[a];"),
    "small_dft_transposed": ("orc_omega(r, mo * p, &fr[2 * (mo * r + p)]", "orc_omega(r, mo * (p + 1), &fr[2 * (mo * r + p)]"),
}


def pin_suite():
    """Return the list of pins that fail (empty for a correct oracle)."""
    failed = []
    rng = np.random.default_rng(7)

    def c(shape):
        return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)

    def check(name, ok):
        if not ok:
            failed.append(name)

    try:
        for n, rho in ((12, [2, 3, 2]), (16, [4, 4]), (15, [5, 3])):
            x = c(n)
            check("fft_def_%d" % n, np.abs(oracle.fft(x, [rho]) - brute_dft(x)).max() < 1e-11)
            check("ifft_def_%d" % n, np.abs(oracle.fft(x, [rho], inverse=True) - brute_dft(x, True)).max() < 1e-12)
            check("perm_%d" % n, np.array_equal(oracle.perm_index(rho), D.pos_table(rho)))
        x = c((4, 6))
        check("fft_def_2d", np.abs(oracle.fft(x) - brute_dft(x)).max() < 1e-11)
        for shape in ((6,), (3, 4)):
            x, h = c(shape), c(shape)
            ref = brute_conv(x, h)
            check("direct_%s" % (shape,), rel_l2(oracle.conv_direct(x, h), ref) < 1e-13)
            check("fftconv_%s" % (shape,), rel_l2(oracle.conv_fft(x, h), ref) < 1e-13)
    except Exception as e:  # a mutant that crashes is caught too
        failed.append("exception:%s" % e)
    return failed


def test_real_oracle_passes_pin_suite():
    assert pin_suite() == []


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    src = oracle.source_text()
    assert src.count(old) == 1, name
    lib = oracle.compile_variant(src.replace(old, new), str(tmp_path / ("m_%s.so" % name)))
    here = os.path.dirname(os.path.abspath(__file__))
    code = ("import sys; sys.path[:0] = [%r, %r]\n"
            "import oracle, test_oracle_mutants as m\n"
            "with oracle.use_library(%r):\n"
            "    f = m.pin_suite()\n"
            "print('FAILED_PINS', len(f))\n"
            "sys.stdout.flush()\n"
            "import os; os._exit(0)\n") % (here, os.path.dirname(here), lib)
    env = dict(os.environ, OMP_NUM_THREADS="2")
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True,
                       timeout=120, env=env)
    caught = r.returncode != 0 or "FAILED_PINS 0" not in r.stdout
    assert caught, "planted mistake %s went unnoticed" % name
