"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU
only): the oracle's C routines (gcc) and the library's host-only entry
points -- planner, error paths, twiddles, tuning parser, batched argument
checks -- (the planner unit rebuilt with host-side sanitizers by hipcc and
linked against the regular kernel objects; no device call is made).  Any
sanitizer report or wrong status fails the test."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CPP = os.path.join(ROOT, "tests", "cpp")
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
           UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
SAN = ["-fsanitize=address", "-fsanitize=undefined", "-fno-sanitize-recover=all"]


def run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    return r.returncode, r.stdout + r.stderr


@pytest.mark.skipif(shutil.which("gcc") is None, reason="no gcc")
def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_san")
    rc, out = run(["gcc", "-O1", "-g"] + SAN +
                  [os.path.join(CPP, "oracle_sanitized.c"),
                   os.path.join(ROOT, "oracle", "oracle.c"), "-lm", "-o", exe])
    assert rc == 0, out
    rc, out = run([exe], env=ENV)
    assert rc == 0 and "0 failures" in out and "runtime error" not in out, out


def test_planner_under_sanitizers(tmp_path):
    hipcc = "/opt/rocm/bin/hipcc"
    build = os.path.join(ROOT, "paper_2506_12718_amd", "_build")
    objs = [os.path.join(build, f)
            for f in ("pafc_kernels.hip.o", "pafc_pipe.hip.o", "pafc_pipe_batch.hip.o")]
    if not os.path.exists(hipcc) or not all(os.path.exists(o) for o in objs):
        pytest.skip("needs hipcc and the library's kernel objects (build first)")
    inc = ["-I" + os.path.join(ROOT, "include"),
           "-I" + os.path.join(ROOT, "paper_2506_12718_amd", "csrc")]
    # host-side sanitizers only: each -fsanitize= follows -Xarch_host
    host_san = [f for s in SAN for f in ("-Xarch_host", s)]
    dev = ["-x", "hip", "--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang",
           "-packed-fp32-ops"]
    api = str(tmp_path / "api.o")
    rc, out = run([hipcc, "-O1", "-g", "-std=c++17", "-fPIC", "-Wno-unused-command-line-argument"]
                  + inc + dev + host_san +
                  ["-c", os.path.join(ROOT, "paper_2506_12718_amd", "csrc", "pafc_api.cpp"),
                   "-o", api])
    assert rc == 0, out
    drv = str(tmp_path / "drv.o")  # host code only: the C ABI header
    rc, out = run(["g++", "-O1", "-g", "-std=c++17"] + inc + SAN +
                  ["-c", os.path.join(CPP, "host_entry_points.cpp"), "-o", drv])
    assert rc == 0, out
    exe = str(tmp_path / "host_san")
    rc, out = run([hipcc, "--offload-arch=gfx950", "-Wno-unused-command-line-argument"] +
                  host_san + [drv, api] + objs + ["-o", exe])
    assert rc == 0, out
    rc, out = run([exe], env=ENV, timeout=600)
    assert rc == 0 and "0 failures" in out and "runtime error" not in out, out
