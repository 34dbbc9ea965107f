"""The per-state validation rules on the host, under AddressSanitizer and
UndefinedBehaviorSanitizer (CPU only).

tests/native/validate_check.cpp calls the library's validate_state (the same
__host__ __device__ function the kernels inline) on malformed ragged-CSR
states whose knot arrays are allocated at exactly n_knots entries, so an
offset or count that sent the validator past them would be reported by the
sanitizer.  The status words must match the documented LPS_ST_* bits.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

ST_COUNT, ST_ORDER, ST_COVER, ST_NONFINITE, ST_AMPLITUDE = 1, 2, 4, 8, 16
EXPECTED = [0,              # valid
            ST_COUNT,       # range past the end of the knot arrays
            ST_COUNT,       # no knots at all
            ST_COUNT,       # offset before the start
            ST_COUNT,       # negative count
            ST_COUNT,       # one knot
            ST_COUNT,       # more than k_max knots
            ST_NONFINITE,   # non-finite abscissa
            ST_ORDER,       # unsorted abscissae
            ST_COVER,       # edge knots do not enclose the band
            ST_AMPLITUDE,   # A_OMS <= 0
            ST_NONFINITE]   # a disabled spline, then a non-finite height


@pytest.mark.skipif(not (os.path.exists(HIPCC) or shutil.which("hipcc")), reason="hipcc not available")
def test_validate_state_under_host_sanitizers(tmp_path):
    exe = str(tmp_path / "validate_check")
    cmd = [HIPCC, "-x", "hip", "--offload-arch=gfx950", "-O1", "-g", "-std=c++17",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all",
           "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_2507_06300_amd", "csrc"),
           os.path.join(ROOT, "tests", "native", "validate_check.cpp"), "-o", exe]
    b = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert b.returncode == 0, b.stdout + b.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120, env=env)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr
    got = [int(v) for v in r.stdout.split()]
    assert got == EXPECTED, got
