"""The host setup code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

Builds tests/asan_host_setup.cpp together with the library's host setup source
(host code only, sanitizers on the host pass) and runs it: KL eigenpairs,
chaos tables, cell coefficients, multigrid hierarchies, coarsest inverses and
every coupling plan, and the 2x2 split's coupled hierarchy (K_k on every level, symmetric partner
tables, the coarsest A_hat inverse checked against the assembled matrix) for a spread of options and
both discretisations.
"""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="needs hipcc")
def test_host_setup_is_clean_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "asan_host_setup")
    cmd = ["hipcc", "-x", "hip", "--offload-host-only", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all",
           os.path.join(ROOT, "tests", "asan_host_setup.cpp"),
           os.path.join(ROOT, "paper_1304_1755_amd", "csrc", "sg_setup.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert "ALL OK" in r.stdout
