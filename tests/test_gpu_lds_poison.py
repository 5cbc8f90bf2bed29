"""The LDS-poison debug build (libsgbt_poison.so, built with -DSG_LDS_POISON by
paper_1304_1755_amd/build.py): every kernel with an LDS tile fills its LDS with NaN before use, so
a value read before it was written turns the output into NaN.  This test runs GPU parity suites of
the apply, the V-cycles in every kernel form, the preconditioners (including the 2x2 split), the
edge shapes, the solves and the adjoint gradient against that build, in a child process that
loads it through SGBT_LIBRARY: they must pass there as they do against the normal build.
"""

import os
import subprocess
import sys

import pytest

from gpu_util import note

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
POISON_LIB = os.path.join(ROOT, "paper_1304_1755_amd", "libsgbt_poison.so")

SUITES = [
    "tests/test_gpu_apply.py::test_apply_matches_oracle",
    "tests/test_gpu_apply.py::test_apply_degenerate_shapes",
    "tests/test_gpu_mg.py",
    "tests/test_gpu_edges.py",
    "tests/test_gpu_split.py::test_split_preconditioner_matches_oracle",
    "tests/test_gpu_paper_mode.py::test_lexicographic_vcycle_matches_oracle",
    "tests/test_gpu_solve.py::test_c2_bt_gmres_and_bd_pcg",
    "tests/test_gpu_solve.py::test_c3_copy_mixed_precision",
    "tests/test_gpu_adjoint.py::test_gradient_matches_oracle_small",
]


def test_parity_suites_pass_with_poisoned_lds():
    note("lds poison build: parity suites in a child process")
    assert os.path.exists(POISON_LIB), f"{POISON_LIB} is missing: build it with __graft_entry__.build()"
    env = dict(os.environ, SGBT_LIBRARY=POISON_LIB)
    cmd = [sys.executable, "-u", "-m", "pytest", "-x", "-q", "-m", "gpu", "-p", "no:cacheprovider",
           "--timeout", "300", "--timeout-method", "thread", *SUITES]
    r = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    tail = "\n".join((r.stdout + r.stderr).splitlines()[-30:])
    print(tail, flush=True)
    assert r.returncode == 0, tail
    assert " passed" in r.stdout and "failed" not in r.stdout, tail
