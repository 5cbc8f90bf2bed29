"""The C-ABI library loads on any machine and exports every symbol its header declares."""

import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "sgbt.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(sg_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = _declared()
    for must in ("sg_setup", "sg_apply", "sg_precond_diag", "sg_precond_tri", "sg_solve"):
        assert must in names


def test_library_exports_every_declared_symbol():
    import paper_1304_1755_amd as sgbt
    lib = sgbt.load_library()
    for name in _declared():
        assert hasattr(lib, name), name
    assert sorted(sgbt.EXPORTED) == _declared()


def test_invalid_options_are_rejected_without_a_device():
    import paper_1304_1755_amd as sgbt
    with pytest.raises(sgbt.SGError) as e:
        sgbt.setup_host(30, 2, 2, 0.3)      # n not a multiple of 4
    assert e.value.code == sgbt.SG_EINVAL
    with pytest.raises(sgbt.SGError):
        sgbt.setup_host(32, 9, 2, 0.3)      # m > 8
    with pytest.raises(sgbt.SGError):
        sgbt.setup_host(32, 2, 2, 0.3, coarsest=12)   # 32 is not 12 * 2^L


def test_discretisation_option_is_checked_without_a_device():
    import ctypes

    import numpy as np

    import paper_1304_1755_amd as sgbt
    lib = sgbt.load_library()
    opt = sgbt.Options(n_cells=16, m=2, p=2, sigma=0.1, corr_len=1.0, colour_mode=0, nu1=2, nu2=2,
                       coarsest_cells=4, discretization=7)
    assert lib.sg_setup_host(ctypes.byref(opt), None, None, None, None, None, None, None, None) == sgbt.SG_EINVAL
    # the Sec. 6 setting takes a0 = 1: a nodal mean field is refused
    a0 = np.ones(17 * 17)
    opt.discretization = sgbt.SG_DISC_P1
    P = ctypes.POINTER(ctypes.c_double)
    assert lib.sg_setup_host(ctypes.byref(opt), a0.ctypes.data_as(P), None, None, None, None, None, None,
                             None) == sgbt.SG_EINVAL
    assert lib.sg_setup_host(ctypes.byref(opt), None, None, None, None, None, None, None, None) == sgbt.SG_OK


def test_bench_refuses_more_than_one_gpu():
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr
