"""The allocation-free QoI entry point (sg_qoi_noalloc) against sg_qoi, through the C ABI.

Two calls in a row on one GPU, the second with a smaller input (fewer nodes and
modes), each compared with sg_qoi on the same solution: the two share their
kernels and fixed-order reductions, so the results agree exactly.
"""

import numpy as np
import pytest
import torch

from gpu_util import note

pytestmark = pytest.mark.gpu


def _case(n, m, p, sigma):
    import paper_1304_1755_amd as sgbt
    import sg_inputs
    g = sgbt.Problem(n, m, p, sigma, a0_nodal=sg_inputs.a0_noise_field(n))
    U, info = g.solve(precond="tri", restart=30, rtol=1e-10, max_it=300)
    assert info["status"] == 0
    J_ref, q_ref = g.qoi(U)
    q = torch.full((g.P,), np.nan, dtype=torch.float64, device="cuda")
    J = torch.full((1,), np.nan, dtype=torch.float64, device="cuda")
    g.qoi_noalloc(U, q, J)
    torch.cuda.synchronize()
    qh, Jh = q.cpu().numpy(), float(J.cpu().numpy()[0])
    g.close()
    return qh, Jh, q_ref, J_ref


def test_noalloc_qoi_matches_qoi_on_two_calls():
    note("no-alloc qoi: n=64 m=4 p=3 then n=32 m=2 p=2")
    q1, J1, r1, R1 = _case(64, 4, 3, 0.3)
    q2, J2, r2, R2 = _case(32, 2, 2, 0.2)   # second call: fewer nodes and modes
    assert q1.shape == (35,) and q2.shape == (6,)
    assert np.array_equal(q1, r1) and J1 == R1, (np.max(np.abs(q1 - r1)), J1 - R1)
    assert np.array_equal(q2, r2) and J2 == R2, (np.max(np.abs(q2 - r2)), J2 - R2)


def test_noalloc_qoi_rejects_p1_and_null():
    import paper_1304_1755_amd as sgbt
    note("no-alloc qoi: error paths")
    g = sgbt.Problem(16, 2, 2, 0.1, corr_len=1.0, coarsest=4, disc="p1")
    U = g.empty()
    U.zero_()
    q = torch.zeros((g.P,), dtype=torch.float64, device="cuda")
    J = torch.zeros((1,), dtype=torch.float64, device="cuda")
    with pytest.raises(sgbt.SGError) as e:
        g.qoi_noalloc(U, q, J)
    assert e.value.code == sgbt.SG_EINVAL
    g.close()
    lib = sgbt.load_library()
    assert lib.sg_qoi_noalloc(None, None, None, None) == sgbt.SG_EINVAL
