"""GPU parity at the edges of the supported shapes, for both discretisations.

The smallest grid (n = 4: three interior nodes per side, one row pair and a
half), the coarsest grid of 2 cells, a single chaos mode (m = 0 or p = 0),
the widest block (m = 5, p = 5: P = 252, four wavefronts with 60 lanes in the
last), m = 8 with p = 1, and p = 8 with m = 1: operator apply and residual,
the block-triangular and block-symmetric preconditioners, and a solve
checked against the oracle's assembled matrix.
"""

import numpy as np
import pytest

import sg_inputs
from gpu_util import note, rel_max, to_dev, to_host
from oracle import mg, paper_mode, precond, system

pytestmark = pytest.mark.gpu

CASES = [
    # disc, n, m, p, sigma, coarsest
    ("q1", 4, 2, 2, 0.3, 2),
    ("q1", 8, 0, 0, 0.0, 2),
    ("q1", 16, 5, 5, 0.2, 4),
    ("q1", 16, 8, 1, 0.2, 8),
    ("q1", 32, 1, 8, 0.4, 8),
    ("p1", 4, 2, 2, 0.3, 2),
    ("p1", 8, 3, 0, 0.2, 2),
    ("p1", 16, 5, 5, 0.1, 4),
    ("p1", 32, 8, 1, 0.2, 4),
]


def _problems(disc, n, m, p, sigma, coarsest):
    import paper_1304_1755_amd as sgbt
    if disc == "q1":
        g = sgbt.Problem(n, m, p, sigma, coarsest=coarsest)
        o = system.build_problem(n, m, p, sigma)
        H = mg.Hierarchy(o.K[0], n, coarsest=coarsest)
    else:
        g = sgbt.Problem(n, m, p, sigma, corr_len=1.0, coarsest=coarsest, disc="p1")
        o = paper_mode.build_problem_paper(n, m, p, sigma)
        H = mg.Hierarchy(o.K[0], n, coarsest=coarsest, transfer="p1")
    return g, o, H


@pytest.mark.parametrize("disc,n,m,p,sigma,coarsest", CASES)
def test_edge_shapes_match_oracle(disc, n, m, p, sigma, coarsest):
    note(f"edge {disc} n={n} m={m} p={p} coarsest={coarsest}")
    g, o, H = _problems(disc, n, m, p, sigma, coarsest)
    assert (g.N, g.P) == (o.N, o.P)
    U = sg_inputs.uniform_block(g.N, g.P, seed=3)
    F = sg_inputs.uniform_block(g.N, g.P, seed=4)
    ref = system.apply(o, U.T).T
    assert rel_max(to_host(g.apply(to_dev(U))), ref) < 1e-13
    assert rel_max(to_host(g.residual(to_dev(F), to_dev(U))), F - ref) < 1e-13
    for kind, fn in (("tri", precond.precond_tri), ("sym", precond.precond_sym)):
        Z = to_host(g.precond(to_dev(F), kind=kind))
        assert rel_max(Z, fn(o, F.T, H.vcycle).T) < 1e-11, kind
    A = system.assemble_A(o)
    Fr = o.rhs().ravel()
    X, info = g.solve(precond="tri", restart=20, rtol=1e-10, max_it=200)
    assert info["status"] == 0
    Xh = to_host(X).T.ravel()
    assert np.linalg.norm(Fr - A @ Xh) / np.linalg.norm(Fr) < 1e-10
    g.close()
