"""GPU parity of the matrix-free SG operator (Sec. 3.1, eq. (tensor-product)) against the oracle.

Tolerance: relative max-norm 1e-10 for the double apply; the float-input
variant is compared with the oracle applied to the same float-rounded input.
Full sizes use the separable-input closed form Y = sum_r sum_k (K_k v_r)(G_k w_r)^T.
"""

import numpy as np
import pytest
import torch

import sg_inputs
from gpu_util import oracle_problem, note, rel_max, to_dev, to_host
from oracle import system

pytestmark = pytest.mark.gpu

TOL = 1e-10


def _prob(cfg, **over):
    import paper_1304_1755_amd as sgbt
    c = dict(sg_inputs.CONFIGS[cfg])
    c.update(over)
    a0 = sg_inputs.a0_noise_field(c["n"]) if cfg == "c5" else None
    g = sgbt.Problem(c["n"], c["m"], c["p"], c["sigma"], c["corr_len"], a0_nodal=a0)
    o = system.build_problem(c["n"], c["m"], c["p"], c["sigma"], c["corr_len"], a0_nodal=a0)
    return g, o


@pytest.mark.parametrize("cfg", ["c1", "c2", "c5", "c3_65", "c4_129"])
def test_apply_matches_oracle(cfg):
    note(f"apply f64 {cfg}")
    g, o = _prob(cfg)
    assert (g.N, g.P) == (o.N, o.P)
    U = sg_inputs.uniform_block(g.N, g.P, seed=1234)
    Y = to_host(g.apply(to_dev(U)))
    ref = system.apply(o, U.T).T
    assert rel_max(Y, ref) < TOL
    note(f"apply mixed {cfg}")
    U32 = U.astype(np.float32)
    Ym = to_host(g.apply(to_dev(U32, torch.float32), prec=2))
    refm = system.apply(o, U32.astype(np.float64).T).T
    assert rel_max(Ym, refm) < TOL
    note(f"residual {cfg}")
    F = sg_inputs.uniform_block(g.N, g.P, seed=99)
    R = to_host(g.residual(to_dev(F), to_dev(U)))
    assert np.max(np.abs(R - (F - ref))) < TOL * np.max(np.abs(ref))
    g.close()


@pytest.mark.parametrize("sigma,m,p", [(0.0, 0, 0), (0.3, 1, 4), (0.3, 3, 0), (0.5, 2, 6)])
def test_apply_degenerate_shapes(sigma, m, p):
    import paper_1304_1755_amd as sgbt
    note(f"apply degenerate m={m} p={p}")
    n = 16
    g = sgbt.Problem(n, m, p, sigma)
    o = system.build_problem(n, m, p, sigma)
    U = sg_inputs.uniform_block(g.N, g.P, seed=3)
    Y = to_host(g.apply(to_dev(U)))
    assert rel_max(Y, system.apply(o, U.T).T) < TOL
    g.close()


def test_rhs_is_e0_times_load():
    import paper_1304_1755_amd as sgbt
    note("rhs")
    g = sgbt.Problem(32, 2, 2, 0.3)
    o = system.build_problem(32, 2, 2, 0.3)
    F = to_host(g.rhs())
    assert np.array_equal(F, o.rhs().T)
    g.close()


@pytest.mark.parametrize("cfg", ["c3", "c4"])
def test_apply_full_size_separable(cfg):
    note(f"apply full size separable {cfg}")
    import paper_1304_1755_amd as sgbt
    c = sg_inputs.CONFIGS[cfg]
    g = sgbt.Problem(c["n"], c["m"], c["p"], c["sigma"], c["corr_len"])
    o = oracle_problem(cfg)
    V, W = sg_inputs.separable_factors(g.N, g.P, rank=2)
    U = V.T @ W                                     # (N, P)
    Y = to_host(g.apply(to_dev(U)))
    ref = np.zeros((g.N, g.P))
    for r in range(2):
        for Gk, Kk in zip(o.G, o.K):
            ref += np.outer(Kk @ V[r], Gk @ W[r])
    assert rel_max(Y, ref) < TOL
    g.close()
