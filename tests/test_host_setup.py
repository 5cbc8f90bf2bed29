"""The library's host-side setup (run without a device) against the oracle.

The two sides are independent implementations: KL roots by bisection vs
Brent's method, Galerkin coarsening on stencils vs sparse P^T K P, an own
Cholesky inverse vs LAPACK.
"""

import numpy as np
import pytest

import sg_inputs
from oracle import fem, kl, mg, system


def _matrix_rows(K, n):
    """(N, 9) stencil view of an interior-node matrix; out-of-grid entries NaN."""
    nx = n - 1
    out = np.full((nx * nx, 9), np.nan)
    K = K.tocsr()
    for y in range(nx):
        for x in range(nx):
            i = y * nx + x
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    X, Y = x + dx, y + dy
                    if 0 <= X < nx and 0 <= Y < nx:
                        out[i, (dy + 1) * 3 + dx + 1] = K[i, Y * nx + X]
    return out


@pytest.mark.parametrize("cfg", ["c1", "c2", "c5"])
def test_cell_coefficients_and_kl(cfg):
    import paper_1304_1755_amd as sgbt
    c = sg_inputs.CONFIGS[cfg]
    a0 = sg_inputs.a0_noise_field(c["n"]) if cfg == "c5" else None
    hs = sgbt.setup_host(c["n"], c["m"], c["p"], c["sigma"], c["corr_len"], a0_nodal=a0)
    oc, data = fem.cell_coefficients(c["n"], c["m"], c["sigma"], c["corr_len"], a0_nodal=a0)
    assert np.max(np.abs(hs["cell"] - oc)) < 1e-13
    assert np.max(np.abs(hs["lam"] - data["lams"]) / data["lams"]) < 1e-13
    amin = np.min(oc[0] - np.abs(oc[1:]).sum(axis=0))
    assert abs(hs["a_min_h"] - amin) < 1e-13


def test_custom_amplitudes():
    import paper_1304_1755_amd as sgbt
    amps = np.array([0.3, -0.2, 0.1])
    hs = sgbt.setup_host(16, 3, 2, 0.7, 0.5, kl_amp=amps)
    oc, _ = fem.cell_coefficients(16, 3, 0.7, 0.5, amps=amps)
    assert np.max(np.abs(hs["cell"] - oc)) < 1e-14


@pytest.mark.parametrize("n,coarsest,a0", [(32, 8, False), (64, 8, True), (16, 4, True)])
def test_multigrid_hierarchy(n, coarsest, a0):
    import paper_1304_1755_amd as sgbt
    a0n = sg_inputs.a0_noise_field(n) if a0 else None
    hs = sgbt.setup_host(n, 2, 1, 0.3, 0.5, a0_nodal=a0n, coarsest=coarsest)
    pr = system.build_problem(n, 2, 1, 0.3, a0_nodal=a0n)
    H = mg.Hierarchy(pr.K[0], n, coarsest=coarsest)
    ref0 = _matrix_rows(H.K[0], n)
    ok = ~np.isnan(ref0)
    assert np.max(np.abs(hs["fine"][ok] - ref0[ok])) < 1e-14
    ref1 = _matrix_rows(H.K[1], n // 2)
    ok1 = ~np.isnan(ref1)
    assert np.max(np.abs(hs["l1"][ok1] - ref1[ok1])) < 1e-13
    Kc = H.K[-1].toarray()
    assert np.max(np.abs(hs["cinv"] - np.linalg.inv(Kc))) < 1e-11 * np.max(np.abs(hs["cinv"]))


def test_exact_coarsest_is_the_whole_grid():
    import paper_1304_1755_amd as sgbt
    n = 16
    hs = sgbt.setup_host(n, 2, 2, 0.3, 0.5, coarsest=n)
    pr = system.build_problem(n, 2, 2, 0.3)
    assert np.max(np.abs(hs["cinv"] @ pr.K[0].toarray() - np.eye((n - 1) ** 2))) < 1e-12


def test_not_coercive_is_a_warning():
    import paper_1304_1755_amd as sgbt
    hs = sgbt.setup_host(16, 4, 2, 3.0, 0.5)
    assert hs["code"] == sgbt.SG_WNOTCOERCIVE and hs["a_min_h"] < 0


@pytest.mark.parametrize("n,m,p,sigma", [(16, 3, 2, 0.3), (32, 6, 1, 0.1)])
def test_p1_setup_matches_the_papers_discretisation(n, m, p, sigma):
    # SG_DISC_P1 against the oracle's Sec. 6 problem: triangle coefficients, the 5-point fine
    # K_0, its Galerkin coarsening with the P1 transfer, and the coarsest inverse
    import paper_1304_1755_amd as sgbt
    from oracle import paper_mode
    hs = sgbt.setup_host(n, m, p, sigma, 1.0, coarsest=4, disc="p1")
    pr = paper_mode.build_problem_paper(n, m, p, sigma)
    assert hs["cell"].shape == pr.cellc.shape
    assert np.max(np.abs(hs["cell"] - pr.cellc)) < 1e-13
    amin = np.min(pr.cellc[0] - np.sqrt(3.0) * np.abs(pr.cellc[1:]).sum(axis=0))
    assert abs(hs["a_min_h"] - amin) < 1e-13
    H = mg.Hierarchy(pr.K[0], n, coarsest=4, transfer="p1")
    ref0 = _matrix_rows(H.K[0], n)
    ok = ~np.isnan(ref0)
    assert np.max(np.abs(hs["fine"][ok] - ref0[ok])) < 1e-14
    ref1 = _matrix_rows(H.K[1], n // 2)
    ok1 = ~np.isnan(ref1)
    assert np.max(np.abs(hs["l1"][ok1] - ref1[ok1])) < 1e-13
    # the P1 coarse operator keeps the triangulation's 7-point pattern: no NW / SE entries
    assert np.max(np.abs(hs["l1"][:, [2, 6]])) < 1e-14
    Kc = H.K[-1].toarray()
    assert np.max(np.abs(hs["cinv"] - np.linalg.inv(Kc))) < 1e-11 * np.max(np.abs(hs["cinv"]))
