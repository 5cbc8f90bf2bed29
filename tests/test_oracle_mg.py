"""Pins for the oracle's multigrid V-cycle.

Pinned against: Galerkin coarsening of the constant-coefficient Q1
operator reproducing the coarse Q1 stencil (nested FE spaces), brute-force
scalar Gauss-Seidel loops on tiny grids, fixed-point and symmetry
properties of the cycle, exactness when the fine grid is the coarsest one,
and the contraction of the V(2,2) error propagator.
"""

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import fem, mg


def test_rap_constant_coefficient_is_coarse_q1():
    n = 16
    K = fem.assemble_stiffness(n, np.ones(n * n))
    H = mg.Hierarchy(K, n, coarsest=4)
    for Kc, nc in zip(H.K[1:], H.ns[1:]):
        ref = fem.assemble_stiffness(nc, np.ones(nc * nc))
        assert abs(Kc - ref).max() < 1e-14


def _brute_gs(K, f, u, order_groups, jacobi_in_group):
    """Scalar loops: visit groups in order; inside a group either sequential GS or a frozen snapshot."""
    K = K.toarray()
    u = u.copy()
    for grp in order_groups:
        snap = u.copy()
        for i in grp:
            src = snap if jacobi_in_group else u
            s = f[i]
            for j in range(len(u)):
                if j != i:
                    s -= K[i, j] * src[j]
            u[i] = s / K[i, i]
    return u


@pytest.mark.parametrize("mode", ["four", "rb"])
def test_colour_sweep_matches_scalar_loops(mode):
    n = 8
    rng = np.random.default_rng(5)
    K = fem.assemble_stiffness(n, rng.uniform(0.5, 2.0, n * n))
    H = mg.Hierarchy(K, n, coarsest=8, colour_mode=mode)
    f = rng.standard_normal((n - 1) ** 2)
    u0 = rng.standard_normal((n - 1) ** 2)
    groups = mg.colours(n, mode)
    fwd = H.smooth(0, u0.copy(), f, reverse=False)
    assert np.max(np.abs(fwd - _brute_gs(K, f, u0, groups, mode == "rb"))) < 1e-13
    bwd = H.smooth(0, u0.copy(), f, reverse=True)
    assert np.max(np.abs(bwd - _brute_gs(K, f, u0, groups[::-1], mode == "rb"))) < 1e-13


def test_lexicographic_sweep_matches_scalar_loops():
    # lexicographic point Gauss-Seidel (nodes x-fastest, one at a time): forward in node order
    # before the coarse correction, backward in reverse node order after it
    n = 8
    rng = np.random.default_rng(11)
    K = fem.assemble_stiffness(n, rng.uniform(0.5, 2.0, n * n))
    H = mg.Hierarchy(K, n, coarsest=8, colour_mode="lex")
    N = (n - 1) ** 2
    f = rng.standard_normal(N)
    u0 = rng.standard_normal(N)
    singles = [[i] for i in range(N)]
    fwd = H.smooth(0, u0.copy(), f, reverse=False)
    assert np.max(np.abs(fwd - _brute_gs(K, f, u0, singles, False))) < 1e-13
    bwd = H.smooth(0, u0.copy(), f, reverse=True)
    assert np.max(np.abs(bwd - _brute_gs(K, f, u0, singles[::-1], False))) < 1e-13
    # a plausible slip, the wrong direction, is caught
    assert np.max(np.abs(bwd - fwd)) > 1e-3


def test_four_colours_never_touch():
    n = 10
    K = fem.assemble_stiffness(n, np.ones(n * n)).toarray()
    for c in mg.colours(n, "four"):
        blk = K[np.ix_(c, c)]
        assert np.count_nonzero(blk - np.diag(np.diag(blk))) == 0


def _vcycle_matrix(H, N):
    return np.stack([H.vcycle(e) for e in np.eye(N)], axis=1)


@pytest.mark.parametrize("mode", ["four", "rb", "lex"])
def test_vcycle_symmetric_positive_definite_and_contracting(mode):
    n = 16
    rng = np.random.default_rng(6)
    K = fem.assemble_stiffness(n, rng.uniform(0.5, 2.0, n * n))
    H = mg.Hierarchy(K, n, coarsest=4, colour_mode=mode, nu1=2, nu2=2)
    N = (n - 1) ** 2
    V = _vcycle_matrix(H, N)
    assert np.max(np.abs(V - V.T)) < 1e-12 * np.max(np.abs(V))
    assert np.linalg.eigvalsh(0.5 * (V + V.T)).min() > 0
    # error propagator I - V K, contraction factor in the energy norm
    Kd = K.toarray()
    Lc = np.linalg.cholesky(Kd)
    E = np.eye(N) - V @ Kd
    rho = np.linalg.norm(Lc.T @ E @ np.linalg.inv(Lc.T), 2)
    assert rho < 0.2


def test_exact_solution_is_a_fixed_point():
    n = 16
    K = fem.assemble_stiffness(n, np.random.default_rng(7).uniform(0.5, 2.0, n * n))
    H = mg.Hierarchy(K, n, coarsest=4)
    f = np.random.default_rng(8).standard_normal((n - 1) ** 2)
    u = spla.spsolve(K.tocsc(), f)
    for rev in (False, True):
        assert np.max(np.abs(H.smooth(0, u.copy(), f, rev) - u)) < 1e-13


def test_single_level_cycle_is_exact_and_batched():
    n = 8
    K = fem.assemble_stiffness(n, np.random.default_rng(9).uniform(0.5, 2.0, n * n))
    H = mg.Hierarchy(K, n, coarsest=8)
    F = np.random.default_rng(10).standard_normal(((n - 1) ** 2, 3))
    U = H.vcycle(F)
    assert np.max(np.abs(K @ U - F)) < 1e-12
    H2 = mg.Hierarchy(K, n, coarsest=2)
    Ub = H2.vcycle(F)
    for j in range(3):
        assert np.max(np.abs(Ub[:, j] - H2.vcycle(F[:, j]))) < 1e-15
