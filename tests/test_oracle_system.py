"""Pins for the oracle's Galerkin system, its solution and the PCE statistics.

Pinned against: symmetry / positive definiteness (Sec. 3), the sigma = 0
reduction to the deterministic problem, the closed form for spatially
constant KL fields, the exact stochastic-collocation identity for m = 1
(Gauss-Legendre nodes), and tensor Gauss quadrature of the PCE moments.
"""

import itertools

import numpy as np
import pytest
import scipy.sparse.linalg as spla
from numpy.polynomial import legendre as npleg

from oracle import fem, indexset, qoi, system


def test_A_symmetric_positive_definite():
    pr = system.build_problem(16, 3, 2, 0.3)
    A = system.assemble_A(pr)
    assert abs(A - A.T).max() == 0.0
    ev = np.linalg.eigvalsh(A.toarray())
    assert ev.min() > 0.0


def test_matrix_free_apply_matches_assembled():
    pr = system.build_problem(8, 3, 3, 0.4)
    A = system.assemble_A(pr)
    U = np.random.default_rng(1).uniform(-1, 1, (pr.P, pr.N))
    assert np.max(np.abs(system.apply(pr, U).ravel() - A @ U.ravel())) < 1e-13


def test_sigma_zero_is_the_deterministic_solve():
    pr = system.build_problem(16, 3, 2, 0.0)
    U = system.solve_direct(pr)
    u_det = spla.spsolve(pr.K[0].tocsc(), pr.f)
    assert np.max(np.abs(U[0] - u_det)) < 1e-14
    assert np.max(np.abs(U[1:])) < 1e-14


def test_constant_kl_fields_closed_form():
    # c_{k,e} = gamma_k on every cell => A = (I + sum gamma_k G_k) (x) K_unit
    pr = system.build_problem(8, 3, 3, 0.3)
    gam = np.array([1.0, 0.2, -0.15, 0.1])
    pr.cellc = np.repeat(gam[:, None], pr.n * pr.n, axis=1)
    pr.K = [fem.assemble_stiffness(pr.n, pr.cellc[k]) for k in range(pr.m + 1)]
    U = system.solve_direct(pr)
    Kunit = fem.assemble_stiffness(pr.n, np.ones(pr.n * pr.n))
    Mmat = (sum(g * G for g, G in zip(gam, pr.G))).toarray()
    e0 = np.zeros(pr.P)
    e0[0] = 1.0
    expect = np.outer(np.linalg.solve(Mmat, e0), spla.spsolve(Kunit.tocsc(), pr.f))
    assert np.max(np.abs(U - expect)) < 1e-14


@pytest.mark.parametrize("p", [1, 3, 5])
def test_m1_galerkin_equals_collocation_at_gauss_nodes(p):
    # m = 1: G_1 is the Jacobi matrix of order p+1, so the Galerkin solution
    # evaluated at its Gauss-Legendre nodes equals the deterministic solutions there.
    pr = system.build_problem(16, 1, p, 0.5)
    U = system.solve_direct(pr)
    nodes, _ = npleg.leggauss(p + 1)
    for xq in nodes:
        u_det = spla.spsolve((pr.K[0] + xq * pr.K[1]).tocsc(), pr.f)
        psi = np.array([np.sqrt(2 * j + 1) * npleg.legval(xq, np.eye(p + 1)[j]) for j in range(p + 1)])
        u_sg = psi @ U
        assert np.max(np.abs(u_sg - u_det)) < 1e-13


def test_pce_moments_by_tensor_quadrature():
    # eq. (PCE_u) with an orthonormal basis: E[u] = U_0, E[u^2] = sum U_a^2
    m, p = 2, 3
    pr = system.build_problem(8, m, p, 0.4)
    U = system.solve_direct(pr)
    x, w = npleg.leggauss(p + 1)
    mean = np.zeros(pr.N)
    second = np.zeros(pr.N)
    for (i1, x1), (i2, x2) in itertools.product(enumerate(x), enumerate(x)):
        wq = w[i1] * w[i2] / 4.0
        psi = np.array([np.sqrt((2 * a + 1) * (2 * b + 1))
                        * npleg.legval(x1, np.eye(p + 1)[a]) * npleg.legval(x2, np.eye(p + 1)[b])
                        for (a, b) in indexset.multi_indices(m, p)])
        u = psi @ U
        mean += wq * u
        second += wq * u * u
    E, V = qoi.mean_variance(U)
    assert np.max(np.abs(mean - E)) < 1e-15
    assert np.max(np.abs(second - mean ** 2 - V)) < 1e-15


def test_coercivity_margins_of_the_workloads():
    # a_min,h > 0 guarantees SPD local G-combinations; the workloads must satisfy it
    for n, m, p, s, L, lo in [(32, 2, 2, 0.3, 0.5, 0.6), (128, 4, 3, 0.5, 0.5, 0.2),
                              (64, 6, 4, 0.4, 0.5, 0.15), (256, 8, 3, 0.5, 0.25, 0.0)]:
        c, _ = fem.cell_coefficients(n, m, s, L)
        assert np.min(c[0] - np.abs(c[1:]).sum(axis=0)) > lo
