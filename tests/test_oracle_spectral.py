"""Pins for the oracle's preconditioners against the spectral results of Sec. 5.

* Theorem 1: the spectrum of A B_T^{-1} is real and in (0, 1].
* For block-tridiagonal (consistently ordered) A, block Gauss-Seidel and block
  Jacobi spectra are related by Young's theorem, so
  sigma(B_T^{-1} A) = {1} u {1 - (1 - nu)^2 : nu in sigma(B_D^{-1} A)}.
* Lemma 1 for the paper's 2x2 split with exact A-hat.
* Theorem 2 (p = 1): sigma(B_T^{-1} A) = {1} u sigma(I - c sum_k (K_0^{-1} K_k)^2)
  with c = 1/3 for xi ~ U[-1, 1], and the printed lower bound.
* The ideal preconditioner with the exact Schur complement gives GMRES
  convergence in at most two iterations (remark after eq. (block-LU)).
* The level sweep equals a direct solve with the assembled block
  lower-triangular matrix.
"""

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse.linalg as spla

from oracle import krylov, precond, system


def _dense(prob):
    A = system.assemble_A(prob).toarray()
    BT = precond.assemble_BT(prob).toarray()
    BD = precond.assemble_BD(prob).toarray()
    return A, BT, BD


@pytest.mark.parametrize("sigma", [0.2, 0.5])
def test_theorem1_and_young_relation(sigma):
    pr = system.build_problem(6, 3, 3, sigma)
    A, BT, BD = _dense(pr)
    mu = np.linalg.eigvals(np.linalg.solve(BT, A))
    # the eigenvalue 1 is defective (Jordan blocks), so it is computed to O(sqrt(eps))
    assert np.max(np.abs(mu.imag)) < 1e-6
    mu = np.sort(mu.real)
    assert mu.min() > 0.0 and mu.max() < 1.0 + 1e-6
    nu = sla.eigh(A, BD, eigvals_only=True)
    young = 1.0 - (1.0 - nu) ** 2
    # set equality away from 1 (both directions); eigenvalues of the
    # nonsymmetric B_T^{-1} A carry O(sqrt(eps)) error, hence the tolerance
    far_mu = mu[mu < 1 - 1e-5]
    far_y = young[young < 1 - 1e-5]
    assert len(far_mu) > 0
    for v in far_mu:
        assert np.min(np.abs(far_y - v)) < 1e-6
    for v in far_y:
        assert np.min(np.abs(mu - v)) < 1e-6


def test_lemma1_two_by_two_split():
    pr = system.build_problem(6, 2, 3, 0.4)
    A = system.assemble_A(pr).toarray()
    nA = pr.offsets[-2] * pr.N
    Ahat, Wt, W, D = A[:nA, :nA], A[:nA, nA:], A[nA:, :nA], A[nA:, nA:]
    B = np.zeros_like(A)
    B[:nA, :nA] = Ahat
    B[nA:, :nA] = W
    B[nA:, nA:] = D
    mu = np.linalg.eigvals(A @ np.linalg.inv(B))
    assert np.max(np.abs(mu.imag)) < 1e-8
    S = D - W @ np.linalg.solve(Ahat, Wt)
    gen = sla.eigh(S, D, eigvals_only=True)
    assert gen.min() > 0 and gen.max() <= 1 + 1e-12
    cand = np.concatenate([[1.0], gen])
    for v in mu.real:
        assert np.min(np.abs(cand - v)) < 1e-7


def test_theorem2_p1():
    pr = system.build_problem(8, 3, 1, 0.5)
    A, BT, _ = _dense(pr)
    mu = np.sort(np.linalg.eigvals(np.linalg.solve(BT, A)).real)
    K0 = pr.K[0].toarray()
    T = sum(np.linalg.matrix_power(np.linalg.solve(K0, pr.K[k].toarray()), 2) for k in range(1, pr.m + 1))
    ev = np.sort(np.linalg.eigvals(np.eye(pr.N) - T / 3.0).real)
    cand = np.concatenate([ev, np.ones(len(mu) - len(ev))])
    assert np.max(np.abs(np.sort(cand) - mu)) < 1e-9
    # printed bound: mu > 1 - c sum_k lambda_k ||b_k||^2_inf / abar^2, c = 1/3,
    # with the discrete sup of |c_k / c_0| over cells in place of sqrt(lambda_k)||b_k||/abar
    bound = 1.0 - sum(np.max(np.abs(pr.cellc[k] / pr.cellc[0])) ** 2 for k in range(1, pr.m + 1)) / 3.0
    assert mu.min() >= bound - 1e-12


def test_ideal_block_triangular_two_iterations():
    pr = system.build_problem(6, 2, 2, 0.4)
    A = system.assemble_A(pr).toarray()
    nA = pr.offsets[-2] * pr.N
    Ahat, Wt, W, D = A[:nA, :nA], A[:nA, nA:], A[nA:, :nA], A[nA:, nA:]
    SD = D - W @ np.linalg.solve(Ahat, Wt)
    Bid = np.zeros_like(A)
    Bid[:nA, :nA] = Ahat
    Bid[nA:, :nA] = W
    Bid[nA:, nA:] = SD
    F = pr.rhs().ravel()
    x, info = krylov.fgmres(lambda v: A @ v, F, lambda v: np.linalg.solve(Bid, v),
                            restart=10, tol=1e-12)
    assert info["converged"] and info["iters"] <= 2


def test_level_sweep_equals_block_lower_solve():
    pr = system.build_problem(8, 3, 3, 0.4)
    R = np.random.default_rng(2).standard_normal((pr.P, pr.N))
    Z = precond.precond_tri(pr, R, precond.ExactK0(pr.K[0]))
    BT = precond.assemble_BT(pr)
    Zd = spla.spsolve(BT.tocsc(), R.ravel()).reshape(pr.P, pr.N)
    assert np.max(np.abs(Z - Zd)) < 1e-12 * np.max(np.abs(Zd))
    Zdiag = precond.precond_diag(pr, R, precond.ExactK0(pr.K[0]))
    BD = precond.assemble_BD(pr)
    assert np.max(np.abs(Zdiag.ravel() - spla.spsolve(BD.tocsc(), R.ravel()))) < 1e-12 * np.max(np.abs(Zdiag))
