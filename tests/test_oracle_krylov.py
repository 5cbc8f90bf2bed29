"""Pins for the oracle's Krylov solvers.

Pinned against: the direct solution, and the defining minimum-residual
property of GMRES checked by brute force (least squares over an explicit
Krylov basis), plus the CG energy-norm monotonicity.
"""

import numpy as np
import pytest

from oracle import krylov, mg, precond, system


def _operators(pr, inner="exact", kind="tri"):
    A = system.assemble_A(pr)
    if inner == "exact":
        K0inv = precond.ExactK0(pr.K[0])
    else:
        H = mg.Hierarchy(pr.K[0], pr.n, coarsest=4)
        K0inv = H.vcycle
    if kind == "tri":
        M = lambda v: precond.precond_tri(pr, v.reshape(pr.P, pr.N), K0inv).ravel()  # noqa: E731
    else:
        M = lambda v: precond.precond_diag(pr, v.reshape(pr.P, pr.N), K0inv).ravel()  # noqa: E731
    return A, M


@pytest.mark.parametrize("inner", ["exact", "vcycle"])
def test_fgmres_reaches_direct_solution(inner):
    pr = system.build_problem(16, 3, 3, 0.4)
    A, M = _operators(pr, inner)
    F = pr.rhs().ravel()
    x, info = krylov.fgmres(lambda v: A @ v, F, M, restart=30, tol=1e-10)
    assert info["converged"]
    U = system.solve_direct(pr, A=A)
    assert np.linalg.norm(x - U.ravel()) / np.linalg.norm(U) < 1e-8
    assert np.linalg.norm(F - A @ x) / np.linalg.norm(F) < 1e-10


def test_gmres_minimises_residual_over_krylov_space():
    pr = system.build_problem(8, 2, 2, 0.4)
    A, M = _operators(pr, "exact")
    Ad = A.toarray()
    F = pr.rhs().ravel()
    _x, info = krylov.fgmres(lambda v: Ad @ v, F, M, restart=50, tol=1e-13)
    nF = np.linalg.norm(F)
    # explicit basis of K_j(A M, F), orthonormalised for conditioning
    basis = [F / nF]
    for j, est in enumerate(info["est"][:6]):
        Q, _ = np.linalg.qr(np.stack(basis, axis=1))
        AMQ = np.stack([Ad @ M(q) for q in Q.T], axis=1)
        y, *_ = np.linalg.lstsq(AMQ, F, rcond=None)
        best = np.linalg.norm(F - AMQ @ y) / nF
        assert abs(best - est) < 1e-10 + 1e-7 * best
        w = Ad @ M(basis[-1])
        basis.append(w / np.linalg.norm(w))


def test_restarts_still_converge():
    pr = system.build_problem(16, 3, 3, 0.5)
    A, M = _operators(pr, "vcycle")
    F = pr.rhs().ravel()
    x, info = krylov.fgmres(lambda v: A @ v, F, M, restart=3, tol=1e-9)
    assert info["converged"] and info["restarts"] >= 1
    assert np.linalg.norm(F - A @ x) / np.linalg.norm(F) < 1e-9


@pytest.mark.parametrize("inner", ["exact", "vcycle"])
def test_pcg_block_diagonal(inner):
    pr = system.build_problem(16, 3, 3, 0.3)
    A, M = _operators(pr, inner, kind="diag")
    F = pr.rhs().ravel()
    x, info = krylov.pcg(lambda v: A @ v, F, M, tol=1e-10)
    assert info["converged"]
    U = system.solve_direct(pr, A=A)
    assert np.linalg.norm(x - U.ravel()) / np.linalg.norm(U) < 1e-8


def test_block_triangular_needs_fewer_iterations_than_block_diagonal():
    # the qualitative claim of Sec. 6 (Tables 2 and 3) on a small case with large sigma
    pr = system.build_problem(32, 4, 3, 0.5)
    A, Mt = _operators(pr, "vcycle", "tri")
    _, Md = _operators(pr, "vcycle", "diag")
    F = pr.rhs().ravel()
    _, it_t = krylov.fgmres(lambda v: A @ v, F, Mt, restart=30, tol=1e-8)
    _, it_d = krylov.pcg(lambda v: A @ v, F, Md, tol=1e-8)
    assert it_t["converged"] and it_d["converged"]
    assert it_t["iters"] < it_d["iters"]


def test_symmetric_block_gs_preconditioner():
    # B_S (Sec. 4.2): the sweep form equals the assembled (D+L) D^{-1} (D+U) with exact
    # blocks, is symmetric positive definite, and PCG with it converges
    import scipy.sparse.linalg as spla
    pr = system.build_problem(8, 3, 3, 0.4)
    R = np.random.default_rng(3).standard_normal((pr.P, pr.N))
    inner = precond.ExactK0(pr.K[0])
    Z = precond.precond_sym(pr, R, inner)
    BS = precond.assemble_BS(pr)
    Zd = spla.spsolve(BS.tocsc(), R.ravel()).reshape(pr.P, pr.N)
    assert np.max(np.abs(Z - Zd)) < 1e-11 * np.max(np.abs(Zd))
    Bd = BS.toarray()
    assert np.max(np.abs(Bd - Bd.T)) < 1e-12 * np.max(np.abs(Bd))
    assert np.linalg.eigvalsh(0.5 * (Bd + Bd.T)).min() > 0
    # with V-cycle blocks the operator is still symmetric (symmetric cycle)
    H = mg.Hierarchy(pr.K[0], pr.n, coarsest=4)
    Sv = np.stack([precond.precond_sym(pr, e.reshape(pr.P, pr.N), H.vcycle).ravel()
                   for e in np.eye(pr.P * pr.N)[:: max(1, pr.P * pr.N // 40)]])
    idx = np.arange(0, pr.P * pr.N, max(1, pr.P * pr.N // 40))
    sub = Sv[:, idx]
    assert np.max(np.abs(sub - sub.T)) < 1e-12 * np.max(np.abs(sub))


@pytest.mark.parametrize("inner", ["exact", "vcycle"])
def test_gpcg1_equals_pcg_for_a_symmetric_preconditioner(inner):
    pr = system.build_problem(16, 3, 3, 0.3)
    A, M = _operators(pr, inner, kind="diag")
    F = pr.rhs().ravel()
    xc, ic = krylov.pcg(lambda v: A @ v, F, M, tol=1e-10)
    xg, ig = krylov.gpcg1(lambda v: A @ v, F, M, tol=1e-10)
    assert ic["converged"] and ig["converged"]
    assert abs(ic["iters"] - ig["iters"]) <= 1
    n = min(len(ic["est"]), len(ig["est"]))
    assert np.allclose(ic["est"][:n - 1], ig["est"][:n - 1], rtol=1e-6)


def test_gpcg1_and_block_gs_with_bt_converge():
    pr = system.build_problem(16, 3, 3, 0.4)
    A, Mt = _operators(pr, "vcycle", "tri")
    F = pr.rhs().ravel()
    U = system.solve_direct(pr, A=A).ravel()
    for solver in (krylov.gpcg1, krylov.block_gs):
        x, info = solver(lambda v: A @ v, F, Mt, tol=1e-9, max_it=500)
        assert info["converged"]
        assert np.linalg.norm(x - U) / np.linalg.norm(U) < 1e-7
    _, ig = krylov.gpcg1(lambda v: A @ v, F, Mt, tol=1e-9)
    _, ib = krylov.block_gs(lambda v: A @ v, F, Mt, tol=1e-9, max_it=500)
    assert ig["iters"] < ib["iters"]   # the Krylov method beats the stationary iteration
