"""Stochastic Galerkin system in Kronecker form (oracle; test infrastructure only).

Sec. 3.1, eq. (tensor-product): A = G_0 (x) K_0 + sum_k G_k (x) K_k, with the
right-hand side F = e_0 (x) f_h for a deterministic load (the weak form of
Sec. 2.2 tested against psi_i gives int f psi_i rho = delta_{i,0}).

Vectors here are mode-major, as the Kronecker product orders them: entry
alpha*N + i is node i of mode alpha, i.e. a (P, N) array U with
A vec(U) = vec(sum_k G_k U K_k^T).
"""

from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import fem, indexset


@dataclass
class Problem:
    n: int                 # cells per side; N = (n-1)^2 interior nodes
    m: int                 # KL terms
    p: int                 # total polynomial degree
    sigma: float
    corr_len: float = 0.5
    a0_nodal: np.ndarray = None   # (n+1)^2 nodal mean field, or None for abar = 1
    amps: np.ndarray = None       # KL amplitudes s_k, or None for sqrt(lambda_k)
    # filled by build()
    N: int = 0
    P: int = 0
    index: list = field(default_factory=list)
    offsets: list = field(default_factory=list)
    G: list = field(default_factory=list)
    cellc: np.ndarray = None
    kldata: dict = None
    K: list = field(default_factory=list)
    f: np.ndarray = None

    def build(self):
        self.N = (self.n - 1) ** 2
        self.index = indexset.multi_indices(self.m, self.p)
        self.P = len(self.index)
        self.offsets = indexset.level_offsets(self.m, self.p)
        self.G = indexset.g_matrices(self.m, self.p)
        self.cellc, self.kldata = fem.cell_coefficients(
            self.n, self.m, self.sigma, self.corr_len, self.a0_nodal, self.amps)
        self.K = [fem.assemble_stiffness(self.n, self.cellc[k]) for k in range(self.m + 1)]
        self.f = fem.load_vector_unit(self.n)
        return self

    def rhs(self):
        """F = e_0 (x) f_h as a (P, N) array."""
        F = np.zeros((self.P, self.N))
        F[0] = self.f
        return F

    def a_min_h(self):
        """min over cells of c_0 - sum_k |c_k| (positive => every local G-matrix is SPD)."""
        return float(np.min(self.cellc[0] - np.abs(self.cellc[1:]).sum(axis=0)))


def build_problem(n, m, p, sigma, corr_len=0.5, a0_nodal=None, amps=None):
    return Problem(n=n, m=m, p=p, sigma=sigma, corr_len=corr_len,
                   a0_nodal=a0_nodal, amps=amps).build()


def assemble_A(prob):
    """A = sum_k kron(G_k, K_k) in CSR (eq. (tensor-product))."""
    A = None
    for Gk, Kk in zip(prob.G, prob.K):
        term = sp.kron(Gk, Kk, format="csr")
        A = term if A is None else A + term
    A.sum_duplicates()
    return A.tocsr()


def apply(prob, U):
    """Y = sum_k G_k U K_k^T for a (P, N) array U (the matrix-free form of A vec(U))."""
    U = np.asarray(U, dtype=np.float64).reshape(prob.P, prob.N)
    Y = np.zeros_like(U)
    for Gk, Kk in zip(prob.G, prob.K):
        Y += Gk @ (Kk @ U.T).T
    return Y


def solve_direct(prob, F=None, A=None, rtol=1e-14):
    """Galerkin solution U* of A vec(U) = vec(F), returned as (P, N).

    Dense LU up to 6000 unknowns, sparse LU up to 60000; larger systems use
    conjugate gradients (A is SPD, Sec. 3) preconditioned by exact K_0 solves
    on every mode, run to a relative residual of `rtol`, close to rounding.
    """
    if F is None:
        F = prob.rhs()
    if A is None:
        A = assemble_A(prob)
    b = np.asarray(F, dtype=np.float64).reshape(-1)
    n = A.shape[0]
    if n <= 6000:
        x = sla.solve(A.toarray(), b, assume_a="sym")
    elif n <= 60000:
        x = spla.spsolve(A.tocsc(), b)
    else:
        lu = spla.splu(prob.K[0].tocsc())
        M = spla.LinearOperator((n, n), matvec=lambda v: lu.solve(
            np.ascontiguousarray(v.reshape(prob.P, prob.N).T)).T.ravel())
        x, info = spla.cg(A, b, rtol=rtol, atol=0.0, M=M, maxiter=2000)
        if info != 0:
            raise RuntimeError(f"reference CG did not reach {rtol}: info={info}")
    return x.reshape(prob.P, prob.N)
