"""The block-triangular preconditioner of Sec. 4.2 with its 2x2 split taken literally
(oracle; test infrastructure only).

Sec. 4.2 splits the chaos space into the polynomials of degree <= p-1 and those of
degree p, which gives the 2x2 block structure of eq. (hierarchical_structure),
A = [[A_hat, W^T], [W, D]], and defines B_T = [[A_hat, 0], [W, D]] (one block
Gauss-Seidel step from a zero guess).  Applying B_T^{-1} to r = (r1, r2):

    z1 = A_hat^{-1} r1,    z2 = D^{-1} (r2 - W z1).

A_hat is itself a stochastic Galerkin matrix (the degree p-1 system), and
D = I (x) K_0 because G_k(alpha, alpha) = 0 for k >= 1.  The paper solves the
diagonal blocks "inexactly by the standard multigrid V-cycle"; this module
offers two ways for A_hat, so that the reading can be compared with Table 3:

* exact: A_hat^{-1} by conjugate gradients preconditioned with one exact K_0
  solve per mode, to a relative residual of 1e-13;
* vcycle: one V(nu1, nu2) multigrid cycle for the coupled system A_hat, with the
  Galerkin coarse operator of every K_k (coarse A_hat_l = sum_k G_hat_k (x) P^T K_k P),
  the transfer I (x) P, the coarsest level solved directly, and point Gauss-Seidel
  on the assembled A_hat_l in its natural (mode-major: mode, then node
  x-fastest) order, forward before and backward after the coarse correction.

The D blocks take `inner`, an approximate K_0^{-1} on (N, B) blocks (one V-cycle
per mode, as in the level sweep of ``precond``).  The symmetric variant
B_S = B_T blockdiag(A_hat, D)^{-1} B_T^T (last display of Sec. 4.2) applies the
forward step above, then z1 <- z1 - A_hat^{-1} W^T z2.

Arrays are mode-major (P, N), as in ``system``.
"""

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def split(prob):
    """(A_hat, W, Pa): the degree <= p-1 block, the coupling block W (rows: degree p), and the
    number Pa of modes of degree <= p-1."""
    Pa = prob.offsets[prob.p]
    Ahat = sp.csr_matrix((Pa * prob.N, Pa * prob.N))
    W = sp.csr_matrix(((prob.P - Pa) * prob.N, Pa * prob.N))
    for Gk, Kk in zip(prob.G, prob.K):
        Gk = sp.csr_matrix(Gk)
        Ahat = Ahat + sp.kron(Gk[:Pa, :Pa], Kk, format="csr")
        W = W + sp.kron(Gk[Pa:, :Pa], Kk, format="csr")
    return Ahat.tocsr(), W.tocsr(), Pa


class ExactAhat:
    """A_hat^{-1} by CG with one exact K_0 solve per mode as preconditioner."""

    def __init__(self, prob, Ahat, Pa, tol=1e-13):
        self.A, self.Pa, self.N, self.tol = Ahat, Pa, prob.N, tol
        self.lu = spla.splu(prob.K[0].tocsc())

    def __call__(self, r):
        r = np.asarray(r, dtype=np.float64).ravel()
        M = lambda v: self.lu.solve(v.reshape(self.Pa, self.N).T).T.ravel()  # noqa: E731
        x = np.zeros_like(r)
        res = r.copy()
        z = M(res)
        p = z.copy()
        rz = res @ z
        nr = np.linalg.norm(r)
        for _ in range(2000):
            if np.linalg.norm(res) <= self.tol * nr:
                break
            q = self.A @ p
            a = rz / (p @ q)
            x += a * p
            res -= a * q
            z = M(res)
            rzn = res @ z
            p = z + (rzn / rz) * p
            rz = rzn
        return x


class CoupledVcycle:
    """One V(nu1, nu2) cycle for the coupled system A_hat (see the module docstring)."""

    def __init__(self, prob, Pa, prolong, coarsest=4, nu1=2, nu2=2):
        self.nu1, self.nu2 = nu1, nu2
        Ghat = [sp.csr_matrix(Gk)[:Pa, :Pa] for Gk in prob.G]
        Ks = [K.tocsr() for K in prob.K]
        n = prob.n
        self.A, self.T, self.L, self.U = [], [], [], []
        while True:
            Al = sp.csr_matrix((Pa * Ks[0].shape[0],) * 2)
            for Gk, Kk in zip(Ghat, Ks):
                Al = Al + sp.kron(Gk, Kk, format="csr")
            Al = Al.tocsr()
            self.A.append(Al)
            self.L.append(sp.tril(Al, 0, format="csr"))
            self.U.append(sp.triu(Al, 0, format="csr"))
            if n <= coarsest:
                break
            Pm = prolong(n // 2)
            self.T.append(sp.kron(sp.identity(Pa, format="csr"), Pm, format="csr"))
            Ks = [(Pm.T @ K @ Pm).tocsr() for K in Ks]
            n //= 2
        self.coarse = sla.cho_factor(self.A[-1].toarray(), lower=True)

    def smooth(self, l, u, f, reverse):
        """One point Gauss-Seidel sweep on A_hat_l in mode-major order (backward if reverse)."""
        if not reverse:
            return u + spla.spsolve_triangular(self.L[l], f - self.A[l] @ u, lower=True)
        return u + spla.spsolve_triangular(self.U[l], f - self.A[l] @ u, lower=False)

    def _cycle(self, l, f):
        if l == len(self.A) - 1:
            return sla.cho_solve(self.coarse, f)
        A = self.A[l]
        u = np.zeros_like(f)
        for _ in range(self.nu1):
            u = self.smooth(l, u, f, reverse=False)
        ec = self._cycle(l + 1, self.T[l].T @ (f - A @ u))
        u += self.T[l] @ ec
        for _ in range(self.nu2):
            u = self.smooth(l, u, f, reverse=True)
        return u

    def __call__(self, r):
        return self._cycle(0, np.asarray(r, dtype=np.float64).ravel())


def precond_tri_2x2(prob, R, W, Pa, ahat_inv, inner):
    """Z = B_T^{-1} R with B_T = [[A_hat, 0], [W, D]]; R, Z (P, N)."""
    R = np.asarray(R, dtype=np.float64)
    Z = np.empty_like(R)
    Z[:Pa] = ahat_inv(R[:Pa].ravel()).reshape(Pa, prob.N)
    r2 = R[Pa:].ravel() - W @ Z[:Pa].ravel()
    Z[Pa:] = inner(np.ascontiguousarray(r2.reshape(prob.P - Pa, prob.N).T)).T
    return Z


def precond_sym_2x2(prob, R, W, Pa, ahat_inv, inner):
    """Z = B_S^{-1} R with B_S = B_T blockdiag(A_hat, D)^{-1} B_T^T; R, Z (P, N)."""
    Z = precond_tri_2x2(prob, R, W, Pa, ahat_inv, inner)
    Z[:Pa] -= ahat_inv((W.T @ Z[Pa:].ravel())).reshape(Pa, prob.N)
    return Z
