"""Geometric multigrid V-cycle for the mean stiffness K_0 (oracle; test infrastructure only).

The paper inverts each diagonal block K_0 inexactly by one multigrid V-cycle
(Sec. 4.1 and Sec. 4.2: "may be solved inexactly by the standard multigrid
V-cycle"; Sec. 6: one V(2,2) cycle with point Gauss-Seidel smoothing).  It
names no other component, so the readings used here are:

* grids n, n/2, ..., n_c cells per side; bilinear prolongation P (exact
  interpolation of the coarse Q1 space; for the P1 triangulation of Sec. 6,
  transfer="p1" gives linear interpolation on the triangles), restriction
  R = P^T, Galerkin coarse operators K_{l-1} = P^T K_l P;
* Gauss-Seidel by colours of the interior grid indices (I, J):
  'four'  : colour (I mod 2) + 2 (J mod 2), a true Gauss-Seidel sweep for the
            9-point stencil because equal colours never touch;
  'rb'    : colour (I + J) mod 2, each colour updated from the values at the
            start of that colour (diagonal neighbours share a colour);
  'lex'   : lexicographic point Gauss-Seidel;
  pre-smoothing visits the colours forward, post-smoothing backward, so the
  cycle is a symmetric operator;
* zero initial guess, one cycle; coarsest grid solved by dense Cholesky.
"""

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def prolong_1d(nc):
    """(2nc-1) x (nc-1) bilinear interpolation between interior nodes."""
    nf = 2 * nc
    rows, cols, vals = [], [], []
    for i in range(1, nc):              # coarse grid index
        I = 2 * i                       # fine grid index of the same point
        for d, w in ((-1, 0.5), (0, 1.0), (1, 0.5)):
            rows.append(I + d - 1)
            cols.append(i - 1)
            vals.append(w)
    return sp.csr_matrix((vals, (rows, cols)), shape=(nf - 1, nc - 1))


def prolongation(nc):
    """2-D bilinear prolongation, interior x-fastest numbering on both grids."""
    p1 = prolong_1d(nc)
    return sp.kron(p1, p1, format="csr")


def prolongation_p1(nc):
    """Linear interpolation on the triangulation whose squares are split south-west to
    north-east (the natural P1 transfer): a fine node on a coarse node copies it, one on a
    horizontal, vertical or diagonal coarse edge takes the mean of that edge's two ends.
    Interior x-fastest numbering on both grids; Dirichlet coarse nodes drop out."""
    nf = 2 * nc
    rows, cols, vals = [], [], []

    def coarse(i, j):
        return (j - 1) * (nc - 1) + (i - 1) if 1 <= i <= nc - 1 and 1 <= j <= nc - 1 else None

    for J in range(1, nf):
        for I in range(1, nf):
            if I % 2 == 0 and J % 2 == 0:
                ends = [(I // 2, J // 2, 1.0)]
            elif J % 2 == 0:                      # horizontal coarse edge
                ends = [((I - 1) // 2, J // 2, 0.5), ((I + 1) // 2, J // 2, 0.5)]
            elif I % 2 == 0:                      # vertical coarse edge
                ends = [(I // 2, (J - 1) // 2, 0.5), (I // 2, (J + 1) // 2, 0.5)]
            else:                                 # diagonal: south-west and north-east corners
                ends = [((I - 1) // 2, (J - 1) // 2, 0.5), ((I + 1) // 2, (J + 1) // 2, 0.5)]
            for i, j, w in ends:
                c = coarse(i, j)
                if c is not None:
                    rows.append((J - 1) * (nf - 1) + (I - 1))
                    cols.append(c)
                    vals.append(w)
    return sp.csr_matrix((vals, (rows, cols)), shape=((nf - 1) ** 2, (nc - 1) ** 2))


def colours(n, mode):
    """List of index arrays, one per colour, in pre-smoothing order."""
    I, J = np.meshgrid(np.arange(1, n), np.arange(1, n), indexing="xy")
    I = I.ravel()
    J = J.ravel()
    if mode == "four":
        c = (I % 2) + 2 * (J % 2)
        return [np.nonzero(c == q)[0] for q in range(4)]
    if mode == "rb":
        c = (I + J) % 2
        return [np.nonzero(c == q)[0] for q in range(2)]
    raise ValueError(mode)


class Hierarchy:
    def __init__(self, K0, n, coarsest=8, colour_mode="four", nu1=2, nu2=2, transfer="bilinear"):
        assert n % coarsest == 0 and ((n // coarsest) & (n // coarsest - 1)) == 0
        self.colour_mode = colour_mode
        self.nu1, self.nu2 = nu1, nu2
        self.ns = [n]
        self.K = [K0.tocsr()]
        self.P = []
        make_p = {"bilinear": prolongation, "p1": prolongation_p1}[transfer]
        while self.ns[-1] > coarsest:
            nc = self.ns[-1] // 2
            P = make_p(nc)
            self.P.append(P)
            Kc = (P.T @ self.K[-1] @ P).tocsr()
            Kc.sum_duplicates()
            self.K.append(Kc)
            self.ns.append(nc)
        self.chol = sla.cho_factor(self.K[-1].toarray(), lower=True)
        self.diag = [K.diagonal() for K in self.K]
        if colour_mode != "lex":
            self.cols = [colours(nl, colour_mode) for nl in self.ns]
            self.Krows = [[K[c] for c in cl] for K, cl in zip(self.K, self.cols)]
        else:
            self.Klow = [sp.tril(K, 0, format="csr") for K in self.K]
            self.Kupp = [sp.triu(K, 0, format="csr") for K in self.K]

    def smooth(self, l, u, f, reverse):
        K = self.K[l]
        if self.colour_mode == "lex":
            # lexicographic Gauss-Seidel: forward (pre) or backward (post)
            if not reverse:
                L = self.Klow[l]
                u += spla.spsolve_triangular(L, f - K @ u, lower=True)
            else:
                U = self.Kupp[l]
                u += spla.spsolve_triangular(U, f - K @ u, lower=False)
            return u
        order = range(len(self.cols[l]))
        if reverse:
            order = reversed(list(order))
        d = self.diag[l]
        for q in order:
            c = self.cols[l][q]
            r = f[c] - self.Krows[l][q] @ u
            u[c] += r / d[c][:, None] if u.ndim == 2 else r / d[c]
        return u

    def vcycle(self, f, l=0):
        """One V(nu1, nu2) cycle with zero initial guess; f is (N_l,) or (N_l, B)."""
        f = np.asarray(f, dtype=np.float64)
        if l == len(self.K) - 1:
            return sla.cho_solve(self.chol, f)
        u = np.zeros_like(f)
        for _ in range(self.nu1):
            u = self.smooth(l, u, f, reverse=False)
        r = f - self.K[l] @ u
        ec = self.vcycle(self.P[l].T @ r, l + 1)
        u = u + self.P[l] @ ec
        for _ in range(self.nu2):
            u = self.smooth(l, u, f, reverse=True)
        return u
