"""Block preconditioners B_D, B_T and B_S (oracle; test infrastructure only).

Sec. 4.1: B_D = G_0 (x) K_0 (one K_0 solve per mode).
Sec. 4.2: B_T is the lower block-triangular part of A, i.e. one block
Gauss-Seidel step from a zero guess.  Reading taken here: the blocks are the
polynomial degree levels (the 2x2 split of eq. (hierarchical_structure)
applied recursively down to degree 0), and every diagonal block is
I (x) K_0 because G_k(alpha, alpha) = 0 for k >= 1; each diagonal solve is
exact or one V-cycle.  Because the G_k (k >= 1) vanish inside a degree level,
this equals the mode-by-mode lower block-triangular part of A.

Sec. 4.2 (last display): B_S = B_L blockdiag^{-1} B_U, the block symmetric
Gauss-Seidel preconditioner for PCG.  With the level-wise reading, B_S^{-1} r
is a forward sweep y_d = inner(r_d - L_{d,d-1} y_{d-1}) followed by a backward
sweep z_d = y_d - inner(U_{d,d+1} z_{d+1}) (z_p = y_p), where L and U are the
strictly lower and upper block parts of A by degree level (U = L^T).  With
exact inner solves this is (D + U)^{-1} D (D + L)^{-1}.

Arrays are mode-major (P, N), as in ``system``.
"""

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


class ExactK0:
    """Exact inverse of K_0 applied column-wise."""

    def __init__(self, K0):
        self.lu = spla.splu(K0.tocsc())

    def __call__(self, f):
        # f: (N,) or (N, B)
        return self.lu.solve(np.asarray(f, dtype=np.float64))


def apply_block_inverse(inner, R):
    """Apply `inner` (an approximate K_0^{-1} acting on (N, B) blocks) to every mode of R (P, N)."""
    return inner(np.ascontiguousarray(R.T)).T.copy()


def precond_diag(prob, R, inner):
    """Z = B_D^{-1} R, with K_0^{-1} replaced by `inner`."""
    return apply_block_inverse(inner, np.asarray(R, dtype=np.float64))


def precond_tri(prob, R, inner):
    """Z = B_T^{-1} R by the forward sweep over degree levels.

    For d = 0..p:  Z_d = inner( R_d - sum_{k>=1} [G_k]_{d,d-1} (x) K_k  Z_{d-1} ).
    """
    R = np.asarray(R, dtype=np.float64)
    Z = np.zeros_like(R)
    off = prob.offsets
    for d in range(prob.p + 1):
        cur = slice(off[d], off[d + 1])
        rhs = R[cur].copy()
        if d > 0:
            prev = slice(off[d - 1], off[d])
            for k in range(1, prob.m + 1):
                Gb = prob.G[k][cur, prev]
                if Gb.nnz:
                    rhs -= Gb @ (prob.K[k] @ Z[prev].T).T
        Z[cur] = apply_block_inverse(inner, rhs)
    return Z


def precond_sym(prob, R, inner):
    """Z = B_S^{-1} R: the forward level sweep of precond_tri, then the backward sweep."""
    Y = precond_tri(prob, R, inner)
    Z = Y.copy()
    off = prob.offsets
    for d in range(prob.p - 1, -1, -1):
        cur = slice(off[d], off[d + 1])
        nxt = slice(off[d + 1], off[d + 2])
        t = np.zeros((off[d + 1] - off[d], prob.N))
        for k in range(1, prob.m + 1):
            Gb = prob.G[k][cur, nxt]
            if Gb.nnz:
                t += Gb @ (prob.K[k] @ Z[nxt].T).T
        Z[cur] = Y[cur] - apply_block_inverse(inner, t)
    return Z


def assemble_BS(prob):
    """(D + L) D^{-1} (D + U) with D = I (x) K_0 and L, U the strict block parts by level."""
    BL = assemble_BT(prob)
    BD = assemble_BD(prob).tocsc()
    return (BL @ spla.spsolve(BD, BL.T.tocsc())).tocsr()


def degree_of_mode(prob):
    lev = np.empty(prob.P, dtype=np.int64)
    for d in range(prob.p + 1):
        lev[prob.offsets[d]:prob.offsets[d + 1]] = d
    return lev


def assemble_BT(prob):
    """Block lower-triangular part of A by degree level, assembled (for small cases)."""
    lev = degree_of_mode(prob)
    B = None
    for Gk, Kk in zip(prob.G, prob.K):
        Gc = Gk.tocoo()
        keep = lev[Gc.row] >= lev[Gc.col]
        Gl = sp.csr_matrix((Gc.data[keep], (Gc.row[keep], Gc.col[keep])), shape=Gk.shape)
        term = sp.kron(Gl, Kk, format="csr")
        B = term if B is None else B + term
    return B.tocsr()


def assemble_BD(prob):
    return sp.kron(prob.G[0], prob.K[0], format="csr")
