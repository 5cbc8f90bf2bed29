"""Multi-index set and stochastic matrices (oracle; test infrastructure only).

Follows Sec. 2.2 (the total-degree gPC space Xi_p, dimension (m+p)!/(m!p!))
and Sec. 3.1, eq. (def-stochastic) (G_0 and G_k as expectations of products
of basis polynomials), with Legendre chaos for xi_k ~ U[-1, 1].

Ordering reading: modes are sorted by total degree (so that every degree
level is a contiguous range, matching the hierarchical split of Sec. 3.3,
eq. (hierarchical_structure)); inside one degree, by alpha_1 descending,
then alpha_2 descending, and so on.
"""

from math import comb, sqrt

import numpy as np
import scipy.sparse as sp


def dimension(m, p):
    """N_xi = (m+p)! / (m! p!)  (Sec. 2.2)."""
    return comb(m + p, p)


def _degree_slice(m, d):
    """All alpha in N^m with |alpha| == d, alpha_1 descending, then alpha_2 ..."""
    if m == 0:
        return [()] if d == 0 else []
    out = []
    for a1 in range(d, -1, -1):
        for rest in _degree_slice(m - 1, d - a1):
            out.append((a1,) + rest)
    return out


def multi_indices(m, p):
    """Graded list of multi-indices with |alpha| <= p."""
    out = []
    for d in range(p + 1):
        out.extend(_degree_slice(m, d))
    return out


def level_offsets(m, p):
    """Start of each degree level in the graded order, plus the total (length p+2)."""
    offs = [0]
    for d in range(p + 1):
        offs.append(offs[-1] + comb(m + d - 1, d) if m > 0 else offs[-1] + (d == 0))
    return offs


def legendre_coupling(n):
    """<xi psi_n psi_{n+1}> for orthonormal Legendre polynomials, density 1/2 on [-1, 1].

    From the three-term recurrence (n+1) L_{n+1} = (2n+1) xi L_n - n L_{n-1}
    with psi_n = sqrt(2n+1) L_n:  xi psi_n = b_{n+1} psi_{n+1} + b_n psi_{n-1},
    b_n = n / sqrt((2n-1)(2n+1)).  Hence the value is b_{n+1}.
    """
    return (n + 1) / sqrt((2 * n + 1) * (2 * n + 3))


def g_matrices(m, p):
    """[G_0, G_1, ..., G_m] as CSR matrices of size P x P (eq. (def-stochastic)).

    G_0 = I by orthonormality (Sec. 3.2).  For k >= 1 the product structure
    of psi_alpha gives G_k(alpha, beta) != 0 only for beta = alpha +- e_k,
    with value <xi psi_a psi_{a+1}> taken at a = min(alpha_k, beta_k).
    """
    idx = multi_indices(m, p)
    P = len(idx)
    pos = {a: i for i, a in enumerate(idx)}
    mats = [sp.identity(P, format="csr", dtype=np.float64)]
    for k in range(m):
        rows, cols, vals = [], [], []
        for i, a in enumerate(idx):
            b = list(a)
            b[k] += 1
            b = tuple(b)
            j = pos.get(b)
            if j is not None:
                v = legendre_coupling(a[k])
                rows += [i, j]
                cols += [j, i]
                vals += [v, v]
        mats.append(sp.csr_matrix((vals, (rows, cols)), shape=(P, P)))
    return mats
