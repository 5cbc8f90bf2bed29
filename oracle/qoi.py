"""PCE statistics, the subdomain QoI and its adjoint gradient (oracle; test infrastructure only).

Sec. 2.2, eq. (PCE_u): u = sum_j u_j(x) psi_j(xi); with the orthonormal basis
(Sec. 3.2) E[u] = u_0 and Var[u] = sum_{j>0} u_j^2.

QoI reading: Q = (1/|S|) int_S u dx over S = [1/4, 3/4]^2, integrated exactly
for the bilinear interpolant, and J = E[Q] + Var[Q] = q_0 + sum_{a>0} q_a^2
with q_a = w_S . U_a.  The gradient is the adjoint one: A lambda = dJ/dU
(A is symmetric, Sec. 3), and with A = sum_k G_k (x) sum_e c_{k,e} K_ref^e,
dJ/dc_{k,e} = - sum_{a,b} G_k(a,b) lambda_{a,e}^T K_ref U_{b,e}.  The chain
rule through c_{k,e} = sigma s_k b_k(x_e) and c_{0,e} = mean of the four
vertex values of a0 gives the parameter gradients.
"""

import numpy as np

from . import fem, system


def subdomain_weights(n):
    """w_S on interior nodes: exact integral of each hat function over S, divided by |S|."""
    assert n % 4 == 0
    h = 1.0 / n
    a, b = n // 4, 3 * n // 4
    I = np.arange(1, n)
    w1 = np.where((I > a) & (I < b), h, 0.0) + np.where((I == a) | (I == b), 0.5 * h, 0.0)
    return (np.outer(w1, w1) / 0.25).ravel()  # J-major rows, I fastest


def mean_variance(U):
    U = np.asarray(U)
    return U[0].copy(), (U[1:] ** 2).sum(axis=0)


def qoi(prob, U):
    w = subdomain_weights(prob.n)
    q = U @ w
    return float(q[0] + np.sum(q[1:] ** 2)), q


def _to_full(n, V):
    """(B, N) interior values -> (B, (n+1)^2) with zero boundary."""
    imap = fem.interior_map(n)
    full = np.zeros((V.shape[0], (n + 1) ** 2))
    inside = imap >= 0
    full[:, inside] = V[:, imap[inside]]
    return full


def cell_gradient(prob, U, lam):
    """dJ/dc_{k,e} = - sum_{a,b} G_k(a,b) lam_{a,e}^T K_ref U_{b,e}; shape (m+1, n*n)."""
    n = prob.n
    verts = fem.cell_vertices(n)
    lf = _to_full(n, lam)[:, verts]                 # (P, cells, 4)
    out = np.empty((prob.m + 1, n * n))
    for k, Gk in enumerate(prob.G):
        T = Gk @ U                                   # (P, N)
        tf = _to_full(n, T)[:, verts]                # (P, cells, 4)
        kt = tf @ fem.K_REF.T                        # K_ref applied per cell
        out[k] = -np.einsum("pcv,pcv->c", lf, kt)
    return out


def qoi_and_gradient(prob, U=None, A=None):
    """J, and its gradient w.r.t. sigma, the KL amplitudes and the interior a0 values."""
    if A is None:
        A = system.assemble_A(prob)
    if U is None:
        U = system.solve_direct(prob, A=A)
    J, q = qoi(prob, U)
    w = subdomain_weights(prob.n)
    g = np.outer(np.concatenate([[1.0], 2.0 * q[1:]]), w)
    lam = system.solve_direct(prob, F=g, A=A)
    dc = cell_gradient(prob, U, lam)
    n, m = prob.n, prob.m
    b = fem.kl_at_cells(n, m, prob.corr_len)        # (m, cells)
    s = prob.kldata["amps"]
    dsigma = float(np.sum(dc[1:] * b * s[:, None])) if m else 0.0
    damp = prob.sigma * np.sum(dc[1:] * b, axis=1) if m else np.zeros(0)
    # a0 enters c_0 as the mean of the four cell vertices
    verts = fem.cell_vertices(n)
    da0_full = np.zeros((n + 1) ** 2)
    np.add.at(da0_full, verts.ravel(), np.repeat(0.25 * dc[0], 4))
    imap = fem.interior_map(n)
    inside = imap >= 0
    da0 = np.zeros((n - 1) ** 2)
    da0[imap[inside]] = da0_full[inside]
    return dict(J=J, q=q, U=U, lam=lam, dc=dc, dsigma=dsigma, damp=np.asarray(damp), da0=da0)
