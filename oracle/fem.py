"""Q1 finite elements on the unit square (oracle; test infrastructure only).

Spatial stiffness matrices of Sec. 3.1, eq. (def-stiffness):
K_0(r,s) = int abar grad phi_s . grad phi_r and
K_k(r,s) = sqrt(lambda_k) int b_k grad phi_s . grad phi_r.

Readings taken here (the paper uses linear triangles; the workload uses
bilinear Q1 elements on a uniform n x n grid):
* every coefficient is taken constant on a cell, equal to its value at the
  cell centre (mean field: the average of the four vertex values);
* homogeneous Dirichlet conditions are imposed by dropping boundary nodes;
* interior nodes are numbered lexicographically, x fastest;
* the KL amplitude s_k defaults to sqrt(lambda_k) and sigma multiplies it,
  so c_{k,e} = sigma * s_k * b_k(x_e).
"""

import numpy as np
import scipy.sparse as sp

from . import kl

# Element stiffness of grad.grad on a square cell (independent of h in 2-D),
# vertices counter-clockwise from the lower-left corner.
K_REF = np.array(
    [
        [4.0, -1.0, -2.0, -1.0],
        [-1.0, 4.0, -1.0, -2.0],
        [-2.0, -1.0, 4.0, -1.0],
        [-1.0, -2.0, -1.0, 4.0],
    ]
) / 6.0


def cell_vertices(n):
    """(n*n, 4) array of full-grid node ids (j*(n+1)+i), vertices CCW."""
    ci, cj = np.meshgrid(np.arange(n), np.arange(n), indexing="xy")
    ci = ci.ravel()
    cj = cj.ravel()
    n1 = n + 1
    v0 = cj * n1 + ci
    return np.stack([v0, v0 + 1, v0 + 1 + n1, v0 + n1], axis=1)


def cell_centres(n):
    h = 1.0 / n
    ci, cj = np.meshgrid(np.arange(n), np.arange(n), indexing="xy")
    return (ci.ravel() + 0.5) * h, (cj.ravel() + 0.5) * h


def interior_map(n):
    """Full-grid node id -> interior index, -1 on the boundary."""
    n1 = n + 1
    ii, jj = np.meshgrid(np.arange(n1), np.arange(n1), indexing="xy")
    ii = ii.ravel()
    jj = jj.ravel()
    inside = (ii > 0) & (ii < n) & (jj > 0) & (jj < n)
    out = -np.ones(n1 * n1, dtype=np.int64)
    out[inside] = (jj[inside] - 1) * (n - 1) + (ii[inside] - 1)
    return out


def cell_coefficients(n, m, sigma, corr_len, a0_nodal=None, amps=None):
    """(m+1, n*n) array: row 0 the mean field per cell, rows k the sigma*s_k*b_k(x_e).

    Also returns the KL data (picked modes, 1-D table, eigenvalues, amplitudes).
    """
    x1, x2 = cell_centres(n)
    c = np.empty((m + 1, n * n))
    if a0_nodal is None:
        c[0] = 1.0
    else:
        a0 = np.asarray(a0_nodal, dtype=np.float64).reshape(-1)
        assert a0.size == (n + 1) ** 2
        c[0] = a0[cell_vertices(n)].mean(axis=1)
    picked, modes1 = kl.kl_modes_2d(corr_len, m) if m > 0 else ([], [])
    lams = np.array([lam for (_i, _j, lam) in picked])
    s = np.sqrt(lams) if amps is None else np.asarray(amps, dtype=np.float64)
    for k in range(m):
        c[k + 1] = sigma * s[k] * kl.eval_2d(picked, modes1, k, x1, x2)
    return c, dict(picked=picked, modes1=modes1, lams=lams, amps=s)


def kl_at_cells(n, m, corr_len):
    """(m, n*n) values of the KL eigenfunctions b_k at cell centres."""
    x1, x2 = cell_centres(n)
    picked, modes1 = kl.kl_modes_2d(corr_len, m)
    return np.stack([kl.eval_2d(picked, modes1, k, x1, x2) for k in range(m)]) if m else np.zeros((0, n * n))


def assemble_stiffness(n, cellc):
    """Interior-node CSR matrix sum_e cellc[e] * K_REF^e (Dirichlet rows/cols dropped)."""
    verts = cell_vertices(n)
    imap = interior_map(n)
    rows = np.repeat(verts, 4, axis=1).ravel()
    cols = np.tile(verts, (1, 4)).ravel()
    vals = (cellc[:, None] * K_REF.ravel()[None, :]).ravel()
    ri = imap[rows]
    cj = imap[cols]
    keep = (ri >= 0) & (cj >= 0)
    N = (n - 1) ** 2
    K = sp.coo_matrix((vals[keep], (ri[keep], cj[keep])), shape=(N, N)).tocsr()
    K.sum_duplicates()
    return K


def load_vector_unit(n):
    """int f phi_i for f = 1: each interior hat function integrates to h^2."""
    h = 1.0 / n
    return np.full((n - 1) ** 2, h * h)
