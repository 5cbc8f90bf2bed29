"""The paper's own discretisation (Sec. 6) as an oracle problem (test infrastructure only).

Sec. 6 sets the model problem of Sec. 2 on D = (-1/2, 1/2)^2 with
f = 2 (1/2 - x^2 - y^2), zero Dirichlet data, the mean coefficient 1, the
exponential covariance with L = 1, xi_k uniform with unit variance, linear
(P1) finite elements on a uniform triangulation, and one V(2,2) cycle with
point Gauss-Seidel per diagonal block; the Krylov methods stop when the
relative Euclidean residual falls below 1e-10 from a zero initial guess.

Readings taken here (the paper does not state them):
* each grid square is split by its south-west to north-east diagonal; both
  right isosceles triangles then give every K_k a 5-point pattern, which the
  nonzero counts of Table 1 confirm;
* coefficients are constant per triangle, equal to their value at the
  centroid (the analogue of the cell-centre rule used for Q1);
* the covariance is the separable one of the Q1 workload (l1 distance), with
  L = 1, and the variance-one law xi ~ U(-sqrt 3, sqrt 3) multiplies the
  Legendre coupling entries by sqrt 3;
* the load vector is integrated exactly (f phi_i is a cubic on each triangle;
  the four-point rule of degree three below is exact for it);
* multigrid: linear interpolation on the triangulation (mg transfer "p1"),
  R = P^T, Galerkin coarse operators, lexicographic point Gauss-Seidel, the
  coarsest grid of 4 cells per side solved exactly.

Node numbering: interior nodes x-fastest, as in `fem`.
"""

import numpy as np
import scipy.sparse as sp

from . import indexset, kl
from .fem import interior_map
from .system import Problem

# degree-3 rule on the reference triangle (barycentric points, weights summing to 1)
_TRI_Q = [((1 / 3, 1 / 3, 1 / 3), -27 / 48)] + [
    (b, 25 / 48) for b in ((0.6, 0.2, 0.2), (0.2, 0.6, 0.2), (0.2, 0.2, 0.6))
]


def triangles(n):
    """(2 n^2, 3) full-grid vertex ids (j*(n+1)+i) of the SW-NE split, and the owning cell."""
    n1 = n + 1
    ci, cj = np.meshgrid(np.arange(n), np.arange(n), indexing="xy")
    ci = ci.ravel()
    cj = cj.ravel()
    sw = cj * n1 + ci
    se, ne, nw = sw + 1, sw + 1 + n1, sw + n1
    lower = np.stack([sw, se, ne], axis=1)
    upper = np.stack([sw, ne, nw], axis=1)
    return np.concatenate([lower, upper]), np.concatenate([np.arange(n * n), np.arange(n * n)])


def vertex_coords(n):
    """Physical coordinates of the full grid on (-1/2, 1/2)^2, x-fastest."""
    t = np.linspace(-0.5, 0.5, n + 1)
    x, y = np.meshgrid(t, t, indexing="xy")
    return x.ravel(), y.ravel()


def centroids(n):
    tri, _ = triangles(n)
    x, y = vertex_coords(n)
    return x[tri].mean(axis=1), y[tri].mean(axis=1)


def assemble_p1(n, coef):
    """Interior-node CSR of sum_t coef[t] int_t grad phi_i . grad phi_j (Dirichlet dropped)."""
    tri, _ = triangles(n)
    x, y = vertex_coords(n)
    X, Y = x[tri], y[tri]                                   # (T, 3)
    # gradients of the barycentric coordinates: grad lambda_i = (y_j - y_k, x_k - x_j) / (2|T|)
    area2 = (X[:, 1] - X[:, 0]) * (Y[:, 2] - Y[:, 0]) - (X[:, 2] - X[:, 0]) * (Y[:, 1] - Y[:, 0])
    gx = np.stack([Y[:, 1] - Y[:, 2], Y[:, 2] - Y[:, 0], Y[:, 0] - Y[:, 1]], axis=1) / area2[:, None]
    gy = np.stack([X[:, 2] - X[:, 1], X[:, 0] - X[:, 2], X[:, 1] - X[:, 0]], axis=1) / area2[:, None]
    local = (gx[:, :, None] * gx[:, None, :] + gy[:, :, None] * gy[:, None, :]) * (0.5 * np.abs(area2))[:, None, None]
    vals = (np.asarray(coef)[:, None, None] * local).ravel()
    rows = np.repeat(tri, 3, axis=1).ravel()
    cols = np.tile(tri, (1, 3)).ravel()
    imap = interior_map(n)
    ri, cj = imap[rows], imap[cols]
    keep = (ri >= 0) & (cj >= 0)
    N = (n - 1) ** 2
    K = sp.coo_matrix((vals[keep], (ri[keep], cj[keep])), shape=(N, N)).tocsr()
    K.sum_duplicates()
    # entries that cancel exactly (e.g. the centre node of a KL mode odd in x) keep a
    # rounding residue of ~1e-17; they are zero by definition
    if K.nnz:
        K.data[np.abs(K.data) <= 1e-13 * np.max(np.abs(K.data))] = 0.0
    K.eliminate_zeros()
    return K


def paper_load(x, y):
    """f = 2 (1/2 - x^2 - y^2); -Laplace of (1/4 - x^2)(1/4 - y^2)."""
    return 2.0 * (0.5 - x * x - y * y)


def load_vector_p1(n, f=paper_load):
    """int f phi_i over every triangle by the degree-3 rule (exact for quadratic f)."""
    tri, _ = triangles(n)
    x, y = vertex_coords(n)
    X, Y = x[tri], y[tri]
    area = 0.5 * np.abs((X[:, 1] - X[:, 0]) * (Y[:, 2] - Y[:, 0]) - (X[:, 2] - X[:, 0]) * (Y[:, 1] - Y[:, 0]))
    local = np.zeros(tri.shape)
    for bary, w in _TRI_Q:
        b = np.asarray(bary)
        px, py = X @ b, Y @ b
        local += w * area[:, None] * paper_load(px, py)[:, None] * b[None, :]
    imap = interior_map(n)
    F = np.zeros((n - 1) ** 2)
    ids = imap[tri.ravel()]
    keep = ids >= 0
    np.add.at(F, ids[keep], local.ravel()[keep])
    return F


def build_problem_paper(n, m, p, sigma, corr_len=1.0):
    """Problem of Sec. 6: P1 on (-1/2, 1/2)^2, f = 2(1/2 - x^2 - y^2), xi ~ U(-sqrt 3, sqrt 3)."""
    pr = Problem(n=n, m=m, p=p, sigma=sigma, corr_len=corr_len)
    pr.N = (n - 1) ** 2
    pr.index = indexset.multi_indices(m, p)
    pr.P = len(pr.index)
    pr.offsets = indexset.level_offsets(m, p)
    G = indexset.g_matrices(m, p)
    pr.G = [G[0]] + [np.sqrt(3.0) * Gk for Gk in G[1:]]
    cx, cy = centroids(n)
    coef = np.empty((m + 1, cx.size))
    coef[0] = 1.0
    picked, modes1 = kl.kl_modes_2d(corr_len, m) if m > 0 else ([], [])
    lams = np.array([lam for (_i, _j, lam) in picked])
    for k in range(m):
        # kl.eval_2d takes unit-square coordinates (centred at 1/2)
        coef[k + 1] = sigma * np.sqrt(lams[k]) * kl.eval_2d(picked, modes1, k, cx + 0.5, cy + 0.5)
    pr.cellc = coef
    pr.kldata = dict(picked=picked, modes1=modes1, lams=lams, amps=np.sqrt(lams))
    pr.K = [assemble_p1(n, coef[k]) for k in range(m + 1)]
    pr.f = load_vector_p1(n)
    return pr
