"""Pins for the oracle's Q1 stiffness matrices and load vector.

Pinned against: the textbook constant-coefficient Q1 stencil, 2x2 Gauss
quadrature of the bilinear forms with explicit shape-function gradients,
and the discrete form of the eigenvalue enclosure of Lemma 2.
"""

import numpy as np
import pytest
import scipy.linalg as sla

from oracle import fem


def _gauss_bilinear_form(n, cellc, u_full, v_full):
    """sum_e c_e int_e grad u . grad v by 2x2 Gauss, explicit bilinear gradients."""
    h = 1.0 / n
    g = 0.5 / np.sqrt(3.0)
    tot = 0.0
    verts = fem.cell_vertices(n)
    for e in range(n * n):
        u = u_full[verts[e]]
        v = v_full[verts[e]]
        for sx in (0.5 - g, 0.5 + g):
            for sy in (0.5 - g, 0.5 + g):
                # reference coords (sx, sy) in [0,1]^2, vertices (0,0),(1,0),(1,1),(0,1)
                dNx = np.array([-(1 - sy), (1 - sy), sy, -sy]) / h
                dNy = np.array([-(1 - sx), -sx, sx, (1 - sx)]) / h
                tot += cellc[e] * (np.dot(dNx, u) * np.dot(dNx, v) + np.dot(dNy, u) * np.dot(dNy, v)) * h * h / 4
    return tot


def test_k_ref_properties():
    K = fem.K_REF
    assert np.array_equal(K, K.T)
    assert np.allclose(K.sum(axis=1), 0.0, atol=1e-15)
    assert np.allclose(np.sort(np.linalg.eigvalsh(K)), [0.0, 2.0 / 3.0, 1.0, 1.0], atol=1e-14)


def test_constant_coefficient_stencil():
    n = 8
    K = fem.assemble_stiffness(n, np.ones(n * n)).toarray()
    i = 3 * (n - 1) + 3  # interior node away from the boundary
    row = K[i].reshape(n - 1, n - 1)[2:5, 2:5]
    expect = np.full((3, 3), -1.0 / 3.0)
    expect[1, 1] = 8.0 / 3.0
    assert np.allclose(row, expect, atol=1e-15)
    assert np.count_nonzero(K[i]) == 9


def test_bilinear_form_equals_gauss_quadrature():
    n = 6
    rng = np.random.default_rng(0)
    cellc = rng.uniform(0.5, 2.0, n * n)
    K = fem.assemble_stiffness(n, cellc)
    imap = fem.interior_map(n)
    inside = imap >= 0
    for _ in range(3):
        u = rng.standard_normal((n - 1) ** 2)
        v = rng.standard_normal((n - 1) ** 2)
        uf = np.zeros((n + 1) ** 2)
        vf = np.zeros((n + 1) ** 2)
        uf[inside] = u[imap[inside]]
        vf[inside] = v[imap[inside]]
        assert abs(u @ (K @ v) - _gauss_bilinear_form(n, cellc, uf, vf)) < 1e-12


def test_load_vector_integrates_interpolant():
    # u^T f_h = int u_h dx for f = 1, with the integral of the bilinear
    # interpolant taken by 2x2 Gauss quadrature and explicit shape functions.
    n = 8
    rng = np.random.default_rng(3)
    u = rng.standard_normal((n - 1) ** 2)
    imap = fem.interior_map(n)
    inside = imap >= 0
    uf = np.zeros((n + 1) ** 2)
    uf[inside] = u[imap[inside]]
    h = 1.0 / n
    g = 0.5 / np.sqrt(3.0)
    tot = 0.0
    for vtx in fem.cell_vertices(n):
        for sx in (0.5 - g, 0.5 + g):
            for sy in (0.5 - g, 0.5 + g):
                N = np.array([(1 - sx) * (1 - sy), sx * (1 - sy), sx * sy, (1 - sx) * sy])
                tot += np.dot(N, uf[vtx]) * h * h / 4
    assert abs(u @ fem.load_vector_unit(n) - tot) < 1e-15


@pytest.mark.parametrize("sigma", [0.3, 0.5])
def test_lemma2_discrete_enclosure(sigma):
    # Lemma 2 (discrete form): sigma(K_0^{-1} K_k) lies in [min_e c_k/c_0, max_e c_k/c_0]
    n, m = 8, 4
    c, _ = fem.cell_coefficients(n, m, sigma, 0.5)
    K0 = fem.assemble_stiffness(n, c[0]).toarray()
    for k in range(1, m + 1):
        Kk = fem.assemble_stiffness(n, c[k]).toarray()
        ev = sla.eigh(Kk, K0, eigvals_only=True)
        r = c[k] / c[0]
        assert ev.min() >= r.min() - 1e-12 and ev.max() <= r.max() + 1e-12


def test_mean_field_from_nodal_a0():
    n = 4
    a0 = np.arange((n + 1) ** 2, dtype=float)
    c, _ = fem.cell_coefficients(n, 0, 0.0, 0.5, a0_nodal=a0)
    # cell (1, 2): vertices (1,2),(2,2),(2,3),(1,3) on the 5x5 grid
    e = 2 * n + 1
    assert c[0, e] == pytest.approx((a0[11] + a0[12] + a0[17] + a0[16]) / 4)


@pytest.mark.parametrize("n,m", [(8, 6), (16, 8)])
def test_cell_coefficients_respect_mode_parity(n, m):
    # cosine factors are even and sine factors odd about the centre of the
    # square, so reflecting the cell grid maps c_{k,e} to +-c_{k,e}; this pins
    # the evaluation point (the cell centre) and the centring t = x - 1/2.
    c, data = fem.cell_coefficients(n, m, 0.4, 0.5)
    for k in range(1, m + 1):
        i, j, _ = data["picked"][k - 1]
        sx = 1.0 if data["modes1"][i][0] == "cos" else -1.0
        sy = 1.0 if data["modes1"][j][0] == "cos" else -1.0
        f = c[k].reshape(n, n)                      # [cj, ci]
        assert np.allclose(f[:, ::-1], sx * f, atol=1e-15, rtol=1e-13)
        assert np.allclose(f[::-1, :], sy * f, atol=1e-15, rtol=1e-13)
        assert np.max(np.abs(f)) > 0.05


def test_cell_coefficients_reproduce_the_covariance():
    # Mercer: sum_k (sigma s_k b_k(x)) (sigma s_k b_k(y)) with s_k = sqrt(lambda_k) tends to the
    # covariance sigma^2 exp(-|x1 - y1|/L - |x2 - y2|/L) (Sec. 2.1, eq. (exponential-covariance),
    # separable reading).  Truncated after m modes the error is at most
    # sigma^2 max_k |b_k|^2 sum_{k>m} lambda_k <= 4 sigma^2 (1 - sum_{k<=m} lambda_k), since every
    # 1-D eigenfunction is bounded by sqrt 2 and the 1-D eigenvalues sum to one.  A wrong
    # amplitude (lambda for sqrt lambda, a stray factor) or normalisation breaks the limit.
    n, m, sigma, L = 4, 1000, 0.7, 0.5
    c, data = fem.cell_coefficients(n, m, sigma, L)
    cov = c[1:].T @ c[1:]
    x1, x2 = fem.cell_centres(n)
    ref = sigma ** 2 * np.exp(-(np.abs(x1[:, None] - x1[None, :]) + np.abs(x2[:, None] - x2[None, :])) / L)
    bound = 4 * sigma ** 2 * (1.0 - data["lams"].sum())
    assert bound < 0.05 * sigma ** 2
    assert np.max(np.abs(cov - ref)) <= bound
