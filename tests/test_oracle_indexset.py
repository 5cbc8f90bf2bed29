"""Pins for the oracle's multi-index set and stochastic matrices.

Pinned against: the paper's worked dimension and Table 1 sizes (golden file),
tensor Gauss-Legendre quadrature of the defining integrals, and the textbook
spectrum of Jacobi matrices (Gauss-Legendre nodes).
"""

import itertools
import os
from math import comb

import numpy as np
import pytest
from numpy.polynomial import legendre as npleg

from oracle import indexset

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_numbers.txt")


def golden():
    out = {}
    for line in open(GOLDEN):
        line = line.split("#", 1)[0].strip()
        if "=" in line:
            k, v = (s.strip() for s in line.split("=", 1))
            out[k] = v
    return out


def test_dimension_matches_paper_example():
    g = golden()
    assert indexset.dimension(6, 4) == int(g["dim_m6_p4"])
    assert len(indexset.multi_indices(6, 4)) == int(g["dim_m6_p4"])


def test_table1_sizes_from_level_structure():
    # h = 1/64 -> 63 x 63 interior nodes; A-hat is the degree <= p-1 system,
    # D the top-degree block (eq. (hierarchical_structure)).
    g = golden()
    Nx = 63 * 63
    off = indexset.level_offsets(6, 4)
    assert Nx * off[-1] == int(g["table1_size_A"])
    assert Nx * off[-2] == int(g["table1_size_Ahat"])
    assert Nx * (off[-1] - off[-2]) == int(g["table1_size_D"])
    assert Nx * (off[-1] - off[-2]) == int(g["table1_size_W_rows"])
    assert Nx * off[-2] == int(g["table1_size_W_cols"])
    # B_D and D are block diagonal with K_0 blocks; with the paper's linear
    # triangles K_0 is the 5-point stencil, nnz = 5 Nx - 4*63.
    nnz_k0_p1 = 5 * Nx - 4 * 63
    assert off[-1] * nnz_k0_p1 == int(g["table1_nnz_BD"])
    assert (off[-1] - off[-2]) * nnz_k0_p1 == int(g["table1_nnz_D"])


@pytest.mark.parametrize("m,p", [(2, 2), (4, 3), (6, 4), (8, 3), (5, 3), (1, 5), (3, 0)])
def test_graded_order_and_levels(m, p):
    idx = indexset.multi_indices(m, p)
    off = indexset.level_offsets(m, p)
    assert len(idx) == comb(m + p, p) == off[-1]
    assert len(set(idx)) == len(idx)
    brute = [a for a in itertools.product(range(p + 1), repeat=m) if sum(a) <= p]
    assert sorted(brute) == sorted(idx)
    for d in range(p + 1):
        lev = idx[off[d]:off[d + 1]]
        assert len(lev) == comb(m + d - 1, d)
        assert all(sum(a) == d for a in lev)
        assert lev == sorted(lev, reverse=True)  # alpha_1 descending, then alpha_2, ...


def _psi(alpha, pts):
    """Orthonormal Legendre product basis evaluated at points (Q, m)."""
    val = np.ones(pts.shape[0])
    for k, a in enumerate(alpha):
        c = np.zeros(a + 1)
        c[a] = 1.0
        val *= np.sqrt(2 * a + 1) * npleg.legval(pts[:, k], c)
    return val


@pytest.mark.parametrize("m,p", [(1, 4), (2, 2), (2, 3), (3, 2)])
def test_g_matrices_equal_tensor_quadrature(m, p):
    # eq. (def-stochastic): G_k(i,j) = E[xi_k psi_j psi_i], xi ~ U[-1,1]^m (density 2^-m)
    x, w = npleg.leggauss(p + 2)
    pts = np.array(list(itertools.product(x, repeat=m)))
    wts = np.prod(np.array(list(itertools.product(w, repeat=m))), axis=1) / 2.0 ** m
    idx = indexset.multi_indices(m, p)
    Psi = np.stack([_psi(a, pts) for a in idx])            # (P, Q)
    G = indexset.g_matrices(m, p)
    G0q = (Psi * wts) @ Psi.T
    assert np.max(np.abs(G[0].toarray() - G0q)) < 1e-13
    for k in range(m):
        Gkq = (Psi * wts * pts[:, k]) @ Psi.T
        assert np.max(np.abs(G[k + 1].toarray() - Gkq)) < 1e-13


@pytest.mark.parametrize("m,p", [(2, 2), (4, 3), (6, 4), (8, 3), (5, 3)])
def test_g_structure_and_spectrum(m, p):
    G = indexset.g_matrices(m, p)
    P = comb(m + p, p)
    assert np.array_equal(G[0].toarray(), np.eye(P))
    total = sum(G[1:]).tocsr()
    assert total.nnz == 2 * m * comb(m + p - 1, p - 1)
    for k in range(1, m + 1):
        Gk = G[k].toarray()
        assert np.array_equal(Gk, Gk.T)
        assert np.all(np.diag(Gk) == 0.0)
        # chains along direction k have length L = p + 1 - |alpha'| and are
        # Jacobi matrices of orthonormal Legendre polynomials: their spectrum
        # is the Gauss-Legendre rule of order L.
        expect = []
        for L in range(1, p + 2):
            nchains = comb((m - 1) + (p + 1 - L) - 1, p + 1 - L) if m > 1 else int(L == p + 1)
            expect += list(npleg.leggauss(L)[0]) * nchains
        ev = np.linalg.eigvalsh(Gk)
        assert len(expect) == P
        assert np.max(np.abs(np.sort(ev) - np.sort(expect))) < 1e-13


def test_g_vanishes_inside_a_level():
    m, p = 4, 3
    G = indexset.g_matrices(m, p)
    off = indexset.level_offsets(m, p)
    for k in range(1, m + 1):
        Gk = G[k].toarray()
        for d in range(p + 1):
            blk = Gk[off[d]:off[d + 1], off[d]:off[d + 1]]
            assert not blk.any()
            for e in range(p + 1):
                if abs(e - d) > 1:
                    assert not Gk[off[d]:off[d + 1], off[e]:off[e + 1]].any()
