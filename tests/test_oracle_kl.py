"""Pins for the oracle's Karhunen-Loeve eigenpairs.

Pinned against the defining integral equation (adaptive quadrature), L2
orthonormality, a Nystrom discretisation of the covariance operator, the
trace of the unit kernel, and a brute-force choice of the largest products.
"""

import numpy as np
import pytest
from scipy import integrate

from oracle import kl


@pytest.mark.parametrize("L", [0.5, 0.25, 1.0])
def test_integral_equation_and_orthonormality(L):
    c = 1.0 / L
    modes = kl.eigen_1d(L, 8)
    lams = [md[2] for md in modes]
    assert all(a > b for a, b in zip(lams, lams[1:]))
    for md in modes:
        lam = md[2]
        for s in (-0.41, -0.13, 0.0, 0.22, 0.47):
            f = lambda t: np.exp(-c * abs(s - t)) * kl.eval_1d(md, t)  # noqa: E731
            v = integrate.quad(f, -0.5, s, epsabs=1e-14, epsrel=1e-13, limit=200)[0] + \
                integrate.quad(f, s, 0.5, epsabs=1e-14, epsrel=1e-13, limit=200)[0]
            assert abs(v - lam * kl.eval_1d(md, s)) < 1e-11
    for a in range(8):
        for b in range(a, 8):
            v = integrate.quad(lambda t: kl.eval_1d(modes[a], t) * kl.eval_1d(modes[b], t),
                               -0.5, 0.5, epsabs=1e-14, epsrel=1e-13, limit=200)[0]
            assert abs(v - (1.0 if a == b else 0.0)) < 1e-11


def test_nystrom_eigenvalues():
    L = 0.5
    n = 4000
    t = (np.arange(n) + 0.5) / n - 0.5
    Kmat = np.exp(-np.abs(t[:, None] - t[None, :]) / L) / n
    ev = np.sort(np.linalg.eigvalsh(Kmat))[::-1][:6]
    lams = np.array([md[2] for md in kl.eigen_1d(L, 6)])
    assert np.max(np.abs(ev - lams) / lams) < 2e-5


def test_trace_of_unit_kernel():
    # sum of all eigenvalues = int k(t,t) dt = 1; the tail after M modes is O(1/M)
    lams = np.array([md[2] for md in kl.eigen_1d(0.5, 4000)])
    s = lams.sum()
    assert s < 1.0 and 1.0 - s < 1e-3


@pytest.mark.parametrize("L,m", [(0.5, 2), (0.5, 4), (0.5, 6), (0.25, 8), (0.5, 5)])
def test_two_d_selection_is_the_largest_products(L, m):
    picked, modes1 = kl.kl_modes_2d(L, m)
    lam1 = [md[2] for md in kl.eigen_1d(L, 20)]
    allprods = sorted([lam1[i] * lam1[j] for i in range(20) for j in range(20)], reverse=True)
    got = [lam for (_i, _j, lam) in picked]
    assert np.allclose(got, allprods[:m], rtol=1e-14, atol=0)
    # tie rule: equal products keep (i, j) ascending, x1 factor first
    for (i1, j1, l1), (i2, j2, l2) in zip(picked, picked[1:]):
        assert l1 > l2 or (l1 == l2 and (i1, j1) < (i2, j2))
