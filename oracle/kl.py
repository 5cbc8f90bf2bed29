"""Karhunen-Loeve expansion of the separable exponential covariance (oracle).

Sec. 2.1, eq. (truncated-KLE): a_m = abar + sum_k sqrt(lambda_k) b_k(x) xi_k,
with eigenpairs of the covariance operator, and eq. (exponential-covariance)
for the kernel.  Reading taken here: the distance |x - y| is the l1 distance,
so the 2-D kernel exp(-|x1-y1|/L - |x2-y2|/L) is the product of two 1-D
kernels on the centred interval t in [-1/2, 1/2]; the 2-D eigenpairs are
products of 1-D ones, both the cosine (even) and sine (odd) families, and the
m largest products are kept (ties broken by the 1-D index pair, x1 factor
first).  sigma multiplies the field, not the eigenvalues.

1-D eigenproblem on [-a, a] with kernel exp(-c|s-t|), c = 1/L: with
lambda = 2c / (omega^2 + c^2) the eigenfunctions are cos(omega t) where
c - omega tan(omega a) = 0, and sin(omega t) where omega + c tan(omega a) = 0.
The roots are found here by bracketing (one root per half period).
"""

import numpy as np
from scipy.optimize import brentq


HALF = 0.5  # half-width a of the centred unit interval


def _even_eq(w, c):
    # c cos(w a) - w sin(w a) = 0  <=>  c - w tan(w a) = 0
    return c * np.cos(w * HALF) - w * np.sin(w * HALF)


def _odd_eq(w, c):
    # w cos(w a) + c sin(w a) = 0  <=>  w + c tan(w a) = 0
    return w * np.cos(w * HALF) + c * np.sin(w * HALF)


def eigen_1d(corr_len, count):
    """First `count` 1-D eigenpairs, ordered by decreasing eigenvalue.

    Returns a list of (kind, omega, lam, norm) with kind 'cos' or 'sin'.  The
    eigenfunction is cos(omega t)/norm or sin(omega t)/norm on t in [-1/2, 1/2].
    """
    c = 1.0 / corr_len
    out = []
    j = 0
    while len(out) < count:
        # with a = 1/2 the even roots lie in (2 j pi, 2 j pi + pi),
        # the odd roots in (2 j pi + pi, 2 j pi + 2 pi).
        lo, hi = 2 * j * np.pi, 2 * j * np.pi + np.pi
        w = brentq(_even_eq, lo, hi, args=(c,), xtol=1e-15, rtol=1e-15, maxiter=500)
        nrm = np.sqrt(HALF + np.sin(2 * w * HALF) / (2 * w))
        out.append(("cos", w, 2 * c / (w * w + c * c), nrm))
        if len(out) == count:
            break
        lo, hi = 2 * j * np.pi + np.pi, 2 * j * np.pi + 2 * np.pi
        w = brentq(_odd_eq, lo, hi, args=(c,), xtol=1e-15, rtol=1e-15, maxiter=500)
        nrm = np.sqrt(HALF - np.sin(2 * w * HALF) / (2 * w))
        out.append(("sin", w, 2 * c / (w * w + c * c), nrm))
        j += 1
    return out


def eval_1d(mode, t):
    kind, w, _lam, nrm = mode
    t = np.asarray(t, dtype=np.float64)
    return (np.cos(w * t) if kind == "cos" else np.sin(w * t)) / nrm


def kl_modes_2d(corr_len, m):
    """The m dominant 2-D modes: list of (i, j, lam_i * lam_j) and the 1-D table."""
    modes1 = eigen_1d(corr_len, m + 1)
    cands = []
    for i in range(m + 1):
        for j in range(m + 1):
            cands.append((-(modes1[i][2] * modes1[j][2]), i, j))
    cands.sort()
    picked = [(i, j, -negl) for (negl, i, j) in cands[:m]]
    return picked, modes1


def eval_2d(picked, modes1, k, x1, x2):
    """phi_k at physical points (x1, x2) in the unit square (centred at 1/2)."""
    i, j, _ = picked[k]
    return eval_1d(modes1[i], np.asarray(x1) - 0.5) * eval_1d(modes1[j], np.asarray(x2) - 0.5)
