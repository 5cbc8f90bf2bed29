"""Pins for the oracle's QoI and adjoint gradient.

Pinned against: exact integrals of bilinear functions over the subdomain,
central finite differences with direct solves, the scaling identity
sigma dJ/dsigma = sum_k s_k dJ/ds_k (c_k is bilinear in sigma and s_k), and
the symmetry dJ/dsigma = 0 at sigma = 0.
"""

import numpy as np
import pytest

from oracle import qoi, system


def test_subdomain_weights_integrate_bilinear_exactly():
    n = 16
    h = 1.0 / n
    w = qoi.subdomain_weights(n)
    I, J = np.meshgrid(np.arange(1, n), np.arange(1, n), indexing="xy")
    x, y = (I * h).ravel(), (J * h).ravel()
    assert abs(w.sum() - 1.0) < 1e-15                    # mean of 1 over S
    assert abs(w @ (x * y) - 0.25) < 1e-15               # ((0.75^2-0.25^2)/2)^2 / |S|
    assert abs(w @ x - 0.5) < 1e-15


def _J(n, m, p, sigma, amps=None, a0=None):
    pr = system.build_problem(n, m, p, sigma, a0_nodal=a0, amps=amps)
    return qoi.qoi(pr, system.solve_direct(pr))[0]


def test_gradient_matches_central_differences():
    n, m, p, sigma = 8, 2, 2, 0.3
    rng = np.random.default_rng(11)
    a0 = 1.0 + 0.05 * rng.standard_normal((n + 1) ** 2)
    pr = system.build_problem(n, m, p, sigma, a0_nodal=a0)
    g = qoi.qoi_and_gradient(pr)
    amps = pr.kldata["amps"]
    h = 1e-6
    fd = (_J(n, m, p, sigma + h, a0=a0) - _J(n, m, p, sigma - h, a0=a0)) / (2 * h)
    assert abs(fd - g["dsigma"]) < 1e-7 * max(1.0, abs(fd))
    for k in range(m):
        e = np.zeros(m)
        e[k] = h
        fd = (_J(n, m, p, sigma, amps=amps + e, a0=a0) - _J(n, m, p, sigma, amps=amps - e, a0=a0)) / (2 * h)
        assert abs(fd - g["damp"][k]) < 1e-7 * max(1.0, abs(fd))
    # a0: random interior direction
    v = rng.standard_normal((n - 1) ** 2)
    v /= np.linalg.norm(v)
    from oracle import fem
    imap = fem.interior_map(n)
    inside = imap >= 0
    vf = np.zeros((n + 1) ** 2)
    vf[inside] = v[imap[inside]]
    fd = (_J(n, m, p, sigma, a0=a0 + h * vf) - _J(n, m, p, sigma, a0=a0 - h * vf)) / (2 * h)
    assert abs(fd - g["da0"] @ v) < 1e-7 * max(1.0, abs(fd))


@pytest.mark.parametrize("sigma", [0.0, 0.35])
def test_scaling_identity_and_symmetry(sigma):
    pr = system.build_problem(8, 3, 2, sigma)
    g = qoi.qoi_and_gradient(pr)
    s = pr.kldata["amps"]
    assert abs(sigma * g["dsigma"] - np.dot(s, g["damp"])) < 1e-13
    if sigma == 0.0:
        assert abs(g["dsigma"]) < 1e-14
        assert np.max(np.abs(g["damp"])) < 1e-14
