"""GPU adjoint gradient of J = E[Q] + Var[Q] against the oracle and central differences."""

import numpy as np
import pytest
import torch

import sg_inputs
from gpu_util import note, to_host
from oracle import qoi, system

pytestmark = pytest.mark.gpu

SOLVE = dict(precond="tri", prec=0, restart=40, rtol=1e-13, max_it=400)


def test_gradient_matches_oracle_small():
    import paper_1304_1755_amd as sgbt
    note("adjoint small vs oracle")
    n, m, p, sigma = 16, 2, 2, 0.3
    a0 = sg_inputs.a0_noise_field(n)
    g = sgbt.Problem(n, m, p, sigma, a0_nodal=a0)
    o = system.build_problem(n, m, p, sigma, a0_nodal=a0)
    ref = qoi.qoi_and_gradient(o)
    U, info = g.solve(**SOLVE)
    J, q = g.qoi(U)
    assert abs(J - ref["J"]) < 1e-11 * abs(ref["J"])
    gr = g.qoi_grad(U, **SOLVE)
    assert abs(gr["dsigma"] - ref["dsigma"]) < 1e-8 * max(1, abs(ref["dsigma"]))
    assert np.max(np.abs(gr["damp"] - ref["damp"])) < 1e-8 * max(1, np.max(np.abs(ref["damp"])))
    assert np.max(np.abs(gr["da0"] - ref["da0"])) < 1e-8 * np.max(np.abs(ref["da0"]))
    g.close()


# Finite differences of J need J to be a smooth function of the parameters.
# At 257^2 the relative residual cannot go below about 1e-11 (rounding in
# A U ~ F with |A||U| >> |F|), so a tolerance-driven stop would make the
# iteration count, and J, jump between the +h and -h solves.  The FD
# evaluations therefore run a fixed number of FGMRES steps (one cycle, no
# restart), which brings the residual to its rounding floor, and the
# gradient is taken at a solution computed the same way.
FIXED = dict(precond="tri", prec=0, restart=60, rtol=1e-30, max_it=60)


def _J(cfg, sigma, amps, a0):
    import paper_1304_1755_amd as sgbt
    g = sgbt.Problem(cfg["n"], cfg["m"], cfg["p"], sigma, cfg["corr_len"], a0_nodal=a0, kl_amp=amps)
    U, info = g.solve(**FIXED)
    J, _ = g.qoi(U)
    g.close()
    return J


def test_gradient_against_central_differences_c5():
    import paper_1304_1755_amd as sgbt
    note("adjoint c5 finite differences")
    cfg = sg_inputs.CONFIGS["c5"]
    n, m = cfg["n"], cfg["m"]
    a0 = sg_inputs.a0_noise_field(n)
    g = sgbt.Problem(n, m, cfg["p"], cfg["sigma"], cfg["corr_len"], a0_nodal=a0)
    amps = np.sqrt(np.array(g.kl_lambda))
    U, info = g.solve(**FIXED)
    note(f"c5 forward solve: {info['iters']} it, status {info['status']}, residual {info['rel_res_true']:.2e}")
    assert info["rel_res_true"] < 1e-10
    gr = g.qoi_grad(U, **FIXED)
    note(f"c5 adjoint solve: {gr['adj_info']['iters']} it, residual {gr['adj_info']['rel_res_true']:.2e}")
    assert gr["adj_info"]["rel_res_true"] < 1e-10
    g.close()
    grad = np.concatenate([[gr["dsigma"]], gr["damp"], gr["da0"]])
    gnorm = np.linalg.norm(grad)
    h = 1e-6
    inner = np.zeros((n + 1, n + 1))

    def fd_along(v):
        inner[1:n, 1:n] = v[1 + m:].reshape(n - 1, n - 1)
        va0 = inner.ravel().copy()
        Jp = _J(cfg, cfg["sigma"] + h * v[0], amps + h * v[1:1 + m], a0 + h * va0)
        Jm = _J(cfg, cfg["sigma"] - h * v[0], amps - h * v[1:1 + m], a0 - h * va0)
        return (Jp - Jm) / (2 * h)

    # 20 seeded random unit directions over all 1 + m + (n-1)^2 parameters:
    # normwise bar |grad.v - FD| <= 1e-6 ||grad|| ||v||
    worst = 0.0
    for t, v in enumerate(sg_inputs.unit_directions(20, grad.size, seed=7)):
        fd = fd_along(v)
        ad = float(grad @ v)
        err = abs(ad - fd) / gnorm
        worst = max(worst, err)
        note(f"fd direction {t}: adjoint {ad:.12e} fd {fd:.12e} normwise {err:.2e} "
             f"componentwise {abs(ad - fd) / abs(fd):.2e}")
    assert worst <= 1e-6
    # directions in (sigma, s): derivatives well above the FP64 noise of J/h,
    # componentwise bar |grad.v - FD| <= 1e-6 |FD|
    sub = sg_inputs.unit_directions(4, 1 + m, seed=8)
    for t, vs in enumerate(sub):
        v = np.zeros(grad.size)
        v[:1 + m] = vs
        fd = fd_along(v)
        ad = float(grad @ v)
        note(f"(sigma, s) direction {t}: adjoint {ad:.12e} fd {fd:.12e} rel {abs(ad - fd) / abs(fd):.2e}")
        assert abs(ad - fd) <= 1e-6 * abs(fd)


def test_autograd_function():
    import paper_1304_1755_amd as sgbt
    note("autograd function")
    n, m, p = 16, 2, 2
    o = system.build_problem(n, m, p, 0.3)
    sigma = torch.tensor(0.3, dtype=torch.float64, requires_grad=True)
    amps = torch.tensor(o.kldata["amps"], dtype=torch.float64, requires_grad=True)
    a0 = torch.ones((n + 1) ** 2, dtype=torch.float64, requires_grad=True)
    J = sgbt.SGQoI.apply(sigma, amps, a0, dict(n=n, m=m, p=p, solve=SOLVE))
    J.backward()
    ref = qoi.qoi_and_gradient(o)
    assert abs(J.item() - ref["J"]) < 1e-11 * abs(ref["J"])
    assert abs(sigma.grad.item() - ref["dsigma"]) < 1e-8 * max(1, abs(ref["dsigma"]))
    ga0 = a0.grad.reshape(n + 1, n + 1)[1:n, 1:n].reshape(-1).numpy()
    assert np.max(np.abs(ga0 - ref["da0"])) < 1e-8 * np.max(np.abs(ref["da0"]))
    assert torch.all(a0.grad.reshape(n + 1, n + 1)[0] == 0)
