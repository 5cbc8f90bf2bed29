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


def test_gradient_matches_oracle_c5():
    # the adjoint workload itself (257^2, m = 5, p = 3, P = 56, sigma = 0.3, seeded a0 noise): every
    # component of the GPU gradient (dJ/dsigma, the 5 dJ/ds_k and all 65,025 interior dJ/da0)
    # against the oracle's adjoint gradient (direct solves), element by element
    import paper_1304_1755_amd as sgbt
    note("adjoint c5 vs oracle gradient")
    cfg = sg_inputs.CONFIGS["c5"]
    n, m, p = cfg["n"], cfg["m"], cfg["p"]
    a0 = sg_inputs.a0_noise_field(n)
    g = sgbt.Problem(n, m, p, cfg["sigma"], cfg["corr_len"], a0_nodal=a0)
    U, info = g.solve(**FIXED)
    gr = g.qoi_grad(U, **FIXED)
    g.close()
    note(f"c5 gpu: J {gr['J']:.15e}, forward {info['iters']} it, adjoint {gr['adj_info']['iters']} it")
    o = system.build_problem(n, m, p, cfg["sigma"], cfg["corr_len"], a0_nodal=a0)
    ref = qoi.qoi_and_gradient(o)
    note(f"c5 oracle: J {ref['J']:.15e}")
    assert abs(gr["J"] - ref["J"]) < 1e-10 * abs(ref["J"])
    assert abs(gr["dsigma"] - ref["dsigma"]) < 1e-8 * abs(ref["dsigma"])
    assert np.max(np.abs(gr["damp"] - ref["damp"])) < 1e-8 * np.max(np.abs(ref["damp"]))
    err_a0 = np.max(np.abs(gr["da0"] - ref["da0"])) / np.max(np.abs(ref["da0"]))
    note(f"c5 gradient: max rel error of dJ/da0 {err_a0:.2e}")
    assert err_a0 < 1e-8


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
    # the interior nodal values of a0 are the differentiable input; the boundary
    # vertices are data (here 1); every input gets the oracle's gradient
    import paper_1304_1755_amd as sgbt
    note("autograd function")
    n, m, p = 16, 2, 2
    a0 = sg_inputs.a0_noise_field(n)
    o = system.build_problem(n, m, p, 0.3, a0_nodal=a0)
    sigma = torch.tensor(0.3, dtype=torch.float64, requires_grad=True)
    amps = torch.tensor(o.kldata["amps"], dtype=torch.float64, requires_grad=True)
    inner = torch.tensor(a0.reshape(n + 1, n + 1)[1:n, 1:n].ravel(), dtype=torch.float64, requires_grad=True)
    J = sgbt.SGQoI.apply(sigma, amps, inner, dict(n=n, m=m, p=p, a0_boundary=a0, solve=SOLVE))
    J.backward()
    ref = qoi.qoi_and_gradient(o)
    assert abs(J.item() - ref["J"]) < 1e-11 * abs(ref["J"])
    assert abs(sigma.grad.item() - ref["dsigma"]) < 1e-8 * max(1, abs(ref["dsigma"]))
    assert np.max(np.abs(amps.grad.numpy() - ref["damp"])) < 1e-8 * max(1, np.max(np.abs(ref["damp"])))
    assert np.max(np.abs(inner.grad.numpy() - ref["da0"])) < 1e-8 * np.max(np.abs(ref["da0"]))


def test_boundary_a0_is_data_not_a_parameter():
    # a0 on the boundary vertices changes J (the cells next to the boundary average it in), so it
    # cannot silently receive a zero gradient: the autograd Function takes it as fixed data
    import paper_1304_1755_amd as sgbt
    note("boundary a0 is data")
    n, m, p = 16, 2, 2
    a0 = sg_inputs.a0_noise_field(n)
    inner = torch.tensor(a0.reshape(n + 1, n + 1)[1:n, 1:n].ravel(), dtype=torch.float64)
    amps = torch.tensor(system.build_problem(n, m, p, 0.3).kldata["amps"], dtype=torch.float64)
    cfg = dict(n=n, m=m, p=p, solve=SOLVE)
    J1 = sgbt.SGQoI.apply(torch.tensor(0.3, dtype=torch.float64), amps, inner, cfg).item()
    bnd = np.full((n + 1) ** 2, 1.5)
    J2 = sgbt.SGQoI.apply(torch.tensor(0.3, dtype=torch.float64), amps, inner, dict(cfg, a0_boundary=bnd)).item()
    full = a0.reshape(n + 1, n + 1).copy()
    full[0, :] = full[-1, :] = full[:, 0] = full[:, -1] = 1.5
    ref = qoi.qoi_and_gradient(system.build_problem(n, m, p, 0.3, a0_nodal=full.ravel()))
    assert abs(J2 - ref["J"]) < 1e-11 * abs(ref["J"])
    assert abs(J1 - J2) > 1e-6 * abs(J1)
    with pytest.raises(ValueError):
        sgbt.SGQoI.apply(torch.tensor(0.3, dtype=torch.float64), amps, torch.ones((n + 1) ** 2, dtype=torch.float64), cfg)
