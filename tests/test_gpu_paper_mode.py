"""GPU parity for the paper's own discretisation (Sec. 6, SG_DISC_P1) against the oracle.

Linear elements on the south-west to north-east triangulation, the load
f = 2 (1/2 - x^2 - y^2), unit-variance uniform xi_k (G_k scaled by sqrt 3),
L = 1, and the P1 multigrid transfer: operator apply and residual, the load
vector, batched V-cycles, and the Krylov solvers of Table 3 with their
iteration counts checked against the printed ones.
"""

import numpy as np
import pytest

import sg_inputs
from gpu_util import note, rel_max, to_dev, to_host
from oracle import krylov, mg, paper_mode, precond, system
from test_oracle_indexset import golden

pytestmark = pytest.mark.gpu

_ORACLE = {}


def _pair(n, m, p, sigma, coarsest=4):
    import paper_1304_1755_amd as sgbt
    key = (n, m, p, sigma)
    if key not in _ORACLE:
        _ORACLE.clear()
        _ORACLE[key] = paper_mode.build_problem_paper(n, m, p, sigma)
    g = sgbt.Problem(n, m, p, sigma, corr_len=1.0, coarsest=coarsest, disc="p1")
    return g, _ORACLE[key]


@pytest.mark.parametrize("n,m,p,sigma", [(64, 4, 3, 0.3), (16, 6, 4, 0.2), (32, 1, 1, 0.4), (16, 0, 0, 0.0)])
def test_apply_and_residual_match_oracle(n, m, p, sigma):
    # several 32-column segments with a ragged tail (n = 64: 63 nodes per row), an odd last
    # row pair, P = 35, 210 (four wavefronts per node), 2 and 1 modes
    note(f"p1 apply n={n} m={m} p={p}")
    import torch
    g, o = _pair(n, m, p, sigma)
    assert (g.N, g.P) == (o.N, o.P)
    U = sg_inputs.uniform_block(g.N, g.P, seed=11)
    ref = system.apply(o, U.T).T
    Y = to_host(g.apply(to_dev(U)))
    assert rel_max(Y, ref) < 1e-13
    Ym = to_host(g.apply(to_dev(U, dtype=torch.float32), prec=2))
    ref32 = system.apply(o, U.astype(np.float32).astype(np.float64).T).T
    assert rel_max(Ym, ref32) < 1e-13
    F = sg_inputs.uniform_block(g.N, g.P, seed=12)
    R = to_host(g.residual(to_dev(F), to_dev(U)))
    assert rel_max(R, F - ref) < 1e-13
    g.close()


def test_apply_full_size_separable():
    # the Sec. 6 discretisation at the bench's grid (513 x 513 vertices, m = 6, p = 4, P = 210,
    # 54.8M unknowns, the launch configuration of the timed apply): for a separable input
    # U = sum_r v_r w_r^T the exact result is sum_r sum_k (K_k v_r)(G_k w_r)^T, formed from the
    # oracle's K_k and G_k
    note("p1 apply full size separable")
    import paper_1304_1755_amd as sgbt
    g = sgbt.Problem(512, 6, 4, 0.2, corr_len=1.0, coarsest=4, disc="p1")
    o = paper_mode.build_problem_paper(512, 6, 4, 0.2)
    V, W = sg_inputs.separable_factors(g.N, g.P, rank=2)
    Y = to_host(g.apply(to_dev(V.T @ W)))
    ref = np.zeros((g.N, g.P))
    for r in range(2):
        for Gk, Kk in zip(o.G, o.K):
            ref += np.outer(Kk @ V[r], Gk @ W[r])
    assert rel_max(Y, ref) < 1e-12
    g.close()


def test_load_vector_matches_oracle():
    note("p1 rhs")
    g, o = _pair(32, 3, 2, 0.1)
    F = to_host(g.rhs())
    assert np.max(np.abs(F[:, 0] - o.f)) < 1e-15 * max(1.0, np.max(np.abs(o.f))) + 1e-17
    assert np.all(F[:, 1:] == 0.0)
    g.close()


@pytest.mark.parametrize("n,width,prec", [(64, 35, 0), (64, 7, 0), (128, 20, 1), (128, 5, 1), (16, 10, 0)])
def test_vcycle_matches_oracle(n, width, prec):
    # widths >= 16 take the walking transfer kernels, narrower ones the per-node kernels; the
    # double cycle fuses grids up to 31 x 31 interior nodes, the float one up to 63 x 63
    note(f"p1 vcycle n={n} width={width} prec={prec}")
    import torch
    g, o = _pair(n, 4, 3, 0.3)  # P = 35 >= width
    H = mg.Hierarchy(o.K[0], n, coarsest=4, colour_mode="four", nu1=2, nu2=2, transfer="p1")
    f = sg_inputs.uniform_block(g.N, width, seed=21)
    ref = np.stack([H.vcycle(f[:, j]) for j in range(width)], axis=1)
    dt = torch.float64 if prec == 0 else torch.float32
    u = to_host(g.vcycle(to_dev(f, dtype=dt), prec=prec))
    assert rel_max(u, ref) < (1e-12 if prec == 0 else 2e-5)
    g.close()


@pytest.mark.parametrize("kind", ["diag", "tri", "sym"])
def test_preconditioners_match_oracle(kind):
    note(f"p1 precond {kind}")
    g, o = _pair(32, 3, 3, 0.3)
    H = mg.Hierarchy(o.K[0], 32, coarsest=4, colour_mode="four", transfer="p1")
    fn = {"diag": precond.precond_diag, "tri": precond.precond_tri, "sym": precond.precond_sym}[kind]
    R = sg_inputs.uniform_block(g.N, g.P, seed=41)
    ref = fn(o, R.T, H.vcycle).T
    Z = to_host(g.precond(to_dev(R), kind=kind))
    assert rel_max(Z, ref) < 1e-11
    g.close()


def test_solution_matches_direct_solve():
    note("p1 solve direct")
    g, o = _pair(32, 3, 2, 0.3)
    A = system.assemble_A(o)
    U, info = g.solve(solver="fgmres", precond="tri", restart=10, rtol=1e-10, max_it=200)
    Ustar = system.solve_direct(o, A=A)
    assert info["status"] == 0 and info["rel_res_true"] < 1e-10
    assert rel_max(to_host(U).T, Ustar) < 1e-8
    g.close()


def oracle_table3(colour, sigma):
    """The oracle's Table 3 counts (block GS, BD-PCG, BT-GPCG, BT-GMRes(10), BS-PCG) stored by
    tests/golden/make_oracle_table3.py, which calls only the oracle."""
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "oracle_table3_counts.txt")
    with open(path) as fh:
        for line in fh:
            line = line.split("#")[0].strip()
            if line.startswith(f"{colour}_sigma_{sigma} ="):
                return [int(v) for v in line.split("=", 1)[1].split()]
    raise KeyError((colour, sigma))


def _oracle_counts(pr, names):
    A = system.assemble_A(pr)
    H = mg.Hierarchy(pr.K[0], pr.n, coarsest=4, colour_mode="four", transfer="p1")
    F = pr.rhs().ravel()
    Av = lambda v: A @ v  # noqa: E731

    def M(fn):
        return lambda v: fn(pr, v.reshape(pr.P, pr.N), H.vcycle).ravel()

    run = {
        "bgs": lambda: krylov.block_gs(Av, F, M(precond.precond_tri), tol=1e-10, max_it=300),
        "bd-pcg": lambda: krylov.pcg(Av, F, M(precond.precond_diag), tol=1e-10),
        "bt-gpcg": lambda: krylov.gpcg1(Av, F, M(precond.precond_tri), tol=1e-10),
        "bt-gmres": lambda: krylov.fgmres(Av, F, M(precond.precond_tri), restart=10, tol=1e-10),
        "bs-pcg": lambda: krylov.pcg(Av, F, M(precond.precond_sym), tol=1e-10),
    }
    return [run[k]()[1]["iters"] for k in names]


@pytest.mark.parametrize("sigma", [0.1, 0.2, 0.3, 0.4])
def test_table3_iteration_counts(sigma):
    # Table 3 (p = 4, m = 6, h = 1/64, 833,490 unknowns): block Gauss-Seidel, BD-PCG,
    # BT-GPCG, BT-GMRes(10), BS-PCG to a relative residual of 1e-10 from zero, with the
    # four-colour point Gauss-Seidel smoother (forward before, backward after the coarse
    # correction).  The counts must equal the oracle's, running the same algorithm, within one
    # (the printed counts are only reported: they were obtained with another smoother).
    note(f"p1 table 3 sigma {sigma}")
    paper = [int(v) for v in golden()[f"table3_iters_sigma_{sigma}"].split()]
    g, o = _pair(64, 6, 4, sigma)
    assert g.N * g.P == int(golden()["table1_size_A"])
    runs = [dict(solver="bgs", precond="tri"), dict(solver="pcg", precond="diag"),
            dict(solver="gpcg", precond="tri"), dict(solver="fgmres", precond="tri", restart=10),
            dict(solver="pcg", precond="sym")]
    got = []
    for kw in runs:
        _, info = g.solve(rtol=1e-10, max_it=300, **kw)
        assert info["status"] == 0 and info["rel_res_true"] < 1e-10, (kw, info["status"])
        got.append(info["iters"])
    g.close()
    ref = oracle_table3("four", sigma)
    note(f"p1 table 3 sigma {sigma}: gpu {got}, oracle {ref}, paper {paper}")
    for it, r in zip(got, ref):
        assert abs(it - r) <= 1, (got, ref)


def test_table2_counts_are_robust_in_h_and_p():
    # Table 2 (sigma = 0.1, m = 4): the iteration counts of BD-PCG, BT-GPCG, BS-PCG and BT-GMRes do not
    # grow with the mesh (h = 1/32, 1/64, 1/128) or the chaos degree (p = 2, 3, 4); the paper
    # prints one count per solver for all of them.  Here: counts no larger than the printed ones,
    # independent of h within one for every p, growing by at most two from p = 2 to p = 4 (the
    # mean-based B_D sees the spread of the G_k spectra widen with p; the four-colour smoother
    # leaves it visible below the printed 13), and equal to the oracle's four-colour counts
    # within one on the smallest mesh.
    note("p1 table 2")
    import paper_1304_1755_amd as sgbt
    g0 = golden()
    # the table prints one column for BT-GPCG and BS-PCG
    paper = [int(g0["table2_iters_BD_PCG"]), int(g0["table2_iters_BT_GPCG"]), int(g0["table2_iters_BT_GMRes"]),
             int(g0["table2_iters_BT_GPCG"])]
    runs = [dict(solver="pcg", precond="diag"), dict(solver="gpcg", precond="tri"),
            dict(solver="fgmres", precond="tri", restart=10), dict(solver="pcg", precond="sym")]
    counts = {}
    for n in (32, 64, 128):
        for p in (2, 3, 4):
            g = sgbt.Problem(n, 4, p, 0.1, corr_len=1.0, coarsest=4, disc="p1")
            its = []
            for kw in runs:
                _, info = g.solve(rtol=1e-10, max_it=300, **kw)
                assert info["status"] == 0 and info["rel_res_true"] < 1e-10, (n, p, kw)
                its.append(info["iters"])
            g.close()
            counts[(n, p)] = its
    note(f"p1 table 2 counts {counts} (paper {paper})")
    for j in range(4):
        col = [v[j] for v in counts.values()]
        assert max(col) <= paper[j], (j, counts, paper)
        assert max(col) - min(col) <= 2, (j, counts)
        for p in (2, 3, 4):
            in_h = [counts[(n, p)][j] for n in (32, 64, 128)]
            assert max(in_h) - min(in_h) <= 1, (j, p, counts)
    o = paper_mode.build_problem_paper(32, 4, 3, 0.1)
    ref = _oracle_counts(o, ["bd-pcg", "bt-gpcg", "bt-gmres", "bs-pcg"])
    for it, r in zip(counts[(32, 3)], ref):
        assert abs(it - r) <= 1, (counts[(32, 3)], ref)


@pytest.mark.parametrize("disc,n,width,prec", [("p1", 64, 35, 0), ("p1", 64, 6, 1), ("q1", 64, 21, 0),
                                                 ("q1", 128, 35, 1)])
def test_lexicographic_vcycle_matches_oracle(disc, n, width, prec):
    # lexicographic point Gauss-Seidel (our reading of Sec. 6's point Gauss-Seidel), forward before and backward
    # after the coarse correction; separate-launch levels and the fused coarse cycle
    note(f"lex vcycle {disc} n={n} width={width} prec={prec}")
    import torch
    import paper_1304_1755_amd as sgbt
    if disc == "p1":
        g = sgbt.Problem(n, 4, 3, 0.3, corr_len=1.0, coarsest=4, disc="p1", colour="lex")
        o = paper_mode.build_problem_paper(n, 4, 3, 0.3)
        H = mg.Hierarchy(o.K[0], n, coarsest=4, colour_mode="lex", transfer="p1")
    else:
        g = sgbt.Problem(n, 4, 3, 0.3, coarsest=8, colour="lex")
        o = system.build_problem(n, 4, 3, 0.3)
        H = mg.Hierarchy(o.K[0], n, coarsest=8, colour_mode="lex")
    f = sg_inputs.uniform_block(g.N, width, seed=23)
    ref = H.vcycle(f)
    dt = torch.float64 if prec == 0 else torch.float32
    u = to_host(g.vcycle(to_dev(f, dtype=dt), prec=prec))
    assert rel_max(u, ref) < (1e-11 if prec == 0 else 2e-5)
    g.close()


@pytest.mark.parametrize("sigma", [0.1, 0.2, 0.3, 0.4])
def test_table3_with_lexicographic_smoother(sigma):
    # Table 3 with the lexicographic V(2,2) (our reading of Sec. 6's point Gauss-Seidel): the five
    # solvers' counts equal the oracle's (same smoother) within one at every sigma; at sigma = 0.1
    # they are also within one of the printed ones (at larger sigma this reading of B_T gives more
    # block Gauss-Seidel / BT iterations than printed, on the oracle as on the GPU)
    note(f"p1 table 3 lexicographic sigma {sigma}")
    import paper_1304_1755_amd as sgbt
    paper = [int(v) for v in golden()[f"table3_iters_sigma_{sigma}"].split()]
    g = sgbt.Problem(64, 6, 4, sigma, corr_len=1.0, coarsest=4, disc="p1", colour="lex")
    runs = [dict(solver="bgs", precond="tri"), dict(solver="pcg", precond="diag"),
            dict(solver="gpcg", precond="tri"), dict(solver="fgmres", precond="tri", restart=10),
            dict(solver="pcg", precond="sym")]
    got = []
    for kw in runs:
        _, info = g.solve(rtol=1e-10, max_it=300, **kw)
        assert info["status"] == 0 and info["rel_res_true"] < 1e-10, (kw, info["status"])
        got.append(info["iters"])
    g.close()
    ref = oracle_table3("lex", sigma)
    note(f"p1 table 3 lexicographic sigma {sigma}: gpu {got}, oracle {ref}, paper {paper}")
    for it, r, pp in zip(got, ref, paper):
        assert abs(it - r) <= 1, (got, ref)
        if sigma == 0.1:
            assert abs(it - pp) <= 1, (got, paper)


def test_table2_with_lexicographic_smoother():
    # Table 2 (sigma = 0.1, m = 4, h = 1/32 .. 1/128, p = 2 .. 4) with the lexicographic V(2,2):
    # every count within one of the printed one (BD-PCG 13, BT-GPCG 9, BT-GMRes 8, BS-PCG 9),
    # whatever h and p
    note("p1 table 2 lexicographic")
    import paper_1304_1755_amd as sgbt
    g0 = golden()
    paper = [int(g0["table2_iters_BD_PCG"]), int(g0["table2_iters_BT_GPCG"]), int(g0["table2_iters_BT_GMRes"]),
             int(g0["table2_iters_BT_GPCG"])]
    runs = [dict(solver="pcg", precond="diag"), dict(solver="gpcg", precond="tri"),
            dict(solver="fgmres", precond="tri", restart=10), dict(solver="pcg", precond="sym")]
    counts = {}
    for n in (32, 64, 128):
        for p in (2, 3, 4):
            g = sgbt.Problem(n, 4, p, 0.1, corr_len=1.0, coarsest=4, disc="p1", colour="lex")
            its = []
            for kw in runs:
                _, info = g.solve(rtol=1e-10, max_it=300, **kw)
                assert info["status"] == 0 and info["rel_res_true"] < 1e-10, (n, p, kw)
                its.append(info["iters"])
            g.close()
            counts[(n, p)] = its
    note(f"p1 table 2 lexicographic counts {counts} (paper {paper})")
    for its in counts.values():
        for it, pp in zip(its, paper):
            assert abs(it - pp) <= 1, (counts, paper)


def test_mixed_precision_solve_reaches_tolerance():
    note("p1 mixed solve")
    g, o = _pair(64, 4, 3, 0.3)
    U, info = g.solve(solver="fgmres", precond="tri", prec=2, restart=10, rtol=1e-10, max_it=200)
    _, i64 = g.solve(solver="fgmres", precond="tri", restart=10, rtol=1e-10, max_it=200)
    assert info["status"] == 0 and info["rel_res_true"] < 1e-10
    assert abs(info["iters"] - i64["iters"]) <= 1
    F = o.rhs().ravel()
    r = F - system.apply(o, to_host(U).T).ravel()
    assert np.linalg.norm(r) / np.linalg.norm(F) < 1e-10
    g.close()


def test_p1_rejects_unsupported_options():
    import paper_1304_1755_amd as sgbt
    with pytest.raises(sgbt.SGError):
        sgbt.Problem(16, 2, 2, 0.1, corr_len=1.0, coarsest=4, disc="p1", colour="rb")
    with pytest.raises(sgbt.SGError):
        sgbt.Problem(16, 2, 2, 0.1, corr_len=1.0, coarsest=4, disc="p1", a0_nodal=np.ones(17 * 17))
    g = sgbt.Problem(16, 2, 2, 0.1, corr_len=1.0, coarsest=4, disc="p1")
    U, _ = g.solve(rtol=1e-8)
    with pytest.raises(sgbt.SGError):
        g.qoi(U)
    g.close()
