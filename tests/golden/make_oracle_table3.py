"""Write oracle_table3_counts.txt: the oracle's iteration counts for the five Table 3 solvers.

The paper's Sec. 6 problem (linear triangles, h = 1/64, m = 6, p = 4, L = 1, 833,490 unknowns,
tol 1e-10 from a zero guess): block Gauss-Seidel with B_T, BD-PCG, BT-GPCG[1], BT-GMRes(10) and
BS-PCG, sigma = 0.1 .. 0.4, under two readings of B_T:
  four_*, lex_*: B_T as the lower block-triangular part of A by degree level, every diagonal
    block I (x) K_0 solved by one V(2,2) cycle with four-colour or lexicographic point
    Gauss-Seidel, right-preconditioned FGMRES(10) stopping on the true residual;
  literal_*: B_T = [[A_hat, 0], [W, D]] (the 2x2 split of Sec. 4.2), A_hat solved by one coupled
    V(2,2) cycle with point Gauss-Seidel in mode-major order, D by one lexicographic V(2,2) per
    mode, and GMRes(10) preconditioned from the left with the tolerance on the preconditioned
    residual.
Only the oracle is called; the tests compare with these.  Run:
python tests/golden/make_oracle_table3.py (about twenty minutes on one core).
"""

import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import bt_literal, krylov, mg, paper_mode, precond, system  # noqa: E402

SOLVERS = ["bgs", "bd-pcg", "bt-gpcg", "bt-gmres", "bs-pcg"]


def counts(sigma, colour):
    pr = paper_mode.build_problem_paper(64, 6, 4, sigma)
    A = system.assemble_A(pr)
    H = mg.Hierarchy(pr.K[0], pr.n, coarsest=4, colour_mode=colour, transfer="p1")
    F = pr.rhs().ravel()

    def Av(v):
        return A @ v

    def M(fn):
        return lambda v: fn(pr, v.reshape(pr.P, pr.N), H.vcycle).ravel()

    run = {
        "bgs": lambda: krylov.block_gs(Av, F, M(precond.precond_tri), tol=1e-10, max_it=300),
        "bd-pcg": lambda: krylov.pcg(Av, F, M(precond.precond_diag), tol=1e-10),
        "bt-gpcg": lambda: krylov.gpcg1(Av, F, M(precond.precond_tri), tol=1e-10),
        "bt-gmres": lambda: krylov.fgmres(Av, F, M(precond.precond_tri), restart=10, tol=1e-10),
        "bs-pcg": lambda: krylov.pcg(Av, F, M(precond.precond_sym), tol=1e-10),
    }
    out = []
    for k in SOLVERS:
        _x, info = run[k]()
        assert info["converged"], (sigma, colour, k)
        out.append(info["iters"])
    return out


def literal_counts(sigma):
    pr = paper_mode.build_problem_paper(64, 6, 4, sigma)
    A = system.assemble_A(pr)
    _Ahat, W, Pa = bt_literal.split(pr)
    H = mg.Hierarchy(pr.K[0], pr.n, coarsest=4, colour_mode="lex", transfer="p1")
    V = bt_literal.CoupledVcycle(pr, Pa, mg.prolongation_p1, coarsest=4)
    F = pr.rhs().ravel()

    def Av(v):
        return A @ v

    def Mt(v):
        return bt_literal.precond_tri_2x2(pr, v.reshape(pr.P, pr.N), W, Pa, V, H.vcycle).ravel()

    def Ms(v):
        return bt_literal.precond_sym_2x2(pr, v.reshape(pr.P, pr.N), W, Pa, V, H.vcycle).ravel()

    def Md(v):
        return precond.precond_diag(pr, v.reshape(pr.P, pr.N), H.vcycle).ravel()

    runs = [lambda: krylov.block_gs(Av, F, Mt, tol=1e-10, max_it=300),
            lambda: krylov.pcg(Av, F, Md, tol=1e-10),
            lambda: krylov.gpcg1(Av, F, Mt, tol=1e-10),
            lambda: krylov.gmres_left(Av, F, Mt, restart=10, tol=1e-10),
            lambda: krylov.pcg(Av, F, Ms, tol=1e-10)]
    out = []
    for run in runs:
        _x, info = run()
        assert info["converged"], sigma
        out.append(info["iters"])
    return out


def main():
    lines = ["# The oracle's iteration counts for Table 3's solvers (block GS, BD-PCG, BT-GPCG, BT-GMRes(10),",
             "# BS-PCG) on the Sec. 6 problem, h = 1/64, m = 6, p = 4, tol 1e-10, one V(2,2) per block;",
             "# four_/lex_: level-wise B_T, four-colour / lexicographic smoother; literal_: the 2x2 B_T of",
             "# Sec. 4.2 with a coupled V(2,2) on A_hat and left-preconditioned GMRes (see the script).",
             "# Written by make_oracle_table3.py (oracle only).",
             "# key = counts"]
    for colour in ("four", "lex"):
        for sigma in (0.1, 0.2, 0.3, 0.4):
            c = counts(sigma, colour)
            lines.append(f"{colour}_sigma_{sigma} = " + " ".join(str(v) for v in c))
            print(lines[-1], flush=True)
    for sigma in (0.1, 0.2, 0.3, 0.4):
        lines.append(f"literal_sigma_{sigma} = " + " ".join(str(v) for v in literal_counts(sigma)))
        print(lines[-1], flush=True)
    with open(os.path.join(HERE, "oracle_table3_counts.txt"), "w") as fh:
        fh.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
