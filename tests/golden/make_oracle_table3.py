"""Write oracle_table3_counts.txt: the oracle's iteration counts for the five Table 3 solvers.

The paper's Sec. 6 problem (linear triangles, h = 1/64, m = 6, p = 4, L = 1, 833,490 unknowns,
tol 1e-10 from a zero guess): block Gauss-Seidel with B_T, BD-PCG, BT-GPCG[1], BT-GMRes(10) and
BS-PCG, each block solved by one V(2,2) cycle with four-colour or lexicographic point
Gauss-Seidel, sigma = 0.1 .. 0.4.  Only the oracle is called; the GPU tests compare their counts
with these.  Run: python tests/golden/make_oracle_table3.py (a few minutes on one core).
"""

import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import krylov, mg, paper_mode, precond, system  # noqa: E402

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


def main():
    lines = ["# The oracle's iteration counts for Table 3's solvers (block GS, BD-PCG, BT-GPCG, BT-GMRes(10),",
             "# BS-PCG) on the Sec. 6 problem, h = 1/64, m = 6, p = 4, tol 1e-10, one V(2,2) per block.",
             "# Written by make_oracle_table3.py (oracle only).",
             "# key = counts"]
    for colour in ("four", "lex"):
        for sigma in (0.1, 0.2, 0.3, 0.4):
            c = counts(sigma, colour)
            lines.append(f"{colour}_sigma_{sigma} = " + " ".join(str(v) for v in c))
            print(lines[-1], flush=True)
    with open(os.path.join(HERE, "oracle_table3_counts.txt"), "w") as fh:
        fh.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
