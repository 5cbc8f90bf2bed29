"""Write oracle_table2_counts.txt: the oracle's iteration counts for the Table 2 solvers under the
2x2 split of Sec. 4.2.

The paper's Sec. 6 problem with sigma = 0.1, m = 4, L = 1, tol 1e-10 from a zero guess, for
h = 1/32, 1/64, 1/128 and p = 2, 3, 4: BD-PCG (one lexicographic V(2,2) per mode), BT-GPCG[1] and
BT-GMRes(10) with B_T = [[A_hat, 0], [W, D]] (A_hat by one coupled lexicographic V(2,2), D by one
V(2,2) per mode; GMRes preconditioned from the left, the tolerance on the preconditioned
residual), and BS-PCG with the symmetric B_S of the same split.  Only the oracle is called; the
GPU tests compare with these.  Run: python tests/golden/make_oracle_table2.py (about fifteen
minutes on one core).
"""

import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import bt_literal, krylov, mg, paper_mode, precond, system  # noqa: E402


def split_counts(n, p, sigma=0.1, m=4):
    pr = paper_mode.build_problem_paper(n, m, p, sigma)
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

    runs = [lambda: krylov.pcg(Av, F, Md, tol=1e-10),
            lambda: krylov.gpcg1(Av, F, Mt, tol=1e-10),
            lambda: krylov.gmres_left(Av, F, Mt, restart=10, tol=1e-10),
            lambda: krylov.pcg(Av, F, Ms, tol=1e-10)]
    out = []
    for run in runs:
        _x, info = run()
        assert info["converged"], (n, p)
        out.append(info["iters"])
    return out


def main():
    sizes = [int(v) for v in sys.argv[1:]] or [32, 64, 128]
    lines = ["# The oracle's iteration counts for Table 2's solvers (BD-PCG, BT-GPCG, BT-GMRes(10), BS-PCG)",
             "# on the Sec. 6 problem, sigma = 0.1, m = 4, tol 1e-10, one lexicographic V(2,2) per block,",
             "# with B_T and B_S of the 2x2 split of Sec. 4.2 (A_hat by a coupled V(2,2)) and GMRes(10)",
             "# preconditioned from the left.  Written by make_oracle_table2.py (oracle only).",
             "# split_n<cells>_p<degree> = counts"]
    for n in sizes:
        for p in (2, 3, 4):
            lines.append(f"split_n{n}_p{p} = " + " ".join(str(v) for v in split_counts(n, p)))
            print(lines[-1], flush=True)
    with open(os.path.join(HERE, "oracle_table2_counts.txt"), "w") as fh:
        fh.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
