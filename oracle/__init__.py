"""FP64 CPU oracle for stochastic Galerkin solves with block preconditioners.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously correct
reference for the method of Zheng, Lin and Xu, "Block triangular
preconditioning for stochastic Galerkin method" (arXiv:1304.1755).  Only the
test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import it.  It shares no code, tables or constants with the
HIP library in ``paper_1304_1755_amd``; the only thing both sides consume is
the seeded input generator package ``sg_inputs``.

Modules (each function cites the part of the paper it follows):

* ``indexset`` -- total-degree multi-index set and the stochastic matrices
  G_0, G_k (Sec. 2.2, eq. (def-stochastic), Sec. 3.2).
* ``kl``       -- Karhunen-Loeve eigenpairs of the separable exponential
  covariance (Sec. 2.1, eqs. (truncated-KLE), (exponential-covariance)).
* ``fem``      -- Q1 stiffness matrices K_0, K_k and the load vector
  (Sec. 3.1, eq. (def-stiffness)).
* ``system``   -- the Kronecker-form Galerkin matrix A (eq. (tensor-product))
  and its direct solution.
* ``mg``       -- geometric multigrid V-cycle for K_0 (Sec. 4.1, Sec. 6).
* ``precond``  -- block-diagonal B_D and block-triangular B_T (Sec. 4).
* ``krylov``   -- GMRES / FGMRES (right preconditioned) and PCG (Sec. 4, 6).
* ``qoi``      -- PCE statistics (eq. (PCE_u)), the subdomain QoI and its
  adjoint gradient.
"""

from . import indexset, kl, fem, system, mg, precond, krylov, qoi  # noqa: F401
