/*
 * sgbt -- stochastic Galerkin solves with block-triangular preconditioning on AMD MI355X (gfx950).
 *
 * C ABI of libsgbt.so.  The library solves the stochastic Galerkin system of
 * Zheng, Lin and Xu, "Block triangular preconditioning for stochastic Galerkin
 * method" (arXiv:1304.1755):
 *
 *     A U = F,   A = G_0 (x) K_0 + sum_{k=1..m} G_k (x) K_k          (Sec. 3.1, eq. (tensor-product))
 *
 * for -div(a grad u) = f with zero Dirichlet data on a uniform n x n grid, a
 * truncated Karhunen-Loeve coefficient a = a0 + sigma sum_k s_k b_k(x) xi_k
 * (Sec. 2.1, eq. (truncated-KLE)) and orthonormal Legendre chaos of total
 * degree p (Sec. 2.2).  Two discretisations (sg_options.discretization):
 *   SG_DISC_Q1: bilinear elements on the unit square, f = 1, xi_k ~ U[-1, 1],
 *     cell-centre coefficients, bilinear multigrid transfer;
 *   SG_DISC_P1: the setting of Sec. 6: linear elements on the triangulation
 *     that splits every square along its south-west to north-east diagonal,
 *     D = (-1/2, 1/2)^2, f = 2 (1/2 - x^2 - y^2), xi_k uniform with variance
 *     one (so the coupling entries of G_k, k >= 1, carry a factor sqrt 3),
 *     one coefficient value per triangle (at its centroid), and the linear
 *     interpolation of the triangulation as multigrid transfer.  Every K_k is
 *     then a 5-point operator.
 *
 * Data layout of every block vector ("N x P, node-major"): N = (n-1)^2
 * interior nodes numbered x-fastest, P = (m+p)!/(m!p!) chaos modes in graded
 * order (by total degree; inside a degree by alpha_1 descending, then
 * alpha_2 ...).  Element (node i, mode a) lives at index i*P + a.  Every degree
 * level d is the contiguous column range [off[d], off[d+1]) of each row.
 *
 * Pointers: arguments documented as "device" are HIP device pointers that the
 * caller allocates and owns (for instance torch tensors); "host" arguments are
 * ordinary host memory.  The context owns everything else it allocates.
 * Each context has one HIP stream (the one passed to sg_setup, or the null
 * stream); all work is enqueued on it and calls return without waiting,
 * except where a result is written to host memory.  A context is not
 * thread-safe.
 *
 * Errors: every int-returning call returns 0 on success, a positive warning
 * or a negative error code below; it never aborts.  sg_last_error() returns a
 * message for the last failure in the calling thread.
 */
#ifndef SGBT_H
#define SGBT_H

#ifdef __cplusplus
extern "C" {
#endif

#define SG_OK 0
#define SG_WNOTCOERCIVE 1 /* setup: min over elements of c_0 - xi_max sum_k |c_k| is <= 0, with xi_max = 1
                             (SG_DISC_Q1) or sqrt 3 (SG_DISC_P1): A may be indefinite */
#define SG_EINVAL (-1)    /* invalid argument (sizes, null pointers, unsupported combination) */
#define SG_ENOMEM (-2)    /* device or host allocation failed */
#define SG_EHIP (-3)      /* a HIP runtime call failed; see sg_last_error() */
#define SG_ENOTCONV (-4)  /* solver stopped at max_it above the tolerance (result still written) */
#define SG_ENAN (-5)      /* a residual norm became NaN or Inf */
#define SG_EBREAKDOWN (-6) /* the Krylov recurrence broke down without a usable step (a zero or
                              negative curvature (A p, p) in the CG-type solvers, or no Arnoldi column
                              in the first FGMRES step); U holds the last iterate */

/* precisions */
#define SG_F64 0   /* all arithmetic and storage in double */
#define SG_F32 1   /* float storage and float arithmetic (preconditioner-side variants only) */
#define SG_MIXED 2 /* float preconditioner work, double Krylov / true residual (see each call) */

/* smoother colourings for the multigrid V-cycle */
#define SG_COLOUR_FOUR 0 /* colour (I mod 2) + 2 (J mod 2): exact Gauss-Seidel for the 9-point stencil */
#define SG_COLOUR_RB 1   /* colour (I + J) mod 2, each colour updated from its start-of-colour values */
#define SG_COLOUR_LEX 2  /* lexicographic point Gauss-Seidel (x fastest), forward before and backward after
                            the coarse correction: a reading of the point Gauss-Seidel that Sec. 6 names
                            (the paper gives no ordering).  Sequential fronts: for grids of the paper's
                            sizes, not for throughput */

/* discretisations (see above) */
#define SG_DISC_Q1 0
#define SG_DISC_P1 1

typedef struct sg_ctx sg_ctx;

typedef struct {
    int n_cells;        /* n: cells per side; n = coarsest_cells * 2^L, n % 4 == 0, n <= 4096 */
    int m;              /* KL terms, 0..8 */
    int p;              /* total chaos degree, 0..8, with P = (m+p)!/(m!p!) <= 256 */
    double sigma;       /* standard deviation scale of the field (Sec. 2.1, eq. (exponential-covariance)) */
    double corr_len;    /* correlation length L > 0 */
    int colour_mode;    /* SG_COLOUR_FOUR, SG_COLOUR_RB or SG_COLOUR_LEX */
    int nu1, nu2;       /* pre- and post-smoothing sweeps of the V-cycle, 0..8 */
    int coarsest_cells; /* cells per side of the coarsest grid (>= 2); equal to n_cells gives exact K_0 solves */
    int discretization; /* SG_DISC_Q1 (0) or SG_DISC_P1 (1); SG_DISC_P1 takes a0 = 1 (a0_nodal NULL),
                           SG_COLOUR_FOUR or SG_COLOUR_LEX, and has no sg_qoi / sg_qoi_grad */
} sg_options;

typedef struct {
    int solver;   /* 0: right-preconditioned FGMRES(restart); 1: PCG (precond 0, 2 or 4);
                     2: GPCG[1] (one stored direction); 3: block Gauss-Seidel iteration
                     x <- x + B^{-1}(F - A x); 4: GMRES(restart) preconditioned from the left,
                     stopping when ||B^{-1}(F - A U)|| / ||B^{-1} F|| < rtol (the convention of the
                     MATLAB environment Sec. 6 names; a reading of its GMRes(10)).
                     Solvers 1-4 need prec SG_F64. */
    int precond;  /* 0: block-diagonal B_D (Sec. 4.1); 1: block-triangular B_T (Sec. 4.2), one
                     block per degree level; 2: block symmetric Gauss-Seidel B_S (Sec. 4.2), same
                     blocks; 3: B_T with the 2 x 2 split of Sec. 4.2 (see sg_precond_split);
                     4: its symmetric B_S.  3 and 4 need prec SG_F64 and SG_COLOUR_LEX. */
    int prec;     /* SG_F64: double V-cycles; SG_MIXED: float V-cycles, double Krylov and residuals */
    int restart;  /* GMRES restart length (solvers 0 and 4), 1..64 */
    int max_it;   /* maximum total iterations */
    double rtol;  /* stop when ||F - A U||_2 / ||F||_2 < rtol (true residual, double); solver 4
                     stops on the preconditioned residual (see solver) and reports the true one */
    int use_x0;   /* 0: start from U = 0; 1: U holds the initial guess */
    int timing;   /* 1: time the phases with HIP events (fills t_* below) */
} sg_solve_opts;

typedef struct {
    int iters;              /* total Krylov iterations */
    int restarts;           /* FGMRES cycles beyond the first */
    int status;             /* return code of the solve */
    int n_hist;             /* entries used in rel_res_hist */
    double rel_res_true;    /* final ||F - A U|| / ||F|| in double */
    double rel_res_hist[1024]; /* per-iteration residual estimate (recurrence), relative */
    double t_total_ms;      /* wall time of the solve */
    double t_apply_ms;      /* sum of operator-apply kernel times (timing = 1) */
    double t_prec_ms;       /* sum of preconditioner times (timing = 1) */
    double t_orth_ms;       /* sum of orthogonalisation times (timing = 1) */
    int n_apply;            /* operator applies timed */
    int n_prec;             /* preconditioner applications */
} sg_solve_info;

/* Build a context: KL eigenpairs of the separable exponential covariance,
 * chaos tables, cell coefficients, the multigrid hierarchy of K_0 (Galerkin
 * coarse operators) and the coarsest-grid factorisation; uploads them to the
 * current HIP device.  a0_nodal: host, (n+1)^2 nodal mean field x-fastest, or
 * NULL for a0 = 1.  kl_amp: host, m amplitudes s_k, or NULL for
 * s_k = sqrt(lambda_k).  hip_stream: a hipStream_t or NULL.  Returns
 * SG_WNOTCOERCIVE (ctx still valid) when the discrete coercivity margin is
 * not positive. */
int sg_setup(const sg_options* opt, const double* a0_nodal, const double* kl_amp,
             void* hip_stream, sg_ctx** out);

/* Sizes and tables.  Any output pointer may be NULL.  level_offsets: host,
 * p+2 ints; multi_index: host, P*m ints (row a = alpha of mode a);
 * kl_lambda: host, m doubles; a_min_h: host, 1 double. */
int sg_query(const sg_ctx* ctx, int* N, int* P, int* level_offsets, int* multi_index,
             double* kl_lambda, double* a_min_h);

/* Host copy of the element coefficients c_{k,e} (Sec. 3.1, eq. (def-stiffness)
 * with element-constant coefficients).  SG_DISC_Q1: (m+1) rows of n*n cells,
 * cell (cx, cy) at cy*n + cx; out: host, (m+1)*n*n doubles.  SG_DISC_P1:
 * (m+1) rows of 2*n*n triangles, the lower triangle (SW, SE, NE corners) of
 * cell (cx, cy) at cy*n + cx and its upper triangle (SW, NE, NW) at
 * n*n + cy*n + cx; out: host, (m+1)*2*n*n doubles. */
int sg_get_cell_coeffs(const sg_ctx* ctx, double* out);

/* F = e_0 (x) f_h (Sec. 2.2 Galerkin right-hand side): f = 1 for SG_DISC_Q1,
 * f = 2 (1/2 - x^2 - y^2) integrated exactly for SG_DISC_P1 (Sec. 6).
 * F: device, N*P doubles. */
int sg_rhs(sg_ctx* ctx, double* F);

/* Y = A U, matrix-free (Sec. 3.1, eq. (tensor-product)).
 * prec SG_F64: U, Y device doubles.  SG_MIXED: U device floats, Y device
 * doubles, double arithmetic.  U and Y must not overlap. */
int sg_apply(sg_ctx* ctx, const void* U, void* Y, int prec);

/* R = F - A U in one pass, all device doubles (true residual). */
int sg_residual(sg_ctx* ctx, const double* F, const double* U, double* R);

/* One batched V-cycle for K_0 (Sec. 4.1, Sec. 6) on `width` right-hand sides:
 * u approximately K_0^{-1} f, zero initial guess.  f, u: device, N x width
 * node-major with row strides ldf, ldu (elements).  prec SG_F64: doubles;
 * SG_F32: floats.  1 <= width <= P. */
int sg_vcycle(sg_ctx* ctx, const void* f, int ldf, void* u, int ldu, int width, int prec);

/* Z = B_D^{-1} R with every K_0 solve replaced by one V-cycle (Sec. 4.1).
 * prec SG_F64: R, Z device doubles.  SG_MIXED: R device doubles, Z device floats. */
int sg_precond_diag(sg_ctx* ctx, const void* R, void* Z, int prec);

/* Z = B_T^{-1} R: forward block Gauss-Seidel sweep over degree levels with
 * one V-cycle per diagonal block (Sec. 4.2).  Precisions as sg_precond_diag. */
int sg_precond_tri(sg_ctx* ctx, const void* R, void* Z, int prec);

/* Z = B_S^{-1} R, the block symmetric Gauss-Seidel preconditioner (Sec. 4.2):
 * the forward sweep of sg_precond_tri, then the backward sweep
 * Z_d <- Z_d - V-cycle(sum_k [G_k]_{d,d+1} (x) K_k Z_{d+1}) for d = p-1 .. 0.
 * Symmetric positive definite for double V-cycles (used with PCG).
 * Precisions as sg_precond_diag. */
int sg_precond_sym(sg_ctx* ctx, const void* R, void* Z, int prec);

/* Z = B^{-1} R for the 2 x 2 split of Sec. 4.2, eq. (hierarchical_structure):
 * A = [[A_hat, W^T], [W, D]] with A_hat the stochastic Galerkin matrix of the
 * modes of degree <= p-1 and D = I (x) K_0 that of the degree-p modes.
 * symmetric 0: B = B_T = [[A_hat, 0], [W, D]], so z1 = A_hat^{-1} r1 and
 * z2 = D^{-1}(r2 - W z1).  symmetric 1: B = B_S = B_T blockdiag(A_hat, D)^{-1} B_T^T
 * (the last display of Sec. 4.2), i.e. afterwards z1 <- z1 - A_hat^{-1} W^T z2.
 * Every diagonal block is solved inexactly by one multigrid V(nu1, nu2) cycle,
 * as Table 3's caption has it: A_hat by a cycle for the coupled system (Galerkin
 * coarse operators sum_k G_k (x) P^T K_k P, transfer I (x) P, point Gauss-Seidel
 * on the assembled A_hat_l in its natural order -- mode by mode, inside a mode
 * node by node, x fastest -- forward before and backward after the coarse
 * correction, the coarsest level solved directly), D by one K_0 V-cycle per mode.
 * R, Z: device doubles, N x P node-major, not overlapping.  Double precision only.  The first
 * call builds the coupled hierarchy (host Galerkin products, the coarsest A_hat
 * inverted) and allocates its buffers (about 4 N P doubles).  SG_EINVAL when
 * p < 1, the context's colour mode is not SG_COLOUR_LEX, or the coarsest A_hat
 * has more than 2048 unknowns ((coarsest_cells - 1)^2 times the number of
 * modes of degree <= p-1). */
int sg_precond_split(sg_ctx* ctx, const double* R, double* Z, int symmetric);

/* Solve A U = F (Sec. 4.2 with Sec. 6 stopping rule).  F, U: device doubles
 * (U holds x0 if opts->use_x0).  info: host, may be NULL.  Returns SG_OK,
 * SG_ENOTCONV, SG_ENAN or SG_EBREAKDOWN (U holds the last iterate) or an
 * error.  Work queued earlier on the context's stream is finished before the
 * solve's clock (info->t_total_ms) starts. */
int sg_solve(sg_ctx* ctx, const double* F, double* U, const sg_solve_opts* opts, sg_solve_info* info);

/* SG_DISC_Q1 only (SG_EINVAL otherwise).
 * QoI of eq. (PCE_u) statistics: q_a = w_S . U_a with w_S the exact
 * integration weights of S = [1/4, 3/4]^2 divided by |S|, and
 * J = q_0 + sum_{a>0} q_a^2 (mean plus variance of the subdomain mean).
 * U: device doubles.  q: host, P doubles (may be NULL).  J: host. */
int sg_qoi(sg_ctx* ctx, const double* U, double* q, double* J);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): sg_qoi with
 * no allocation at all.  Its scratch (reduction partials and adjoint weights)
 * is a static per-device array of 1024 * 256 + 256 doubles (2 MiB), held by
 * every GPU the library runs on until the process ends, and its results stay
 * on the device.  U: device doubles, N x P.  q: device, P doubles (q_a).
 * J: device, 1 double.  Enqueued on the context's stream; returns without
 * waiting.  SG_DISC_Q1 only.  SG_EINVAL for null pointers, SG_DISC_P1, or a P
 * whose partials exceed the array (cannot happen for P <= 256).  All calls on
 * one GPU share the array: calls that overlap in time (any contexts, any
 * streams) race; serialize them.  Nothing needs clearing between calls (every
 * scratch entry is written before it is read). */
int sg_qoi_noalloc(sg_ctx* ctx, const double* U, double* q, double* J);

/* SG_DISC_Q1 only (SG_EINVAL otherwise).
 * Adjoint gradient of J at the solution U: solves A lambda = dJ/dU with the
 * same solver options, then dJ/dc_{k,e} = -sum G_k(a,b) lambda_{a,e}^T K_ref U_{b,e}
 * and the chain rule to sigma, the KL amplitudes s_k and the interior nodal
 * values of a0.  U: device doubles (a converged solution).  Outputs host:
 * J (1), dJ_dsigma (1), dJ_damp (m), dJ_da0 ((n-1)^2, interior nodes x-fastest).
 * adj_info: host, may be NULL.  Returns SG_ENOTCONV (outputs written) when
 * the adjoint solve stopped at max_it above rtol. */
int sg_qoi_grad(sg_ctx* ctx, const double* U, const sg_solve_opts* opts, double* J,
                double* dJ_dsigma, double* dJ_damp, double* dJ_da0, sg_solve_info* adj_info);

/* Host-only run of the setup arithmetic of sg_setup, without any device:
 * for checking the tables on machines without a GPU.  Outputs (host, each may
 * be NULL): cell_coeffs as sg_get_cell_coeffs; fine_stencil N*9 and
 * level1_stencil N_1*9 (9-point rows of K_0 and of its first Galerkin coarse
 * operator, (dy,dx) row-major, N_1 = (n/2-1)^2, left untouched when the fine
 * grid is the coarsest); coarsest_inverse Nc*Nc (row-major inverse of the
 * coarsest operator); kl_lambda m; a_min_h 1. */
int sg_setup_host(const sg_options* opt, const double* a0_nodal, const double* kl_amp, double* cell_coeffs,
                  double* fine_stencil, double* level1_stencil, double* coarsest_inverse, double* kl_lambda,
                  double* a_min_h);

/* Wait for all work enqueued on the context's stream. */
int sg_sync(sg_ctx* ctx);

/* Release the context and its device memory. */
void sg_destroy(sg_ctx* ctx);

/* Message for the last failure in this thread ("" if none). */
const char* sg_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* SGBT_H */
