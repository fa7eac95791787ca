/*
 * CPU oracle for matching-based AMG preconditioned CG on IgA stiffness systems.
 *
 * TEST INFRASTRUCTURE ONLY.  This code is the slow, plain, obviously-correct
 * FP64 statement of what the method computes.  Only the test-suite, the smoke
 * check and the CPU-baseline leg of the benchmark may load it.  It shares no
 * code, header, table or helper with the HIP library; the two meet only through
 * the seeded input generator (random draws, no arithmetic of the method).
 *
 * Paper: D'Ambra, Durastante, Filippone, "Parallel matching-based AMG
 * preconditioners for elliptic equations discretized by IgA" (arXiv 2511.21268).
 * Each function cites the passage it follows.  Where the paper is silent the
 * reading taken is stated beside the code.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp (no FMA contraction anywhere, so the
 * aggregates and coarse matrices are fixed to the bit by the evaluation orders
 * written below).
 *
 * Parity pins (tests/test_oracle_*.py): every function below is checked against
 * closed forms, invariants, library routines or brute force.  None is unpinned
 * except the iteration counts of the configurations, which the paper does not
 * print for this preconditioner (see the header of krylov.c).
 */
#ifndef AMG_ORACLE_H
#define AMG_ORACLE_H
#include <stdint.h>

/* ---------------- iga.c : B-spline discretization (Sec. 2) ---------------- */

/* Gauss-Legendre nodes/weights on [-1,1], q points (Newton on P_q). */
int  or_gauss_legendre(int q, double *x, double *w);
/* Open uniform knot vector with n elements, degree p: length n+2p+1. */
void or_knots(int p, int n, double *t);
/* Value and derivative of B-spline N_{i,p} at x by the Cox-de Boor recursion. */
double or_bspline(const double *t, int i, int p, double x);
double or_bspline_deriv(const double *t, int i, int p, double x);
/* 1D mass M1 and stiffness K1 (dense m x m, m=n+p, row-major), and the integrals
 * of each basis function (the 1D load vector for f = 1), by (p+1)-point Gauss
 * quadrature per element. */
void or_matrices_1d(int p, int n, double *M, double *K, double *Fint);
/* Size of the Dirichlet-reduced tensor system: N = (n+p-2)^d and its nnz. */
void or_poisson_size(int d, int p, int n, int64_t *N, int64_t *nnz);
/* Size with Dirichlet only on the faces flagged in dir[2k] (low) and
 * dir[2k+1] (high) of direction k (x = 0, y = 1, z = 2); dir NULL = all faces. */
void or_tensor_size(int d, int p, int n, const int *dir, int64_t *N, int64_t *nnz);
/* As or_poisson_kron with the face flags of or_tensor_size (all zero: the
 * singular Neumann matrix of the full basis). */
int  or_poisson_kron_bc(int d, int p, int n, const int *dir, int64_t *rp, int32_t *ci,
                        double *v, double *F);
/* Constant-coefficient Poisson, homogeneous Dirichlet on every face:
 * K = sum of Kronecker products of K1 and M1 (lexicographic, x fastest),
 * the first and last basis function of every direction removed.  CSR out,
 * arrays sized by or_poisson_size.  Also F for f = 1 when F != NULL. */
int  or_poisson_kron(int d, int p, int n, int64_t *rp, int32_t *ci, double *v, double *F);
/* 3D stiffness with coefficient kappa by (p+1)^3-point Gauss quadrature, by the
 * plain element loop (every quadrature point, every local pair).  kappa is given
 * by its parameters: kappa(x) = exp(0.5 * sum_k a[k] cos(2 pi m_k . x)), nk terms
 * (nk = 0 gives kappa = 1).  Output in the same CSR pattern as or_poisson_kron,
 * plus F for f = 1.  Intended for small n only. */
int  or_diffusion_quad3d(int p, int n, int nk, const double *a, const int32_t *mk,
                         int64_t *rp, int32_t *ci, double *v, double *F);

/* The same integral by sum factorization per element (three 1D contractions per
 * gradient term); the form used at the benchmark sizes. */
int  or_diffusion_sf3d(int p, int n, int nk, const double *a, const int32_t *mk,
                       int64_t *rp, int32_t *ci, double *v, double *F);

/* ---------------- cube.c : the paper's cube benchmark (Sec. 5.1) ---------------- */

/* Size of the cube system: Dirichlet on x = 0, x = 1, y = 0 (Table 1(b)). */
void or_cube_size(int p, int n, int64_t *N, int64_t *nnz);
/* Interior system K u0 = F of -Lap u = f with u = exp(x+z) sin(y): K in CSR
 * (or_poisson_kron_bc pattern), F with the source, the Neumann integrals of
 * sides 4-6 and minus the lifting; lift (length (n+p)^3, full-space order)
 * holds the Dirichlet coefficients (L2 projection of g_D), zero elsewhere. */
int  or_cube_system(int p, int n, int64_t *rp, int32_t *ci, double *v, double *F, double *lift);
/* Full-space coefficients u_h = lift + u0 on the interior functions. */
void or_cube_embed(int p, int n, const double *u0, const double *lift, double *ufull);
/* L2 norm of u_h - u and of u over the cube by (p+4)^3 Gauss points per element. */
int  or_cube_error(int p, int n, const double *ufull, double *err, double *norm);

/* ---------------- amg.c : hierarchy (Sec. 3, 3.1) ---------------- */

typedef struct {
    int sweeps_per_level;   /* m pairwise sweeps per level (aggregates <= 2^m) */
    int max_coarse;         /* coarsest size for the dense Cholesky            */
    int max_levels;
    int nu_pre, nu_post;    /* l1-Jacobi sweeps                                 */
    int match_positive_only;/* 1: only edges with c > 1 are eligible           */
    int smoother;           /* 0: l1-Jacobi, 1: degree-4 polynomial,
                               2: fourth-kind Chebyshev of degree cheb_degree */
    int smooth_prolong;     /* 1: smoothed prolongator (I - omega D^{-1} K) P  */
    int cheb_degree;        /* smoother 2: degree = matrix products per sweep */
    int coarse_solver;      /* 0: dense Cholesky; 1: CG with Jacobi            */
    int coarse_itmax;       /* coarse_solver 1: iteration limit (30)          */
    double omega;           /* prolongator damping (4/3)                      */
    double coarse_tol;      /* coarse_solver 1: relative residual (1e-4)      */
} or_params;

void or_params_default(or_params *p);

typedef struct {
    int64_t n, nnz;
    int64_t *rp; int32_t *ci; double *v;
    double *invd;           /* 1 / l1 diagonal                                */
    double *w;              /* test vector on this level                      */
    int32_t *agg;           /* aggregate (coarse index) of each row; ell < L  */
    double *pc;             /* prolongator coefficient of each row; ell < L   */
    double poly[4];         /* polynomial smoother coefficients (smoother 1)  */
    int64_t *prp; int32_t *pci; double *pv;   /* smoothed prolongator, n x n_c
                               CSR (smooth_prolong; NULL otherwise)           */
    int64_t pnnz;
} or_level;

typedef struct {
    or_params prm;
    int nlev;               /* levels 0..nlev-1; the last one is factored     */
    or_level *lev;
    double *chol;           /* dense lower Cholesky factor, nL x nL row-major */
} or_hier;

/* c_ij of eq. (cij) for the stored entry k_ij (i<j, from row i). */
double or_cij(double kij, double kii, double kjj, double wi, double wj);
/* Greedy matching on an explicit edge list (weights c, ends ei < ej): sort
 * into the strict order below, then take each edge whose ends are both free. */
int  or_greedy_edges(int64_t n, int64_t ne, const double *c, const int32_t *ei,
                     const int32_t *ej, int positive_only, int32_t *mate);
/* Greedy matching in the strict order (c desc, min index asc, max index asc),
 * by a full sort of the eligible edges.  mate[i] = partner or -1. */
int  or_match(int64_t n, const int64_t *rp, const int32_t *ci, const double *v,
              const double *w, int positive_only, int32_t *mate);
/* Count the edges that violate the greedy characterisation of `mate`: an
 * eligible edge not in the matching none of whose endpoints is matched through
 * an edge that comes earlier in the order, or a matched pair that is not an
 * eligible edge.  Zero iff mate is the greedy matching. */
int64_t or_check_greedy(int64_t n, const int64_t *rp, const int32_t *ci, const double *v,
                        const double *w, int positive_only, const int32_t *mate);
/* Number coarse nodes by scanning rows, and build the pairwise prolongator
 * (eq. prolongation) and the restricted test vector.  Returns n_c. */
int64_t or_pairwise_p(int64_t n, const int32_t *mate, const double *w,
                      int32_t *agg, double *pc, double *wc);
void or_l1_invdiag(int64_t n, const int64_t *rp, const int32_t *ci, const double *v, double *invd);
/* Dense Cholesky, in place lower factor.  Returns 0 or -2 (pivot <= 0). */
int  or_cholesky(int n, double *a);
void or_chol_solve(int n, const double *L, const double *b, double *x);

/* Build the hierarchy.  K is copied.  w NULL means ones.
 * Returns 0, -1 (bad argument), -2 (not SPD), -6 (coarsening stalled). */
int  or_setup(int64_t n, const int64_t *rp, const int32_t *ci, const double *v,
              const double *w, const or_params *prm, or_hier **out);
void or_free(or_hier *h);
/* Threads of the row-parallel SpMV (OpenMP; results do not depend on it). */
void or_set_threads(int n);
/* Print one line per level built (progress of long set-ups) when v != 0. */
void or_set_verbose(int v);
int  or_nlevels(const or_hier *h);
void or_level_info(const or_hier *h, int l, int64_t *n, int64_t *nnz);
void or_level_matrix(const or_hier *h, int l, int64_t *rp, int32_t *ci, double *v);
void or_level_agg(const or_hier *h, int l, int32_t *agg, double *pc, double *invd, double *w);
void or_coarse_factor(const or_hier *h, double *L);
int  or_set_poly(or_hier *h, int l, const double *coef);
/* Size and copy of the smoothed prolongator of level l (nnz 0: none). */
int64_t or_level_pnnz(const or_hier *h, int l);
void or_level_prolongator(const or_hier *h, int l, int64_t *rp, int32_t *ci, double *v);

/* ---------------- krylov.c : V-cycle and CG (Sec. 3, 4) ---------------- */

void or_spmv(int64_t n, const int64_t *rp, const int32_t *ci, const double *v,
             const double *x, double *y);
double or_dot(int64_t n, const double *x, const double *y);
/* 0 (default): dots summed in ascending index order; 1: descending */
void or_set_dot_order(int descending);
/* z = B r, one V-cycle from level l with zero initial guess. */
void or_vcycle(const or_hier *h, int l, const double *r, double *z);
/* Preconditioned CG (flexible = 0) or FCG(1) (flexible = 1) on level 0.
 * u: in initial guess, out solution.  Returns 0 converged, 1 not converged,
 * -5 breakdown.  hist (may be NULL) receives ||r_k||/||F|| for k = 0..iters. */
int  or_pcg(const or_hier *h, const double *F, double *u, double tol, int itmax,
            int flexible, int *iters, double *relres, double *hist);
/* Test vector by relaxation on K w = 0 (Sec. 3.1, "Edge weights and projection
 * onto the fine subspace"): `sweeps` l1-Jacobi sweeps w <- w - D^{-1} (K w) from
 * the given random start w0 (row sums ascending from +0.0, no contraction). */
void or_bootstrap_w(int64_t n, const int64_t *rp, const int32_t *ci, const double *v, const double *w0,
                    int sweeps, double *w);
/* Fourth-kind Chebyshev smoother of the given degree for K x = f with the
 * l1 diagonal (invd = 1/d): x in: initial guess (ignored, taken as 0, when
 * x0_zero), out: the smoothed iterate. */
void or_cheb4(int64_t n, const int64_t *rp, const int32_t *ci, const double *v, const double *invd,
              const double *f, double *x, int x0_zero, int degree);
/* CG with the Jacobi preconditioner diag(K)^{-1} from x = 0: stops when
 * ||r|| <= tol ||b|| (recursive residual) or after itmax iterations.
 * Returns the iteration count. */
int  or_cg_jacobi(int64_t n, const int64_t *rp, const int32_t *ci, const double *v, const double *b,
                  double *x, double tol, int itmax);
/* Block flexible CG (O'Leary's block CG with the flexible coefficients) for s
 * right-hand sides F (n x s, column j at F + j n), preconditioned by the
 * V-cycle; U in: initial guesses, out: solutions.  Columns whose residual
 * reaches tol ||F_j|| leave the block.  iters[j], relres[j] per column.
 * Returns 0 all converged, 1 not converged, -5 breakdown (Gram matrix not
 * positive definite). */
int  or_block_fcg(const or_hier *h, int s, const double *F, double *U, double tol, int itmax, int *iters,
                  double *relres);
/* l1-Jacobi-preconditioned polynomial smoother error polynomial check. */
int  or_poly_accept(const double *coef);

/* ---------------- mlp.c : learned-smoother network ---------------- */

int    or_mlp_nparam(void);
double or_bf16_value(uint16_t b);
void   or_mlp_forward(const uint16_t *wb, const double *X, int B, double *Y);
/* loss (mean squared error) and, if grad != NULL, its gradient */
double or_mlp_loss_grad(const uint16_t *wb, const double *X, const double *T, int B, double *grad);
double or_mlp_loss_grad_w(const double *w, const double *X, const double *T, int B, double *grad);

#endif
