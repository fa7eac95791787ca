/*
 * Oracle, part 3: the solve phase (paper Sec. 3: smoother sweep eq. (smoother),
 * the five steps of the two-level correction applied recursively as a V-cycle,
 * the l1-Jacobi iteration of Sec. 3.2; Sec. 4 Krylov call: CG, and flexible CG
 * for a variable preconditioner).  TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * Readings:
 *  - V-cycle: zero initial guess on every level; nu_pre sweeps, restrict the
 *    residual with P^T, recurse (dense Cholesky solve on the coarsest level),
 *    prolongate and correct, nu_post sweeps.  The first sweep from the zero
 *    guess is u = D^{-1} f (K 0 = 0);
 *  - l1-Jacobi sweep: u <- u + D^{-1} (f - K u);
 *  - degree-4 polynomial smoother: u <- u + sum_{k=0..3} a_k (D^{-1}K)^k D^{-1} r
 *    with r = f - K u, evaluated by Horner's rule; its error polynomial is
 *    e(t) = 1 - sum_k a_k t^{k+1} on the spectrum t of D^{-1}K, in (0, 1];
 *  - fourth-kind Chebyshev smoother (Sec. 3.2: Chebyshev acceleration of
 *    l1-Jacobi without spectral estimates, after Lottes' fourth-kind
 *    polynomials; the paper's optimized coefficients are not given, the
 *    unoptimized fourth-kind polynomial is taken): k sweeps leave the error
 *    e_k = W_k(I - 2 D^{-1}K) e_0 / (2k+1), W_k the fourth-kind Chebyshev
 *    polynomial, W_k(cos t) = sin((k + 1/2) t) / sin(t/2), on the spectrum of
 *    D^{-1}K in (0, 1].  Written as the three-term recurrence of W_k on the
 *    iterates with the true residual r_j = f - K x_j:
 *      x_1 = x_0 + (4/3) D^{-1} r_0,
 *      (2j+3) x_{j+1} = 2(2j+1) x_j + 4(2j+1) D^{-1} r_j - (2j-1) x_{j-1};
 *    nu_pre / nu_post count such smoothers; the same polynomial before and
 *    after keeps the V-cycle symmetric;
 *  - coarsest level (coarse_solver 1, Sec. 5.1): CG preconditioned by one
 *    Jacobi sweep z = diag(K)^{-1} r from x = 0 (a Jacobi weight cancels in
 *    CG), to ||r|| <= coarse_tol ||f|| or coarse_itmax iterations; the
 *    V-cycle is then a variable preconditioner (use FCG);
 *  - test vector (Sec. 3.1): a few l1-Jacobi sweeps on K w = 0 from a random
 *    start that the caller draws (the relaxation named by the paper is damped
 *    Jacobi or Gauss-Seidel; l1-Jacobi is the path's own damped Jacobi);
 *  - restriction and prolongation with a smoothed prolongator: f_c = P'^T r
 *    summed over the rows i ascending, u_i += sum_J P'_iJ e_J ascending J;
 *  - block flexible CG for s right-hand sides (O'Leary's block CG, with the
 *    coefficients of FCG(1) so that a variable preconditioner is allowed):
 *    Q = K P, G = P^T Q, alpha = G^{-1} P^T R, X += P alpha, R -= Q alpha,
 *    Z = B R, beta = -G^{-1} Q^T Z, P = Z + P beta, all over the active
 *    columns (G^{-1} by Cholesky of the active block); a column whose
 *    residual reaches tol ||F_j|| leaves the block (its X and R freeze), and
 *    beta is formed over the columns still active after that test;
 *  - CG: Hestenes-Stiefel PCG; FCG(1): alpha = (p,r)/(p,q),
 *    beta = -(z_{k+1}, q_k)/(p_k, q_k);
 *  - stop when ||r_k||_2 <= tol ||F||_2 on the recursive residual; iters counts
 *    the completed updates of u; F = 0 returns u = 0 after 0 iterations;
 *  - SpMV row sums and dots are sequential in ascending index order (the SpMV
 *    is parallel over rows only, so any thread count gives the same bits);
 *    or_set_dot_order(1) sums the dots in descending index order instead: a
 *    second, equally plain rounding order of the same algorithm (the paper
 *    fixes none), used by the tests to measure how far rounding order alone
 *    moves the iterates of a given system.
 *
 * Parity unpinned: iteration counts of the benchmark configurations (the paper
 * prints counts only for its own preconditioner, tolerance and boundary data).
 */
#include "oracle.h"
#include <math.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif
void or_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

void or_spmv(int64_t n, const int64_t *rp, const int32_t *ci, const double *v,
             const double *x, double *y)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++) {
        double s = 0.0;
        for (int64_t e = rp[i]; e < rp[i + 1]; e++) s = s + v[e] * x[ci[e]];
        y[i] = s;
    }
}

static int dot_descending = 0;
void or_set_dot_order(int descending) { dot_descending = descending ? 1 : 0; }

double or_dot(int64_t n, const double *x, const double *y)
{
    double s = 0.0;
    if (dot_descending)
        for (int64_t i = n - 1; i >= 0; i--) s = s + x[i] * y[i];
    else
        for (int64_t i = 0; i < n; i++) s = s + x[i] * y[i];
    return s;
}

/* correction c = p(D^{-1}K) D^{-1} r of the smoother in use */
static void smoother_apply(const or_level *L, int poly, const double *r, double *c, double *tmp)
{
    int64_t n = L->n;
    if (!poly) {
        for (int64_t i = 0; i < n; i++) c[i] = L->invd[i] * r[i];
        return;
    }
    /* Horner: c = a3 s; c = a_k s + D^{-1} K c for k = 2, 1, 0; s = D^{-1} r */
    for (int64_t i = 0; i < n; i++) c[i] = L->poly[3] * (L->invd[i] * r[i]);
    for (int k = 2; k >= 0; k--) {
        or_spmv(n, L->rp, L->ci, L->v, c, tmp);
        for (int64_t i = 0; i < n; i++)
            c[i] = L->poly[k] * (L->invd[i] * r[i]) + L->invd[i] * tmp[i];
    }
}

static void sweep(const or_level *L, int poly, const double *f, double *u,
                  double *r, double *c, double *tmp)
{
    or_spmv(L->n, L->rp, L->ci, L->v, u, r);
    for (int64_t i = 0; i < L->n; i++) r[i] = f[i] - r[i];
    smoother_apply(L, poly, r, c, tmp);
    for (int64_t i = 0; i < L->n; i++) u[i] = u[i] + c[i];
}

void or_bootstrap_w(int64_t n, const int64_t *rp, const int32_t *ci, const double *v, const double *w0,
                    int sweeps, double *w)
{
    double *invd = malloc(sizeof(double) * n), *s = malloc(sizeof(double) * n);
    or_l1_invdiag(n, rp, ci, v, invd);
    memcpy(w, w0, sizeof(double) * n);
    for (int k = 0; k < sweeps; k++) {
        or_spmv(n, rp, ci, v, w, s);
        for (int64_t i = 0; i < n; i++) w[i] = w[i] - invd[i] * s[i];
    }
    free(invd); free(s);
}

void or_cheb4(int64_t n, const int64_t *rp, const int32_t *ci, const double *v, const double *invd,
              const double *f, double *x, int x0_zero, int degree)
{
    double *xp = malloc(sizeof(double) * n), *r = malloc(sizeof(double) * n);
    double *xn = malloc(sizeof(double) * n);
    if (x0_zero)
        for (int64_t i = 0; i < n; i++) x[i] = 0.0;
    for (int j = 0; j < degree; j++) {
        or_spmv(n, rp, ci, v, x, r);
        for (int64_t i = 0; i < n; i++) r[i] = f[i] - r[i];
        if (j == 0) {
            for (int64_t i = 0; i < n; i++) {
                xp[i] = x[i];
                x[i] = x[i] + (4.0 / 3.0) * (invd[i] * r[i]);
            }
            continue;
        }
        const double a = 2.0 * (2 * j + 1), b = 4.0 * (2 * j + 1), c = (double)(2 * j - 1), d = (double)(2 * j + 3);
        for (int64_t i = 0; i < n; i++) xn[i] = (a * x[i] + b * (invd[i] * r[i]) - c * xp[i]) / d;
        for (int64_t i = 0; i < n; i++) { xp[i] = x[i]; x[i] = xn[i]; }
    }
    free(xp); free(r); free(xn);
}

int or_cg_jacobi(int64_t n, const int64_t *rp, const int32_t *ci, const double *v, const double *b,
                 double *x, double tol, int itmax)
{
    double *r = malloc(sizeof(double) * n), *z = malloc(sizeof(double) * n);
    double *p = malloc(sizeof(double) * n), *q = malloc(sizeof(double) * n);
    double *dj = malloc(sizeof(double) * n);
    for (int64_t i = 0; i < n; i++) {
        double kii = 0.0;
        for (int64_t e = rp[i]; e < rp[i + 1]; e++)
            if (ci[e] == i) kii = v[e];
        dj[i] = 1.0 / kii;
        x[i] = 0.0;
        r[i] = b[i];
    }
    int it = 0;
    const double nb = sqrt(or_dot(n, b, b));
    if (nb > 0.0) {
        for (int64_t i = 0; i < n; i++) { z[i] = dj[i] * r[i]; p[i] = z[i]; }
        double rz = or_dot(n, r, z);
        while (it < itmax) {
            or_spmv(n, rp, ci, v, p, q);
            double pq = or_dot(n, p, q);
            if (!(pq > 0.0)) break;
            double alpha = rz / pq;
            for (int64_t i = 0; i < n; i++) {
                x[i] = x[i] + alpha * p[i];
                r[i] = r[i] - alpha * q[i];
            }
            it++;
            if (sqrt(or_dot(n, r, r)) <= tol * nb) break;
            for (int64_t i = 0; i < n; i++) z[i] = dj[i] * r[i];
            double rzn = or_dot(n, r, z);
            double beta = rzn / rz;
            rz = rzn;
            for (int64_t i = 0; i < n; i++) p[i] = z[i] + beta * p[i];
        }
    }
    free(r); free(z); free(p); free(q); free(dj);
    return it;
}

static void coarsest_solve(const or_hier *h, const or_level *L, const double *f, double *u)
{
    if (h->prm.coarse_solver == 1)
        or_cg_jacobi(L->n, L->rp, L->ci, L->v, f, u, h->prm.coarse_tol, h->prm.coarse_itmax);
    else
        or_chol_solve((int)L->n, h->chol, f, u);
}

void or_vcycle(const or_hier *h, int l, const double *f, double *u)
{
    const or_level *L = &h->lev[l];
    int64_t n = L->n;
    if (l == h->nlev - 1) {
        coarsest_solve(h, L, f, u);
        return;
    }
    int poly = h->prm.smoother == 1, cheb = h->prm.smoother == 2;
    double *r = malloc(sizeof(double) * n), *c = malloc(sizeof(double) * n);
    double *tmp = malloc(sizeof(double) * n);
    /* 1. pre-smoothing from u = 0 */
    if (cheb) {
        for (int s = 0; s < h->prm.nu_pre; s++)
            or_cheb4(n, L->rp, L->ci, L->v, L->invd, f, u, s == 0, h->prm.cheb_degree);
        if (h->prm.nu_pre <= 0)
            for (int64_t i = 0; i < n; i++) u[i] = 0.0;
    } else if (h->prm.nu_pre > 0) {
        smoother_apply(L, poly, f, u, tmp);
        for (int s = 1; s < h->prm.nu_pre; s++) sweep(L, poly, f, u, r, c, tmp);
    } else {
        for (int64_t i = 0; i < n; i++) u[i] = 0.0;
    }
    /* 2. restrict the residual */
    or_spmv(n, L->rp, L->ci, L->v, u, r);
    for (int64_t i = 0; i < n; i++) r[i] = f[i] - r[i];
    int64_t nc = h->lev[l + 1].n;
    double *fc = calloc(nc, sizeof(double)), *ec = malloc(sizeof(double) * nc);
    if (L->prp) {
        for (int64_t i = 0; i < n; i++)
            for (int64_t e = L->prp[i]; e < L->prp[i + 1]; e++)
                fc[L->pci[e]] = fc[L->pci[e]] + L->pv[e] * r[i];
    } else {
        for (int64_t i = 0; i < n; i++) fc[L->agg[i]] = fc[L->agg[i]] + L->pc[i] * r[i];
    }
    /* 3. coarse solve */
    or_vcycle(h, l + 1, fc, ec);
    /* 4. prolongate and correct */
    if (L->prp) {
        for (int64_t i = 0; i < n; i++) {
            double s = 0.0;
            for (int64_t e = L->prp[i]; e < L->prp[i + 1]; e++) s = s + L->pv[e] * ec[L->pci[e]];
            u[i] = u[i] + s;
        }
    } else {
        for (int64_t i = 0; i < n; i++) u[i] = u[i] + L->pc[i] * ec[L->agg[i]];
    }
    /* 5. post-smoothing */
    for (int s = 0; s < h->prm.nu_post; s++) {
        if (cheb) or_cheb4(n, L->rp, L->ci, L->v, L->invd, f, u, 0, h->prm.cheb_degree);
        else sweep(L, poly, f, u, r, c, tmp);
    }
    free(r); free(c); free(tmp); free(fc); free(ec);
}

int or_pcg(const or_hier *h, const double *F, double *u, double tol, int itmax,
           int flexible, int *iters, double *relres, double *hist)
{
    const or_level *L = &h->lev[0];
    int64_t n = L->n;
    *iters = 0;
    double nF = sqrt(or_dot(n, F, F));
    if (nF == 0.0) {
        for (int64_t i = 0; i < n; i++) u[i] = 0.0;
        *relres = 0.0;
        if (hist) hist[0] = 0.0;
        return 0;
    }
    double *r = malloc(sizeof(double) * n), *z = malloc(sizeof(double) * n);
    double *p = malloc(sizeof(double) * n), *q = malloc(sizeof(double) * n);
    or_spmv(n, L->rp, L->ci, L->v, u, r);
    for (int64_t i = 0; i < n; i++) r[i] = F[i] - r[i];
    double rr = or_dot(n, r, r);
    if (hist) hist[0] = sqrt(rr) / nF;
    int rc = 1;
    if (sqrt(rr) <= tol * nF) { rc = 0; goto done; }
    or_vcycle(h, 0, r, z);
    double rz = or_dot(n, r, z);
    if (!(rz > 0.0) || !isfinite(rz)) { rc = -5; goto done; }
    for (int64_t i = 0; i < n; i++) p[i] = z[i];
    for (int k = 1; k <= itmax; k++) {
        or_spmv(n, L->rp, L->ci, L->v, p, q);
        double pq = or_dot(n, p, q);
        if (!(pq > 0.0) || !isfinite(pq)) { rc = -5; break; }
        double alpha = flexible ? or_dot(n, p, r) / pq : rz / pq;
        for (int64_t i = 0; i < n; i++) {
            u[i] = u[i] + alpha * p[i];
            r[i] = r[i] - alpha * q[i];
        }
        rr = or_dot(n, r, r);
        *iters = k;
        if (hist) hist[k] = sqrt(rr) / nF;
        if (sqrt(rr) <= tol * nF) { rc = 0; break; }
        if (k == itmax) break;
        or_vcycle(h, 0, r, z);
        double beta;
        if (flexible) {
            beta = -or_dot(n, z, q) / pq;
        } else {
            double rzn = or_dot(n, r, z);
            if (!(rzn > 0.0) || !isfinite(rzn)) { rc = -5; break; }
            beta = rzn / rz;
            rz = rzn;
        }
        for (int64_t i = 0; i < n; i++) p[i] = z[i] + beta * p[i];
    }
done:
    *relres = sqrt(rr) / nF;
    free(r); free(z); free(p); free(q);
    return rc;
}

/* Acceptance of a degree-4 polynomial smoother: with e(t) = 1 - sum a_k t^{k+1},
 * require |e(t)| <= 1 on [0,1] and e(t) < 1 for t > 0, on 10^4 equal steps and
 * the end points.  Then p(t) = (1 - e(t))/t > 0 on (0,1], so the smoother
 * p(D^{-1}K) D^{-1} is SPD and non-expansive in the energy norm. */
int or_poly_accept(const double *a)
{
    for (int s = 0; s <= 10000; s++) {
        double t = s / 10000.0;
        double pt = ((a[3] * t + a[2]) * t + a[1]) * t + a[0];
        double e = 1.0 - t * pt;
        if (!isfinite(e) || fabs(e) > 1.0) return 0;
        if (s > 0 && !(e < 1.0)) return 0;
    }
    return 1;
}

int or_set_poly(or_hier *h, int l, const double *coef)
{
    if (l < 0 || l >= h->nlev) return -1;
    if (!or_poly_accept(coef)) return 1;
    for (int k = 0; k < 4; k++) h->lev[l].poly[k] = coef[k];
    return 0;
}

/* Cholesky of the s x s SPD block G (row-major, leading dimension ld) into L;
 * returns -1 on a non-positive pivot. */
static int small_chol(int s, const double *G, int ld, double *L)
{
    for (int i = 0; i < s; i++)
        for (int j = 0; j <= i; j++) {
            double t = G[i * ld + j];
            for (int k = 0; k < j; k++) t -= L[i * s + k] * L[j * s + k];
            if (i == j) {
                if (!(t > 0.0) || !isfinite(t)) return -1;
                L[i * s + i] = sqrt(t);
            } else {
                L[i * s + j] = t / L[j * s + j];
            }
        }
    return 0;
}

/* Y = G^{-1} B for the s x m right side B (row-major s x m), with L from small_chol. */
static void small_solve(int s, const double *L, int m, double *B)
{
    for (int c = 0; c < m; c++) {
        for (int i = 0; i < s; i++) {
            double t = B[i * m + c];
            for (int k = 0; k < i; k++) t -= L[i * s + k] * B[k * m + c];
            B[i * m + c] = t / L[i * s + i];
        }
        for (int i = s - 1; i >= 0; i--) {
            double t = B[i * m + c];
            for (int k = i + 1; k < s; k++) t -= L[k * s + i] * B[k * m + c];
            B[i * m + c] = t / L[i * s + i];
        }
    }
}

int or_block_fcg(const or_hier *h, int s, const double *F, double *U, double tol, int itmax, int *iters,
                 double *relres)
{
    const or_level *L0 = &h->lev[0];
    const int64_t n = L0->n;
    double *R = malloc(sizeof(double) * n * s), *Z = malloc(sizeof(double) * n * s);
    double *P = malloc(sizeof(double) * n * s), *Q = malloc(sizeof(double) * n * s);
    double *G = malloc(sizeof(double) * s * s), *Lc = malloc(sizeof(double) * s * s);
    double *A = malloc(sizeof(double) * s * s), *nf = malloc(sizeof(double) * s), *rr = malloc(sizeof(double) * s);
    int *act = malloc(sizeof(int) * s), *idx = malloc(sizeof(int) * s);
    int rc = 1;
    for (int j = 0; j < s; j++) {
        const double *f = F + (int64_t)j * n;
        double *r = R + (int64_t)j * n;
        or_spmv(n, L0->rp, L0->ci, L0->v, U + (int64_t)j * n, r);
        for (int64_t i = 0; i < n; i++) r[i] = f[i] - r[i];
        nf[j] = sqrt(or_dot(n, f, f));
        rr[j] = or_dot(n, r, r);
        iters[j] = 0;
        act[j] = !(nf[j] == 0.0 || sqrt(rr[j]) <= tol * nf[j]);
    }
    int na = 0;
    for (int j = 0; j < s; j++) na += act[j];
    if (na == 0) { rc = 0; goto done; }
    for (int j = 0; j < s; j++)
        if (act[j]) {
            or_vcycle(h, 0, R + (int64_t)j * n, Z + (int64_t)j * n);
            memcpy(P + (int64_t)j * n, Z + (int64_t)j * n, sizeof(double) * n);
        }
    for (int k = 1; k <= itmax; k++) {
        int m = 0;
        for (int j = 0; j < s; j++) if (act[j]) idx[m++] = j;
        for (int a = 0; a < m; a++)
            or_spmv(n, L0->rp, L0->ci, L0->v, P + (int64_t)idx[a] * n, Q + (int64_t)idx[a] * n);
        /* G = P^T Q and A = P^T R over the active columns */
        for (int a = 0; a < m; a++)
            for (int b = 0; b < m; b++) {
                G[a * m + b] = or_dot(n, P + (int64_t)idx[a] * n, Q + (int64_t)idx[b] * n);
                A[a * m + b] = or_dot(n, P + (int64_t)idx[a] * n, R + (int64_t)idx[b] * n);
            }
        if (small_chol(m, G, m, Lc)) { rc = -5; goto done; }
        small_solve(m, Lc, m, A);            /* alpha = G^{-1} P^T R */
        for (int b = 0; b < m; b++) {
            double *x = U + (int64_t)idx[b] * n, *r = R + (int64_t)idx[b] * n;
            for (int64_t i = 0; i < n; i++) {
                double dx = 0.0, dr = 0.0;
                for (int a = 0; a < m; a++) {
                    dx = dx + P[(int64_t)idx[a] * n + i] * A[a * m + b];
                    dr = dr + Q[(int64_t)idx[a] * n + i] * A[a * m + b];
                }
                x[i] = x[i] + dx;
                r[i] = r[i] - dr;
            }
            const int j = idx[b];
            rr[j] = or_dot(n, r, r);
            iters[j] = k;
            if (sqrt(rr[j]) <= tol * nf[j]) act[j] = 0;
        }
        na = 0;
        for (int j = 0; j < s; j++) na += act[j];
        if (na == 0) { rc = 0; break; }
        if (k == itmax) break;
        /* beta over the columns still active: -G'^{-1} Q'^T Z' */
        int m2 = 0;
        int *pos = malloc(sizeof(int) * m);
        for (int a = 0; a < m; a++) if (act[idx[a]]) pos[m2++] = a;
        for (int a = 0; a < m2; a++)
            or_vcycle(h, 0, R + (int64_t)idx[pos[a]] * n, Z + (int64_t)idx[pos[a]] * n);
        double *G2 = malloc(sizeof(double) * m2 * m2), *B = malloc(sizeof(double) * m2 * m2);
        for (int a = 0; a < m2; a++)
            for (int b = 0; b < m2; b++) {
                G2[a * m2 + b] = G[pos[a] * m + pos[b]];
                B[a * m2 + b] = -or_dot(n, Q + (int64_t)idx[pos[a]] * n, Z + (int64_t)idx[pos[b]] * n);
            }
        if (small_chol(m2, G2, m2, Lc)) { free(pos); free(G2); free(B); rc = -5; goto done; }
        small_solve(m2, Lc, m2, B);
        /* P_j = Z_j + sum_a P_a beta_aj, written after all reads of the old P */
        double *Pn = malloc(sizeof(double) * n * m2);
        for (int b = 0; b < m2; b++)
            for (int64_t i = 0; i < n; i++) {
                double t = 0.0;
                for (int a = 0; a < m2; a++) t = t + P[(int64_t)idx[pos[a]] * n + i] * B[a * m2 + b];
                Pn[(int64_t)b * n + i] = Z[(int64_t)idx[pos[b]] * n + i] + t;
            }
        for (int b = 0; b < m2; b++) memcpy(P + (int64_t)idx[pos[b]] * n, Pn + (int64_t)b * n, sizeof(double) * n);
        free(Pn); free(pos); free(G2); free(B);
    }
done:
    for (int j = 0; j < s; j++) relres[j] = nf[j] > 0.0 ? sqrt(rr[j]) / nf[j] : 0.0;
    free(R); free(Z); free(P); free(Q); free(G); free(Lc); free(A); free(nf); free(rr); free(act); free(idx);
    return rc;
}
