/*
 * Oracle, part 2: the AMG hierarchy by compatible weighted matching (paper
 * Sec. 3 and 3.1: eq. (galerkin_matrix_projection), eq. (cij), eq. (maxprod),
 * eq. (prolongation), the m-step composition P = P1 P2 ... Pm, the l1-Jacobi
 * diagonal of Sec. 3.2).  TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * Readings where the paper is silent or ambiguous:
 *  - edges are the stored off-diagonal entries with k_ij != 0; for i < j the
 *    value stored in row i is used (coarse matrices are symmetric only up to
 *    rounding);
 *  - c_ij evaluation order: num = ((2 k_ij) w_i) w_j,
 *    den = (k_ii w_i) w_i + (k_jj w_j) w_j, c = 1 - num/den, no FMA;
 *  - "maximum product matching computed by a greedy algorithm on log c":
 *    greedy over every eligible edge (finite c) in the strict order c
 *    descending, then min(i,j) ascending, then max(i,j) ascending; an edge is
 *    taken iff both endpoints are free.  With positive_only, only edges with
 *    c > 1 (log c > 0) are eligible;
 *  - coarse numbering: scan i ascending, a free row opens the next coarse index
 *    and its partner joins it;  singleton with w_s = 0 gets coefficient 1;
 *  - the restricted test vector is w_c = ||(w_i, w_j)||_2 for a pair and |w_s|
 *    for a singleton (equal to P^T w in exact arithmetic);
 *  - Galerkin summation order: coarse row I, members ascending, each member's
 *    entries ascending, acc[agg(j)] += (pc_i k_ij) pc_j from +0.0; exact zeros
 *    are kept as stored entries;
 *  - one level = m pairwise sweeps (m = 2: aggregates of at most 4); the
 *    hierarchy stops when a level has at most max_coarse rows (dense Cholesky
 *    there); if a level shrinks by less than 10% the previous level becomes the
 *    coarsest when it has at most 2000 rows, otherwise the setup fails;
 *  - l1 diagonal: d_i = k_ii, then + |k_ij| for j ascending, j != i;
 *  - smoothed prolongator (Sec. 3.1, "Variants and efficiency"), on request:
 *    P' = (I - omega D^{-1} K) P with the tentative P of the m composed sweeps,
 *    D the l1 diagonal (the paper's only D; lambda(D^{-1}K) <= 1, so
 *    omega = 4/3 needs no spectral estimate).  Entry by entry:
 *    T_iJ = sum over row i's stored j with agg(j) = J, ascending j, of k_ij pc_j
 *    from +0.0; P'_iJ = [J = agg(i)] pc_i - (omega invd_i) T_iJ on the pattern
 *    of T (exact zeros kept).  The coarse matrix is then (P'^T K) P':
 *    B_Ij = sum over i ascending of P'_iI k_ij, then
 *    K_c,IJ = sum over j ascending of B_Ij P'_jJ, each from +0.0; the
 *    unsmoothed product of the last sweep is not used.  The test vector of the
 *    next level is still the pairwise restriction.
 */
#include "oracle.h"
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

static int verbose = 0;
void or_set_verbose(int v) { verbose = v; }

void or_params_default(or_params *p)
{
    p->sweeps_per_level = 2;
    p->max_coarse = 200;
    p->max_levels = 40;
    p->nu_pre = 1;
    p->nu_post = 1;
    p->match_positive_only = 0;
    p->smoother = 0;
    p->smooth_prolong = 0;
    p->cheb_degree = 8;
    p->coarse_solver = 0;
    p->coarse_itmax = 30;
    p->omega = 4.0 / 3.0;
    p->coarse_tol = 1e-4;
}

double or_cij(double kij, double kii, double kjj, double wi, double wj)
{
    double num = ((2.0 * kij) * wi) * wj;
    double den = (kii * wi) * wi + (kjj * wj) * wj;
    return 1.0 - num / den;
}

typedef struct { double c; int32_t i, j; } edge_t;

/* strict total order: larger c first, then smaller i, then smaller j */
static int edge_cmp(const void *pa, const void *pb)
{
    const edge_t *a = pa, *b = pb;
    if (a->c > b->c) return -1;
    if (a->c < b->c) return 1;
    if (a->i != b->i) return a->i < b->i ? -1 : 1;
    if (a->j != b->j) return a->j < b->j ? -1 : 1;
    return 0;
}

static double *diag_of(int64_t n, const int64_t *rp, const int32_t *ci, const double *v)
{
    double *d = malloc(sizeof(double) * n);
    for (int64_t i = 0; i < n; i++) {
        d[i] = 0.0;
        for (int64_t e = rp[i]; e < rp[i + 1]; e++)
            if (ci[e] == i) d[i] = v[e];
    }
    return d;
}

static int eligible(double c, int positive_only)
{
    if (!isfinite(c)) return 0;
    if (positive_only && !(c > 1.0)) return 0;
    return 1;
}

static void greedy_scan(int64_t n, edge_t *E, int64_t k, int32_t *mate)
{
    qsort(E, k, sizeof(edge_t), edge_cmp);
    for (int64_t i = 0; i < n; i++) mate[i] = -1;
    for (int64_t e = 0; e < k; e++)
        if (mate[E[e].i] < 0 && mate[E[e].j] < 0) {
            mate[E[e].i] = E[e].j;
            mate[E[e].j] = E[e].i;
        }
}

int or_greedy_edges(int64_t n, int64_t ne, const double *c, const int32_t *ei,
                    const int32_t *ej, int positive_only, int32_t *mate)
{
    edge_t *E = malloc(sizeof(edge_t) * (ne > 0 ? ne : 1));
    int64_t k = 0;
    for (int64_t e = 0; e < ne; e++) {
        if (!eligible(c[e], positive_only)) continue;
        E[k].c = c[e]; E[k].i = ei[e] < ej[e] ? ei[e] : ej[e]; E[k].j = ei[e] < ej[e] ? ej[e] : ei[e];
        k++;
    }
    greedy_scan(n, E, k, mate);
    free(E);
    return 0;
}

int or_match(int64_t n, const int64_t *rp, const int32_t *ci, const double *v,
             const double *w, int positive_only, int32_t *mate)
{
    double *d = diag_of(n, rp, ci, v);
    int64_t ne = 0;
    for (int64_t i = 0; i < n; i++)
        for (int64_t e = rp[i]; e < rp[i + 1]; e++)
            if (ci[e] > i && v[e] != 0.0) ne++;
    edge_t *E = malloc(sizeof(edge_t) * (ne > 0 ? ne : 1));
    int64_t k = 0;
    for (int64_t i = 0; i < n; i++)
        for (int64_t e = rp[i]; e < rp[i + 1]; e++) {
            int64_t j = ci[e];
            if (j <= i || v[e] == 0.0) continue;
            double c = or_cij(v[e], d[i], d[j], w[i], w[j]);
            if (!eligible(c, positive_only)) continue;
            E[k].c = c; E[k].i = (int32_t)i; E[k].j = (int32_t)j;
            k++;
        }
    greedy_scan(n, E, k, mate);
    free(E);
    free(d);
    return 0;
}

/* a precedes b in the matching order */
static int precedes(double ca, int64_t ia, int64_t ja, double cb, int64_t ib, int64_t jb)
{
    if (ca != cb) return ca > cb;
    if (ia != ib) return ia < ib;
    return ja < jb;
}

int64_t or_check_greedy(int64_t n, const int64_t *rp, const int32_t *ci, const double *v,
                        const double *w, int positive_only, const int32_t *mate)
{
    double *d = diag_of(n, rp, ci, v);
    /* c of each vertex's matched edge (NaN when unmatched or not an edge) */
    double *cm = malloc(sizeof(double) * n);
    int64_t bad = 0;
    for (int64_t i = 0; i < n; i++) {
        cm[i] = NAN;
        int64_t j = mate[i];
        if (j < 0) continue;
        if (j >= n || mate[j] != i || j == i) { bad++; continue; }
        int64_t a = i < j ? i : j, b = i < j ? j : i;
        int found = 0;
        for (int64_t e = rp[a]; e < rp[a + 1]; e++)
            if (ci[e] == b && v[e] != 0.0) {
                double c = or_cij(v[e], d[a], d[b], w[a], w[b]);
                if (eligible(c, positive_only)) { cm[i] = c; found = 1; }
            }
        if (!found) bad++;
    }
    for (int64_t i = 0; i < n; i++)
        for (int64_t e = rp[i]; e < rp[i + 1]; e++) {
            int64_t j = ci[e];
            if (j <= i || v[e] == 0.0) continue;
            if (mate[i] == j) continue;
            double c = or_cij(v[e], d[i], d[j], w[i], w[j]);
            if (!eligible(c, positive_only)) continue;
            int blocked = 0;
            int64_t ends[2] = {i, j};
            for (int s = 0; s < 2; s++) {
                int64_t u = ends[s], x = mate[u];
                if (x < 0 || isnan(cm[u])) continue;
                int64_t a = u < x ? u : x, b = u < x ? x : u;
                if (precedes(cm[u], a, b, c, i, j)) blocked = 1;
            }
            if (!blocked) bad++;
        }
    free(cm);
    free(d);
    return bad;
}

int64_t or_pairwise_p(int64_t n, const int32_t *mate, const double *w,
                      int32_t *agg, double *pc, double *wc)
{
    int64_t nc = 0;
    for (int64_t i = 0; i < n; i++) agg[i] = -1;
    for (int64_t i = 0; i < n; i++) {
        if (agg[i] >= 0) continue;
        agg[i] = (int32_t)nc;
        if (mate[i] >= 0) agg[mate[i]] = (int32_t)nc;
        nc++;
    }
    for (int64_t i = 0; i < n; i++) {
        int64_t j = mate[i];
        if (j >= 0) {
            double s = sqrt(w[i] * w[i] + w[j] * w[j]);
            pc[i] = w[i] / s;
            wc[agg[i]] = s;
        } else {
            pc[i] = (w[i] != 0.0) ? w[i] / fabs(w[i]) : 1.0;
            wc[agg[i]] = fabs(w[i]);
        }
    }
    return nc;
}

typedef struct { int64_t n, nnz; int64_t *rp; int32_t *ci; double *v; } csr_t;

static int cmp_i32(const void *a, const void *b)
{
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/* K_c = P^T K P for P with one entry per row: column agg[i] holds pc[i]. */
static csr_t galerkin(const csr_t *K, int64_t nc, const int32_t *agg, const double *pc)
{
    csr_t C;
    C.n = nc;
    /* members of each coarse row, ascending */
    int64_t *mp = calloc(nc + 1, sizeof(int64_t));
    int64_t *mem = malloc(sizeof(int64_t) * K->n);
    for (int64_t i = 0; i < K->n; i++) mp[agg[i] + 1]++;
    for (int64_t I = 0; I < nc; I++) mp[I + 1] += mp[I];
    int64_t *fill = malloc(sizeof(int64_t) * nc);
    for (int64_t I = 0; I < nc; I++) fill[I] = mp[I];
    for (int64_t i = 0; i < K->n; i++) mem[fill[agg[i]]++] = i;
    free(fill);

    double *acc = malloc(sizeof(double) * nc);
    char *mark = calloc(nc, 1);
    int32_t *touched = malloc(sizeof(int32_t) * nc);
    int64_t cap = K->nnz > 16 ? K->nnz : 16;
    C.rp = malloc(sizeof(int64_t) * (nc + 1));
    C.ci = malloc(sizeof(int32_t) * cap);
    C.v = malloc(sizeof(double) * cap);
    C.rp[0] = 0;
    int64_t pos = 0;
    for (int64_t I = 0; I < nc; I++) {
        int64_t nt = 0;
        for (int64_t m = mp[I]; m < mp[I + 1]; m++) {
            int64_t i = mem[m];
            for (int64_t e = K->rp[i]; e < K->rp[i + 1]; e++) {
                int64_t j = K->ci[e];
                int32_t J = agg[j];
                double t = (pc[i] * K->v[e]) * pc[j];
                if (!mark[J]) { mark[J] = 1; acc[J] = 0.0; touched[nt++] = J; }
                acc[J] = acc[J] + t;
            }
        }
        qsort(touched, nt, sizeof(int32_t), cmp_i32);
        if (pos + nt > cap) {
            while (pos + nt > cap) cap *= 2;
            C.ci = realloc(C.ci, sizeof(int32_t) * cap);
            C.v = realloc(C.v, sizeof(double) * cap);
        }
        for (int64_t k = 0; k < nt; k++) {
            C.ci[pos] = touched[k];
            C.v[pos] = acc[touched[k]];
            mark[touched[k]] = 0;
            pos++;
        }
        C.rp[I + 1] = pos;
    }
    C.nnz = pos;
    free(acc); free(mark); free(touched); free(mp); free(mem);
    return C;
}

/* P' = (I - omega D^{-1} K) P for the one-entry-per-row tentative P. */
static csr_t smooth_p(const csr_t *K, const double *invd, int64_t nc, const int32_t *agg, const double *pc,
                      double omega)
{
    csr_t P;
    P.n = K->n;
    P.rp = malloc(sizeof(int64_t) * (K->n + 1));
    P.ci = malloc(sizeof(int32_t) * (K->nnz > 0 ? K->nnz : 1));
    P.v = malloc(sizeof(double) * (K->nnz > 0 ? K->nnz : 1));
    double *acc = malloc(sizeof(double) * nc);
    char *mark = calloc(nc, 1);
    int32_t *cols = malloc(sizeof(int32_t) * (nc > 0 ? nc : 1));
    int64_t pos = 0;
    P.rp[0] = 0;
    for (int64_t i = 0; i < K->n; i++) {
        int64_t nt = 0;
        for (int64_t e = K->rp[i]; e < K->rp[i + 1]; e++) {
            int32_t J = agg[K->ci[e]];
            if (!mark[J]) { mark[J] = 1; acc[J] = 0.0; cols[nt++] = J; }
            acc[J] = acc[J] + K->v[e] * pc[K->ci[e]];
        }
        qsort(cols, nt, sizeof(int32_t), cmp_i32);
        const double s = omega * invd[i];
        for (int64_t k = 0; k < nt; k++) {
            int32_t J = cols[k];
            double tent = (J == agg[i]) ? pc[i] : 0.0;
            P.ci[pos] = J;
            P.v[pos] = tent - s * acc[J];
            mark[J] = 0;
            pos++;
        }
        P.rp[i + 1] = pos;
    }
    P.nnz = pos;
    free(acc); free(mark); free(cols);
    return P;
}

/* K_c = (P^T K) P for a general sparse P (n x nc). */
static csr_t galerkin_general(const csr_t *K, const csr_t *P, int64_t nc)
{
    const int64_t n = K->n;
    /* columns of P: for coarse J the rows i (ascending) with their values */
    int64_t *tp = calloc(nc + 1, sizeof(int64_t));
    for (int64_t e = 0; e < P->nnz; e++) tp[P->ci[e] + 1]++;
    for (int64_t J = 0; J < nc; J++) tp[J + 1] += tp[J];
    int64_t *ti = malloc(sizeof(int64_t) * (P->nnz > 0 ? P->nnz : 1));
    double *tv = malloc(sizeof(double) * (P->nnz > 0 ? P->nnz : 1));
    int64_t *fill = malloc(sizeof(int64_t) * (nc > 0 ? nc : 1));
    for (int64_t J = 0; J < nc; J++) fill[J] = tp[J];
    for (int64_t i = 0; i < n; i++)
        for (int64_t e = P->rp[i]; e < P->rp[i + 1]; e++) {
            int64_t q = fill[P->ci[e]]++;
            ti[q] = i;
            tv[q] = P->v[e];
        }
    free(fill);
    double *accB = malloc(sizeof(double) * n), *accC = malloc(sizeof(double) * nc);
    char *markB = calloc(n, 1), *markC = calloc(nc, 1);
    int32_t *colB = malloc(sizeof(int32_t) * n), *colC = malloc(sizeof(int32_t) * (nc > 0 ? nc : 1));
    csr_t C;
    C.n = nc;
    int64_t cap = K->nnz > 16 ? K->nnz : 16;
    C.rp = malloc(sizeof(int64_t) * (nc + 1));
    C.ci = malloc(sizeof(int32_t) * cap);
    C.v = malloc(sizeof(double) * cap);
    C.rp[0] = 0;
    int64_t pos = 0;
    for (int64_t I = 0; I < nc; I++) {
        /* B_I = sum_i P_iI K_i, i ascending */
        int64_t nb = 0;
        for (int64_t q = tp[I]; q < tp[I + 1]; q++) {
            int64_t i = ti[q];
            for (int64_t e = K->rp[i]; e < K->rp[i + 1]; e++) {
                int32_t j = K->ci[e];
                if (!markB[j]) { markB[j] = 1; accB[j] = 0.0; colB[nb++] = j; }
                accB[j] = accB[j] + tv[q] * K->v[e];
            }
        }
        qsort(colB, nb, sizeof(int32_t), cmp_i32);
        /* C_I = sum_j B_Ij P_j, j ascending */
        int64_t ncol = 0;
        for (int64_t k = 0; k < nb; k++) {
            int32_t j = colB[k];
            for (int64_t e = P->rp[j]; e < P->rp[j + 1]; e++) {
                int32_t J = P->ci[e];
                if (!markC[J]) { markC[J] = 1; accC[J] = 0.0; colC[ncol++] = J; }
                accC[J] = accC[J] + accB[j] * P->v[e];
            }
            markB[j] = 0;
        }
        qsort(colC, ncol, sizeof(int32_t), cmp_i32);
        if (pos + ncol > cap) {
            while (pos + ncol > cap) cap *= 2;
            C.ci = realloc(C.ci, sizeof(int32_t) * cap);
            C.v = realloc(C.v, sizeof(double) * cap);
        }
        for (int64_t k = 0; k < ncol; k++) {
            C.ci[pos] = colC[k];
            C.v[pos] = accC[colC[k]];
            markC[colC[k]] = 0;
            pos++;
        }
        C.rp[I + 1] = pos;
    }
    C.nnz = pos;
    free(tp); free(ti); free(tv); free(accB); free(accC); free(markB); free(markC); free(colB); free(colC);
    return C;
}

void or_l1_invdiag(int64_t n, const int64_t *rp, const int32_t *ci, const double *v, double *invd)
{
    for (int64_t i = 0; i < n; i++) {
        double d = 0.0;
        for (int64_t e = rp[i]; e < rp[i + 1]; e++)
            if (ci[e] == i) d = v[e];
        for (int64_t e = rp[i]; e < rp[i + 1]; e++)
            if (ci[e] != i) d = d + fabs(v[e]);
        invd[i] = 1.0 / d;
    }
}

/* Cholesky-Banachiewicz on the lower triangle of a (row-major n x n); the
 * strict upper triangle is zeroed so a holds L on return. */
int or_cholesky(int n, double *a)
{
    for (int i = 0; i < n; i++) {
        for (int j = 0; j <= i; j++) {
            double s = a[(int64_t)i * n + j];
            for (int k = 0; k < j; k++) s -= a[(int64_t)i * n + k] * a[(int64_t)j * n + k];
            if (i == j) {
                if (!(s > 0.0)) return -2;
                a[(int64_t)i * n + i] = sqrt(s);
            } else {
                a[(int64_t)i * n + j] = s / a[(int64_t)j * n + j];
            }
        }
        for (int j = i + 1; j < n; j++) a[(int64_t)i * n + j] = 0.0;
    }
    return 0;
}

void or_chol_solve(int n, const double *L, const double *b, double *x)
{
    double *y = malloc(sizeof(double) * (n > 0 ? n : 1));
    for (int i = 0; i < n; i++) {
        double s = b[i];
        for (int k = 0; k < i; k++) s -= L[(int64_t)i * n + k] * y[k];
        y[i] = s / L[(int64_t)i * n + i];
    }
    for (int i = n - 1; i >= 0; i--) {
        double s = y[i];
        for (int k = i + 1; k < n; k++) s -= L[(int64_t)k * n + i] * x[k];
        x[i] = s / L[(int64_t)i * n + i];
    }
    free(y);
}

static int validate(int64_t n, const int64_t *rp, const int32_t *ci, const double *v)
{
    if (n <= 0 || n > 2147483647LL || rp[0] != 0) return -1;
    for (int64_t i = 0; i < n; i++) {
        if (rp[i + 1] < rp[i]) return -1;
        int has_diag = 0;
        for (int64_t e = rp[i]; e < rp[i + 1]; e++) {
            if (ci[e] < 0 || ci[e] >= n) return -1;
            if (e > rp[i] && ci[e] <= ci[e - 1]) return -1;
            if (!isfinite(v[e])) return -1;
            if (ci[e] == i) { has_diag = 1; if (!(v[e] > 0.0)) return -1; }
        }
        if (!has_diag) return -1;
    }
    return 0;
}

static void level_from(or_level *L, csr_t K, double *w)
{
    memset(L, 0, sizeof(*L));
    L->n = K.n; L->nnz = K.nnz; L->rp = K.rp; L->ci = K.ci; L->v = K.v; L->w = w;
    L->poly[0] = 1.0;   /* the polynomial (1,0,0,0) is plain l1-Jacobi */
    L->invd = malloc(sizeof(double) * K.n);
    or_l1_invdiag(K.n, K.rp, K.ci, K.v, L->invd);
}

static int factor_level(or_hier *h, int l)
{
    or_level *L = &h->lev[l];
    int nl = (int)L->n;
    if (h->prm.coarse_solver == 1) { h->nlev = l + 1; return 0; }
    h->chol = calloc((size_t)nl * nl, sizeof(double));
    for (int i = 0; i < nl; i++)
        for (int64_t e = L->rp[i]; e < L->rp[i + 1]; e++)
            if (L->ci[e] <= i) h->chol[(int64_t)i * nl + L->ci[e]] = L->v[e];
    h->nlev = l + 1;
    return or_cholesky(nl, h->chol);
}

int or_setup(int64_t n, const int64_t *rp, const int32_t *ci, const double *v,
             const double *w, const or_params *prm, or_hier **out)
{
    *out = NULL;
    if (validate(n, rp, ci, v)) return -1;
    or_hier *h = calloc(1, sizeof(or_hier));
    if (prm) h->prm = *prm; else or_params_default(&h->prm);
    int maxl = h->prm.max_levels > 0 ? h->prm.max_levels : 1;
    h->lev = calloc(maxl, sizeof(or_level));
    csr_t K;
    K.n = n; K.nnz = rp[n];
    K.rp = malloc(sizeof(int64_t) * (n + 1)); memcpy(K.rp, rp, sizeof(int64_t) * (n + 1));
    K.ci = malloc(sizeof(int32_t) * K.nnz); memcpy(K.ci, ci, sizeof(int32_t) * K.nnz);
    K.v = malloc(sizeof(double) * K.nnz); memcpy(K.v, v, sizeof(double) * K.nnz);
    double *w0 = malloc(sizeof(double) * n);
    for (int64_t i = 0; i < n; i++) w0[i] = w ? w[i] : 1.0;
    level_from(&h->lev[0], K, w0);
    int rc = 0;
    for (int l = 0;; l++) {
        or_level *L = &h->lev[l];
        if (L->n <= h->prm.max_coarse) { rc = factor_level(h, l); break; }
        if (l == maxl - 1) {
            if (L->n <= 2000) rc = factor_level(h, l); else { h->nlev = l + 1; rc = -6; }
            break;
        }
        /* m pairwise sweeps, composed */
        csr_t cur = { L->n, L->nnz, L->rp, L->ci, L->v };
        double *cw = L->w;
        int32_t *agg = malloc(sizeof(int32_t) * L->n);
        double *pc = malloc(sizeof(double) * L->n);
        int64_t nc = L->n;
        for (int s = 0; s < h->prm.sweeps_per_level; s++) {
            int32_t *mate = malloc(sizeof(int32_t) * cur.n);
            int32_t *ag = malloc(sizeof(int32_t) * cur.n);
            double *pcs = malloc(sizeof(double) * cur.n);
            double *wc = malloc(sizeof(double) * cur.n);
            or_match(cur.n, cur.rp, cur.ci, cur.v, cw, h->prm.match_positive_only, mate);
            nc = or_pairwise_p(cur.n, mate, cw, ag, pcs, wc);
            csr_t C = galerkin(&cur, nc, ag, pcs);
            if (s == 0) {
                for (int64_t i = 0; i < L->n; i++) { agg[i] = ag[i]; pc[i] = pcs[i]; }
            } else {
                for (int64_t i = 0; i < L->n; i++) {
                    pc[i] = pc[i] * pcs[agg[i]];
                    agg[i] = ag[agg[i]];
                }
                free(cur.rp); free(cur.ci); free(cur.v); free(cw);
            }
            cur = C;
            cw = wc;
            free(mate); free(ag); free(pcs);
        }
        if ((double)nc > 0.9 * (double)L->n) {
            free(cur.rp); free(cur.ci); free(cur.v); free(cw); free(agg); free(pc);
            if (L->n <= 2000) rc = factor_level(h, l); else { h->nlev = l + 1; rc = -6; }
            break;
        }
        L->agg = agg;
        L->pc = pc;
        if (h->prm.smooth_prolong) {
            csr_t Kl = { L->n, L->nnz, L->rp, L->ci, L->v };
            csr_t P = smooth_p(&Kl, L->invd, nc, agg, pc, h->prm.omega);
            free(cur.rp); free(cur.ci); free(cur.v);
            cur = galerkin_general(&Kl, &P, nc);
            L->prp = P.rp; L->pci = P.ci; L->pv = P.v; L->pnnz = P.nnz;
        }
        level_from(&h->lev[l + 1], cur, cw);
        if (verbose) {
            fprintf(stderr, "oracle setup: level %d done: n=%lld nnz=%lld\n", l + 1, (long long)cur.n,
                    (long long)cur.nnz);
            fflush(stderr);
        }
    }
    *out = h;
    return rc;
}

void or_free(or_hier *h)
{
    if (!h) return;
    int maxl = h->prm.max_levels > 0 ? h->prm.max_levels : 1;
    for (int l = 0; l < maxl; l++) {
        or_level *L = &h->lev[l];
        free(L->rp); free(L->ci); free(L->v); free(L->invd); free(L->w);
        free(L->agg); free(L->pc);
        free(L->prp); free(L->pci); free(L->pv);
    }
    free(h->lev);
    free(h->chol);
    free(h);
}

int or_nlevels(const or_hier *h) { return h->nlev; }

void or_level_info(const or_hier *h, int l, int64_t *n, int64_t *nnz)
{
    *n = h->lev[l].n;
    *nnz = h->lev[l].nnz;
}

void or_level_matrix(const or_hier *h, int l, int64_t *rp, int32_t *ci, double *v)
{
    const or_level *L = &h->lev[l];
    memcpy(rp, L->rp, sizeof(int64_t) * (L->n + 1));
    memcpy(ci, L->ci, sizeof(int32_t) * L->nnz);
    memcpy(v, L->v, sizeof(double) * L->nnz);
}

void or_level_agg(const or_hier *h, int l, int32_t *agg, double *pc, double *invd, double *w)
{
    const or_level *L = &h->lev[l];
    if (agg && L->agg) memcpy(agg, L->agg, sizeof(int32_t) * L->n);
    if (pc && L->pc) memcpy(pc, L->pc, sizeof(double) * L->n);
    if (invd) memcpy(invd, L->invd, sizeof(double) * L->n);
    if (w) memcpy(w, L->w, sizeof(double) * L->n);
}

void or_coarse_factor(const or_hier *h, double *L)
{
    int nl = (int)h->lev[h->nlev - 1].n;
    memcpy(L, h->chol, sizeof(double) * nl * nl);
}

int64_t or_level_pnnz(const or_hier *h, int l) { return h->lev[l].prp ? h->lev[l].pnnz : 0; }

void or_level_prolongator(const or_hier *h, int l, int64_t *rp, int32_t *ci, double *v)
{
    const or_level *L = &h->lev[l];
    if (!L->prp) return;
    memcpy(rp, L->prp, sizeof(int64_t) * (L->n + 1));
    memcpy(ci, L->pci, sizeof(int32_t) * L->pnnz);
    memcpy(v, L->pv, sizeof(double) * L->pnnz);
}
