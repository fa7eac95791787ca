/*
 * Oracle, part 5: the paper's cube benchmark (Sec. 5.1, "Cube"): -Lap u = f
 * on [0,1]^3 with the exact solution u = exp(x+z) sin(y):
 *   f   = -exp(x+z) sin(y),           g_D = exp(x+z) sin(y) on sides 1-3,
 *   g_N = exp(x+z) cos(y)  on side 4, -exp(x+z) sin(y) on side 5,
 *         exp(x+z) sin(y)  on side 6,
 * discretized as in Sec. 2.2: k_ij = int grad phi_j . grad phi_i and
 * f_i = int f phi_i + int_{Gamma_N} g_N phi_i (eq. (matrix_and_vector_values)),
 * Dirichlet data through a lifting (Sec. 2.4).  TEST INFRASTRUCTURE ONLY.
 *
 * Readings where the paper is silent:
 *  - sides 1..6 are x = 0, x = 1, y = 0, y = 1, z = 0, z = 1 (the Neumann data
 *    above are then the outward normal derivatives of u, and the three
 *    Dirichlet faces give the matrix sizes of Table 1(b));
 *  - lifting: the coefficients of the functions supported on Gamma_D are those
 *    of the L2 projection of g_D = u onto the full tensor spline space (a
 *    quasi-optimal boundary approximation); the interior system carries
 *    f_i - sum_{j in D} k_ij c_j;
 *  - load and error integrals by Gauss-Legendre with p+4 points per direction
 *    and element (the data are not polynomial).
 * Full-space index G = i + m (j + m k), m = n + p, x fastest; the interior
 * (reduced) system is the one of or_poisson_kron_bc with the Dirichlet faces
 * x = 0, x = 1, y = 0.
 */
#include "oracle.h"
#include <math.h>
#include <stdlib.h>
#include <string.h>

/* int_0^1 g(x) N_i(x) dx for every basis function, by q-point Gauss per element */
static void load_1d(int p, int n, double (*g)(double), double *out)
{
    const int m = n + p, q = p + 4;
    double *t = malloc(sizeof(double) * (n + 2 * p + 1));
    double xg[32], wg[32];
    or_knots(p, n, t);
    or_gauss_legendre(q, xg, wg);
    memset(out, 0, sizeof(double) * m);
    for (int e = 0; e < n; e++) {
        const int s = p + e;
        const double a = t[s], h = t[s + 1] - t[s];
        for (int k = 0; k < q; k++) {
            const double x = a + (xg[k] + 1.0) * 0.5 * h, w = wg[k] * 0.5 * h;
            const double gx = g(x);
            for (int l = 0; l <= p; l++) out[s - p + l] += w * (gx * or_bspline(t, s - p + l, p, x));
        }
    }
    free(t);
}

static double fexp(double x) { return exp(x); }
static double fsin(double x) { return sin(x); }

/* x = A^{-1} b for the dense SPD m x m matrix A (Cholesky, A copied) */
static int spd_solve(int m, const double *A, const double *b, double *x)
{
    double *L = malloc(sizeof(double) * m * m);
    memcpy(L, A, sizeof(double) * m * m);
    if (or_cholesky(m, L)) { free(L); return -1; }
    for (int i = 0; i < m; i++) {
        double s = b[i];
        for (int k = 0; k < i; k++) s -= L[i * m + k] * x[k];
        x[i] = s / L[i * m + i];
    }
    for (int i = m - 1; i >= 0; i--) {
        double s = x[i];
        for (int k = i + 1; k < m; k++) s -= L[k * m + i] * x[k];
        x[i] = s / L[i * m + i];
    }
    free(L);
    return 0;
}

static const int CUBE_DIR[6] = {1, 1, 1, 0, 0, 0};   /* x lo, x hi, y lo Dirichlet */

static int is_dirichlet(int i, int j, int m) { return i == 0 || i == m - 1 || j == 0; }

void or_cube_size(int p, int n, int64_t *N, int64_t *nnz)
{
    or_tensor_size(3, p, n, CUBE_DIR, N, nnz);
}

int or_cube_system(int p, int n, int64_t *rp, int32_t *ci, double *v, double *F, double *lift)
{
    if (p < 1 || n < 1 || p > 10) return -1;
    const int m = n + p;
    if (or_poisson_kron_bc(3, p, n, CUBE_DIR, rp, ci, v, NULL)) return -1;
    double *M = malloc(sizeof(double) * m * m), *K = malloc(sizeof(double) * m * m);
    double *one = malloc(sizeof(double) * m), *E = malloc(sizeof(double) * m), *S = malloc(sizeof(double) * m);
    double *ax = malloc(sizeof(double) * m), *ay = malloc(sizeof(double) * m);
    or_matrices_1d(p, n, M, K, one);
    load_1d(p, n, fexp, E);              /* int e^x N_i  (also e^z) */
    load_1d(p, n, fsin, S);              /* int sin(y) N_j          */
    /* L2 projection of u = e^x sin(y) e^z: (M x M x M) c = E x S x E, separable */
    if (spd_solve(m, M, E, ax) || spd_solve(m, M, S, ay)) {
        free(M); free(K); free(one); free(E); free(S); free(ax); free(ay);
        return -2;
    }
    const int64_t full = (int64_t)m * m * m;
    memset(lift, 0, sizeof(double) * full);
    for (int k = 0; k < m; k++)
        for (int j = 0; j < m; j++)
            for (int i = 0; i < m; i++)
                if (is_dirichlet(i, j, m)) lift[i + (int64_t)m * (j + (int64_t)m * k)] = (ax[i] * ay[j]) * ax[k];
    /* interior functions: i = 1..m-2, j = 1..m-1, k = 0..m-1 (reduced order, x fastest) */
    const int mx = m - 2, my = m - 1;
    const double e1 = exp(1.0), c1 = cos(1.0);
    for (int k = 0; k < m; k++)
        for (int j = 1; j < m; j++)
            for (int i = 1; i < m - 1; i++) {
                /* source: f = -e^x sin(y) e^z */
                double fi = -((E[i] * S[j]) * E[k]);
                /* side 4 (y = 1): g_N = e^{x+z} cos(1); only N_{m-1}(1) = 1 is nonzero there */
                if (j == m - 1) fi += c1 * (E[i] * E[k]);
                /* side 5 (z = 0): g_N = -e^x sin(y); N_0(0) = 1 */
                if (k == 0) fi += -(E[i] * S[j]);
                /* side 6 (z = 1): g_N = e^{x+1} sin(y); N_{m-1}(1) = 1 */
                if (k == m - 1) fi += e1 * (E[i] * S[j]);
                /* minus the lifting: sum over the Dirichlet functions of the full-space k_ij c_j */
                double s = 0.0;
                for (int kk = (k - p < 0 ? 0 : k - p); kk <= (k + p > m - 1 ? m - 1 : k + p); kk++)
                    for (int jj = (j - p < 0 ? 0 : j - p); jj <= (j + p > m - 1 ? m - 1 : j + p); jj++)
                        for (int ii = (i - p < 0 ? 0 : i - p); ii <= (i + p > m - 1 ? m - 1 : i + p); ii++) {
                            if (!is_dirichlet(ii, jj, m)) continue;
                            const double kij = (K[k * m + kk] * M[j * m + jj]) * M[i * m + ii] +
                                               (M[k * m + kk] * K[j * m + jj]) * M[i * m + ii] +
                                               (M[k * m + kk] * M[j * m + jj]) * K[i * m + ii];
                            s += kij * lift[ii + (int64_t)m * (jj + (int64_t)m * kk)];
                        }
                F[(i - 1) + (int64_t)mx * ((j - 1) + (int64_t)my * k)] = fi - s;
            }
    free(M); free(K); free(one); free(E); free(S); free(ax); free(ay);
    return 0;
}

void or_cube_embed(int p, int n, const double *u0, const double *lift, double *ufull)
{
    const int m = n + p, mx = m - 2, my = m - 1;
    memcpy(ufull, lift, sizeof(double) * (size_t)m * m * m);
    for (int k = 0; k < m; k++)
        for (int j = 1; j < m; j++)
            for (int i = 1; i < m - 1; i++)
                ufull[i + (int64_t)m * (j + (int64_t)m * k)] = u0[(i - 1) + (int64_t)mx * ((j - 1) + (int64_t)my * k)];
}

int or_cube_error(int p, int n, const double *ufull, double *err, double *norm)
{
    const int m = n + p, q = p + 4;
    double *t = malloc(sizeof(double) * (n + 2 * p + 1));
    double xg[32], wg[32];
    or_knots(p, n, t);
    or_gauss_legendre(q, xg, wg);
    /* basis values at the q points of every element: B[e][qi][l] */
    double *B = malloc(sizeof(double) * n * q * (p + 1)), *X = malloc(sizeof(double) * n * q);
    double *W = malloc(sizeof(double) * n * q);
    for (int e = 0; e < n; e++) {
        const int s = p + e;
        const double a = t[s], h = t[s + 1] - t[s];
        for (int k = 0; k < q; k++) {
            const double x = a + (xg[k] + 1.0) * 0.5 * h;
            X[e * q + k] = x;
            W[e * q + k] = wg[k] * 0.5 * h;
            for (int l = 0; l <= p; l++) B[(e * q + k) * (p + 1) + l] = or_bspline(t, s - p + l, p, x);
        }
    }
    double e2 = 0.0, u2 = 0.0;
    for (int ez = 0; ez < n; ez++)
        for (int ey = 0; ey < n; ey++)
            for (int ex = 0; ex < n; ex++)
                for (int qz = 0; qz < q; qz++)
                    for (int qy = 0; qy < q; qy++)
                        for (int qx = 0; qx < q; qx++) {
                            double uh = 0.0;
                            for (int c = 0; c <= p; c++)
                                for (int b = 0; b <= p; b++)
                                    for (int a = 0; a <= p; a++)
                                        uh += ufull[(ex + a) + (int64_t)m * ((ey + b) + (int64_t)m * (ez + c))] *
                                              ((B[(ex * q + qx) * (p + 1) + a] * B[(ey * q + qy) * (p + 1) + b]) *
                                               B[(ez * q + qz) * (p + 1) + c]);
                            const double x = X[ex * q + qx], y = X[ey * q + qy], z = X[ez * q + qz];
                            const double w = (W[ex * q + qx] * W[ey * q + qy]) * W[ez * q + qz];
                            const double u = exp(x + z) * sin(y);
                            e2 += w * (uh - u) * (uh - u);
                            u2 += w * u * u;
                        }
    *err = sqrt(e2);
    *norm = sqrt(u2);
    free(t); free(B); free(X); free(W);
    return 0;
}
