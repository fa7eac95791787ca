/*
 * Oracle, part 1: IgA discretization of the model problem (paper Sec. 2,
 * eq. (poisson), the Galerkin entries k_ij / f_i of Sec. 2.2 and eq.
 * (matrix_and_vector_values)).  TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * Readings where the paper is silent:
 *  - knots: open uniform, p+1 repeated end knots, n equal elements on [0,1]
 *    (maximum regularity C^{p-1}, Sec. 5 set-up);
 *  - quadrature: Gauss-Legendre with p+1 points per direction and element,
 *    exact for the degree <= 2p integrands of M and K;
 *  - Dirichlet: homogeneous on every face, the first and last basis function of
 *    each direction is removed (rows and columns); N = (n+p-2)^d, which matches
 *    the matrix sizes of Tables 1b and 3b for the paper's mixed faces;
 *  - ordering: lexicographic with x fastest, g = ix + m (iy + m iz).
 */
#include "oracle.h"
#include <math.h>
#include <stdlib.h>
#include <string.h>

/* Gauss-Legendre: roots of P_q by Newton from the Chebyshev-like guess
 * cos(pi (k + 3/4) / (q + 1/2)); P_q and P_q' by the Bonnet recurrence.
 * Nodes are returned in ascending order. */
int or_gauss_legendre(int q, double *x, double *w)
{
    if (q < 1) return -1;
    for (int k = 0; k < q; k++) {
        double z = cos(M_PI * (k + 0.75) / (q + 0.5));
        double pq = 0.0, dp = 1.0;
        for (int it = 0; it < 200; it++) {
            double p0 = 1.0, p1 = z;
            for (int j = 2; j <= q; j++) {
                double p2 = ((2.0 * j - 1.0) * z * p1 - (j - 1.0) * p0) / j;
                p0 = p1;
                p1 = p2;
            }
            pq = p1;
            dp = q * (z * p1 - p0) / (z * z - 1.0);
            double dz = pq / dp;
            z -= dz;
            if (fabs(dz) < 1e-16) break;
        }
        {   /* derivative at the converged root for the weight */
            double p0 = 1.0, p1 = z;
            for (int j = 2; j <= q; j++) {
                double p2 = ((2.0 * j - 1.0) * z * p1 - (j - 1.0) * p0) / j;
                p0 = p1;
                p1 = p2;
            }
            dp = q * (z * p1 - p0) / (z * z - 1.0);
        }
        x[k] = -z;
        w[k] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
    return 0;
}

void or_knots(int p, int n, double *t)
{
    for (int i = 0; i <= p; i++) t[i] = 0.0;
    for (int k = 1; k < n; k++) t[p + k] = (double)k / (double)n;
    for (int i = 0; i <= p; i++) t[n + p + i] = 1.0;
}

/* Cox-de Boor: N_{i,0} = 1 on [t_i, t_{i+1}); N_{i,k} blends N_{i,k-1} and
 * N_{i+1,k-1}; a term with a zero knot difference is dropped (0/0 := 0). */
double or_bspline(const double *t, int i, int p, double x)
{
    if (p == 0) return (t[i] <= x && x < t[i + 1]) ? 1.0 : 0.0;
    double a = 0.0, b = 0.0;
    double d1 = t[i + p] - t[i];
    double d2 = t[i + p + 1] - t[i + 1];
    if (d1 > 0.0) a = (x - t[i]) / d1 * or_bspline(t, i, p - 1, x);
    if (d2 > 0.0) b = (t[i + p + 1] - x) / d2 * or_bspline(t, i + 1, p - 1, x);
    return a + b;
}

double or_bspline_deriv(const double *t, int i, int p, double x)
{
    if (p == 0) return 0.0;
    double a = 0.0, b = 0.0;
    double d1 = t[i + p] - t[i];
    double d2 = t[i + p + 1] - t[i + 1];
    if (d1 > 0.0) a = p / d1 * or_bspline(t, i, p - 1, x);
    if (d2 > 0.0) b = p / d2 * or_bspline(t, i + 1, p - 1, x);
    return a - b;
}

/* Element loop of Sec. 2.2 in 1D: on each knot span [t_s, t_{s+1}],
 * s = p + e, the functions N_{s-p..s} are the nonzero ones.  Products
 * N_a N_b are formed before the weight so that M and K are bitwise symmetric. */
void or_matrices_1d(int p, int n, double *M, double *K, double *Fint)
{
    int m = n + p;
    double *t = malloc(sizeof(double) * (n + 2 * p + 1));
    double xg[16], wg[16];
    or_knots(p, n, t);
    or_gauss_legendre(p + 1, xg, wg);
    memset(M, 0, sizeof(double) * m * m);
    memset(K, 0, sizeof(double) * m * m);
    memset(Fint, 0, sizeof(double) * m);
    for (int e = 0; e < n; e++) {
        int s = p + e;
        double a = t[s], b = t[s + 1], h = b - a;
        for (int q = 0; q <= p; q++) {
            double xq = a + (xg[q] + 1.0) * 0.5 * h;
            double wq = wg[q] * 0.5 * h;
            double N[16], dN[16];
            for (int l = 0; l <= p; l++) {
                N[l] = or_bspline(t, s - p + l, p, xq);
                dN[l] = or_bspline_deriv(t, s - p + l, p, xq);
            }
            for (int i = 0; i <= p; i++) {
                int gi = s - p + i;
                Fint[gi] += wq * N[i];
                for (int j = 0; j <= p; j++) {
                    int gj = s - p + j;
                    M[gi * m + gj] += wq * (N[i] * N[j]);
                    K[gi * m + gj] += wq * (dN[i] * dN[j]);
                }
            }
        }
    }
    free(t);
}

static int64_t band_count(int md, int p)
{
    int64_t c = 0;
    for (int i = 0; i < md; i++)
        for (int j = 0; j < md; j++)
            if (abs(i - j) <= p) c++;
    return c;
}

/* Functions kept in direction k: the n+p of the full basis minus one per
 * Dirichlet face (dir[2k] low face, dir[2k+1] high face). */
static void reduced_dims(int d, int p, int n, const int *dir, int *md, int *off)
{
    for (int k = 0; k < 3; k++) { md[k] = 1; off[k] = 0; }
    for (int k = 0; k < d; k++) {
        int lo = dir ? dir[2 * k] : 1, hi = dir ? dir[2 * k + 1] : 1;
        md[k] = n + p - lo - hi;
        off[k] = lo;
    }
}

void or_tensor_size(int d, int p, int n, const int *dir, int64_t *N, int64_t *nnz)
{
    int md[3], off[3];
    reduced_dims(d, p, n, dir, md, off);
    int64_t nn = 1, nz = 1;
    for (int k = 0; k < d; k++) { nn *= md[k]; nz *= band_count(md[k], p); }
    *N = nn;
    *nnz = nz;
}

void or_poisson_size(int d, int p, int n, int64_t *N, int64_t *nnz)
{
    or_tensor_size(d, p, n, NULL, N, nnz);
}

/* Pattern of the reduced tensor system: row (iz,iy,ix), columns with
 * |jd - id| <= p in every direction, in ascending lexicographic order. */
static void tensor_pattern(const int *md, int p, int64_t *rp, int32_t *ci)
{
    int64_t N = (int64_t)md[0] * md[1] * md[2];
    int64_t pos = 0;
    rp[0] = 0;
    for (int64_t g = 0; g < N; g++) {
        int id[3];
        id[0] = (int)(g % md[0]);
        id[1] = (int)((g / md[0]) % md[1]);
        id[2] = (int)(g / ((int64_t)md[0] * md[1]));
        int lo[3], hi[3];
        for (int k = 0; k < 3; k++) {
            lo[k] = id[k] - p < 0 ? 0 : id[k] - p;
            hi[k] = id[k] + p > md[k] - 1 ? md[k] - 1 : id[k] + p;
        }
        for (int jz = lo[2]; jz <= hi[2]; jz++)
            for (int jy = lo[1]; jy <= hi[1]; jy++)
                for (int jx = lo[0]; jx <= hi[0]; jx++)
                    ci[pos++] = (int32_t)(jx + (int64_t)md[0] * (jy + (int64_t)md[1] * jz));
        rp[g + 1] = pos;
    }
}

int or_poisson_kron_bc(int d, int p, int n, const int *dir, int64_t *rp, int32_t *ci,
                       double *v, double *F)
{
    if (d < 1 || d > 3 || p < 1 || n < 1) return -1;
    int m = n + p, md[3], off[3];
    reduced_dims(d, p, n, dir, md, off);
    for (int k = 0; k < d; k++) if (md[k] < 1) return -1;
    double *M = malloc(sizeof(double) * m * m), *K = malloc(sizeof(double) * m * m);
    double *Fi = malloc(sizeof(double) * m);
    or_matrices_1d(p, n, M, K, Fi);
    tensor_pattern(md, p, rp, ci);
    int64_t N = (int64_t)md[0] * md[1] * md[2];
    /* reduced index a in direction k is full index a + off[k] */
#define M1(k, a, b) M[((a) + off[k]) * m + (b) + off[k]]
#define K1(k, a, b) K[((a) + off[k]) * m + (b) + off[k]]
    for (int64_t g = 0; g < N; g++) {
        int ix = (int)(g % md[0]), iy = (int)((g / md[0]) % md[1]);
        int iz = (int)(g / ((int64_t)md[0] * md[1]));
        for (int64_t e = rp[g]; e < rp[g + 1]; e++) {
            int64_t h = ci[e];
            int jx = (int)(h % md[0]), jy = (int)((h / md[0]) % md[1]);
            int jz = (int)(h / ((int64_t)md[0] * md[1]));
            double val;
            if (d == 1) {
                val = K1(0, ix, jx);
            } else if (d == 2) {
                val = K1(1, iy, jy) * M1(0, ix, jx) + M1(1, iy, jy) * K1(0, ix, jx);
            } else {
                double t1 = (K1(2, iz, jz) * M1(1, iy, jy)) * M1(0, ix, jx);
                double t2 = (M1(2, iz, jz) * K1(1, iy, jy)) * M1(0, ix, jx);
                double t3 = (M1(2, iz, jz) * M1(1, iy, jy)) * K1(0, ix, jx);
                val = (t1 + t2) + t3;
            }
            v[e] = val;
        }
        if (F) {
            if (d == 1) F[g] = Fi[ix + off[0]];
            else if (d == 2) F[g] = Fi[iy + off[1]] * Fi[ix + off[0]];
            else F[g] = (Fi[iz + off[2]] * Fi[iy + off[1]]) * Fi[ix + off[0]];
        }
    }
#undef M1
#undef K1
    free(M); free(K); free(Fi);
    return 0;
}

int or_poisson_kron(int d, int p, int n, int64_t *rp, int32_t *ci, double *v, double *F)
{
    return or_poisson_kron_bc(d, p, n, NULL, rp, ci, v, F);
}

static double kappa_eval(int nk, const double *a, const int32_t *mk, double x, double y, double z)
{
    double s = 0.0;
    for (int k = 0; k < nk; k++) {
        double arg = 2.0 * M_PI * (mk[3 * k] * x + mk[3 * k + 1] * y + mk[3 * k + 2] * z);
        s += a[k] * cos(arg);
    }
    return exp(0.5 * s);
}

/* Position of column h in row g (binary search over the sorted row). */
static int64_t find_pos(const int64_t *rp, const int32_t *ci, int64_t g, int64_t h)
{
    int64_t lo = rp[g], hi = rp[g + 1] - 1;
    while (lo <= hi) {
        int64_t mid = (lo + hi) / 2;
        if (ci[mid] == h) return mid;
        if (ci[mid] < h) lo = mid + 1; else hi = mid - 1;
    }
    return -1;
}

/* Sec. 2.2 element loop in 3D: every element, every one of its (p+1)^3 Gauss
 * points, every pair of the (p+1)^3 local functions; the integrand is
 * kappa * grad N_i . grad N_j with the tensor-product basis on the unit cube
 * (identity geometry map, J_F = I). */
int or_diffusion_quad3d(int p, int n, int nk, const double *a, const int32_t *mk,
                        int64_t *rp, int32_t *ci, double *v, double *F)
{
    int m = n + p, md = m - 2;
    if (p < 1 || n < 1 || md < 1) return -1;
    double *t = malloc(sizeof(double) * (n + 2 * p + 1));
    double xg[16], wg[16];
    or_knots(p, n, t);
    or_gauss_legendre(p + 1, xg, wg);
    int mdv[3] = {md, md, md};
    tensor_pattern(mdv, p, rp, ci);
    int64_t N = (int64_t)md * md * md;
    memset(v, 0, sizeof(double) * rp[N]);
    if (F) memset(F, 0, sizeof(double) * N);
    int q1 = p + 1;
    for (int ez = 0; ez < n; ez++)
    for (int ey = 0; ey < n; ey++)
    for (int ex = 0; ex < n; ex++) {
        int e3[3] = {ex, ey, ez};
        /* per direction: basis values and derivatives at the element's points */
        double Bv[3][16][16], Dv[3][16][16], Xq[3][16], Wq[3][16];
        for (int dir = 0; dir < 3; dir++) {
            int s = p + e3[dir];
            double lo = t[s], h = t[s + 1] - t[s];
            for (int q = 0; q < q1; q++) {
                double xq = lo + (xg[q] + 1.0) * 0.5 * h;
                Xq[dir][q] = xq;
                Wq[dir][q] = wg[q] * 0.5 * h;
                for (int l = 0; l < q1; l++) {
                    Bv[dir][l][q] = or_bspline(t, s - p + l, p, xq);
                    Dv[dir][l][q] = or_bspline_deriv(t, s - p + l, p, xq);
                }
            }
        }
        for (int qz = 0; qz < q1; qz++)
        for (int qy = 0; qy < q1; qy++)
        for (int qx = 0; qx < q1; qx++) {
            double Wt = (Wq[0][qx] * Wq[1][qy]) * Wq[2][qz];
            double kap = kappa_eval(nk, a, mk, Xq[0][qx], Xq[1][qy], Xq[2][qz]);
            double kw = kap * Wt;
            for (int az = 0; az < q1; az++)
            for (int ay = 0; ay < q1; ay++)
            for (int ax = 0; ax < q1; ax++) {
                int fx = ex + ax, fy = ey + ay, fz = ez + az;   /* full indices */
                if (fx == 0 || fx == m - 1 || fy == 0 || fy == m - 1 || fz == 0 || fz == m - 1) continue;
                int64_t g = (fx - 1) + (int64_t)md * ((fy - 1) + (int64_t)md * (fz - 1));
                double Ni = (Bv[0][ax][qx] * Bv[1][ay][qy]) * Bv[2][az][qz];
                double gi0 = (Dv[0][ax][qx] * Bv[1][ay][qy]) * Bv[2][az][qz];
                double gi1 = (Bv[0][ax][qx] * Dv[1][ay][qy]) * Bv[2][az][qz];
                double gi2 = (Bv[0][ax][qx] * Bv[1][ay][qy]) * Dv[2][az][qz];
                if (F) F[g] += Wt * Ni;
                for (int bz = 0; bz < q1; bz++)
                for (int by = 0; by < q1; by++)
                for (int bx = 0; bx < q1; bx++) {
                    int hx = ex + bx, hy = ey + by, hz = ez + bz;
                    if (hx == 0 || hx == m - 1 || hy == 0 || hy == m - 1 || hz == 0 || hz == m - 1) continue;
                    int64_t hh = (hx - 1) + (int64_t)md * ((hy - 1) + (int64_t)md * (hz - 1));
                    double gj0 = (Dv[0][bx][qx] * Bv[1][by][qy]) * Bv[2][bz][qz];
                    double gj1 = (Bv[0][bx][qx] * Dv[1][by][qy]) * Bv[2][bz][qz];
                    double gj2 = (Bv[0][bx][qx] * Bv[1][by][qy]) * Dv[2][bz][qz];
                    double dot = (gi0 * gj0 + gi1 * gj1) + gi2 * gj2;
                    int64_t pos = find_pos(rp, ci, g, hh);
                    v[pos] += kw * dot;
                }
            }
        }
    }
    free(t);
    return 0;
}

/* The same integral as or_diffusion_quad3d, with the quadrature sums of each
 * element factorized direction by direction (sum factorization, Sec. 2.2's
 * fast-assembly remark): for each of the three gradient terms,
 *   T1[qx][qy][az][bz] = sum_qz kw(q) Z_az(qz) Z_bz(qz),
 *   T2[qx][ay][by][az][bz] = sum_qy T1 Y_ay(qy) Y_by(qy),
 *   k_local += sum_qx T2 X_ax(qx) X_bx(qx),
 * with X/Y/Z the value or the derivative table of the direction carrying the
 * derivative.  Same CSR pattern and F as the plain loop. */
int or_diffusion_sf3d(int p, int n, int nk, const double *a, const int32_t *mk,
                      int64_t *rp, int32_t *ci, double *v, double *F)
{
    int m = n + p, md = m - 2, q1 = p + 1;
    if (p < 1 || p > 7 || n < 1 || md < 1) return -1;
    double *t = malloc(sizeof(double) * (n + 2 * p + 1));
    double xg[16], wg[16];
    or_knots(p, n, t);
    or_gauss_legendre(q1, xg, wg);
    int mdv[3] = {md, md, md};
    tensor_pattern(mdv, p, rp, ci);
    int64_t N = (int64_t)md * md * md;
    memset(v, 0, sizeof(double) * rp[N]);
    if (F) memset(F, 0, sizeof(double) * N);
    /* 1D tables per element index and direction are the same for every
     * direction (same knots): B[e][l][q], D[e][l][q], X[e][q], W[e][q] */
    double *B = malloc(sizeof(double) * n * q1 * q1), *D = malloc(sizeof(double) * n * q1 * q1);
    double *X = malloc(sizeof(double) * n * q1), *W = malloc(sizeof(double) * n * q1);
    for (int e = 0; e < n; e++) {
        int s = p + e;
        double lo = t[s], h = t[s + 1] - t[s];
        for (int q = 0; q < q1; q++) {
            double xq = lo + (xg[q] + 1.0) * 0.5 * h;
            X[e * q1 + q] = xq;
            W[e * q1 + q] = wg[q] * 0.5 * h;
            for (int l = 0; l < q1; l++) {
                B[(e * q1 + l) * q1 + q] = or_bspline(t, s - p + l, p, xq);
                D[(e * q1 + l) * q1 + q] = or_bspline_deriv(t, s - p + l, p, xq);
            }
        }
    }
    int nq = q1 * q1 * q1, nl = q1 * q1 * q1;
    double *kw = malloc(sizeof(double) * nq), *Kl = malloc(sizeof(double) * nl * nl);
    double *T1 = malloc(sizeof(double) * q1 * q1 * q1 * q1);
    double *T2 = malloc(sizeof(double) * q1 * q1 * q1 * q1 * q1);
    for (int ez = 0; ez < n; ez++)
    for (int ey = 0; ey < n; ey++)
    for (int ex = 0; ex < n; ex++) {
        const double *Bx = B + ex * q1 * q1, *By = B + ey * q1 * q1, *Bz = B + ez * q1 * q1;
        const double *Dx = D + ex * q1 * q1, *Dy = D + ey * q1 * q1, *Dz = D + ez * q1 * q1;
        for (int qz = 0; qz < q1; qz++)
            for (int qy = 0; qy < q1; qy++)
                for (int qx = 0; qx < q1; qx++) {
                    double Wt = (W[ex * q1 + qx] * W[ey * q1 + qy]) * W[ez * q1 + qz];
                    kw[(qx * q1 + qy) * q1 + qz] = kappa_eval(nk, a, mk, X[ex * q1 + qx], X[ey * q1 + qy],
                                                              X[ez * q1 + qz]) * Wt;
                    if (F) {
                        for (int az = 0; az < q1; az++)
                        for (int ay = 0; ay < q1; ay++)
                        for (int ax = 0; ax < q1; ax++) {
                            int fx = ex + ax, fy = ey + ay, fz = ez + az;
                            if (fx == 0 || fx == m - 1 || fy == 0 || fy == m - 1 || fz == 0 || fz == m - 1) continue;
                            int64_t g = (fx - 1) + (int64_t)md * ((fy - 1) + (int64_t)md * (fz - 1));
                            F[g] += Wt * ((Bx[ax * q1 + qx] * By[ay * q1 + qy]) * Bz[az * q1 + qz]);
                        }
                    }
                }
        memset(Kl, 0, sizeof(double) * nl * nl);
        for (int term = 0; term < 3; term++) {
            const double *Tx = term == 0 ? Dx : Bx, *Ty = term == 1 ? Dy : By, *Tz = term == 2 ? Dz : Bz;
            /* contract qz */
            for (int qx = 0; qx < q1; qx++)
            for (int qy = 0; qy < q1; qy++)
            for (int az = 0; az < q1; az++)
            for (int bz = 0; bz < q1; bz++) {
                double s = 0.0;
                for (int qz = 0; qz < q1; qz++)
                    s += kw[(qx * q1 + qy) * q1 + qz] * (Tz[az * q1 + qz] * Tz[bz * q1 + qz]);
                T1[((qx * q1 + qy) * q1 + az) * q1 + bz] = s;
            }
            /* contract qy */
            for (int qx = 0; qx < q1; qx++)
            for (int ay = 0; ay < q1; ay++)
            for (int by = 0; by < q1; by++)
            for (int az = 0; az < q1; az++)
            for (int bz = 0; bz < q1; bz++) {
                double s = 0.0;
                for (int qy = 0; qy < q1; qy++)
                    s += T1[((qx * q1 + qy) * q1 + az) * q1 + bz] * (Ty[ay * q1 + qy] * Ty[by * q1 + qy]);
                T2[(((qx * q1 + ay) * q1 + by) * q1 + az) * q1 + bz] = s;
            }
            /* contract qx into the local matrix; local index (az, ay, ax) with x fastest */
            for (int az = 0; az < q1; az++)
            for (int ay = 0; ay < q1; ay++)
            for (int ax = 0; ax < q1; ax++)
            for (int bz = 0; bz < q1; bz++)
            for (int by = 0; by < q1; by++)
            for (int bx = 0; bx < q1; bx++) {
                double s = 0.0;
                for (int qx = 0; qx < q1; qx++)
                    s += T2[(((qx * q1 + ay) * q1 + by) * q1 + az) * q1 + bz] * (Tx[ax * q1 + qx] * Tx[bx * q1 + qx]);
                Kl[((az * q1 + ay) * q1 + ax) * nl + ((bz * q1 + by) * q1 + bx)] += s;
            }
        }
        /* scatter into the global matrix */
        for (int az = 0; az < q1; az++)
        for (int ay = 0; ay < q1; ay++)
        for (int ax = 0; ax < q1; ax++) {
            int fx = ex + ax, fy = ey + ay, fz = ez + az;
            if (fx == 0 || fx == m - 1 || fy == 0 || fy == m - 1 || fz == 0 || fz == m - 1) continue;
            int64_t g = (fx - 1) + (int64_t)md * ((fy - 1) + (int64_t)md * (fz - 1));
            for (int bz = 0; bz < q1; bz++)
            for (int by = 0; by < q1; by++)
            for (int bx = 0; bx < q1; bx++) {
                int hx = ex + bx, hy = ey + by, hz = ez + bz;
                if (hx == 0 || hx == m - 1 || hy == 0 || hy == m - 1 || hz == 0 || hz == m - 1) continue;
                int64_t hh = (hx - 1) + (int64_t)md * ((hy - 1) + (int64_t)md * (hz - 1));
                v[find_pos(rp, ci, g, hh)] += Kl[((az * q1 + ay) * q1 + ax) * nl + ((bz * q1 + by) * q1 + bx)];
            }
        }
    }
    free(B); free(D); free(X); free(W); free(kw); free(Kl); free(T1); free(T2); free(t);
    return 0;
}
