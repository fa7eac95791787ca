/* Driver of the oracle for AddressSanitizer / UndefinedBehaviorSanitizer
 * builds (tests/test_sanitizers.py): assembly (Kronecker, quadrature with and
 * without sum factorization, the cube with mixed boundary data), the
 * hierarchy in its variants, V-cycle, PCG / FCG with residual history, block
 * flexible CG, the MLP and the helpers.  Links only the oracle's C files. */
#include "oracle.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>

static int fails = 0;
#define CHECK(c, msg)                                           \
    do {                                                        \
        if (!(c)) {                                             \
            fprintf(stderr, "FAILED: %s (%s)\n", msg, #c);      \
            fails++;                                            \
        }                                                       \
    } while (0)

typedef struct { int64_t n, nnz; int64_t *rp; int32_t *ci; double *v, *F; } sys_t;

static sys_t alloc_sys(int64_t n, int64_t nnz)
{
    sys_t s = {n, nnz, malloc(sizeof(int64_t) * (n + 1)), malloc(sizeof(int32_t) * nnz), malloc(sizeof(double) * nnz),
               malloc(sizeof(double) * n)};
    return s;
}
static void free_sys(sys_t *s) { free(s->rp); free(s->ci); free(s->v); free(s->F); }

static void solve_checks(const sys_t *s, const char *name)
{
    int variants[][4] = {{2, 0, 0, 0}, {2, 1, 0, 0}, {1, 0, 0, 0}, {3, 0, 1, 2}, {2, 0, 0, 1}};
    for (int k = 0; k < 5; k++) {
        or_params prm;
        or_params_default(&prm);
        prm.max_coarse = 30;
        prm.sweeps_per_level = variants[k][0];
        prm.match_positive_only = variants[k][1];
        prm.smooth_prolong = variants[k][2];
        if (variants[k][3] == 2) { prm.smoother = 2; prm.cheb_degree = 4; prm.coarse_solver = 1; }
        if (variants[k][3] == 1) prm.coarse_solver = 1;
        or_hier *h = NULL;
        const int rc = or_setup(s->n, s->rp, s->ci, s->v, NULL, &prm, &h);
        CHECK(rc == 0 && h, name);
        if (rc || !h) continue;
        const int nl = or_nlevels(h);
        for (int l = 0; l < nl; l++) {
            int64_t n, nnz;
            or_level_info(h, l, &n, &nnz);
            CHECK(n > 0 && nnz > 0, name);
        }
        double *u = calloc(s->n, sizeof(double)), *hist = calloc(2001, sizeof(double)), *z = calloc(s->n, sizeof(double));
        int iters = 0;
        double rel = 0.0;
        const int flexible = variants[k][3] ? 1 : 0;
        const int st = or_pcg(h, s->F, u, 1e-8, 2000, flexible, &iters, &rel, hist);
        CHECK(st == 0 && rel <= 1e-8 && iters > 0 && hist[iters] == rel, name);
        or_vcycle(h, 0, s->F, z);
        /* two right-hand sides by block flexible CG */
        double *F2 = malloc(sizeof(double) * 2 * s->n), *U2 = calloc(2 * s->n, sizeof(double));
        for (int64_t i = 0; i < s->n; i++) { F2[i] = s->F[i]; F2[s->n + i] = (double)((i * 7) % 13) - 6.0; }
        int it2[2];
        double rel2[2];
        CHECK(or_block_fcg(h, 2, F2, U2, 1e-8, 2000, it2, rel2) == 0, name);
        free(F2); free(U2); free(u); free(hist); free(z);
        or_free(h);
    }
}

int main(void)
{
    int64_t N, nnz;
    /* 2D and 3D Kronecker assembly */
    for (int d = 2; d <= 3; d++) {
        const int p = d == 2 ? 2 : 3, n = d == 2 ? 16 : 6;
        or_poisson_size(d, p, n, &N, &nnz);
        sys_t s = alloc_sys(N, nnz);
        CHECK(or_poisson_kron(d, p, n, s.rp, s.ci, s.v, s.F) == 0, "kron");
        solve_checks(&s, d == 2 ? "2d p2" : "3d p3");
        free_sys(&s);
    }
    /* quadrature assembly with kappa: element loop and sum factorization */
    {
        const double a[3] = {0.7, -0.4, 1.1};
        const int32_t mk[9] = {1, 0, 0, 0, 2, 1, 3, 1, 2};
        or_poisson_size(3, 3, 4, &N, &nnz);
        sys_t s = alloc_sys(N, nnz), t = alloc_sys(N, nnz);
        CHECK(or_diffusion_quad3d(3, 4, 3, a, mk, s.rp, s.ci, s.v, s.F) == 0, "quad3d");
        CHECK(or_diffusion_sf3d(3, 4, 3, a, mk, t.rp, t.ci, t.v, t.F) == 0, "sf3d");
        double dmax = 0.0;
        for (int64_t k = 0; k < nnz; k++) dmax = fmax(dmax, fabs(s.v[k] - t.v[k]));
        CHECK(dmax < 1e-12, "factorized = element loop");
        solve_checks(&s, "kappa p3");
        free_sys(&s); free_sys(&t);
    }
    /* the cube with mixed boundary conditions */
    {
        or_cube_size(3, 6, &N, &nnz);
        sys_t s = alloc_sys(N, nnz);
        double *lift = calloc(9 * 9 * 9, sizeof(double));
        CHECK(or_cube_system(3, 6, s.rp, s.ci, s.v, s.F, lift) == 0, "cube");
        solve_checks(&s, "cube p3");
        free(lift);
        free_sys(&s);
    }
    /* the MLP */
    {
        const int np = or_mlp_nparam(), B = 5;
        uint16_t *wb = malloc(sizeof(uint16_t) * np);
        for (int i = 0; i < np; i++) wb[i] = (uint16_t)(0x3c00 + (i * 37) % 200);   /* small bf16 values */
        double X[5 * 8], T[5 * 4], Y[5 * 4];
        for (int i = 0; i < 40; i++) X[i] = 0.01 * (i % 9) - 0.03;
        for (int i = 0; i < 20; i++) T[i] = 0.1 * (i % 5);
        double *g = malloc(sizeof(double) * np);
        or_mlp_forward(wb, X, B, Y);
        const double loss = or_mlp_loss_grad(wb, X, T, B, g);
        CHECK(isfinite(loss), "mlp loss");
        free(wb); free(g);
    }
    if (fails) {
        fprintf(stderr, "%d checks failed\n", fails);
        return 1;
    }
    printf("oracle checks ok\n");
    return 0;
}
