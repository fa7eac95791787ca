// Driver of the library's host code for AddressSanitizer / UndefinedBehavior-
// Sanitizer builds (tests/test_sanitizers.py): the IgA generators, CSR
// validation, the hierarchy set-up in its variants (matching, pairwise and
// smoothed prolongators, Galerkin products, relaxed test vector), K P, and
// the SELL-C images with their host walk in every layout, each result checked
// against a plain CSR product.  Links only host_setup.cpp (no HIP).
#include "host.h"

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <string>
#include <vector>

using namespace amgiga;

static int fails = 0;
#define CHECK(c, msg)                                            \
    do {                                                         \
        if (!(c)) {                                              \
            std::fprintf(stderr, "FAILED: %s (%s)\n", msg, #c);  \
            fails++;                                             \
        }                                                        \
    } while (0)

static Csr make(int kind, int p, int n)
{
    Csr A;
    int64_t N = 0, nnz = 0;
    if (kind == 3) iga_cube_size(p, n, &N, &nnz);
    else iga_size(kind == 2 ? 2 : 3, p, n, &N, &nnz);
    A.n = N;
    A.rp.resize(N + 1);
    A.ci.resize(nnz);
    A.v.resize(nnz);
    std::vector<double> F(N);
    int st = 0;
    if (kind == 2 || kind == 0) st = iga_poisson(kind == 2 ? 2 : 3, p, n, A.rp.data(), A.ci.data(), A.v.data(), F.data());
    else if (kind == 3) st = iga_cube(p, n, A.rp.data(), A.ci.data(), A.v.data(), F.data());
    else {
        const double a[3] = {0.7, -0.4, 1.1};
        const int32_t mk[9] = {1, 0, 0, 0, 2, 1, 3, 1, 2};
        st = iga_diffusion(p, n, 3, a, mk, A.rp.data(), A.ci.data(), A.v.data(), F.data());
    }
    CHECK(st == 0, "generator");
    return A;
}

static void csr_mv(const Csr &A, int64_t ncols, const std::vector<double> &x, std::vector<double> &y)
{
    (void)ncols;
    y.assign(A.n, 0.0);
    for (int64_t i = 0; i < A.n; i++)
        for (int64_t k = A.rp[i]; k < A.rp[i + 1]; k++) y[i] += A.v[k] * x[A.ci[k]];
}

static void check_images(const Csr &A, int64_t ncols, const char *name)
{
    std::mt19937_64 rng(7);
    std::normal_distribution<double> nd;
    std::vector<double> x(ncols), y, ref;
    for (auto &e : x) e = nd(rng);
    csr_mv(A, ncols, x, ref);
    double scale = 0.0;
    for (double r : ref) scale = std::max(scale, std::fabs(r));
    for (int C : {64, 16, 4})
        for (int layout = 0; layout <= 3; layout++) {
            if ((layout == 1 || layout == 3) && ncols != A.n) continue;
            if (layout == 3 && C != 64) continue;
            y.assign(A.n, 0.0);
            std::string err;
            int64_t sh = 0, st = 0;
            const int rc = sell_spmv_walk(view(A), ncols, C, layout, x.data(), y.data(), &sh, &st, err);
            CHECK(rc == 0, name);
            if (rc) std::fprintf(stderr, "  %s C=%d layout=%d: %s\n", name, C, layout, err.c_str());
            double d = 0.0;
            for (int64_t i = 0; i < A.n; i++) d = std::max(d, std::fabs(y[i] - ref[i]));
            CHECK(d <= 1e-12 * (1.0 + scale), name);
            CHECK(st >= A.nnz(), name);
        }
}

int main()
{
    struct Case { int kind, p, n; const char *name; };
    const Case cases[] = {{2, 2, 12, "2d p2"}, {0, 3, 6, "3d p3"}, {3, 3, 6, "cube p3"}, {1, 3, 4, "kappa p3"},
                          {2, 5, 40, "2d p5 long runs"}, {0, 1, 66, "3d p1 straddling planes"}};
    for (const Case &c : cases) {
        Csr A = make(c.kind, c.p, c.n);
        std::string err;
        CHECK(validate_csr(view(A), err) == 0, c.name);
        check_images(A, A.n, c.name);
        if (c.n > 20) continue;   // the larger stencils only exercise the images
        std::vector<std::pair<const char *, SetupParams>> variants;
        SetupParams d;
        d.max_coarse = 30;   // several levels even on the small cases
        variants.push_back({"default", d});
        SetupParams pos = d; pos.positive_only = 1; variants.push_back({"positive only", pos});
        SetupParams one = d; one.sweeps = 1; variants.push_back({"one sweep", one});
        SetupParams sm = d; sm.sweeps = 3; sm.smooth = 1; variants.push_back({"smoothed", sm});
        SetupParams bs = d; bs.bootstrap = 3; variants.push_back({"bootstrap", bs});
        std::vector<double> w0(A.n);
        std::mt19937_64 rng(11);
        std::uniform_real_distribution<double> ud(0.5, 1.5);
        for (auto &e : w0) e = ud(rng);
        for (auto &v : variants) {
            HostHierarchy H;
            const int rc = build_hierarchy(view(A), v.second.bootstrap ? w0.data() : nullptr, v.second, H, err);
            CHECK(rc == 0, v.first);
            if (rc) { std::fprintf(stderr, "  %s %s: %s\n", c.name, v.first, err.c_str()); continue; }
            CHECK(H.lev.size() >= 2, v.first);
            for (size_t l = 0; l + 1 < H.lev.size(); l++) {
                const HostLevel &L = H.lev[l];
                CsrView K = l == 0 ? view(A) : view(L.K);
                const int64_t nc = H.lev[l + 1].n;
                for (int32_t g : L.agg) CHECK(g >= 0 && g < nc, "aggregate index");
                Csr kp = kp_product(K, nc, L.agg.data(), L.pc.data());
                std::vector<double> e(nc), pe(L.n), y1, y2;
                for (auto &t : e) t = ud(rng);
                for (int64_t i = 0; i < L.n; i++) pe[i] = L.pc[i] * e[L.agg[i]];
                // (K P) e = K (P e)
                csr_mv(kp, nc, e, y1);
                Csr Kc;
                Kc.n = K.n;
                Kc.rp.assign(K.rp, K.rp + K.n + 1);
                Kc.ci.assign(K.ci, K.ci + K.nnz());
                Kc.v.assign(K.v, K.v + K.nnz());
                csr_mv(Kc, K.n, pe, y2);
                double dmax = 0.0, smax = 0.0;
                for (int64_t i = 0; i < L.n; i++) {
                    dmax = std::max(dmax, std::fabs(y1[i] - y2[i]));
                    smax = std::max(smax, std::fabs(y2[i]));
                }
                CHECK(dmax <= 1e-12 * (1.0 + smax), "K P e = K (P e)");
                if (l > 0) check_images(L.K, L.K.n, "coarse level");
                check_images(kp, nc, "K P");
            }
        }
        std::vector<int32_t> mate(A.n);
        const std::vector<double> ones(A.n, 1.0);
        suitor_match(view(A), ones.data(), 0, mate.data());
        for (int64_t i = 0; i < A.n; i++) CHECK(mate[i] < 0 || (mate[i] < A.n && mate[mate[i]] == i), "matching");
    }
    if (fails) {
        std::fprintf(stderr, "%d checks failed\n", fails);
        return 1;
    }
    std::printf("host checks ok\n");
    return 0;
}
