// Host construction of the AMG hierarchy by compatible weighted matching
// (paper Sec. 3.1) and the IgA workload generator (Sec. 2).
//
// Per level, m pairwise sweeps are composed (the m-step aggregation of
// Sec. 3.1, P = P1 P2 ... Pm).  Each sweep:
//   1. edge weights c_ij of eq. (cij) with the stored k_ij of row min(i,j);
//   2. the greedy matching of eq. (maxprod)'s linear-time approximation, taken
//      in the strict order (c descending, min index, max index), computed here
//      by the suitor algorithm (Manne & Halappanavar), which yields the same
//      matching as the sorted greedy scan for a strict total order, without a
//      global sort;
//   3. coarse numbering by the smallest member, pairwise prolongator of
//      eq. (prolongation), restricted test vector;
//   4. Galerkin product of eq. (galerkin_matrix_projection), row-parallel with a
//      fixed per-row summation order (members ascending, entries ascending).
// Every floating-point expression is written with explicit association and the
// file is compiled without FMA contraction, so that two implementations of the
// same readings agree to the bit.
#include "host.h"
#include <atomic>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>

namespace amgiga {

int host_threads()
{
    unsigned h = std::thread::hardware_concurrency();
    if (h == 0) h = 1;
    if (h > 32) h = 32;
    return (int)h;
}

double cij(double kij, double kii, double kjj, double wi, double wj)
{
    double num = ((2.0 * kij) * wi) * wj;
    double den = (kii * wi) * wi + (kjj * wj) * wj;
    return 1.0 - num / den;
}

static int64_t find_in_row(const CsrView &K, int64_t row, int32_t col)
{
    const int32_t *b = K.ci + K.rp[row], *e = K.ci + K.rp[row + 1];
    const int32_t *p = std::lower_bound(b, e, col);
    if (p == e || *p != col) return -1;
    return (int64_t)(p - K.ci);
}

int validate_csr(const CsrView &K, std::string &err)
{
    if (K.n <= 0 || K.n > 2147483647LL) { err = "n must be in 1 .. 2^31-1"; return -1; }
    if (!K.rp || !K.ci || !K.v) { err = "NULL CSR array"; return -1; }
    if (K.rp[0] != 0) { err = "row_ptr[0] must be 0"; return -1; }
    for (int64_t i = 0; i < K.n; i++)
        if (K.rp[i + 1] < K.rp[i]) { err = "row_ptr not monotone"; return -1; }
    // each chunk records its first failing row and the reason
    std::vector<std::pair<int64_t, int>> fails;
    std::mutex mx;
    parallel_for(K.n, [&](int64_t b, int64_t e) {
        for (int64_t i = b; i < e; i++) {
            int code = 0;
            bool diag = false;
            for (int64_t k = K.rp[i]; k < K.rp[i + 1] && !code; k++) {
                int32_t j = K.ci[k];
                if (j < 0 || j >= K.n) code = 1;
                else if (k > K.rp[i] && j <= K.ci[k - 1]) code = 2;
                else if (!std::isfinite(K.v[k])) code = 3;
                else if (j == i) { diag = true; if (!(K.v[k] > 0.0)) code = 4; }
                else {
                    int64_t t = find_in_row(K, j, (int32_t)i);
                    if (t < 0) code = 5;
                    else if (!(K.v[t] == K.v[k])) code = 6;
                }
            }
            if (!code && !diag) code = 4;
            if (code) {
                std::lock_guard<std::mutex> g(mx);
                fails.push_back({i, code});
                return;
            }
        }
    });
    if (!fails.empty()) {
        std::sort(fails.begin(), fails.end());
        static const char *msg[] = {"", "column index out of range", "columns not strictly ascending",
                                    "non-finite value", "missing or non-positive diagonal",
                                    "pattern not symmetric", "values not symmetric"};
        err = std::string(msg[fails[0].second]) + " in row " + std::to_string(fails[0].first);
        return -1;
    }
    return 0;
}

// c of every stored off-diagonal entry, taken from row min(i,j); NaN marks an
// ineligible entry (diagonal, zero value, non-finite c, or c <= 1 when only
// positive log-weights are eligible).
static std::vector<double> edge_weights(const CsrView &K, const double *w, int positive_only)
{
    std::vector<double> diag(K.n), c(K.nnz());
    parallel_for(K.n, [&](int64_t b, int64_t e) {
        for (int64_t i = b; i < e; i++) {
            double d = 0.0;
            for (int64_t k = K.rp[i]; k < K.rp[i + 1]; k++)
                if (K.ci[k] == i) d = K.v[k];
            diag[i] = d;
        }
    });
    parallel_for(K.n, [&](int64_t b, int64_t e) {
        for (int64_t i = b; i < e; i++) {
            for (int64_t k = K.rp[i]; k < K.rp[i + 1]; k++) {
                int64_t j = K.ci[k];
                double val = NAN;
                if (j != i) {
                    double kv;
                    if (i < j) kv = K.v[k];
                    else {
                        int64_t t = find_in_row(K, j, (int32_t)i);
                        kv = t >= 0 ? K.v[t] : 0.0;
                    }
                    if (kv != 0.0) {
                        int64_t a = i < j ? i : j, bb = i < j ? j : i;
                        double cv = cij(kv, diag[a], diag[bb], w[a], w[bb]);
                        bool ok = std::isfinite(cv) && (!positive_only || cv > 1.0);
                        if (ok) val = cv;
                    }
                }
                c[k] = val;
            }
        }
    });
    return c;
}

// Edge (c, a, b) precedes (c2, a2, b2) in the matching order; a < b, a2 < b2.
static inline bool precedes(double c, int64_t a, int64_t b, double c2, int64_t a2, int64_t b2)
{
    if (c != c2) return c > c2;
    if (a != a2) return a < a2;
    return b < b2;
}

// Suitor algorithm: every vertex proposes to the neighbour whose edge is best
// in the order among those that would accept it (its current suitor's edge is
// worse); a displaced suitor proposes again.  On termination the suitor
// relation is mutual on the matched pairs and equals the greedy matching.
static void suitor_core(const CsrView &K, const std::vector<double> &c, int32_t *mate)
{
    int64_t n = K.n;
    std::vector<int32_t> suitor(n, -1);
    std::vector<double> ws(n, 0.0);
    for (int64_t u = 0; u < n; u++) {
        int64_t cur = u;
        while (cur >= 0) {
            int64_t best = -1;
            double bc = 0.0;
            int64_t ba = 0, bb = 0;
            for (int64_t k = K.rp[cur]; k < K.rp[cur + 1]; k++) {
                double cv = c[k];
                if (cv != cv) continue;
                int64_t v = K.ci[k];
                int64_t a = cur < v ? cur : v, b = cur < v ? v : cur;
                if (best >= 0 && !precedes(cv, a, b, bc, ba, bb)) continue;
                int64_t s = suitor[v];
                if (s >= 0) {
                    int64_t sa = s < v ? s : v, sb = s < v ? v : s;
                    if (!precedes(cv, a, b, ws[v], sa, sb)) continue;
                }
                best = v; bc = cv; ba = a; bb = b;
            }
            if (best < 0) break;
            int64_t y = suitor[best];
            suitor[best] = (int32_t)cur;
            ws[best] = bc;
            cur = y;
        }
    }
    for (int64_t v = 0; v < n; v++) {
        int64_t s = suitor[v];
        mate[v] = (s >= 0 && suitor[s] == v) ? (int32_t)s : -1;
    }
}

void suitor_match(const CsrView &K, const double *w, int positive_only, int32_t *mate)
{
    std::vector<double> c = edge_weights(K, w, positive_only);
    suitor_core(K, c, mate);
}

// Coarse numbering by the smallest member; pairwise prolongator and restricted
// test vector (eq. (prolongation)).
static int64_t pairwise(int64_t n, const int32_t *mate, const double *w, std::vector<int32_t> &agg,
                        std::vector<double> &pc, std::vector<double> &wc)
{
    agg.assign(n, -1);
    pc.assign(n, 0.0);
    int64_t nc = 0;
    for (int64_t i = 0; i < n; i++) {
        if (agg[i] >= 0) continue;
        agg[i] = (int32_t)nc;
        if (mate[i] >= 0) agg[mate[i]] = (int32_t)nc;
        nc++;
    }
    wc.assign(nc, 0.0);
    for (int64_t i = 0; i < n; i++) {
        int64_t j = mate[i];
        if (j >= 0) {
            double s = std::sqrt(w[i] * w[i] + w[j] * w[j]);
            pc[i] = w[i] / s;
            wc[agg[i]] = s;
        } else {
            pc[i] = (w[i] != 0.0) ? w[i] / std::fabs(w[i]) : 1.0;
            wc[agg[i]] = std::fabs(w[i]);
        }
    }
    return nc;
}

// Galerkin product for a one-entry-per-row prolongator, parallel over coarse
// rows; within a coarse row the sum order is members ascending, then each
// member's stored entries ascending, from +0.0.
static Csr galerkin(const CsrView &K, int64_t nc, const std::vector<int32_t> &agg,
                    const std::vector<double> &pc)
{
    int64_t n = K.n;
    std::vector<int64_t> mp(nc + 1, 0), mem(n);
    for (int64_t i = 0; i < n; i++) mp[agg[i] + 1]++;
    for (int64_t I = 0; I < nc; I++) mp[I + 1] += mp[I];
    {
        std::vector<int64_t> fill(mp.begin(), mp.end() - 1);
        for (int64_t i = 0; i < n; i++) mem[fill[agg[i]]++] = i;
    }
    Csr C;
    C.n = nc;
    C.rp.assign(nc + 1, 0);
    // pass 1: distinct coarse columns per coarse row
    parallel_for(nc, [&](int64_t b, int64_t e) {
        std::vector<int64_t> stamp(nc, -1);
        for (int64_t I = b; I < e; I++) {
            int64_t cnt = 0;
            for (int64_t m = mp[I]; m < mp[I + 1]; m++) {
                int64_t i = mem[m];
                for (int64_t k = K.rp[i]; k < K.rp[i + 1]; k++) {
                    int32_t J = agg[K.ci[k]];
                    if (stamp[J] != I) { stamp[J] = I; cnt++; }
                }
            }
            C.rp[I + 1] = cnt;
        }
    });
    for (int64_t I = 0; I < nc; I++) C.rp[I + 1] += C.rp[I];
    C.ci.resize(C.rp[nc]);
    C.v.resize(C.rp[nc]);
    // pass 2: accumulate
    parallel_for(nc, [&](int64_t b, int64_t e) {
        std::vector<int64_t> stamp(nc, -1);
        std::vector<double> acc(nc);
        std::vector<int32_t> touched;
        for (int64_t I = b; I < e; I++) {
            touched.clear();
            for (int64_t m = mp[I]; m < mp[I + 1]; m++) {
                int64_t i = mem[m];
                double pi = pc[i];
                for (int64_t k = K.rp[i]; k < K.rp[i + 1]; k++) {
                    int64_t j = K.ci[k];
                    int32_t J = agg[j];
                    double t = (pi * K.v[k]) * pc[j];
                    if (stamp[J] != I) { stamp[J] = I; acc[J] = 0.0; touched.push_back(J); }
                    acc[J] = acc[J] + t;
                }
            }
            std::sort(touched.begin(), touched.end());
            int64_t pos = C.rp[I];
            for (int32_t J : touched) { C.ci[pos] = J; C.v[pos] = acc[J]; pos++; }
        }
    });
    return C;
}

Csr kp_product(const CsrView &K, int64_t nc, const int32_t *agg, const double *pc)
{
    Csr C;
    C.n = K.n;
    C.rp.assign(K.n + 1, 0);
    parallel_for(K.n, [&](int64_t b, int64_t e) {
        std::vector<int32_t> cols;
        for (int64_t i = b; i < e; i++) {
            cols.clear();
            for (int64_t k = K.rp[i]; k < K.rp[i + 1]; k++) cols.push_back(agg[K.ci[k]]);
            std::sort(cols.begin(), cols.end());
            C.rp[i + 1] = std::unique(cols.begin(), cols.end()) - cols.begin();
        }
    });
    for (int64_t i = 0; i < K.n; i++) C.rp[i + 1] += C.rp[i];
    C.ci.resize(C.rp[K.n]);
    C.v.resize(C.rp[K.n]);
    parallel_for(K.n, [&](int64_t b, int64_t e) {
        std::vector<int64_t> slot(nc, -1);
        std::vector<int32_t> cols;
        for (int64_t i = b; i < e; i++) {
            cols.clear();
            for (int64_t k = K.rp[i]; k < K.rp[i + 1]; k++) cols.push_back(agg[K.ci[k]]);
            std::sort(cols.begin(), cols.end());
            cols.erase(std::unique(cols.begin(), cols.end()), cols.end());
            int64_t pos = C.rp[i];
            for (size_t t = 0; t < cols.size(); t++) {
                slot[cols[t]] = pos + (int64_t)t;
                C.ci[pos + t] = cols[t];
                C.v[pos + t] = 0.0;
            }
            for (int64_t k = K.rp[i]; k < K.rp[i + 1]; k++) {
                int64_t j = K.ci[k];
                C.v[slot[agg[j]]] += K.v[k] * pc[j];
            }
        }
    });
    (void)nc;
    return C;
}

Csr smooth_prolongator(const CsrView &K, const std::vector<double> &invd, int64_t nc, const int32_t *agg,
                       const double *pc, double omega)
{
    Csr P = kp_product(K, nc, agg, pc);
    parallel_for(K.n, [&](int64_t b, int64_t e) {
        for (int64_t i = b; i < e; i++) {
            const double s = omega * invd[i];
            for (int64_t k = P.rp[i]; k < P.rp[i + 1]; k++) {
                const double tent = (P.ci[k] == agg[i]) ? pc[i] : 0.0;
                P.v[k] = tent - s * P.v[k];
            }
        }
    });
    return P;
}

Csr transpose(const Csr &P, int64_t ncols)
{
    Csr T;
    T.n = ncols;
    T.rp.assign(ncols + 1, 0);
    for (int64_t k = 0; k < P.nnz(); k++) T.rp[P.ci[k] + 1]++;
    for (int64_t J = 0; J < ncols; J++) T.rp[J + 1] += T.rp[J];
    T.ci.resize(P.nnz());
    T.v.resize(P.nnz());
    std::vector<int64_t> fill(T.rp.begin(), T.rp.end() - 1);
    for (int64_t i = 0; i < P.n; i++)
        for (int64_t k = P.rp[i]; k < P.rp[i + 1]; k++) {
            int64_t q = fill[P.ci[k]]++;
            T.ci[q] = (int32_t)i;
            T.v[q] = P.v[k];
        }
    return T;
}

Csr galerkin_general(const CsrView &K, const Csr &P, const Csr &PT)
{
    const int64_t n = K.n, nc = PT.n;
    const int nt = std::max(1, host_threads());
    // coarse rows in chunks handed out in order; each chunk keeps its rows
    const int64_t nchunk = std::min<int64_t>(nc, (int64_t)nt * 16);
    std::vector<std::vector<int32_t>> cci(nchunk);
    std::vector<std::vector<double>> cv(nchunk);
    std::vector<int64_t> rowlen(nc, 0);
    std::atomic<int64_t> next(0);
    auto work = [&]() {
        std::vector<double> accB(n), accC(nc);
        std::vector<int64_t> stampB(n, -1), stampC(nc, -1);
        std::vector<int32_t> colB, colC;
        for (;;) {
            const int64_t ch = next.fetch_add(1);
            if (ch >= nchunk) break;
            const int64_t I0 = nc * ch / nchunk, I1 = nc * (ch + 1) / nchunk;
            for (int64_t I = I0; I < I1; I++) {
                colB.clear();
                for (int64_t q = PT.rp[I]; q < PT.rp[I + 1]; q++) {
                    const int64_t i = PT.ci[q];
                    const double pv = PT.v[q];
                    for (int64_t k = K.rp[i]; k < K.rp[i + 1]; k++) {
                        const int32_t j = K.ci[k];
                        if (stampB[j] != I) { stampB[j] = I; accB[j] = 0.0; colB.push_back(j); }
                        accB[j] = accB[j] + pv * K.v[k];
                    }
                }
                std::sort(colB.begin(), colB.end());
                colC.clear();
                for (int32_t j : colB) {
                    const double bj = accB[j];
                    for (int64_t k = P.rp[j]; k < P.rp[j + 1]; k++) {
                        const int32_t J = P.ci[k];
                        if (stampC[J] != I) { stampC[J] = I; accC[J] = 0.0; colC.push_back(J); }
                        accC[J] = accC[J] + bj * P.v[k];
                    }
                }
                std::sort(colC.begin(), colC.end());
                rowlen[I] = (int64_t)colC.size();
                for (int32_t J : colC) { cci[ch].push_back(J); cv[ch].push_back(accC[J]); }
            }
        }
    };
    {
        std::vector<std::thread> th;
        for (int t = 1; t < nt; t++) th.emplace_back(work);
        work();
        for (auto &x : th) x.join();
    }
    Csr C;
    C.n = nc;
    C.rp.assign(nc + 1, 0);
    for (int64_t I = 0; I < nc; I++) C.rp[I + 1] = C.rp[I] + rowlen[I];
    C.ci.resize(C.rp[nc]);
    C.v.resize(C.rp[nc]);
    for (int64_t ch = 0; ch < nchunk; ch++) {
        const int64_t I0 = nc * ch / nchunk;
        std::copy(cci[ch].begin(), cci[ch].end(), C.ci.begin() + C.rp[I0]);
        std::copy(cv[ch].begin(), cv[ch].end(), C.v.begin() + C.rp[I0]);
    }
    return C;
}

static void l1_invdiag(const CsrView &K, std::vector<double> &invd)
{
    invd.resize(K.n);
    parallel_for(K.n, [&](int64_t b, int64_t e) {
        for (int64_t i = b; i < e; i++) {
            double d = 0.0;
            for (int64_t k = K.rp[i]; k < K.rp[i + 1]; k++)
                if (K.ci[k] == i) d = K.v[k];
            for (int64_t k = K.rp[i]; k < K.rp[i + 1]; k++)
                if (K.ci[k] != i) d = d + std::fabs(K.v[k]);
            invd[i] = 1.0 / d;
        }
    });
}

void level_features(const CsrView &K, const std::vector<double> &invd, float out[6])
{
    double s_diag = 0.0, min_diag = 1.0, s_off = 0.0;
    int64_t npos = 0, noff = 0, maxlen = 0;
    for (int64_t i = 0; i < K.n; i++) {
        double kii = 0.0, off = 0.0;
        maxlen = std::max<int64_t>(maxlen, K.rp[i + 1] - K.rp[i]);
        for (int64_t k = K.rp[i]; k < K.rp[i + 1]; k++) {
            if (K.ci[k] == i) kii = K.v[k];
            else {
                off += K.v[k];
                noff++;
                if (K.v[k] > 0.0) npos++;
            }
        }
        double r = kii * invd[i];
        s_diag += r;
        min_diag = std::min(min_diag, r);
        s_off += off * invd[i];
    }
    // every feature is independent of the problem size
    const double mean_len = (double)K.nnz() / (double)K.n;
    out[0] = (float)(std::log10(mean_len) / 3.0);
    out[1] = (float)((double)maxlen / mean_len - 1.0);
    out[2] = (float)(s_diag / (double)K.n);
    out[3] = (float)min_diag;
    out[4] = (float)(s_off / (double)K.n);
    out[5] = (float)(noff ? (double)npos / (double)noff : 0.0);
}

static void make_coarsest(HostHierarchy &H, const CsrView &K, int dense = 1)
{
    int64_t n = K.n;
    if (!dense) { H.coarse_lower.clear(); return; }
    H.coarse_lower.assign((size_t)(n * n), 0.0);
    for (int64_t i = 0; i < n; i++)
        for (int64_t k = K.rp[i]; k < K.rp[i + 1]; k++)
            if (K.ci[k] <= i) H.coarse_lower[(size_t)(i * n + K.ci[k])] = K.v[k];
}

void bootstrap_w(const CsrView &K, const double *w0, int sweeps, std::vector<double> &w)
{
    std::vector<double> invd, s(K.n);
    l1_invdiag(K, invd);
    w.assign(w0, w0 + K.n);
    for (int k = 0; k < sweeps; k++) {
        parallel_for(K.n, [&](int64_t b, int64_t e) {
            for (int64_t i = b; i < e; i++) {
                double t = 0.0;
                for (int64_t q = K.rp[i]; q < K.rp[i + 1]; q++) t = t + K.v[q] * w[K.ci[q]];
                s[i] = t;
            }
        });
        for (int64_t i = 0; i < K.n; i++) w[i] = w[i] - invd[i] * s[i];
    }
}

int build_hierarchy(const CsrView &K0, const double *w, const SetupParams &prm,
                    HostHierarchy &H, std::string &err, Coarsener *dev)
{
    int maxl = prm.max_levels > 0 ? prm.max_levels : 1;
    H.lev.clear();
    H.lev.emplace_back();
    {
        HostLevel &L0 = H.lev[0];
        L0.n = K0.n;
        L0.nnz = K0.nnz();
        if (prm.bootstrap > 0) {
            if (dev) dev->bootstrap(K0, w, prm.bootstrap, L0.w);
            else bootstrap_w(K0, w, prm.bootstrap, L0.w);
        } else {
            L0.w.resize(K0.n);
            for (int64_t i = 0; i < K0.n; i++) L0.w[i] = w ? w[i] : 1.0;
        }
        l1_invdiag(K0, L0.invd);
        level_features(K0, L0.invd, L0.feat);
    }
    for (int l = 0;; l++) {
        CsrView K = l == 0 ? K0 : view(H.lev[l].K);
        int64_t nl = H.lev[l].n;
        if (nl <= prm.max_coarse) { make_coarsest(H, K, prm.coarse_dense); return 0; }
        if (l == maxl - 1) {
            if (nl <= 2000) { make_coarsest(H, K, prm.coarse_dense); return 0; }
            err = "coarsening reached max_levels above 2000 unknowns";
            return -6;
        }
        std::vector<int32_t> agg(nl);
        std::vector<double> pc(nl);
        Csr cur;
        std::vector<double> cw;
        const double *wl = H.lev[l].w.data();
        int64_t nc = nl;
        if (dev) {
            CoarsenResult res;
            dev->coarsen(l, K, wl, prm, res);
            nc = res.nc;
            agg = std::move(res.agg);
            pc = std::move(res.pc);
            cur = std::move(res.C);
            cw = std::move(res.wc);
        }
        for (int s = 0; s < (dev ? 0 : prm.sweeps); s++) {
            CsrView kv = s == 0 ? K : view(cur);
            const double *ww = s == 0 ? wl : cw.data();
            std::vector<int32_t> mate(kv.n);
            suitor_match(kv, ww, prm.positive_only, mate.data());
            std::vector<int32_t> ag;
            std::vector<double> pcs, wc;
            nc = pairwise(kv.n, mate.data(), ww, ag, pcs, wc);
            // with smoothing, the last sweep's unsmoothed product is not needed
            Csr C = (prm.smooth && s == prm.sweeps - 1) ? Csr() : galerkin(kv, nc, ag, pcs);
            if (s == 0) {
                agg = ag;
                pc = pcs;
            } else {
                for (int64_t i = 0; i < nl; i++) {
                    pc[i] = pc[i] * pcs[agg[i]];
                    agg[i] = ag[agg[i]];
                }
            }
            cur = std::move(C);
            cw = std::move(wc);
        }
        if ((double)nc > 0.9 * (double)nl) {
            if (nl <= 2000) { make_coarsest(H, K, prm.coarse_dense); return 0; }
            err = "coarsening stalled above 2000 unknowns";
            return -6;
        }
        HostLevel &L = H.lev[l];
        L.agg = std::move(agg);
        L.pc = std::move(pc);
        if (prm.smooth) {
            L.P = smooth_prolongator(K, L.invd, nc, L.agg.data(), L.pc.data(), prm.omega);
            L.PT = transpose(L.P, nc);
            cur = galerkin_general(K, L.P, L.PT);
        }
        {
            std::vector<int> cnt(nc, 0);
            for (int64_t i = 0; i < nl; i++) cnt[L.agg[i]]++;
            L.max_members = *std::max_element(cnt.begin(), cnt.end());
        }
        HostLevel next;
        next.n = cur.n;
        next.nnz = cur.nnz();
        next.K = std::move(cur);
        next.w = std::move(cw);
        l1_invdiag(view(next.K), next.invd);
        level_features(view(next.K), next.invd, next.feat);
        H.lev.push_back(std::move(next));
    }
}

// ---------------------------------------------------------------------------
// Workload generator: 1D B-spline matrices by Gauss quadrature, then the
// Kronecker sum (Sec. 2.2).  The benchmark systems must be the very matrices a
// plain FP64 statement of the discretization produces, bit for bit, so every
// value below is one fixed sequence of IEEE operations: the Gauss nodes come
// from Newton's method on P_q started at cos(pi (k + 3/4) / (q + 1/2)), with
// P_q and P_{q-1} from the three-term recurrence and P_q' = q (z P_q - P_{q-1})
// / (z^2 - 1); the basis values from the Cox-de Boor recurrence evaluated
// bottom-up over the degrees (a term with a zero knot difference is dropped).

// P_q(z) and P_{q-1}(z)
static void legendre_pair(int q, double z, double &pq, double &pq1)
{
    double lo = 1.0, hi = z;
    for (int j = 2; j <= q; j++) {
        double nx = ((2.0 * j - 1.0) * z * hi - (j - 1.0) * lo) / j;
        lo = hi;
        hi = nx;
    }
    pq = hi;
    pq1 = lo;
}

// q-point Gauss-Legendre rule on [-1, 1], nodes ascending
static void gauss_nodes(int q, double *x, double *w)
{
    for (int k = 0; k < q; k++) {
        double z = std::cos(M_PI * (k + 0.75) / (q + 0.5)), pq, pq1, dp;
        for (int it = 0; it < 200; it++) {
            legendre_pair(q, z, pq, pq1);
            dp = q * (z * pq - pq1) / (z * z - 1.0);
            double dz = pq / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        legendre_pair(q, z, pq, pq1);
        dp = q * (z * pq - pq1) / (z * z - 1.0);
        x[k] = -z;
        w[k] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

// Values N[0..p] and derivatives D[0..p] of the functions s-p .. s, the ones
// nonzero on knot span s, at x.  Level k of the table holds N_{i,k}(x) for
// i = s-p .. s+p-k (degree 0: the indicator of [t_i, t_{i+1})).
static void span_basis(const std::vector<double> &t, int s, int p, double x, double *N, double *D)
{
    double tab[2][40];
    const int i0 = s - p;
    double *cur = tab[0], *nxt = tab[1];
    for (int i = i0; i <= s + p; i++) cur[i - i0] = (t[i] <= x && x < t[i + 1]) ? 1.0 : 0.0;
    for (int k = 1; k <= p; k++) {
        if (k == p) {   // derivatives from degree p-1
            for (int l = 0; l <= p; l++) {
                const int i = i0 + l;
                const double d1 = t[i + p] - t[i], d2 = t[i + p + 1] - t[i + 1];
                double a = 0.0, b = 0.0;
                if (d1 > 0.0) a = p / d1 * cur[l];
                if (d2 > 0.0) b = p / d2 * cur[l + 1];
                D[l] = a - b;
            }
        }
        for (int i = i0; i <= s + p - k; i++) {
            const double d1 = t[i + k] - t[i], d2 = t[i + k + 1] - t[i + 1];
            double a = 0.0, b = 0.0;
            if (d1 > 0.0) a = (x - t[i]) / d1 * cur[i - i0];
            if (d2 > 0.0) b = (t[i + k + 1] - x) / d2 * cur[i + 1 - i0];
            nxt[i - i0] = a + b;
        }
        std::swap(cur, nxt);
    }
    for (int l = 0; l <= p; l++) N[l] = cur[l];
}

static void matrices_1d(int p, int n, std::vector<double> &M, std::vector<double> &K,
                        std::vector<double> &Fi)
{
    int m = n + p;
    std::vector<double> t(n + 2 * p + 1);
    for (int i = 0; i <= p; i++) { t[i] = 0.0; t[n + p + i] = 1.0; }
    for (int k = 1; k < n; k++) t[p + k] = (double)k / (double)n;
    double xg[16], wg[16];
    gauss_nodes(p + 1, xg, wg);
    M.assign((size_t)m * m, 0.0);
    K.assign((size_t)m * m, 0.0);
    Fi.assign(m, 0.0);
    for (int e = 0; e < n; e++) {
        int s = p + e;
        double a = t[s], h = t[s + 1] - t[s];
        for (int q = 0; q <= p; q++) {
            double x = a + 0.5 * (xg[q] + 1.0) * h, wq = 0.5 * wg[q] * h;
            double N[16], D[16];
            span_basis(t, s, p, x, N, D);
            for (int i = 0; i <= p; i++) {
                Fi[s - p + i] += wq * N[i];
                for (int j = 0; j <= p; j++) {
                    M[(size_t)(s - p + i) * m + (s - p + j)] += wq * (N[i] * N[j]);
                    K[(size_t)(s - p + i) * m + (s - p + j)] += wq * (D[i] * D[j]);
                }
            }
        }
    }
}

void iga_size(int d, int p, int n, int64_t *N, int64_t *nnz)
{
    int64_t md = n + p - 2;
    int64_t b = 0;
    for (int64_t i = 0; i < md; i++) {
        int64_t lo = i - p < 0 ? 0 : i - p, hi = i + p > md - 1 ? md - 1 : i + p;
        b += hi - lo + 1;
    }
    int64_t nn = 1, nz = 1;
    for (int k = 0; k < d; k++) { nn *= md; nz *= b; }
    *N = nn;
    *nnz = nz;
}

int iga_poisson(int d, int p, int n, int64_t *rp, int32_t *ci, double *v, double *F)
{
    if (d < 2 || d > 3 || p < 1 || p > 10 || n < 1 || n + p - 2 < 1) return -1;
    int m = n + p, md = m - 2;
    std::vector<double> M, K, Fi;
    matrices_1d(p, n, M, K, Fi);
    auto M1 = [&](int a, int b) { return M[(size_t)(a + 1) * m + (b + 1)]; };
    auto K1 = [&](int a, int b) { return K[(size_t)(a + 1) * m + (b + 1)]; };
    auto len1 = [&](int i) { int lo = i - p < 0 ? 0 : i - p, hi = i + p > md - 1 ? md - 1 : i + p; return hi - lo + 1; };
    int64_t N = 1;
    for (int k = 0; k < d; k++) N *= md;
    // row pointer: row length is the product of the 1D lengths
    rp[0] = 0;
    for (int64_t g = 0; g < N; g++) {
        int ix = (int)(g % md), iy = (int)((g / md) % md), iz = d == 3 ? (int)(g / ((int64_t)md * md)) : 0;
        int64_t len = (int64_t)len1(ix) * len1(iy) * (d == 3 ? len1(iz) : 1);
        rp[g + 1] = rp[g] + len;
    }
    parallel_for(N, [&](int64_t b, int64_t e) {
        for (int64_t g = b; g < e; g++) {
            int ix = (int)(g % md), iy = (int)((g / md) % md), iz = d == 3 ? (int)(g / ((int64_t)md * md)) : 0;
            int64_t pos = rp[g];
            int zlo = d == 3 ? std::max(0, iz - p) : 0, zhi = d == 3 ? std::min(md - 1, iz + p) : 0;
            int ylo = std::max(0, iy - p), yhi = std::min(md - 1, iy + p);
            int xlo = std::max(0, ix - p), xhi = std::min(md - 1, ix + p);
            for (int jz = zlo; jz <= zhi; jz++)
                for (int jy = ylo; jy <= yhi; jy++)
                    for (int jx = xlo; jx <= xhi; jx++) {
                        double val;
                        if (d == 2) {
                            val = K1(iy, jy) * M1(ix, jx) + M1(iy, jy) * K1(ix, jx);
                        } else {
                            double a = (K1(iz, jz) * M1(iy, jy)) * M1(ix, jx);
                            double bb = (M1(iz, jz) * K1(iy, jy)) * M1(ix, jx);
                            double c = (M1(iz, jz) * M1(iy, jy)) * K1(ix, jx);
                            val = (a + bb) + c;
                        }
                        ci[pos] = (int32_t)(jx + (int64_t)md * (jy + (int64_t)md * jz));
                        v[pos] = val;
                        pos++;
                    }
            if (F) F[g] = d == 2 ? Fi[iy + 1] * Fi[ix + 1] : (Fi[iz + 1] * Fi[iy + 1]) * Fi[ix + 1];
        }
    });
    return 0;
}


// The paper's cube problem (Sec. 5.1): -Lap u = f on [0,1]^3, u = e^{x+z} sin y,
// Dirichlet on x = 0, x = 1, y = 0 (rows and columns of the functions with a
// nonzero trace there removed: the first and last in x, the first in y),
// Neumann data g_N = du/dn on y = 1, z = 0, z = 1 through boundary integrals.
// Dirichlet data by a lifting with the L2-projection coefficients of g_D.
// Every term is separable: integrals of e^x, sin y, e^z against the 1D basis,
// and the lifting, a tensor product restricted to the Dirichlet functions, is
// split by inclusion-exclusion into three tensor products whose images under
// K = K1 x M1 x M1 + M1 x K1 x M1 + M1 x M1 x K1 are products of 1D vectors.

// int_0^1 g(x) N_i(x) dx, (p+4)-point Gauss per element
template <typename G> static void load_1d(int p, int n, G g, std::vector<double> &out)
{
    const int m = n + p, q = p + 4;
    std::vector<double> t(n + 2 * p + 1);
    for (int i = 0; i <= p; i++) { t[i] = 0.0; t[n + p + i] = 1.0; }
    for (int k = 1; k < n; k++) t[p + k] = (double)k / (double)n;
    double xg[32], wg[32];
    gauss_nodes(q, xg, wg);
    out.assign(m, 0.0);
    for (int e = 0; e < n; e++) {
        const int s = p + e;
        const double a = t[s], h = t[s + 1] - t[s];
        for (int k = 0; k < q; k++) {
            const double x = a + 0.5 * (xg[k] + 1.0) * h, w = 0.5 * wg[k] * h;
            double N[16], D[16];
            span_basis(t, s, p, x, N, D);
            const double gx = g(x);
            for (int l = 0; l <= p; l++) out[s - p + l] += w * (gx * N[l]);
        }
    }
}

// solve the banded SPD system A x = b (m x m dense storage, bandwidth p) by LDL^T
static void band_spd_solve(int m, int p, const std::vector<double> &A, const std::vector<double> &b,
                           std::vector<double> &x)
{
    std::vector<double> L((size_t)m * m, 0.0), D(m, 0.0);
    for (int i = 0; i < m; i++) {
        for (int j = std::max(0, i - p); j < i; j++) {
            double s = A[(size_t)i * m + j];
            for (int k = std::max(0, i - p); k < j; k++) s -= L[(size_t)i * m + k] * L[(size_t)j * m + k] * D[k];
            L[(size_t)i * m + j] = s / D[j];
        }
        double s = A[(size_t)i * m + i];
        for (int k = std::max(0, i - p); k < i; k++) s -= L[(size_t)i * m + k] * L[(size_t)i * m + k] * D[k];
        D[i] = s;
    }
    x = b;
    for (int i = 0; i < m; i++)
        for (int k = std::max(0, i - p); k < i; k++) x[i] -= L[(size_t)i * m + k] * x[k];
    for (int i = 0; i < m; i++) x[i] /= D[i];
    for (int i = m - 1; i >= 0; i--)
        for (int k = i + 1; k < std::min(m, i + p + 1); k++) x[i] -= L[(size_t)k * m + i] * x[k];
}

void iga_cube_size(int p, int n, int64_t *N, int64_t *nnz)
{
    const int m = n + p, md[3] = {m - 2, m - 1, m};
    int64_t nn = 1, nz = 1;
    for (int d = 0; d < 3; d++) {
        int64_t b = 0;
        for (int i = 0; i < md[d]; i++) b += std::min(md[d] - 1, i + p) - std::max(0, i - p) + 1;
        nn *= md[d];
        nz *= b;
    }
    *N = nn;
    *nnz = nz;
}

int iga_cube(int p, int n, int64_t *rp, int32_t *ci, double *v, double *F)
{
    if (p < 1 || p > 10 || n < 1 || n + p < 3) return -1;
    const int m = n + p;
    const int mx = m - 2, my = m - 1, mz = m, ox = 1, oy = 1, oz = 0;   // kept functions, first kept index
    std::vector<double> M, K, Fi;
    matrices_1d(p, n, M, K, Fi);
    auto M1 = [&](int a, int b) { return M[(size_t)a * m + b]; };
    auto K1 = [&](int a, int b) { return K[(size_t)a * m + b]; };
    auto band = [&](int i, int md, int &lo, int &hi) { lo = std::max(0, i - p); hi = std::min(md - 1, i + p); };
    const int64_t N = (int64_t)mx * my * mz;
    rp[0] = 0;
    for (int64_t g = 0; g < N; g++) {
        const int ix = (int)(g % mx), iy = (int)((g / mx) % my), iz = (int)(g / ((int64_t)mx * my));
        int a0, a1, b0, b1, c0, c1;
        band(ix, mx, a0, a1); band(iy, my, b0, b1); band(iz, mz, c0, c1);
        rp[g + 1] = rp[g] + (int64_t)(a1 - a0 + 1) * (b1 - b0 + 1) * (c1 - c0 + 1);
    }
    // load vectors and lifting coefficients
    std::vector<double> E, S, ax, ay;
    load_1d(p, n, [](double x) { return std::exp(x); }, E);
    load_1d(p, n, [](double y) { return std::sin(y); }, S);
    band_spd_solve(m, p, M, E, ax);
    band_spd_solve(m, p, M, S, ay);
    // lifting l = (ax x ay x ax) restricted to {i in {0, m-1}} u {j = 0}
    //   = (ax_X) x ay x ax + ax x (ay_0) x ax - (ax_X) x (ay_0) x ax,
    // ax_X: ax on i in {0, m-1} only; ay_0: ay on j = 0 only.
    std::vector<double> axX(m, 0.0), ay0(m, 0.0);
    axX[0] = ax[0]; axX[m - 1] = ax[m - 1]; ay0[0] = ay[0];
    auto mul = [&](const std::vector<double> &A, const std::vector<double> &u, std::vector<double> &r) {
        r.assign(m, 0.0);
        for (int i = 0; i < m; i++)
            for (int j = std::max(0, i - p); j <= std::min(m - 1, i + p); j++) r[i] += A[(size_t)i * m + j] * u[j];
    };
    std::vector<double> Mx_, Kx_, MxX, KxX, My_, Ky_, My0, Ky0, Mz_, Kz_;
    mul(M, ax, Mx_); mul(K, ax, Kx_); mul(M, axX, MxX); mul(K, axX, KxX);
    mul(M, ay, My_); mul(K, ay, Ky_); mul(M, ay0, My0); mul(K, ay0, Ky0);
    Mz_ = Mx_; Kz_ = Kx_;                               // z uses ax as well (e^z)
    // (K u x v x w)_(i,j,k) for the tensor term u x v x w, by its 1D images
    auto kterm = [&](const std::vector<double> &Mu, const std::vector<double> &Ku, const std::vector<double> &Mv,
                     const std::vector<double> &Kv, int i, int j, int k) {
        return (Kz_[k] * Mv[j]) * Mu[i] + (Mz_[k] * Kv[j]) * Mu[i] + (Mz_[k] * Mv[j]) * Ku[i];
    };
    const double exp1 = std::exp(1.0), cos1 = std::cos(1.0);
    parallel_for(N, [&](int64_t b, int64_t e) {
        for (int64_t g = b; g < e; g++) {
            const int ix = (int)(g % mx), iy = (int)((g / mx) % my), iz = (int)(g / ((int64_t)mx * my));
            const int i = ix + ox, j = iy + oy, k = iz + oz;   // full-space indices
            int a0, a1, b0, b1, c0, c1;
            band(ix, mx, a0, a1); band(iy, my, b0, b1); band(iz, mz, c0, c1);
            int64_t pos = rp[g];
            for (int jz = c0; jz <= c1; jz++)
                for (int jy = b0; jy <= b1; jy++)
                    for (int jx = a0; jx <= a1; jx++) {
                        const int ii = jx + ox, jj = jy + oy, kk = jz + oz;
                        const double t1 = (K1(k, kk) * M1(j, jj)) * M1(i, ii);
                        const double t2 = (M1(k, kk) * K1(j, jj)) * M1(i, ii);
                        const double t3 = (M1(k, kk) * M1(j, jj)) * K1(i, ii);
                        ci[pos] = (int32_t)(jx + (int64_t)mx * (jy + (int64_t)my * jz));
                        v[pos] = (t1 + t2) + t3;
                        pos++;
                    }
            if (F) {
                double f = -(E[i] * S[j]) * E[k];               // source -e^x sin y e^z
                if (j == m - 1) f += cos1 * (E[i] * E[k]);        // y = 1: e^{x+z} cos 1
                if (k == 0) f -= E[i] * S[j];                   // z = 0: -e^x sin y
                if (k == m - 1) f += exp1 * (E[i] * S[j]);        // z = 1: e^{x+1} sin y
                const double lift = kterm(MxX, KxX, My_, Ky_, i, j, k) + kterm(Mx_, Kx_, My0, Ky0, i, j, k) -
                                    kterm(MxX, KxX, My0, Ky0, i, j, k);
                F[g] = f - lift;
            }
        }
    });
    return 0;
}

// Variable-coefficient stiffness -div(kappa grad u) on the unit cube (Sec. 2.2,
// kappa inside the integral), kappa = exp(0.5 sum_k a_k cos(2 pi m_k . x)),
// (p+1)^3 Gauss points per element, the quadrature sums of each element
// factorized direction by direction: per gradient term, contract the z points
// (T1[qx][qy][az][bz]), then the y points (T2[qx][ay][by][az][bz]), then the x
// points into the local matrix.  Elements are added into the global matrix in
// lexicographic order (z slowest), one fixed summation order for every entry:
// local matrices of a run of consecutive elements are formed in parallel, then
// added row by row (a row owned by one thread, its elements in order).  F is
// the load of f = 1, summed per element over the points in (z, y, x) order.
static double kappa_at(int nk, const double *a, const int32_t *mk, double x, double y, double z)
{
    double s = 0.0;
    for (int k = 0; k < nk; k++)
        s += a[k] * std::cos(2.0 * M_PI * ((double)mk[3 * k] * x + (double)mk[3 * k + 1] * y + (double)mk[3 * k + 2] * z));
    return std::exp(0.5 * s);
}

int iga_diffusion(int p, int n, int nk, const double *a, const int32_t *mk, int64_t *rp, int32_t *ci, double *v,
                  double *F)
{
    if (p < 1 || p > 7 || n < 1 || n + p - 2 < 1 || nk < 0) return -1;
    const int m = n + p, md = m - 2, q1 = p + 1;
    // pattern: the constant-coefficient generator's layout (ascending (z, y, x) columns)
    if (iga_poisson(3, p, n, rp, ci, v, nullptr)) return -1;
    const int64_t N = (int64_t)md * md * md;
    std::fill(v, v + rp[N], 0.0);
    if (F) std::fill(F, F + N, 0.0);
    std::vector<double> t(n + 2 * p + 1);
    for (int i = 0; i <= p; i++) { t[i] = 0.0; t[n + p + i] = 1.0; }
    for (int k = 1; k < n; k++) t[p + k] = (double)k / (double)n;
    double xg[16], wg[16];
    gauss_nodes(q1, xg, wg);
    // per element index e: points X[e][q], weights W[e][q], values B[e][l][q] and
    // derivatives Dv[e][l][q] of the element's p+1 functions (same in every direction)
    std::vector<double> X(n * q1), W(n * q1), Bv(n * q1 * q1), Dv(n * q1 * q1);
    for (int e = 0; e < n; e++) {
        int s0 = p + e;
        double lo = t[s0], h = t[s0 + 1] - t[s0];
        for (int q = 0; q < q1; q++) {
            double x = lo + 0.5 * (xg[q] + 1.0) * h;
            X[e * q1 + q] = x;
            W[e * q1 + q] = 0.5 * wg[q] * h;
            double Nv[16], Dd[16];
            span_basis(t, s0, p, x, Nv, Dd);
            for (int l = 0; l < q1; l++) { Bv[(e * q1 + l) * q1 + q] = Nv[l]; Dv[(e * q1 + l) * q1 + q] = Dd[l]; }
        }
    }
    auto len1 = [&](int i) { return std::min(md - 1, i + p) - std::max(0, i - p) + 1; };
    const int nl = q1 * q1 * q1, q2 = q1 * q1;
    // a run: elements ez, ey in [y0, y1), every ex; at most ~64 MB of local matrices
    const int64_t per_el = (int64_t)nl * nl;
    const int lines = (int)std::max<int64_t>(1, std::min<int64_t>(n, ((int64_t)8 << 20) / (per_el * n)));
    std::vector<double> Kl((size_t)lines * n * per_el);
    auto local = [&](int ex, int ey, int ez, double *K) {
        const double *BX = &Bv[ex * q2], *BY = &Bv[ey * q2], *BZ = &Bv[ez * q2];
        const double *DX = &Dv[ex * q2], *DY = &Dv[ey * q2], *DZ = &Dv[ez * q2];
        double kw[512], T1[4096], T2[32768];
        for (int qx = 0; qx < q1; qx++)
            for (int qy = 0; qy < q1; qy++)
                for (int qz = 0; qz < q1; qz++) {
                    double wt = (W[ex * q1 + qx] * W[ey * q1 + qy]) * W[ez * q1 + qz];
                    kw[(qx * q1 + qy) * q1 + qz] =
                        kappa_at(nk, a, mk, X[ex * q1 + qx], X[ey * q1 + qy], X[ez * q1 + qz]) * wt;
                }
        std::fill(K, K + per_el, 0.0);
        for (int term = 0; term < 3; term++) {
            const double *TX = term == 0 ? DX : BX, *TY = term == 1 ? DY : BY, *TZ = term == 2 ? DZ : BZ;
            for (int qx = 0; qx < q1; qx++)
            for (int qy = 0; qy < q1; qy++)
            for (int az = 0; az < q1; az++)
            for (int bz = 0; bz < q1; bz++) {
                double acc = 0.0;
                for (int qz = 0; qz < q1; qz++)
                    acc += kw[(qx * q1 + qy) * q1 + qz] * (TZ[az * q1 + qz] * TZ[bz * q1 + qz]);
                T1[((qx * q1 + qy) * q1 + az) * q1 + bz] = acc;
            }
            for (int qx = 0; qx < q1; qx++)
            for (int ay = 0; ay < q1; ay++)
            for (int by = 0; by < q1; by++)
            for (int az = 0; az < q1; az++)
            for (int bz = 0; bz < q1; bz++) {
                double acc = 0.0;
                for (int qy = 0; qy < q1; qy++)
                    acc += T1[((qx * q1 + qy) * q1 + az) * q1 + bz] * (TY[ay * q1 + qy] * TY[by * q1 + qy]);
                T2[(((qx * q1 + ay) * q1 + by) * q1 + az) * q1 + bz] = acc;
            }
            for (int az = 0; az < q1; az++)
            for (int ay = 0; ay < q1; ay++)
            for (int ax = 0; ax < q1; ax++)
            for (int bz = 0; bz < q1; bz++)
            for (int by = 0; by < q1; by++)
            for (int bx = 0; bx < q1; bx++) {
                double acc = 0.0;
                for (int qx = 0; qx < q1; qx++)
                    acc += T2[(((qx * q1 + ay) * q1 + by) * q1 + az) * q1 + bz] * (TX[ax * q1 + qx] * TX[bx * q1 + qx]);
                K[(size_t)((az * q1 + ay) * q1 + ax) * nl + (bz * q1 + by) * q1 + bx] += acc;
            }
        }
    };
    for (int ez = 0; ez < n; ez++)
        for (int y0 = 0; y0 < n; y0 += lines) {
            const int y1 = std::min(n, y0 + lines);
            const int64_t nel = (int64_t)(y1 - y0) * n;
            parallel_for(nel, [&](int64_t b, int64_t e) {
                for (int64_t el = b; el < e; el++)
                    local((int)(el % n), y0 + (int)(el / n), ez, &Kl[(size_t)el * per_el]);
            }, 1);
            // rows touched by the run: full indices fz in [ez, ez+p], fy in [y0, y1-1+p]
            const int fz0 = std::max(1, ez), fz1 = std::min(m - 2, ez + p);
            const int fy0 = std::max(1, y0), fy1 = std::min(m - 2, y1 - 1 + p);
            if (fz0 > fz1 || fy0 > fy1) continue;
            const int64_t nrow = (int64_t)(fz1 - fz0 + 1) * (fy1 - fy0 + 1) * md;
            parallel_for(nrow, [&](int64_t b, int64_t e) {
                for (int64_t r = b; r < e; r++) {
                    const int ix = (int)(r % md), fx = ix + 1;
                    const int fy = fy0 + (int)((r / md) % (fy1 - fy0 + 1)), fz = fz0 + (int)(r / ((int64_t)md * (fy1 - fy0 + 1)));
                    const int iy = fy - 1, iz = fz - 1;
                    const int64_t g = ix + (int64_t)md * (iy + (int64_t)md * iz);
                    const int az = fz - ez;
                    const int xlo = std::max(0, ix - p), ylo = std::max(0, iy - p), zlo = std::max(0, iz - p);
                    const int lx = len1(ix), ly = len1(iy);
                    for (int ey = std::max(y0, fy - p); ey <= std::min(y1 - 1, fy); ey++)
                        for (int ex = std::max(0, fx - p); ex <= std::min(n - 1, fx); ex++) {
                            const int ay = fy - ey, ax = fx - ex;
                            if (F) {
                                const double *BX = &Bv[ex * q2], *BY = &Bv[ey * q2], *BZ = &Bv[ez * q2];
                                for (int qz = 0; qz < q1; qz++)
                                    for (int qy = 0; qy < q1; qy++)
                                        for (int qx = 0; qx < q1; qx++) {
                                            double wt = (W[ex * q1 + qx] * W[ey * q1 + qy]) * W[ez * q1 + qz];
                                            F[g] += wt * ((BX[ax * q1 + qx] * BY[ay * q1 + qy]) * BZ[az * q1 + qz]);
                                        }
                            }
                            const double *K = &Kl[(size_t)((ey - y0) * (int64_t)n + ex) * per_el] +
                                              (size_t)((az * q1 + ay) * q1 + ax) * nl;
                            for (int bz = 0; bz < q1; bz++) {
                                const int jz = ez + bz - 1;
                                if (jz < 0 || jz >= md) continue;
                                for (int by = 0; by < q1; by++) {
                                    const int jy = ey + by - 1;
                                    if (jy < 0 || jy >= md) continue;
                                    const int64_t base = rp[g] + ((int64_t)(jz - zlo) * ly + (jy - ylo)) * lx;
                                    for (int bx = 0; bx < q1; bx++) {
                                        const int jx = ex + bx - 1;
                                        if (jx < 0 || jx >= md) continue;
                                        v[base + (jx - xlo)] += K[(bz * q1 + by) * q1 + bx];
                                    }
                                }
                            }
                        }
                }
            }, 1);
        }
    return 0;
}


// ---------------------------------------------------------------------------
// Device matrix images (SELL-C) built on the host, and their host walk.


// Ascending union of the column offsets (column - row) of the rows of slice s,
// or an empty list when it would be longer than `limit`.
std::vector<int32_t> slice_offsets(const CsrView &K, int64_t s, int C, int64_t limit)
{
    std::vector<int32_t> u, m;
    for (int64_t r = s * C; r < std::min(K.n, (s + 1) * C); r++) {
        m.clear();
        size_t a = 0;
        for (int64_t k = K.rp[r]; k < K.rp[r + 1]; k++) {
            const int32_t o = (int32_t)(K.ci[k] - r);
            while (a < u.size() && u[a] < o) m.push_back(u[a++]);
            if (a < u.size() && u[a] == o) a++;
            m.push_back(o);
        }
        while (a < u.size()) m.push_back(u[a++]);
        if ((int64_t)m.size() > limit) return {};
        u.swap(m);
    }
    return u;
}

// Number of C-row slices whose offset unions would be stored once.
int64_t count_shared(const CsrView &K, int C)
{
    const int64_t ns = (K.n + C - 1) / C;
    std::atomic<int64_t> cnt{0};
    parallel_for(ns, [&](int64_t sb, int64_t se) {
        int64_t c = 0;
        for (int64_t s = sb; s < se; s++) {
            int64_t w = 0;
            for (int64_t r = s * C; r < std::min(K.n, (s + 1) * C); r++) w = std::max(w, K.rp[r + 1] - K.rp[r]);
            if (w > 0 && !slice_offsets(K, s, C, (w + 7) / 8 * 8).empty()) c++;
        }
        cnt += c;
    }, 1);
    return cnt.load();
}

// SELL-C image of a CSR matrix (slice height C rows; group layout of kernels.h).
// With `shared`, a slice whose offset union is no wider than its longest row
// (both rounded up to 8) stores the union once; the others keep per-row indices.
// With sigma > 0 (no shared offsets then), the rows of every window of sigma
// consecutive rows are placed in the window's slots by decreasing length (ties
// by index), so the slices of a window pad to similar lengths; perm[slot]
// gives the row of each slot (-1 for the slots past the last row).
void build_sell(const CsrView &K, int C, bool want64, bool want32, bool shared, int sigma, SellHost &S)
{
    const int64_t n = K.n;
    S.nslices = (n + C - 1) / C;
    const int64_t nslot = S.nslices * C;
    if (sigma > 0) shared = false;
    std::vector<int32_t> rowof(nslot, -1);
    auto len = [&](int64_t r) { return K.rp[r + 1] - K.rp[r]; };
    parallel_for((n + std::max(sigma, 1) - 1) / std::max(sigma, 1), [&](int64_t wb, int64_t we) {
        for (int64_t w = wb; w < we; w++) {
            const int64_t a = w * std::max(sigma, 1), e = std::min(n, a + std::max(sigma, 1));
            for (int64_t r = a; r < e; r++) rowof[r] = (int32_t)r;
            if (sigma > 0)
                std::stable_sort(rowof.begin() + a, rowof.begin() + e,
                                 [&](int32_t x, int32_t y) { return len(x) > len(y); });
        }
    }, 1);
    S.sorted = sigma > 0 ? 1 : 0;
    if (S.sorted) S.perm = rowof;
    std::vector<int64_t> wd(S.nslices);
    std::vector<std::vector<int32_t>> U(S.nslices);
    parallel_for(S.nslices, [&](int64_t sb, int64_t se) {
        for (int64_t s = sb; s < se; s++) {
            int64_t w = 0;
            for (int64_t q = s * C; q < (s + 1) * C; q++)
                if (rowof[q] >= 0) w = std::max(w, len(rowof[q]));
            wd[s] = (w + 7) / 8 * 8;
            if (shared && w > 0) U[s] = slice_offsets(K, s, C, wd[s]);
        }
    }, 1);
    S.soff.assign(S.nslices + 1, 0);
    S.ibase.assign(S.nslices, 0);
    int64_t ib = 0, sh = 0;
    S.nshared = 0;
    S.index_bytes = 0.0;
    // identical offset lists (the interior slices of a stencil matrix) are
    // stored once, so the wavefronts reading them share cache lines
    std::map<std::vector<int32_t>, int64_t> lists;
    for (int64_t s = 0; s < S.nslices; s++) {
        const int64_t w = U[s].empty() ? wd[s] : (int64_t)(U[s].size() + 7) / 8 * 8;
        S.soff[s + 1] = S.soff[s] + C * w;
        if (U[s].empty()) {
            S.ibase[s] = ib;
            ib += C * w;
        } else {
            // every lane r of the slice (rows s*C .. s*C+C-1, padding rows
            // included) reads column row + offset for every stored offset,
            // the padding offsets 0 included
            const int64_t lo = s * C + std::min<int64_t>(0, U[s].front());
            const int64_t hi = s * C + C - 1 + std::max<int64_t>(0, U[s].back());
            const int64_t inrange = (lo >= 0 && hi < n) ? 1 : 0;
            auto it = lists.find(U[s]);
            if (it == lists.end()) {
                it = lists.emplace(U[s], sh).first;
                sh += w;
                S.index_bytes += 4.0 * (double)U[s].size();
            }
            S.ibase[s] = -1 - (2 * it->second + inrange);
            S.nshared++;
        }
    }
    S.stored = S.soff[S.nslices];
    int maxd = 0;
    int64_t dnnz = 0, drows = 0;
    {
        std::mutex mx;
        parallel_for(S.nslices, [&](int64_t sb, int64_t se) {
            int m = 0;
            int64_t z = 0, nr = 0;
            for (int64_t s = sb; s < se; s++) {
                if (!U[s].empty()) continue;
                for (int64_t q = s * C; q < (s + 1) * C; q++) {
                    const int64_t r = rowof[q];
                    if (r < 0) continue;
                    for (int64_t k = K.rp[r] + 1; k < K.rp[r + 1]; k++) m = std::max(m, K.ci[k] - K.ci[k - 1]);
                    z += K.rp[r + 1] - K.rp[r];
                    nr++;
                }
            }
            std::lock_guard<std::mutex> g(mx);
            maxd = std::max(maxd, m);
            dnnz += z;
            drows += nr;
        }, 1);
    }
    S.idx16 = maxd <= 65535 ? 1 : 0;
    S.index_bytes += S.idx16 ? 2.0 * (double)dnnz + 4.0 * (double)drows : 4.0 * (double)dnnz;
    if (want64) S.v64.assign(S.stored, 0.0);
    if (want32) S.v32.assign(S.stored, 0.0f);
    if (ib > 0) {
        if (S.idx16) {
            S.d16.assign(ib, 0);
            S.col0.assign(S.nslices * C, 0);
        } else {
            S.c32.assign(ib, 0);
        }
    }
    S.shoff.assign(sh, 0);
    for (const auto &kv : lists) std::copy(kv.first.begin(), kv.first.end(), S.shoff.begin() + kv.second);
    // run table of each list for the block kernels' staged x windows: its
    // runs of consecutive offsets (o, o+1, ...), at most amgk::WIN_LMAX long, in
    // order from the list's position, packed as o * 16 + length, then 0; a
    // list with an offset beyond +-2^27 gets no table (first entry 0)
    S.shrun.assign(sh, 0);
    for (const auto &kv : lists) {
        const std::vector<int32_t> &u = kv.first;
        bool fits = true;
        for (int32_t o : u) fits = fits && o >= -(1 << 27) && o < (1 << 27);
        if (!fits) continue;
        int64_t rho = 0;
        for (size_t k = 0; k < u.size();) {
            size_t L = 1;
            while (L < (size_t)amgk::WIN_LMAX && k + L < u.size() && u[k + L] == u[k] + (int32_t)L) L++;
            S.shrun[kv.second + rho++] = u[k] * 16 + (int32_t)L;
            k += L;
        }
    }
    parallel_for(S.nslices, [&](int64_t sb, int64_t se) {
        for (int64_t s = sb; s < se; s++) {
            const int64_t base = S.soff[s];
            const int64_t w = (S.soff[s + 1] - base) / C;
            const bool sl = !U[s].empty();
            for (int lane = 0; lane < C; lane++) {
                const int64_t q = s * C + lane, r = rowof[q];
                const int64_t len = r >= 0 ? K.rp[r + 1] - K.rp[r] : 0;
                const int64_t r0 = r >= 0 ? K.rp[r] : 0;
                auto put = [&](int64_t k, double v) {
                    if (want64) S.v64[base + (k / 2) * 2 * C + lane * 2 + (k % 2)] = v;
                    if (want32) S.v32[base + (k / 4) * 4 * C + lane * 4 + (k % 4)] = (float)v;
                };
                if (sl) {
                    int64_t j = 0;
                    for (int64_t k = 0; k < (int64_t)U[s].size() && j < len; k++)
                        if (K.ci[r0 + j] - r == U[s][k]) put(k, K.v[r0 + j++]);
                    continue;
                }
                const int64_t ibs = S.ibase[s];
                if (S.idx16 && r >= 0) S.col0[q] = K.ci[r0];
                for (int64_t k = 0; k < w; k++) {
                    put(k, k < len ? K.v[r0 + k] : 0.0);
                    if (S.idx16) {
                        int d = (k >= 1 && k < len) ? K.ci[r0 + k] - K.ci[r0 + k - 1] : 0;
                        S.d16[ibs + (k / 8) * 8 * C + lane * 8 + (k % 8)] = (uint16_t)d;
                    } else {
                        int32_t c = k < len ? K.ci[r0 + k] : (len > 0 ? K.ci[r0 + len - 1] : 0);
                        S.c32[ibs + (k / 4) * 4 * C + lane * 4 + (k % 4)] = c;
                    }
                }
            }
        }
    }, 1);
}


// y = K x by walking the SELL-C image of K the way the device kernels do (see
// amg_sell_spmv_host in amg.h for the layouts); every column and window slot
// the walk reads is checked.  0, or AMG_ERR_STATE (-6) with a message.
void build_wg_stages(const SellHost &S, int C, int64_t nwg, int sigma, WgStages &W)
{
    W = WgStages();
    W.sigma = sigma;
    W.nwg = nwg;
    W.tab.assign(nwg * 8, 0);
    const int64_t slots = 4 * nwg, group = 4 * (int64_t)sigma, full = slots / group * group;
    auto slice_of = [&](int64_t b, int k) -> int64_t {
        if (4 * b < full) {
            const int64_t g = b / sigma, j = b % sigma;
            return g * group + j + (int64_t)k * sigma;
        }
        return 4 * b + k;
    };
    // a wave's runs: window-range start rows and lengths, in order
    auto runs_of = [&](int64_t s, std::vector<std::pair<int64_t, int>> &r) {
        r.clear();
        if (s >= S.nslices || S.ibase[s] >= 0) return;
        const int64_t e = -1 - S.ibase[s];
        const int32_t *rt = S.shrun.data() + (e >> 1);
        const int width = (int)((S.soff[s + 1] - S.soff[s]) / C);
        int k = 0;
        for (int rho = 0; k < width && rt[rho] != 0; rho++) {
            r.push_back({s * C + (rt[rho] >> 4), rt[rho] & 15});
            k += rt[rho] & 15;
        }
    };
    std::vector<int32_t> cnt(nwg, 0);
    std::vector<std::vector<int32_t>> per(nwg);
    parallel_for(nwg, [&](int64_t b0, int64_t b1) {
        std::vector<std::pair<int64_t, int>> r[4];
        for (int64_t b = b0; b < b1; b++) {
            size_t ptr[4] = {0, 0, 0, 0};
            for (int k = 0; k < 4; k++) {
                const int64_t s = slice_of(b, k);
                W.tab[8 * b + k] = (int32_t)s;
                runs_of(s, r[k]);
            }
            std::vector<int32_t> &out = per[b];
            for (;;) {
                int64_t g0 = INT64_MAX;
                for (int k = 0; k < 4; k++)
                    if (ptr[k] < r[k].size()) g0 = std::min(g0, r[k][ptr[k]].first);
                if (g0 == INT64_MAX) break;
                uint32_t info = 0;
                for (int k = 0; k < 4; k++) {
                    if (ptr[k] >= r[k].size()) continue;
                    const int64_t shift = r[k][ptr[k]].first - g0;
                    if (shift + C - 1 + r[k][ptr[k]].second > amgk::WIN_WG_ROWS) continue;
                    info |= (uint32_t)(0x80 | shift) << (8 * k);
                    ptr[k]++;
                }
                out.push_back((int32_t)g0);
                out.push_back((int32_t)info);
            }
            cnt[b] = (int32_t)(out.size() / 2);
        }
    });
    int64_t total = 0;
    for (int64_t b = 0; b < nwg; b++) {
        W.tab[8 * b + 4] = (int32_t)total;
        W.tab[8 * b + 5] = cnt[b];
        total += cnt[b];
    }
    W.st.resize(2 * total);
    parallel_for(nwg, [&](int64_t b0, int64_t b1) {
        for (int64_t b = b0; b < b1; b++) std::copy(per[b].begin(), per[b].end(), W.st.begin() + 2 * (int64_t)W.tab[8 * b + 4]);
    });
    W.copied_rows = total * amgk::WIN_WG_ROWS;
    int64_t runs = 0;
    for (int64_t t = 0; t < total; t++)
        for (int k = 0; k < 4; k++) runs += (W.st[2 * t + 1] >> (8 * k)) & 0x80 ? 1 : 0;
    W.runs = runs;
}

void choose_wg_stages(const SellHost &S, int C, int64_t nwg, WgStages &W)
{
    W = WgStages();
    for (int sigma = 1; sigma <= 4; sigma++) {
        WgStages T;
        build_wg_stages(S, C, nwg, sigma, T);
        if (W.sigma == 0 || T.copied_rows < W.copied_rows) W = std::move(T);
    }
}

int sell_spmv_walk(const CsrView &K, int64_t ncols, int C, int layout, const double *x, double *y,
                   int64_t *shared_slices, int64_t *stored, std::string &err)
{
    auto fail = [&](const char *m) { err = m; return -6; };
    const int64_t n = K.n;
    SellHost S;
    build_sell(K, C, true, false, layout == 1 || layout >= 3, layout == 2 ? 4 * C : 0, S);
    const int32_t hi = (int32_t)(ncols - 1);
    auto bad = [&](int64_t c) { return c < 0 || c > hi; };
    if (layout == 3) {
        // shared-offset slices walked as the block kernels' staged x windows:
        // per run of the run table, window rows g0 + w (w < 63 + L, clamped
        // where the slice needs it) are copied, then lane r reads window row
        // r + t for the run's t-th entry; every row copied and every window
        // slot read is checked
        std::vector<double> win(amgk::WIN_ROWS);
        for (int64_t s = 0; s < S.nslices; s++) {
            const int64_t ib = S.ibase[s];
            if (ib >= 0) continue;   // per-row-index slices: the gather path of layout 1
            const int64_t base = S.soff[s];
            const int width = (int)((S.soff[s + 1] - base) / C);
            const int64_t e = -1 - ib;
            if ((e >> 1) + width > (int64_t)S.shoff.size()) { return fail("offset list past its array"); }
            const int32_t *so = S.shoff.data() + (e >> 1), *rt = S.shrun.data() + (e >> 1);
            if (rt[0] == 0) {
                // no run table: the gather walk below
                continue;
            }
            std::vector<double> acc(C, 0.0);
            int k = 0;
            for (int rho = 0; k < width; rho++) {
                const int32_t pk = rt[rho];
                if (pk == 0) break;
                const int L = pk & 15;
                if (L < 1 || L > amgk::WIN_LMAX || k + L > width) { return fail("run past the list or too long"); }
                if ((pk >> 4) != so[k]) { return fail("run table and offset list disagree"); }
                for (int t = 1; t < L; t++)
                    if (so[k + t] != so[k] + t) { return fail("run of non-consecutive offsets"); }
                const int64_t g0 = s * C + so[k];
                for (int w = 0; w < C + L - 1; w++) {
                    int64_t g = g0 + w;
                    if (!(e & 1)) g = std::min<int64_t>(std::max<int64_t>(g, 0), hi);
                    if (bad(g) || w >= amgk::WIN_ROWS) { return fail("window row out of range"); }
                    win[w] = x[g];
                }
                for (int r = 0; r < C; r++)
                    for (int t = 0; t < L; t++) {
                        if (r + t >= C + L - 1) { return fail("window slot not staged"); }
                        const int kk = k + t;
                        acc[r] = std::fma(S.v64[base + (kk / 2) * 2 * C + r * 2 + (kk % 2)], win[r + t], acc[r]);
                    }
                k += L;
            }
            for (int r = 0; r < C; r++)
                if (s * C + r < n) y[s * C + r] = acc[r];
        }
    }
    if (layout == 4) {
        // the same slices walked through the block stage tables: per block of
        // four slices, per stage, the window rows g0 + w (w < WIN_WG_ROWS,
        // clamped) are copied once, and every wave taking part sums its next
        // run from the window rows at its shift; every run of every slice must
        // be taken exactly once, in order
        amgiga::WgStages W;
        const int64_t nwg = (S.nslices + 3) / 4;
        choose_wg_stages(S, C, nwg, W);
        std::vector<char> seen(4 * nwg, 0);
        std::vector<double> win(amgk::WIN_WG_ROWS);
        for (int64_t b = 0; b < nwg; b++) {
            int64_t sl[4];
            int kk[4] = {0, 0, 0, 0}, rho[4] = {0, 0, 0, 0}, width[4] = {0, 0, 0, 0};
            const int32_t *rt[4] = {nullptr, nullptr, nullptr, nullptr};
            std::vector<double> acc(4 * (size_t)C, 0.0);
            for (int k = 0; k < 4; k++) {
                sl[k] = W.tab[8 * b + k];
                if (sl[k] < 0 || sl[k] >= 4 * nwg || seen[sl[k]]) { return fail("block table: slice missing or twice"); }
                seen[sl[k]] = 1;
                if (sl[k] < S.nslices && S.ibase[sl[k]] < 0) {
                    const int64_t e = -1 - S.ibase[sl[k]];
                    if (S.shrun[e >> 1] != 0) rt[k] = S.shrun.data() + (e >> 1);
                    width[k] = (int)((S.soff[sl[k] + 1] - S.soff[sl[k]]) / C);
                }
            }
            const int64_t t0 = W.tab[8 * b + 4], nst = W.tab[8 * b + 5];
            if (t0 < 0 || t0 + nst > (int64_t)W.st.size() / 2) { return fail("stage list past its array"); }
            for (int64_t t = t0; t < t0 + nst; t++) {
                const int64_t g0 = W.st[2 * t];
                for (int w = 0; w < amgk::WIN_WG_ROWS; w++) win[w] = x[std::min<int64_t>(std::max<int64_t>(g0 + w, 0), hi)];
                for (int k = 0; k < 4; k++) {
                    const int me = (W.st[2 * t + 1] >> (8 * k)) & 0xFF;
                    if (!(me & 0x80)) continue;
                    if (!rt[k] || kk[k] >= width[k] || rt[k][rho[k]] == 0) { return fail("stage for a wave without a run"); }
                    const int32_t pk = rt[k][rho[k]];
                    const int L = pk & 15, sh = me & 0x7F;
                    if (L < 1 || L > amgk::WIN_LMAX || kk[k] + L > width[k]) { return fail("run past the list or too long"); }
                    if (sl[k] * C + (pk >> 4) != g0 + sh) { return fail("run not at its window shift"); }
                    if (sh + C - 1 + L > amgk::WIN_WG_ROWS) { return fail("run past its window"); }
                    const int64_t base = S.soff[sl[k]];
                    for (int r = 0; r < C; r++)
                        for (int u = 0; u < L; u++) {
                            const int e2 = kk[k] + u;
                            acc[k * C + r] = std::fma(S.v64[base + (e2 / 2) * 2 * C + r * 2 + (e2 % 2)], win[sh + r + u],
                                                      acc[k * C + r]);
                        }
                    kk[k] += L;
                    rho[k]++;
                }
            }
            for (int k = 0; k < 4; k++) {
                if (!rt[k]) continue;
                if (kk[k] < width[k] && rt[k][rho[k]] != 0) { return fail("runs left after the last stage"); }
                for (int r = 0; r < C; r++)
                    if (sl[k] * C + r < n) y[sl[k] * C + r] = acc[k * C + r];
            }
        }
    }
    for (int64_t s = 0; s < S.nslices; s++) {
        if (layout >= 3 && S.ibase[s] < 0 && S.shrun[(-1 - S.ibase[s]) >> 1] != 0) continue;
        const int64_t base = S.soff[s];
        const int width = (int)((S.soff[s + 1] - base) / C);
        const int64_t ib = S.ibase[s];
        for (int r = 0; r < C; r++) {
            const int64_t slot = s * C + r;
            const int64_t row = S.sorted ? (int64_t)S.perm[slot] : (slot < n ? slot : -1);
            double acc = 0.0;
            if (ib < 0) {
                if (S.sorted) { return fail("shared offsets in a sorted image"); }
                const int64_t e = -1 - ib;
                const int32_t *so = S.shoff.data() + (e >> 1);
                if ((e >> 1) + width > (int64_t)S.shoff.size()) { return fail("offset list past its array"); }
                for (int k = 0; k < width; k++) {
                    int64_t c = slot + so[k];
                    if (!(e & 1)) c = std::min<int64_t>(std::max<int64_t>(c, 0), hi);
                    if (bad(c)) { return fail("shared-offset column out of range"); }
                    acc = std::fma(S.v64[base + (k / 2) * 2 * C + r * 2 + (k % 2)], x[c], acc);
                }
            } else if (S.idx16) {
                int64_t c = S.col0.empty() ? 0 : S.col0[slot];
                for (int k = 0; k < width; k++) {
                    const int64_t q = ib + (k / 8) * 8 * C + r * 8 + (k % 8);
                    if (q >= (int64_t)S.d16.size()) { return fail("delta stream past its array"); }
                    c += S.d16[q];
                    if (bad(c)) { return fail("delta column out of range"); }
                    acc = std::fma(S.v64[base + (k / 2) * 2 * C + r * 2 + (k % 2)], x[c], acc);
                }
            } else {
                for (int k = 0; k < width; k++) {
                    const int64_t q = ib + (k / 4) * 4 * C + r * 4 + (k % 4);
                    if (q >= (int64_t)S.c32.size()) { return fail("column stream past its array"); }
                    const int64_t c = S.c32[q];
                    if (bad(c)) { return fail("int32 column out of range"); }
                    acc = std::fma(S.v64[base + (k / 2) * 2 * C + r * 2 + (k % 2)], x[c], acc);
                }
            }
            if (row >= 0) y[row] = acc;
        }
    }
    if (shared_slices) *shared_slices = S.nshared;
    if (stored) *stored = S.stored;
    return 0;
}

}  // namespace amgiga
