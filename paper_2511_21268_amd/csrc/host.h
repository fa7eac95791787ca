// Host-side hierarchy of the matching-based AMG (paper Sec. 3.1) and the IgA
// workload generator (Sec. 2).  Compiled by g++ with -ffp-contract=off: the
// aggregates and Galerkin matrices are fixed to the bit by the evaluation order
// written in host_setup.cpp.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

#include "layout.h"

namespace amgiga {

struct Csr {
    int64_t n = 0;
    std::vector<int64_t> rp;
    std::vector<int32_t> ci;
    std::vector<double> v;
    int64_t nnz() const { return rp.empty() ? 0 : rp[n]; }
};

// A borrowed CSR (the caller's arrays, or a Csr's).
struct CsrView {
    int64_t n = 0;
    const int64_t *rp = nullptr;
    const int32_t *ci = nullptr;
    const double *v = nullptr;
    int64_t nnz() const { return rp[n]; }
};

inline CsrView view(const Csr &a) { return CsrView{a.n, a.rp.data(), a.ci.data(), a.v.data()}; }

struct SetupParams {
    int sweeps = 2;
    int max_coarse = 200;
    int max_levels = 40;
    int positive_only = 0;
    int smooth = 0;              // smoothed prolongator (I - omega D^{-1} K) P
    double omega = 4.0 / 3.0;
    int coarse_dense = 1;        // dense lower triangle of the coarsest matrix
    int bootstrap = 0;           // > 0: w from this many relaxation sweeps on K w = 0
};

struct HostLevel {
    int64_t n = 0, nnz = 0;
    Csr K;                       // Galerkin matrix (empty for level 0: caller's)
    std::vector<double> invd;    // 1 / l1 diagonal
    std::vector<double> w;       // test vector of this level
    std::vector<int32_t> agg;    // coarse index of each row (not on coarsest)
    std::vector<double> pc;      // prolongator coefficient of each row
    Csr P, PT;                   // smoothed prolongator (n x nc) and its transpose, if built
    int max_members = 0;         // largest aggregate size into the next level
    float feat[6] = {0, 0, 0, 0, 0, 0};  // level features independent of the depth
};

struct HostHierarchy {
    std::vector<HostLevel> lev;  // lev.back() is the coarsest (factored) level
    std::vector<double> coarse_lower;  // dense n_L x n_L, lower triangle of K_L
};

// One level's coarsening: m composed pairwise sweeps (matching, pairwise
// prolongator, Galerkin product) from (K, w) to the coarse matrix and test
// vector, with the composed aggregate map and coefficients.
struct CoarsenResult {
    int64_t nc = 0;
    std::vector<int32_t> agg;
    std::vector<double> pc, wc;
    Csr C;
};

// Alternative executor of the set-up steps (the device one); results must be
// the host's bits.
struct Coarsener {
    virtual ~Coarsener() {}
    // w = `sweeps` l1-Jacobi sweeps on K w = 0 from w0
    virtual void bootstrap(const CsrView &K0, const double *w0, int sweeps, std::vector<double> &w) = 0;
    virtual void coarsen(int level, const CsrView &K, const double *w, const SetupParams &prm, CoarsenResult &out) = 0;
};

// Status codes follow amg_status.
int validate_csr(const CsrView &K, std::string &err);
int build_hierarchy(const CsrView &K0, const double *w, const SetupParams &prm,
                    HostHierarchy &H, std::string &err, Coarsener *dev = nullptr);
// Test vector on the host: `sweeps` l1-Jacobi sweeps on K w = 0 from w0, each
// row sum ascending from +0.0, w_i <- w_i - invd_i s_i.
void bootstrap_w(const CsrView &K, const double *w0, int sweeps, std::vector<double> &w);

// Features of a level for the learned smoother (the first six of eight; the
// relative depth and the coarsening ratio are added once the hierarchy is known):
// log10(n)/7, (nnz/n)/1000, mean and min of k_ii/d_i, mean of sum_{j!=i} k_ij/d_i,
// fraction of positive off-diagonal entries.
void level_features(const CsrView &K, const std::vector<double> &invd, float out[6]);

// K P for a one-entry-per-row prolongator (agg, pc): n x nc CSR with
// (KP)_{iJ} = sum over the stored j of row i with agg(j) = J of k_ij pc_j,
// accumulated in ascending j, columns ascending.  Used by the fused
// prolongation + post-smoothing pass: f - K (u + P e) = r - (K P) e.
Csr kp_product(const CsrView &K, int64_t nc, const int32_t *agg, const double *pc);

// Smoothed prolongator P' = (I - omega D^{-1} K) P on the pattern of K P:
// P'_iJ = [J = agg(i)] pc_i - (omega invd_i) (K P)_iJ, and its Galerkin
// product (P'^T K) P': B_Ij = sum over i ascending of P'_iI k_ij, then
// K_c,IJ = sum over j ascending of B_Ij P'_jJ (parallel over coarse rows).
Csr smooth_prolongator(const CsrView &K, const std::vector<double> &invd, int64_t nc, const int32_t *agg,
                       const double *pc, double omega);
Csr transpose(const Csr &P, int64_t ncols);
Csr galerkin_general(const CsrView &K, const Csr &P, const Csr &PT);

// Pieces exposed for the unit tests of the library's own setup.
double cij(double kij, double kii, double kjj, double wi, double wj);
void suitor_match(const CsrView &K, const double *w, int positive_only, int32_t *mate);

// Workload generator.
void iga_size(int d, int p, int n, int64_t *N, int64_t *nnz);
int iga_poisson(int d, int p, int n, int64_t *rp, int32_t *ci, double *v, double *F);
void iga_cube_size(int p, int n, int64_t *N, int64_t *nnz);
int iga_cube(int p, int n, int64_t *rp, int32_t *ci, double *v, double *F);
int iga_diffusion(int p, int n, int nk, const double *a, const int32_t *mk, int64_t *rp, int32_t *ci, double *v,
                  double *F);

// SELL-C image of a matrix as the device kernels read it (layout described in
// kernels.h): per-slice value offsets soff, index-stream bases ibase (< 0: a
// shared column-offset list at shoff, with its run table in shrun), values in
// FP64 and/or FP32, 16-bit deltas with first columns or int32 columns, and the
// slot -> row map of sorted images.
struct SellHost {
    int64_t nslices = 0, stored = 0, nshared = 0;
    int sorted = 0;
    std::vector<int32_t> perm;
    double index_bytes = 0.0;   // index data a pass must read (no padding)
    int idx16 = 1;
    std::vector<int64_t> soff, ibase;
    std::vector<double> v64;
    std::vector<float> v32;
    std::vector<uint16_t> d16;
    std::vector<int32_t> c32, col0, shoff, shrun;
};
// Windows shared by the four waves (slices) of a workgroup in the block
// kernels: logical workgroup b holds slices tab[8b .. 8b+3] (ids past the last
// slice: none) and, in order, stages st[2 tab[8b+4]] .. of count tab[8b+5];
// stage t copies X rows st[2t] .. st[2t] + WIN_WG_ROWS - 1 and byte k of st[2t+1]
// says whether wave k sums its next run from it (bit 7) and at which row of the
// window that run's range starts (bits 0-6).  Each wave's runs are taken in
// order.  Slices are grouped by stride sigma: groups of 4 sigma consecutive
// slices make sigma workgroups of every sigma-th slice (so that with sigma
// slices per grid line the windows of neighbouring lines coincide); slices
// past the last full group go four consecutive ones per workgroup.
struct WgStages {
    int sigma = 0;
    int64_t nwg = 0, copied_rows = 0, runs = 0;
    std::vector<int32_t> tab, st;
};
void build_wg_stages(const SellHost &S, int C, int64_t nwg, int sigma, WgStages &W);
// the stride of 1..4 with the fewest copied window rows
void choose_wg_stages(const SellHost &S, int C, int64_t nwg, WgStages &W);
std::vector<int32_t> slice_offsets(const CsrView &K, int64_t s, int C, int64_t limit);
int64_t count_shared(const CsrView &K, int C);
void build_sell(const CsrView &K, int C, bool want64, bool want32, bool shared, int sigma, SellHost &S);
// y = K x walked through the image as the kernels walk it (layouts of
// amg_sell_spmv_host); 0, or -6 with err set when a read would leave its array.
int sell_spmv_walk(const CsrView &K, int64_t ncols, int C, int layout, const double *x, double *y,
                   int64_t *shared_slices, int64_t *stored, std::string &err);

// Runs f(begin, end) over [0, n) split in contiguous chunks on host threads
// (serially when n < serial_below).
template <class F> void parallel_for(int64_t n, F f, int64_t serial_below = 4096);

}  // namespace amgiga

#include <thread>
namespace amgiga {
int host_threads();
template <class F> void parallel_for(int64_t n, F f, int64_t serial_below)
{
    int nt = host_threads();
    if (n < serial_below || nt <= 1) { f((int64_t)0, n); return; }
    std::vector<std::thread> th;
    int64_t chunk = (n + nt - 1) / nt;
    for (int t = 0; t < nt; t++) {
        int64_t b = t * chunk, e = b + chunk < n ? b + chunk : n;
        if (b >= e) break;
        th.emplace_back([=]() { f(b, e); });
    }
    for (auto &x : th) x.join();
}
}  // namespace amgiga
