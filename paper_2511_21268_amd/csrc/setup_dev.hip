// Device execution of the hierarchy set-up (Sec. 3.1): the test vector by
// relaxation on K w = 0, the compatible weighted matching, the pairwise
// prolongator and the Galerkin product, with the same bits as the host
// set-up in host_setup.cpp.  Built without FMA contraction; every sum runs in
// the host's order.
//
//  * Matching: rounds of locally dominant edges.  In each round every free
//    vertex points to its best eligible free neighbour in the strict order
//    (c descending, smaller end ascending, larger end ascending) and mutual
//    pointers are matched.  The best remaining edge is always mutual, so every
//    round with a candidate matches at least one pair (at most n/2 rounds), and
//    an edge matched this way is never preceded in the order by an edge that
//    could take one of its ends: the result is the greedy matching.
//  * Galerkin product for a one-entry-per-row prolongator: the contribution of
//    stored entry e (row i, column j) is (pc_i k_e) pc_j at coarse position
//    (agg_i, agg_j); the host adds the contributions of a position in
//    ascending e.  Entry indices are sorted by position with a stable radix
//    sort, and one thread per position sums its run in that order from +0.0.
#include "setup_dev.h"

#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include <cmath>
#include <cstdint>
#include <stdexcept>
#include <vector>

namespace amgiga {
namespace {

#pragma clang fp contract(off)

struct HipError : std::runtime_error {
    using std::runtime_error::runtime_error;
};
struct InputError : std::runtime_error {
    using std::runtime_error::runtime_error;
};

#define DCHK(x)                                                                                      \
    do {                                                                                             \
        hipError_t e_ = (x);                                                                         \
        if (e_ != hipSuccess) throw HipError(std::string("HIP error in set-up: ") + hipGetErrorString(e_)); \
    } while (0)

template <typename T> struct DBuf {
    T *p = nullptr;
    size_t n = 0;
    DBuf() = default;
    explicit DBuf(size_t k) { alloc(k); }
    void alloc(size_t k)
    {
        release();
        n = k;
        if (k) DCHK(hipMalloc((void **)&p, k * sizeof(T)));
    }
    void release()
    {
        if (p) (void)hipFree(p);
        p = nullptr;
        n = 0;
    }
    ~DBuf() { release(); }
    DBuf(const DBuf &) = delete;
    DBuf &operator=(const DBuf &) = delete;
    DBuf(DBuf &&o) noexcept : p(o.p), n(o.n) { o.p = nullptr; o.n = 0; }
    DBuf &operator=(DBuf &&o) noexcept
    {
        release();
        p = o.p; n = o.n; o.p = nullptr; o.n = 0;
        return *this;
    }
};

inline unsigned grid(int64_t n) { return (unsigned)((n + 255) / 256); }

// ---- kernels --------------------------------------------------------------

__global__ void k_diag(int64_t n, const int64_t *__restrict__ rp, const int32_t *__restrict__ ci,
                       const double *__restrict__ v, double *__restrict__ diag)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double d = 0.0;
    for (int64_t k = rp[i]; k < rp[i + 1]; k++)
        if (ci[k] == i) d = v[k];
    diag[i] = d;
}

// 1 / (k_ii + sum_{j != i} |k_ij|), the sum in ascending j after k_ii
__global__ void k_l1_invdiag(int64_t n, const int64_t *__restrict__ rp, const int32_t *__restrict__ ci,
                             const double *__restrict__ v, double *__restrict__ invd)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double d = 0.0;
    for (int64_t k = rp[i]; k < rp[i + 1]; k++)
        if (ci[k] == i) d = v[k];
    for (int64_t k = rp[i]; k < rp[i + 1]; k++)
        if (ci[k] != i) d = d + fabs(v[k]);
    invd[i] = 1.0 / d;
}

// one relaxation sweep on K w = 0: wout_i = w_i - invd_i sum_j k_ij w_j
__global__ void k_boot_sweep(int64_t n, const int64_t *__restrict__ rp, const int32_t *__restrict__ ci,
                             const double *__restrict__ v, const double *__restrict__ invd,
                             const double *__restrict__ w, double *__restrict__ wout)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double t = 0.0;
    for (int64_t k = rp[i]; k < rp[i + 1]; k++) t = t + v[k] * w[ci[k]];
    wout[i] = w[i] - invd[i] * t;
}

__device__ inline double cij_dev(double kij, double kii, double kjj, double wi, double wj)
{
    double num = ((2.0 * kij) * wi) * wj;
    double den = (kii * wi) * wi + (kjj * wj) * wj;
    return 1.0 - num / den;
}

__device__ inline int64_t find_col(const int64_t *rp, const int32_t *ci, int64_t row, int32_t col)
{
    int64_t lo = rp[row], hi = rp[row + 1] - 1;
    while (lo <= hi) {
        int64_t mid = (lo + hi) >> 1;
        int32_t c = ci[mid];
        if (c == col) return mid;
        if (c < col) lo = mid + 1;
        else hi = mid - 1;
    }
    return -1;
}

// c of every stored entry (value of row min(i, j)); NaN marks an ineligible
// entry.  cnt[0] counts entries below the diagonal without a stored transpose.
__global__ void k_edge_c(int64_t n, const int64_t *__restrict__ rp, const int32_t *__restrict__ ci,
                         const double *__restrict__ v, const double *__restrict__ diag, const double *__restrict__ w,
                         int positive_only, double *__restrict__ cw, unsigned long long *cnt)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    unsigned long long missing = 0;
    for (int64_t k = rp[i]; k < rp[i + 1]; k++) {
        const int64_t j = ci[k];
        double val = __builtin_nan("");
        if (j != i) {
            double kv;
            if (i < j) {
                kv = v[k];
                if (find_col(rp, ci, j, (int32_t)i) < 0) missing++;
            } else {
                const int64_t t = find_col(rp, ci, j, (int32_t)i);
                if (t < 0) missing++;
                kv = t >= 0 ? v[t] : 0.0;
            }
            if (kv != 0.0) {
                const int64_t a = i < j ? i : j, b = i < j ? j : i;
                const double c = cij_dev(kv, diag[a], diag[b], w[a], w[b]);
                const bool ok = isfinite(c) && (!positive_only || c > 1.0);
                if (ok) val = c;
            }
        }
        cw[k] = val;
    }
    if (missing) atomicAdd(cnt, missing);
}

__device__ inline bool precedes(double c, int64_t a, int64_t b, double c2, int64_t a2, int64_t b2)
{
    if (c != c2) return c > c2;
    if (a != a2) return a < a2;
    return b < b2;
}

// every free vertex points to its best eligible free neighbour (or -1)
__global__ void k_ld_point(int64_t n, const int64_t *__restrict__ rp, const int32_t *__restrict__ ci,
                           const double *__restrict__ cw, const int32_t *__restrict__ mate,
                           int32_t *__restrict__ ptr, unsigned int *any)
{
    int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= n) return;
    if (mate[u] >= 0) { ptr[u] = -1; return; }
    int64_t best = -1, ba = 0, bb = 0;
    double bc = 0.0;
    for (int64_t k = rp[u]; k < rp[u + 1]; k++) {
        const double c = cw[k];
        if (c != c) continue;
        const int64_t v = ci[k];
        if (mate[v] >= 0) continue;
        const int64_t a = u < v ? u : v, b = u < v ? v : u;
        if (best >= 0 && !precedes(c, a, b, bc, ba, bb)) continue;
        best = v; bc = c; ba = a; bb = b;
    }
    ptr[u] = (int32_t)best;
    if (best >= 0) atomicOr(any, 1u);
}

__global__ void k_ld_match(int64_t n, const int32_t *__restrict__ ptr, int32_t *__restrict__ mate)
{
    int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= n) return;
    const int32_t v = ptr[u];
    if (v >= 0 && ptr[v] == (int32_t)u) mate[u] = v;
}

__global__ void k_fill_i32(int64_t n, int32_t val, int32_t *__restrict__ d)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) d[i] = val;
}

// 1 where row i opens a coarse index (singleton or the smaller of its pair)
__global__ void k_open(int64_t n, const int32_t *__restrict__ mate, int32_t *__restrict__ flag)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t m = mate[i];
    flag[i] = (m < 0 || i < m) ? 1 : 0;
}

// coarse index by the smallest member, pairwise prolongator coefficient and
// the restricted test vector (eq. (prolongation))
__global__ void k_pairwise(int64_t n, const int32_t *__restrict__ mate, const double *__restrict__ w,
                           const int32_t *__restrict__ idx, int32_t *__restrict__ agg, double *__restrict__ pc,
                           double *__restrict__ wc)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t j = mate[i];
    const int32_t I = (j < 0 || i < j) ? idx[i] : idx[j];
    agg[i] = I;
    if (j >= 0) {
        const double s = sqrt(w[i] * w[i] + w[j] * w[j]);
        pc[i] = w[i] / s;
        if (i < j) wc[I] = s;
    } else {
        pc[i] = (w[i] != 0.0) ? w[i] / fabs(w[i]) : 1.0;
        wc[I] = fabs(w[i]);
    }
}

// sort keys (coarse row, coarse column), entry indices and contributions
__global__ void k_gal_keys(int64_t n, const int64_t *__restrict__ rp, const int32_t *__restrict__ ci,
                           const double *__restrict__ v, const int32_t *__restrict__ agg, const double *__restrict__ pc,
                           uint64_t *__restrict__ keys, int32_t *__restrict__ vals, double *__restrict__ t)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint64_t I = (uint64_t)(uint32_t)agg[i];
    const double pi = pc[i];
    for (int64_t k = rp[i]; k < rp[i + 1]; k++) {
        const int32_t j = ci[k];
        keys[k] = (I << 32) | (uint64_t)(uint32_t)agg[j];
        vals[k] = (int32_t)k;
        t[k] = (pi * v[k]) * pc[j];
    }
}

__global__ void k_run_heads(int64_t m, const uint64_t *__restrict__ keys, int32_t *__restrict__ head)
{
    int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= m) return;
    head[s] = (s == 0 || keys[s] != keys[s - 1]) ? 1 : 0;
}

__global__ void k_run_starts(int64_t m, const int32_t *__restrict__ head, const int64_t *__restrict__ runid,
                             int64_t *__restrict__ start)
{
    int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= m) return;
    if (head[s]) start[runid[s]] = s;
}

// one thread per coarse position: the run's contributions in ascending entry
// index, from +0.0; the column, and a count per coarse row
__global__ void k_run_sums(int64_t nrun, const int64_t *__restrict__ start, const uint64_t *__restrict__ keys,
                           const int32_t *__restrict__ vals, const double *__restrict__ t, int32_t *__restrict__ cci,
                           double *__restrict__ cv, int64_t *__restrict__ rowcnt)
{
    int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= nrun) return;
    double acc = 0.0;
    for (int64_t s = start[g]; s < start[g + 1]; s++) acc = acc + t[vals[s]];
    cv[g] = acc;
    const uint64_t key = keys[start[g]];
    cci[g] = (int32_t)(uint32_t)(key & 0xffffffffull);
    atomicAdd((unsigned long long *)&rowcnt[key >> 32], 1ull);
}

__global__ void k_compose(int64_t n, int32_t *__restrict__ agg, double *__restrict__ pc,
                          const int32_t *__restrict__ ag, const double *__restrict__ pcs)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t a = agg[i];
    pc[i] = pc[i] * pcs[a];
    agg[i] = ag[a];
}

// ---- host driver ----------------------------------------------------------

struct DevCsr {
    int64_t n = 0, nnz = 0;
    DBuf<int64_t> rp;
    DBuf<int32_t> ci;
    DBuf<double> v;
};

template <typename T> void up(DBuf<T> &d, const T *h, size_t k, hipStream_t s)
{
    d.alloc(k);
    if (k) DCHK(hipMemcpyAsync(d.p, h, k * sizeof(T), hipMemcpyHostToDevice, s));
}
template <typename T> void down(std::vector<T> &h, const DBuf<T> &d, size_t k, hipStream_t s)
{
    h.resize(k);
    if (k) DCHK(hipMemcpyAsync(h.data(), d.p, k * sizeof(T), hipMemcpyDeviceToHost, s));
}

class DeviceCoarsener : public Coarsener {
  public:
    DeviceCoarsener(hipStream_t s, DevSetupInfo *info) : s_(s), info_(info) {}

    void bootstrap(const CsrView &K0, const double *w0, int sweeps, std::vector<double> &w) override
    {
        DevCsr &K = level0(K0);
        DBuf<double> invd(K.n), a(K.n), b(K.n);
        hipLaunchKernelGGL(k_l1_invdiag, dim3(grid(K.n)), dim3(256), 0, s_, K.n, K.rp.p, K.ci.p, K.v.p, invd.p);
        DCHK(hipMemcpyAsync(a.p, w0, K.n * sizeof(double), hipMemcpyHostToDevice, s_));
        for (int k = 0; k < sweeps; k++) {
            hipLaunchKernelGGL(k_boot_sweep, dim3(grid(K.n)), dim3(256), 0, s_, K.n, K.rp.p, K.ci.p, K.v.p, invd.p,
                               a.p, b.p);
            std::swap(a.p, b.p);
        }
        DCHK(hipGetLastError());
        down(w, a, K.n, s_);
        DCHK(hipStreamSynchronize(s_));
    }

    void coarsen(int level, const CsrView &Kh, const double *w, const SetupParams &prm, CoarsenResult &out) override
    {
        DevCsr &K0 = level == 0 ? level0(Kh) : cur_;
        if (K0.n != Kh.n || K0.nnz != Kh.nnz()) throw HipError("device set-up: level matrix out of step");
        const int64_t nl = K0.n;
        DBuf<int32_t> agg(nl);
        DBuf<double> pc(nl);
        DBuf<double> wv;
        up(wv, w, nl, s_);
        DevCsr C;
        const DevCsr *K = &K0;
        DBuf<double> wcur = std::move(wv);
        int64_t nc = nl;
        for (int sw = 0; sw < prm.sweeps; sw++) {
            DBuf<int32_t> mate(K->n), ag(K->n);
            DBuf<double> pcs(K->n), wc;
            match(*K, wcur.p, prm.positive_only, mate.p);
            nc = pairwise(*K, mate.p, wcur.p, ag, pcs, wc);
            DevCsr Cn = galerkin(*K, nc, ag.p, pcs.p);
            if (sw == 0) {
                DCHK(hipMemcpyAsync(agg.p, ag.p, nl * sizeof(int32_t), hipMemcpyDeviceToDevice, s_));
                DCHK(hipMemcpyAsync(pc.p, pcs.p, nl * sizeof(double), hipMemcpyDeviceToDevice, s_));
            } else {
                hipLaunchKernelGGL(k_compose, dim3(grid(nl)), dim3(256), 0, s_, nl, agg.p, pc.p, ag.p, pcs.p);
                DCHK(hipGetLastError());
            }
            C = std::move(Cn);
            K = &C;
            wcur = std::move(wc);
        }
        out.nc = nc;
        down(out.agg, agg, nl, s_);
        down(out.pc, pc, nl, s_);
        down(out.wc, wcur, nc, s_);
        out.C.n = C.n;
        down(out.C.rp, C.rp, C.n + 1, s_);
        down(out.C.ci, C.ci, C.nnz, s_);
        down(out.C.v, C.v, C.nnz, s_);
        DCHK(hipStreamSynchronize(s_));
        cur_ = std::move(C);
    }

  private:
    hipStream_t s_;
    DevSetupInfo *info_;
    DevCsr l0_, cur_;
    bool have_l0_ = false;

    DevCsr &level0(const CsrView &K)
    {
        if (!have_l0_) {
            l0_.n = K.n;
            l0_.nnz = K.nnz();
            up(l0_.rp, K.rp, K.n + 1, s_);
            up(l0_.ci, K.ci, K.nnz(), s_);
            up(l0_.v, K.v, K.nnz(), s_);
            have_l0_ = true;
        }
        return l0_;
    }

    template <typename F> size_t cub_bytes(F f)
    {
        size_t b = 0;
        DCHK(f(nullptr, b));
        return b;
    }

    void scan_i32_to_i32(const int32_t *in, int32_t *out, int64_t n)
    {
        size_t b = 0;
        DCHK(hipcub::DeviceScan::ExclusiveSum(nullptr, b, in, out, (int)n, s_));
        DBuf<char> tmp(b ? b : 1);
        DCHK(hipcub::DeviceScan::ExclusiveSum(tmp.p, b, in, out, (int)n, s_));
    }
    void scan_i32_to_i64(const int32_t *in, int64_t *out, int64_t n)
    {
        size_t b = 0;
        DCHK(hipcub::DeviceScan::ExclusiveSum(nullptr, b, in, out, (int)n, s_));
        DBuf<char> tmp(b ? b : 1);
        DCHK(hipcub::DeviceScan::ExclusiveSum(tmp.p, b, in, out, (int)n, s_));
    }
    void scan_i64(const int64_t *in, int64_t *out, int64_t n)
    {
        size_t b = 0;
        DCHK(hipcub::DeviceScan::ExclusiveSum(nullptr, b, in, out, (int)n, s_));
        DBuf<char> tmp(b ? b : 1);
        DCHK(hipcub::DeviceScan::ExclusiveSum(tmp.p, b, in, out, (int)n, s_));
    }

    void match(const DevCsr &K, const double *w, int positive_only, int32_t *mate)
    {
        DBuf<double> diag(K.n), cw(K.nnz ? K.nnz : 1);
        DBuf<unsigned long long> cnt(1);
        DBuf<unsigned int> any(1);
        DBuf<int32_t> ptr(K.n);
        DCHK(hipMemsetAsync(cnt.p, 0, sizeof(unsigned long long), s_));
        hipLaunchKernelGGL(k_diag, dim3(grid(K.n)), dim3(256), 0, s_, K.n, K.rp.p, K.ci.p, K.v.p, diag.p);
        hipLaunchKernelGGL(k_edge_c, dim3(grid(K.n)), dim3(256), 0, s_, K.n, K.rp.p, K.ci.p, K.v.p, diag.p, w,
                           positive_only, cw.p, cnt.p);
        hipLaunchKernelGGL(k_fill_i32, dim3(grid(K.n)), dim3(256), 0, s_, K.n, -1, mate);
        DCHK(hipGetLastError());
        unsigned long long missing = 0;
        DCHK(hipMemcpyAsync(&missing, cnt.p, sizeof(missing), hipMemcpyDeviceToHost, s_));
        DCHK(hipStreamSynchronize(s_));
        if (missing) throw InputError("device set-up needs a structurally symmetric matrix");
        // at most n/2 + 1 rounds: each round with a candidate matches a pair
        int rounds = 0;
        for (int64_t r = 0; r <= K.n / 2 + 1; r++) {
            unsigned int h_any = 0;
            DCHK(hipMemsetAsync(any.p, 0, sizeof(unsigned int), s_));
            hipLaunchKernelGGL(k_ld_point, dim3(grid(K.n)), dim3(256), 0, s_, K.n, K.rp.p, K.ci.p, cw.p, mate,
                               ptr.p, any.p);
            hipLaunchKernelGGL(k_ld_match, dim3(grid(K.n)), dim3(256), 0, s_, K.n, ptr.p, mate);
            DCHK(hipGetLastError());
            DCHK(hipMemcpyAsync(&h_any, any.p, sizeof(h_any), hipMemcpyDeviceToHost, s_));
            DCHK(hipStreamSynchronize(s_));
            rounds++;
            if (!h_any) break;
        }
        if (info_) {
            info_->rounds_total += rounds;
            if (rounds > info_->rounds_max) info_->rounds_max = rounds;
            info_->sweeps++;
        }
    }

    int64_t pairwise(const DevCsr &K, const int32_t *mate, const double *w, DBuf<int32_t> &ag, DBuf<double> &pcs,
                     DBuf<double> &wc)
    {
        const int64_t n = K.n;
        DBuf<int32_t> flag(n), idx(n);
        hipLaunchKernelGGL(k_open, dim3(grid(n)), dim3(256), 0, s_, n, mate, flag.p);
        DCHK(hipGetLastError());
        scan_i32_to_i32(flag.p, idx.p, n);
        int32_t last_idx = 0, last_flag = 0;
        DCHK(hipMemcpyAsync(&last_idx, idx.p + (n - 1), sizeof(int32_t), hipMemcpyDeviceToHost, s_));
        DCHK(hipMemcpyAsync(&last_flag, flag.p + (n - 1), sizeof(int32_t), hipMemcpyDeviceToHost, s_));
        DCHK(hipStreamSynchronize(s_));
        const int64_t nc = (int64_t)last_idx + last_flag;
        wc.alloc(nc);
        hipLaunchKernelGGL(k_pairwise, dim3(grid(n)), dim3(256), 0, s_, n, mate, w, idx.p, ag.p, pcs.p, wc.p);
        DCHK(hipGetLastError());
        return nc;
    }

    DevCsr galerkin(const DevCsr &K, int64_t nc, const int32_t *agg, const double *pc)
    {
        const int64_t m = K.nnz;
        DBuf<uint64_t> keys(m), keys2(m);
        DBuf<int32_t> vals(m), vals2(m), head(m);
        DBuf<double> t(m);
        hipLaunchKernelGGL(k_gal_keys, dim3(grid(K.n)), dim3(256), 0, s_, K.n, K.rp.p, K.ci.p, K.v.p, agg, pc,
                           keys.p, vals.p, t.p);
        DCHK(hipGetLastError());
        int bits = 1;
        while ((int64_t(1) << bits) < nc) bits++;
        const int end_bit = 32 + bits;
        {
            size_t b = 0;
            DCHK(hipcub::DeviceRadixSort::SortPairs(nullptr, b, keys.p, keys2.p, vals.p, vals2.p, (int)m, 0, end_bit,
                                                    s_));
            DBuf<char> tmp(b ? b : 1);
            DCHK(hipcub::DeviceRadixSort::SortPairs(tmp.p, b, keys.p, keys2.p, vals.p, vals2.p, (int)m, 0, end_bit,
                                                    s_));
        }
        keys.release();
        vals.release();
        hipLaunchKernelGGL(k_run_heads, dim3(grid(m)), dim3(256), 0, s_, m, keys2.p, head.p);
        DCHK(hipGetLastError());
        DBuf<int64_t> runid(m);
        scan_i32_to_i64(head.p, runid.p, m);
        int64_t last_run = 0;
        int32_t last_head = 0;
        DCHK(hipMemcpyAsync(&last_run, runid.p + (m - 1), sizeof(int64_t), hipMemcpyDeviceToHost, s_));
        DCHK(hipMemcpyAsync(&last_head, head.p + (m - 1), sizeof(int32_t), hipMemcpyDeviceToHost, s_));
        DCHK(hipStreamSynchronize(s_));
        const int64_t nrun = last_run + last_head;
        DBuf<int64_t> start(nrun + 1);
        hipLaunchKernelGGL(k_run_starts, dim3(grid(m)), dim3(256), 0, s_, m, head.p, runid.p, start.p);
        DCHK(hipMemcpyAsync(start.p + nrun, &m, sizeof(int64_t), hipMemcpyHostToDevice, s_));
        DCHK(hipGetLastError());
        DevCsr C;
        C.n = nc;
        C.nnz = nrun;
        C.ci.alloc(nrun);
        C.v.alloc(nrun);
        C.rp.alloc(nc + 1);
        DBuf<int64_t> cnt(nc + 1);
        DCHK(hipMemsetAsync(cnt.p, 0, (nc + 1) * sizeof(int64_t), s_));
        hipLaunchKernelGGL(k_run_sums, dim3(grid(nrun)), dim3(256), 0, s_, nrun, start.p, keys2.p, vals2.p, t.p,
                           C.ci.p, C.v.p, cnt.p);
        DCHK(hipGetLastError());
        scan_i64(cnt.p, C.rp.p, nc + 1);
        DCHK(hipStreamSynchronize(s_));
        return C;
    }
};

}  // namespace

int build_hierarchy_on_device(const CsrView &K0, const double *w, const SetupParams &prm, HostHierarchy &H,
                              std::string &err, void *stream, DevSetupInfo *info)
{
    if (K0.nnz() >= (int64_t(1) << 31) || K0.n >= (int64_t(1) << 31)) {
        err = "device set-up takes fewer than 2^31 stored entries";
        return -1;
    }
    if (prm.smooth) {
        err = "device set-up builds the tentative prolongator only (smooth_prolong 0)";
        return -1;
    }
    try {
        DeviceCoarsener dc((hipStream_t)stream, info);
        return build_hierarchy(K0, w, prm, H, err, &dc);
    } catch (InputError &e) {
        err = e.what();
        return -1;
    } catch (HipError &e) {
        err = e.what();
        return -3;
    } catch (std::bad_alloc &) {
        err = "host allocation failed";
        return -4;
    }
}

}  // namespace amgiga
