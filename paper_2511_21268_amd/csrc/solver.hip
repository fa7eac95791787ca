// amg_ctx: device hierarchy, V-cycle and CG / FCG drivers, and the C ABI of
// include/amg.h.  Every step of the solve phase runs in the kernels of
// kernels.h / coarse.h on the context's stream; the host only enqueues them and
// reads one small scalar block per iteration to test convergence.
#include "amg.h"
#include "cheb.h"
#include "coarse.h"
#include "host.h"
#include "kernels.h"
#include "kernels_blk.h"
#include "blockcg.h"
#include "mlp.h"
#include "post_res.h"
#include "setup_dev.h"
#include "tail.h"

#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

using namespace amgk;
using amgiga::CsrView;
using amgiga::HostHierarchy;
using amgiga::SellHost;
using amgiga::build_sell;
using amgiga::count_shared;

static thread_local std::string g_err;

// rocTX range over a scope (host side: the solve, each Krylov iteration, each
// V-cycle level's launches), for traces taken with a marker-tracing profiler;
// without one the calls do nothing.
struct TxRange {
    explicit TxRange(const char *m) { roctxRangePushA(m); }
    ~TxRange() { roctxRangePop(); }
};
static const char *level_label(int l)
{
    static const std::vector<std::string> names = [] {
        std::vector<std::string> v;
        for (int i = 0; i < 64; i++) v.push_back("amg level " + std::to_string(i));
        return v;
    }();
    return names[(size_t)std::min(std::max(l, 0), 63)].c_str();
}

namespace {

struct Fail {
    amg_status st;
};

void set_err(const std::string &m) { g_err = m; }

#define HIPCHK(x)                                                                              \
    do {                                                                                       \
        hipError_t e_ = (x);                                                                   \
        if (e_ != hipSuccess) {                                                                \
            set_err(std::string("HIP error: ") + hipGetErrorString(e_) + " at " #x);           \
            throw Fail{e_ == hipErrorOutOfMemory ? AMG_ERR_OOM : AMG_ERR_HIP};                 \
        }                                                                                      \
    } while (0)

template <typename T> T *dalloc(size_t n)
{
    void *p = nullptr;
    if (n == 0) n = 1;
    HIPCHK(hipMalloc(&p, n * sizeof(T)));
    return (T *)p;
}

template <typename T> T *dupload(const T *h, size_t n)
{
    T *d = dalloc<T>(n);
    if (n) HIPCHK(hipMemcpy(d, h, n * sizeof(T), hipMemcpyHostToDevice));
    return d;
}

inline unsigned nblocks(int64_t n, int per = 256) { return (unsigned)((n + per - 1) / per); }
inline unsigned vgrid(int64_t n) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>(1024, (n + 255) / 256)); }

// Host-side sliced-ELL image of one level (layout described in kernels.h).
struct DevMat {
    int64_t n = 0, ncols = 0, nnz = 0, nslices = 0, stored = 0, nshared = 0;
    double index_bytes = 0.0;
    int idx16 = 1, C = SLICE, sorted = 0;
    int64_t *soff = nullptr, *ibase = nullptr;
    int32_t *col0 = nullptr, *c32 = nullptr, *shoff = nullptr, *perm = nullptr, *shrun = nullptr;
    // windows shared by the four slices of a block (batched stencil images)
    int32_t *wgtab = nullptr, *wgst = nullptr;
    int wg_sigma = 0;
    int xwin = 0;   // single-vector K passes through x windows (shared-offset images with run tables)
    double wg_ratio = 0.0;   // rows the shared windows copy / rows per-wave windows copy
    uint16_t *d16 = nullptr;
    double *v64 = nullptr;
    float *v32 = nullptr;
    // CSR image with `lpr` lanes per row (lpr > 0; FP64, int32 columns) instead
    // of SELL: long or few rows of the smoothed hierarchy
    int lpr = 0;
    int64_t *crp = nullptr;
    int32_t *cci = nullptr;
    double *cv = nullptr;
    bool built() const { return soff || crp; }
    template <typename VT> const VT *val() const;
    template <typename IT> const IT *idx() const;
    template <typename VT, typename IT> Sell<VT, IT> sv() const
    {
        return Sell<VT, IT>{n,     ncols, nslices, soff,  ibase, val<VT>(), idx<IT>(), col0,
                            shoff, perm,  shrun,   wgtab, wgst,  xwin};
    }
};
template <> const double *DevMat::val<double>() const { return v64; }
template <> const float *DevMat::val<float>() const { return v32; }
template <> const uint16_t *DevMat::idx<uint16_t>() const { return d16; }
template <> const int32_t *DevMat::idx<int32_t>() const { return c32; }

struct Level {
    int64_t n = 0, nnz = 0;
    DevMat A;     // SELL-64, one lane per row
    DevMat Ab;    // SELL-(64/LPR) image of the block kernels (batched solves), if built
    DevMat KP;    // SELL-64 image of K P (fused prolongation + post-smoothing), ell < L
    DevMat KPb;   // SELL-(64/LPR) image of K P for the block kernels, if built
    DevMat Pm;    // SELL-64 image of the smoothed prolongator (rows n, columns n_c), if built
    DevMat Rm;    // SELL-64 image of its transpose (rows n_c, columns n), if built
    double *invd64 = nullptr;
    float *invd32 = nullptr;
    // transfer to the next level
    int32_t *agg = nullptr, *members = nullptr;
    int mw = 0;
    double *pc64 = nullptr;
    float *pc32 = nullptr;
    // work vectors in the V-cycle precision (single vector, and 16-column blocks)
    void *f = nullptr, *u = nullptr, *u2 = nullptr, *r = nullptr, *c = nullptr, *c2 = nullptr;
    void *bf = nullptr, *bu = nullptr, *bu2 = nullptr, *br = nullptr, *bc = nullptr, *bc2 = nullptr;
    double poly[4] = {1.0, 0.0, 0.0, 0.0};
    int poly_on = 0;
    template <typename VT> VT *invd() const;
    template <typename VT> VT *pc() const;
};
template <> double *Level::invd<double>() const { return invd64; }
template <> float *Level::invd<float>() const { return invd32; }
template <> double *Level::pc<double>() const { return pc64; }
template <> float *Level::pc<float>() const { return pc32; }

}  // namespace

struct amg_ctx {
    amg_params prm;
    hipStream_t stream = nullptr;
    int device = 0;
    int host_only = 0;
    HostHierarchy host;
    std::vector<Level> lev;
    int nlev = 0;
    int nL = 0, ldL = 0;
    double *Linv = nullptr, *LinvT = nullptr;
    // coarsest level for the CG coarse solver: CSR (int32) and 1 / k_ii
    int32_t *cg_rp = nullptr, *cg_ci = nullptr;
    double *cg_v = nullptr, *cg_dj = nullptr;
    int64_t n = 0;
    double *r = nullptr, *z = nullptr, *p = nullptr, *q = nullptr;
    double *partial = nullptr;
    int64_t partial_cap = 0;
    // batched solve (allocated on first use)
    double *bR = nullptr, *bZ = nullptr, *bP = nullptr, *bQ = nullptr, *bU = nullptr, *bF = nullptr;
    double *bY = nullptr, *bsc = nullptr, *hbsc = nullptr, *bpartial = nullptr, *bstrided = nullptr;
    double *bgram = nullptr, *bcoef = nullptr, *bgsave = nullptr;   // block CG: Gram partials, alpha / beta, G
    int blk_lpr = 1, blk_threads = 256;   // block-kernel variant (autotuned when prm.nrhs > 1)
    int blk_win = 4;       // stencil images: staged-window block kernel with this many rows per lane (0: off)
    int blk_img_lpr = 0;   // lanes per row the SELL-(64/lpr) block images were built for (0: none)
    // windows shared by a block's slices where the image has stage tables:
    // bit 0 for the passes over FP64 values, bit 1 over FP32 values
    int blk_share = 3;
    // graph replay of the iteration body (single: [0]=CG [1]=FCG; batched likewise)
    int use_graph = 0;
    int fuse_post = 1;   // fused prolongation + post-smoothing through K P (when built)
    // V-cycle tail in one persistent workgroup (k_vtail): levels tail_start ..
    // nlev-2 and the coarsest; device arrays of their TailLevel descriptors for
    // the single-vector and the 16-column buffers; off by default (measured
    // on the 2.1M-unknown cube: one workgroup walking the last levels takes
    // longer than the per-level launches it replaces, 9 us per V-cycle single
    // vector and 110 us per 16-column V-cycle)
    int use_tail = 0, tail_start = -1;
    void *tail_dev = nullptr, *tail_dev_blk = nullptr;
    hipStream_t gstream = nullptr;
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    double *uw = nullptr;
    hipGraphExec_t gA[2] = {nullptr, nullptr}, gB[2] = {nullptr, nullptr};
    hipGraphExec_t gbA[2] = {nullptr, nullptr}, gbB[2] = {nullptr, nullptr};
    void drop_graphs()
    {
        for (auto *arr : {gA, gB, gbA, gbB})
            for (int i = 0; i < 2; i++)
                if (arr[i]) { (void)hipGraphExecDestroy(arr[i]); arr[i] = nullptr; }
    }
    template <class Body> hipGraphExec_t capture(Body body)
    {
        hipGraph_t g = nullptr;
        HIPCHK(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal));
        try {
            body();
        } catch (...) {
            (void)hipStreamEndCapture(stream, &g);
            if (g) (void)hipGraphDestroy(g);
            throw;
        }
        HIPCHK(hipStreamEndCapture(stream, &g));
        hipGraphExec_t ex = nullptr;
        hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        HIPCHK(e);
        return ex;
    }
    // Run the solve on the library's own stream (graphs cannot be captured on
    // the null stream); ordered after / before the caller's stream by events.
    struct OnGraphStream {
        amg_ctx *c;
        hipStream_t user;
        bool on;
        OnGraphStream(amg_ctx *c_, bool on_) : c(c_), user(c_->stream), on(on_)
        {
            if (!on) return;
            if (!c->gstream) {
                HIPCHK(hipStreamCreateWithFlags(&c->gstream, hipStreamNonBlocking));
                HIPCHK(hipEventCreateWithFlags(&c->ev_in, hipEventDisableTiming));
                HIPCHK(hipEventCreateWithFlags(&c->ev_out, hipEventDisableTiming));
            }
            HIPCHK(hipEventRecord(c->ev_in, user));
            HIPCHK(hipStreamWaitEvent(c->gstream, c->ev_in, 0));
            c->stream = c->gstream;
        }
        ~OnGraphStream()
        {
            if (!on) return;
            (void)hipEventRecord(c->ev_out, c->gstream);
            (void)hipStreamWaitEvent(user, c->ev_out, 0);
            c->stream = user;
        }
    };
    std::vector<std::pair<std::string, double>> tune_log;
    amgiga::DevSetupInfo setup_info;
    double *sc = nullptr;
    double *hsc = nullptr;     // pinned host copy of the scalar block
    std::vector<double> hist;  // ||r_k|| / ||F|| of the last pcg_solve, k = 0 .. iterations
    hipEvent_t ev_iter = nullptr;
    std::vector<void *> allocs;
    // profiling
    int prof = 0;
    std::vector<hipEvent_t> evpool;
    size_t evused = 0;
    std::vector<double> evbytes;
    std::vector<int> evkind;
    int64_t pk_launches[AMG_PASS_KINDS] = {};
    double pk_ms[AMG_PASS_KINDS] = {}, pk_bytes[AMG_PASS_KINDS] = {};
    int64_t prof_launches = 0;
    double prof_ms = 0.0, prof_bytes = 0.0;

    template <typename T> T *alloc(size_t k)
    {
        T *d = dalloc<T>(k);
        allocs.push_back(d);
        return d;
    }
    template <typename T> T *upload(const std::vector<T> &h)
    {
        T *d = dupload(h.data(), h.size());
        allocs.push_back(d);
        return d;
    }
    void release(void *p)
    {
        if (!p) return;
        auto it = std::find(allocs.begin(), allocs.end(), p);
        if (it != allocs.end()) allocs.erase(it);
        (void)hipFree(p);
    }
    void release(DevMat &M)
    {
        release(M.soff); release(M.ibase); release(M.shoff); release(M.shrun); release(M.perm); release(M.col0);
        release(M.wgtab); release(M.wgst);
        release(M.c32);
        release(M.d16);
        release(M.v64); release(M.v32);
        release(M.crp); release(M.cci); release(M.cv);
        M = DevMat();
    }
    // Image of a matrix of the smoothed-aggregation V-cycle: SELL-64 (stencil
    // matrices, and short rows in numbers that fill the GPU), else CSR with
    // 8..64 lanes per row by the mean row length.
    DevMat upload_image(const CsrView &K, int64_t ncols = 0)
    {
        const bool square = ncols <= 0;
        const int64_t ns = (K.n + SLICE - 1) / SLICE;
        const double mean = (double)K.nnz() / (double)std::max<int64_t>(K.n, 1);
        const bool stencil = square && prm.slice_offsets && 2 * count_shared(K, SLICE) >= ns;
        if (stencil || !(mean >= 256.0 || (mean >= 32.0 && ns < 2048))) return upload_sell(K, SLICE, true, false, ncols);
        DevMat A;
        A.n = K.n; A.ncols = square ? K.n : ncols; A.nnz = K.nnz(); A.stored = K.nnz(); A.C = 0;
        A.index_bytes = 4.0 * (double)K.nnz() + 8.0 * (double)(K.n + 1);
        A.lpr = mean >= 512.0 ? 64 : mean >= 256.0 ? 32 : mean >= 64.0 ? 16 : 8;
        A.crp = dupload(K.rp, (size_t)K.n + 1); allocs.push_back(A.crp);
        A.cci = dupload(K.ci, (size_t)K.nnz()); allocs.push_back(A.cci);
        A.cv = dupload(K.v, (size_t)K.nnz()); allocs.push_back(A.cv);
        return A;
    }
    // y = acc, f + acc or f - acc over an image (SELL or CSR), FP64, no dots.
    template <int EPI> void apply(const DevMat &M, const double *x, const double *f, double *y)
    {
        if (M.lpr) {
            const unsigned g = (unsigned)((M.n * M.lpr + 255) / 256);
#define CSR_APPLY(L) hipLaunchKernelGGL((k_csr_apply<L, EPI>), dim3(g), dim3(256), 0, stream, M.n, M.crp, M.cci, \
                                        M.cv, x, f, y)
            switch (M.lpr) {
            case 8: CSR_APPLY(8); break;
            case 16: CSR_APPLY(16); break;
            case 32: CSR_APPLY(32); break;
            default: CSR_APPLY(64); break;
            }
#undef CSR_APPLY
            HIPCHK(hipGetLastError());
            return;
        }
        launch_sell<double, double, double, EPI, 0>(M, (unsigned)((M.nslices + SELL_WAVES - 1) / SELL_WAVES), x, f,
                                                    nullptr, y, nullptr, nullptr, 1.0);
    }
    // SELL-C image of a square level matrix, or with ncols > 0 of a
    // rectangular one (K P).  With prm.slice_offsets: a square matrix whose
    // slices mostly share their column offsets (stencil matrices) keeps row
    // order and stores shared offsets; every other image is sorted by row
    // length within windows of 4 slices (the slices of one 4-wave block).
    // Without: row order and per-entry indices everywhere.
    DevMat upload_sell(const CsrView &K, int C, bool want64, bool want32, int64_t ncols = 0)
    {
        SellHost S;
        const bool square = ncols <= 0;
        if (prm.slice_offsets == 0) {
            build_sell(K, C, want64, want32, false, 0, S);
        } else {
            const int64_t ns = (K.n + C - 1) / C;
            const bool stencil = square && 2 * count_shared(K, C) >= ns;
            build_sell(K, C, want64, want32, stencil, stencil ? 0 : 4 * C, S);
        }
        DevMat A;
        A.n = K.n; A.ncols = square ? K.n : ncols; A.sorted = S.sorted;
        A.nnz = K.nnz(); A.nslices = S.nslices; A.stored = S.stored; A.idx16 = S.idx16; A.C = C;
        A.nshared = S.nshared; A.index_bytes = S.index_bytes;
        A.soff = upload(S.soff);
        A.ibase = upload(S.ibase);
        if (!S.shoff.empty()) {
            A.shoff = upload(S.shoff);
            A.shrun = upload(S.shrun);
            A.xwin = C == SLICE && S.nshared > 0 ? 1 : 0;
            if (C == SLICE && S.nshared > 0) {
                // the block kernels' windows shared by a block's slices
                amgiga::WgStages W;
                amgiga::choose_wg_stages(S, C, (S.nslices + SELL_WAVES - 1) / SELL_WAVES, W);
                const double per_wave = (double)W.runs * amgk::WIN_ROWS;
                if (W.runs > 0 && W.st.size() / 2 < ((size_t)1 << 31)) {
                    A.wgtab = upload(W.tab);
                    A.wgst = upload(W.st);
                    A.wg_sigma = W.sigma;
                    A.wg_ratio = (double)W.copied_rows / per_wave;
                }
            }
        }
        if (S.sorted) A.perm = upload(S.perm);
        if (want64) A.v64 = upload(S.v64);
        if (want32) A.v32 = upload(S.v32);
        if (!S.d16.empty()) A.d16 = upload(S.d16);
        if (!S.col0.empty()) A.col0 = upload(S.col0);
        if (!S.c32.empty()) A.c32 = upload(S.c32);
        return A;
    }
    // Device time of body(), best of two after one warm-up run.
    template <class Body> float time_passes(Body body)
    {
        hipEvent_t e0, e1;
        HIPCHK(hipEventCreate(&e0));
        HIPCHK(hipEventCreate(&e1));
        float best = 1e30f;
        for (int rep = 0; rep < 3; rep++) {
            HIPCHK(hipEventRecord(e0, stream));
            body();
            HIPCHK(hipEventRecord(e1, stream));
            HIPCHK(hipEventSynchronize(e1));
            float ms = 0.f;
            HIPCHK(hipEventElapsedTime(&ms, e0, e1));
            if (rep > 0) best = std::min(best, ms);
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        return best;
    }
    // x windows or the gather walk for the single-vector FP64 K passes,
    // whichever runs faster on this GPU: three residual passes each (measured
    // at c4: x windows 0.999 against 1.025 ms on one box, 0.996 against
    // ~0.97 ms on others -- the gather walk gains more from a faster memory)
    void tune_xwin()
    {
        DevMat &A = lev[0].A;
        if (!A.xwin || !A.v64) return;
        for (double *v : {p, r})
            hipLaunchKernelGGL((k_fill<double>), dim3(vgrid(n)), dim3(256), 0, stream, n, 1.0, v);
        HIPCHK(hipGetLastError());
        const int prof_saved = prof;
        prof = 0;
        auto passes = [&] {
            for (int i = 0; i < 3; i++)
                sell<double, double, double, EPI_RESID, 0>(0, p, r, lev[0].invd<double>(), q, nullptr, nullptr);
        };
        // warm-up (clocks), then the two walks alternately, the best of each
        for (int i = 0; i < 4; i++) passes();
        float t[2] = {1e30f, 1e30f};
        for (int rep = 0; rep < 2; rep++)
            for (int on : {1, 0}) {
                A.xwin = on;
                const float ms = time_passes(passes);
                tune_log.push_back({std::string("x windows ") + (on ? "on" : "off"), ms});
                t[on] = std::min(t[on], ms);
            }
        A.xwin = t[1] <= t[0] ? 1 : 0;
        prof = prof_saved;
    }
    // The level-0 passes of one batched iteration: FP64 outer SpMV and two
    // passes in the V-cycle precision.
    template <typename VT> void level0_passes()
    {
        Level &L = lev[0];
        // the outer product with the dots of the Krylov method in use
        if (prm.krylov) sell_blk<double, double, double, EPI_SPMV, 2>(0, bP, nullptr, nullptr, bQ, nullptr, bR);
        else sell_blk<double, double, double, EPI_SPMV, 1>(0, bP, nullptr, nullptr, bQ, nullptr, nullptr);
        sell_blk<VT, double, VT, EPI_RESID, 0>(0, (const VT *)L.bu, bR, L.invd<VT>(), (VT *)L.br, nullptr, nullptr);
        sell_blk<VT, double, VT, EPI_RESID, 0>(0, (const VT *)L.bu, bR, L.invd<VT>(), (VT *)L.br, nullptr, nullptr);
    }
    // The passes over images that take the lanes-per-row variant: the level-0
    // K P pass, a level-1 residual pass and, without staged windows at level
    // 0, the level-0 passes.
    template <typename VT> void variant_passes(bool with_level0)
    {
        if (with_level0) level0_passes<VT>();
        if (nlev > 1 && lev[0].KP.soff)
            bpost_fused<VT, VT>(0, (const VT *)lev[1].bu, (const VT *)lev[0].bu, (VT *)lev[0].bu2, 0, nullptr, nullptr);
        if (nlev > 2) {
            Level &L = lev[1];
            sell_blk<VT, VT, VT, EPI_RESID, 0>(1, (const VT *)L.bu, (const VT *)L.bf, L.invd<VT>(), (VT *)L.br,
                                               nullptr, nullptr);
        }
    }
    // Autotuner of the block kernels.  Stencil images (shared column offsets,
    // in practice level 0) take the staged-window kernel: its rows per lane
    // (2 or 4) are timed on the level-0 passes.  The other images -- coarse
    // levels and the K P images of the fused post-smoothing -- take 1 lane per
    // row on the SELL-64 images or 4, 8 or 16 on SELL-(64/lanes) images with
    // 256 or 512 threads per block, timed on the level-0 K P pass and a
    // level-1 pass; the fastest variant's images are then built for every level.
    void tune_blocks(const CsrView &K0)
    {
        blk_alloc();
        const bool f32 = fp32();
        for (double *v : {bP, bR})
            hipLaunchKernelGGL((k_fill<double>), dim3(vgrid(n * NB)), dim3(256), 0, stream, n * NB, 1.0, v);
        for (int l = 0; l < std::min(nlev, 2); l++)
            for (void *v : {lev[l].bu, lev[l].bf}) {
                if (f32) hipLaunchKernelGGL((k_fill<float>), dim3(vgrid(lev[l].n * NB)), dim3(256), 0, stream,
                                            lev[l].n * NB, 1.0f, (float *)v);
                else hipLaunchKernelGGL((k_fill<double>), dim3(vgrid(lev[l].n * NB)), dim3(256), 0, stream,
                                        lev[l].n * NB, 1.0, (double *)v);
            }
        HIPCHK(hipGetLastError());
        int prof_saved = prof;
        prof = 0;
        blk_lpr = 1;
        blk_threads = 256;
        const bool win0 = lev[0].A.nshared > 0 && lev[0].A.shrun != nullptr;
        if (win0) {
            int best_r = 4, best_share = 0;
            float best_t = 1e30f;
            for (int share : {0, 1, 2, 3}) {
                if (share && !lev[0].A.wgtab) continue;
                if ((share & 2) && !f32) continue;   // no pass over FP32 values
                blk_share = share;
                for (int R : {2, 4}) {
                    blk_win = R;
                    float t = f32 ? time_passes([&] { level0_passes<float>(); })
                                  : time_passes([&] { level0_passes<double>(); });
                    tune_log.push_back({"shared windows " + std::to_string(share) + ", window rows per lane " +
                                        std::to_string(R), t});
                    if (t < best_t) { best_t = t; best_r = R; best_share = share; }
                }
            }
            blk_win = best_r;
            blk_share = best_share;
        }
        const bool lvl0 = !(win0 && blk_win > 0);
        struct Best { int lpr, thr; float ms; } best{1, 256, 1e30f};
        best.ms = f32 ? time_passes([&] { variant_passes<float>(lvl0); }) : time_passes([&] { variant_passes<double>(lvl0); });
        tune_log.push_back({"lpr=1 threads=256", best.ms});
        // level-0 K P product, formed once for every candidate image
        amgiga::Csr kp0;
        if (nlev > 1) kp0 = amgiga::kp_product(K0, host.lev[1].n, host.lev[0].agg.data(), host.lev[0].pc.data());
        struct Imgs { DevMat a0, a1, kp0; };
        Imgs keep;
        for (int lpr : {4, 8, 16}) {
            Imgs im;
            if (lvl0) im.a0 = upload_sell(K0, 64 / lpr, true, f32);
            if (nlev > 2) im.a1 = upload_sell(amgiga::view(host.lev[1].K), 64 / lpr, !f32, f32);
            if (nlev > 1) im.kp0 = upload_sell(amgiga::view(kp0), 64 / lpr, !f32, f32, host.lev[1].n);
            lev[0].Ab = im.a0;
            if (nlev > 2) lev[1].Ab = im.a1;
            if (nlev > 1) lev[0].KPb = im.kp0;
            bool won = false;
            for (int thr : {256, 512}) {
                blk_lpr = lpr;
                blk_threads = thr;
                float t = f32 ? time_passes([&] { variant_passes<float>(lvl0); })
                              : time_passes([&] { variant_passes<double>(lvl0); });
                tune_log.push_back({"lpr=" + std::to_string(lpr) + " threads=" + std::to_string(thr), t});
                if (t < best.ms) { best = {lpr, thr, t}; won = true; }
            }
            lev[0].Ab = DevMat(); lev[0].KPb = DevMat();
            if (nlev > 2) lev[1].Ab = DevMat();
            if (won) {
                release(keep.a0); release(keep.a1); release(keep.kp0);
                keep = im;
            } else {
                release(im.a0); release(im.a1); release(im.kp0);
            }
        }
        prof = prof_saved;
        blk_lpr = best.lpr;
        blk_threads = best.thr;
        if (best.lpr > 1) {
            lev[0].Ab = keep.a0;
            if (nlev > 2) lev[1].Ab = keep.a1;
            if (nlev > 1) lev[0].KPb = keep.kp0;
            for (int l = 2; l < nlev - 1; l++)
                lev[l].Ab = upload_sell(amgiga::view(host.lev[l].K), 64 / best.lpr, !f32, f32);
            for (int l = 1; l < nlev - 1; l++) {
                amgiga::Csr kp = amgiga::kp_product(amgiga::view(host.lev[l].K), host.lev[l + 1].n,
                                                    host.lev[l].agg.data(), host.lev[l].pc.data());
                lev[l].KPb = upload_sell(amgiga::view(kp), 64 / best.lpr, !f32, f32, host.lev[l + 1].n);
            }
            blk_img_lpr = best.lpr;
        }
        HIPCHK(hipStreamSynchronize(stream));
    }
    ~amg_ctx()
    {
        if (!host_only) (void)hipStreamSynchronize(stream);
        for (void *p : allocs) (void)hipFree(p);
        if (hsc) (void)hipHostFree(hsc);
        if (hbsc) (void)hipHostFree(hbsc);
        drop_graphs();
        if (gstream) { (void)hipStreamSynchronize(gstream); (void)hipStreamDestroy(gstream); }
        if (ev_in) (void)hipEventDestroy(ev_in);
        if (ev_out) (void)hipEventDestroy(ev_out);
        if (ev_iter) (void)hipEventDestroy(ev_iter);
        for (auto e : evpool) (void)hipEventDestroy(e);
    }

    bool fp32() const { return prm.vcycle_fp32 != 0; }

    // ---- profiling of level-0 matrix passes -------------------------------
    void prof_begin()
    {
        if (!prof) return;
        while (evpool.size() < evused + 2) {
            hipEvent_t e;
            HIPCHK(hipEventCreate(&e));
            evpool.push_back(e);
        }
        HIPCHK(hipEventRecord(evpool[evused], stream));
    }
    void prof_end(double bytes, int kind)
    {
        if (!prof) return;
        HIPCHK(hipEventRecord(evpool[evused + 1], stream));
        evbytes.push_back(bytes);
        evkind.push_back(kind);
        evused += 2;
    }
    void prof_collect()
    {
        if (!prof) return;
        for (size_t k = 0; k + 1 < evused; k += 2) {
            float ms = 0.f;
            HIPCHK(hipEventElapsedTime(&ms, evpool[k], evpool[k + 1]));
            prof_ms += ms;
            prof_launches++;
            prof_bytes += evbytes[k / 2];
            const int kd = evkind[k / 2];
            pk_ms[kd] += ms;
            pk_launches[kd]++;
            pk_bytes[kd] += evbytes[k / 2];
        }
        evused = 0;
        evbytes.clear();
        evkind.clear();
    }
    static constexpr int pass_kind(int epi)
    {
        return epi == EPI_SPMV ? AMG_PASS_SPMV : epi == EPI_RESID ? AMG_PASS_RESID
             : epi == EPI_SMOOTH ? AMG_PASS_SMOOTH : epi == EPI_POLY ? AMG_PASS_POLY : AMG_PASS_OTHER;
    }
    // algorithmic bytes of one level-0 pass: matrix without padding + vectors
    double pass_bytes(int vb, int nvec) const
    {
        const DevMat &A = lev[0].A;
        return (double)A.nnz * vb + A.index_bytes + (double)nvec * 8.0 * A.n;
    }

    // ---- the V-cycle tail ------------------------------------------------------
    // Levels from tail_start on qualify when each is small (at most TAIL_ROWS
    // rows and TAIL_NNZ entries: one workgroup walks it in about the time a
    // launch takes) and the coarsest fits the tail's LDS; the tail is used
    // when the V-cycle is the l1-Jacobi one with one pre- and one post-sweep
    // and the fused K P post-smoothing, no polynomial smoother on those levels.
    static constexpr int64_t TAIL_ROWS = 2048, TAIL_NNZ = 60000;
    void choose_tail()
    {
        tail_start = -1;
        if (nlev < 3 || nL > TAIL_MAX_COARSE || general_vcycle()) return;
        for (int l = nlev - 2; l >= 1; l--) {
            if (lev[l].n > TAIL_ROWS || lev[l].nnz > TAIL_NNZ || !lev[l].KP.soff || !lev[l].A.soff) break;
            tail_start = l;
        }
        // descriptors uploaded now, never inside a graph capture
        if (tail_start > 0) tail_dev = fp32() ? tail_descriptors<float>(false) : tail_descriptors<double>(false);
    }
    bool tail_usable() const
    {
        if (!use_tail || tail_start < 1 || !fuse_post || prm.nu_pre != 1 || prm.nu_post != 1) return false;
        for (int l = tail_start; l < nlev - 1; l++)
            if (lev[l].poly_on) return false;
        return true;
    }
    template <typename VT> void *tail_descriptors(bool blk)
    {
        std::vector<TailLevel<VT>> T;
        for (int l = tail_start; l < nlev - 1; l++) {
            Level &L = lev[l];
            TailLevel<VT> d{};
            d.a16 = L.A.idx16;
            if (d.a16) d.A16 = L.A.sv<VT, uint16_t>();
            else d.A32 = L.A.sv<VT, int32_t>();
            d.p16 = L.KP.idx16;
            if (d.p16) d.P16 = L.KP.sv<VT, uint16_t>();
            else d.P32 = L.KP.sv<VT, int32_t>();
            d.mw = L.mw;
            d.n = L.n;
            d.invd = L.invd<VT>();
            d.pc = L.pc<VT>();
            d.agg = L.agg;
            d.members = L.members;
            d.f = (VT *)(blk ? L.bf : L.f);
            d.u = (VT *)(blk ? L.bu : L.u);
            d.u2 = (VT *)(blk ? L.bu2 : L.u2);
            d.r = (VT *)(blk ? L.br : L.r);
            T.push_back(d);
        }
        return upload(T);
    }
    // run the tail; returns the post-smoothed correction of level tail_start
    template <typename VT> VT *run_tail(bool blk)
    {
        const int nt = nlev - 1 - tail_start;
        Level &C = lev[nlev - 1];
        if (blk) {
            hipLaunchKernelGGL((k_vtail_blk<VT>), dim3(1), dim3(TAIL_THREADS), 0, stream,
                               (const TailLevel<VT> *)tail_dev_blk, nt, nL, ldL, Linv, LinvT, (VT *)C.bf,
                               (VT *)C.bu, bY);
        } else {
            hipLaunchKernelGGL((k_vtail<VT>), dim3(1), dim3(TAIL_THREADS), 0, stream, (const TailLevel<VT> *)tail_dev,
                               nt, nL, ldL, Linv, LinvT, (VT *)C.f, (VT *)C.u);
        }
        HIPCHK(hipGetLastError());
        return (VT *)(blk ? lev[tail_start].bu2 : lev[tail_start].u2);
    }

    // ---- kernel launchers --------------------------------------------------
    template <typename VT, typename FT, typename OT, int EPI, int NDOT>
    void sell(int l, const VT *x, const FT *f, const VT *invd, OT *y, const double *g0, const double *g1,
              VT coef = 1)
    {
        const DevMat &A = lev[l].A;
        unsigned nb = (unsigned)((A.nslices + SELL_WAVES - 1) / SELL_WAVES);
        if (l == 0) {
            int nvec = 2 + (EPI == EPI_RESID ? 1 : 0) + (EPI == EPI_SMOOTH ? 2 : 0) + (EPI == EPI_POLY ? 2 : 0) +
                       (NDOT >= 2 ? 1 : 0) + (EPI == EPI_SMOOTH && NDOT >= 1 ? 1 : 0);
            prof_begin();
            launch_sell<VT, FT, OT, EPI, NDOT>(A, nb, x, f, invd, y, g0, g1, coef);
            prof_end(pass_bytes((int)sizeof(VT), nvec), pass_kind(EPI));
        } else {
            launch_sell<VT, FT, OT, EPI, NDOT>(A, nb, x, f, invd, y, g0, g1, coef);
        }
    }
    template <typename VT, typename FT, typename OT, int EPI, int NDOT>
    void launch_sell(const DevMat &A, unsigned nb, const VT *x, const FT *f, const VT *invd, OT *y,
                     const double *g0, const double *g1, VT coef)
    {
        if (A.idx16)
            hipLaunchKernelGGL((k_sell<VT, FT, OT, uint16_t, EPI, NDOT>), dim3(nb), dim3(256), 0, stream,
                               A.sv<VT, uint16_t>(), x, f, invd, y, g0, g1, partial, coef);
        else
            hipLaunchKernelGGL((k_sell<VT, FT, OT, int32_t, EPI, NDOT>), dim3(nb), dim3(256), 0, stream,
                               A.sv<VT, int32_t>(), x, f, invd, y, g0, g1, partial, coef);
        HIPCHK(hipGetLastError());
    }
    unsigned sell_blocks(int l) const { return (unsigned)((lev[l].A.nslices + SELL_WAVES - 1) / SELL_WAVES); }
    // Fused prolongation + first post-smoothing sweep on level l (needs K P).
    template <typename VT, typename OT>
    unsigned post_fused(int l, const VT *e, const VT *u, OT *y, int ndot, const double *g0, const double *g1)
    {
        Level &L = lev[l];
        const DevMat &A = L.KP;
        unsigned nb = (unsigned)((A.nslices + SELL_WAVES - 1) / SELL_WAVES);
        if (l == 0) prof_begin();
#define POST_LAUNCH(IT, IDX, ND)                                                                              \
    hipLaunchKernelGGL((k_sell_post<VT, OT, IT, ND>), dim3(nb), dim3(256), 0, stream, A.sv<VT, IT>(), e, u,     \
                       (const VT *)L.r, L.invd<VT>(), L.agg, L.pc<VT>(), y, g0, g1, partial)
        if (A.idx16) {
            if (ndot == 2) POST_LAUNCH(uint16_t, A.d16, 2);
            else if (ndot == 1) POST_LAUNCH(uint16_t, A.d16, 1);
            else POST_LAUNCH(uint16_t, A.d16, 0);
        } else {
            if (ndot == 2) POST_LAUNCH(int32_t, A.c32, 2);
            else if (ndot == 1) POST_LAUNCH(int32_t, A.c32, 1);
            else POST_LAUNCH(int32_t, A.c32, 0);
        }
#undef POST_LAUNCH
        HIPCHK(hipGetLastError());
        if (l == 0) {
            double bytes = (double)A.nnz * sizeof(VT) + A.index_bytes +
                           (double)sizeof(VT) * lev[1].n +                         // e gathered once
                           (double)sizeof(VT) * A.n * 4 + 4.0 * A.n +               // u, r, invd, pc, agg
                           (double)sizeof(OT) * A.n + 8.0 * A.n * ndot;              // y, dot partners
            prof_end(bytes, AMG_PASS_KP);
        }
        return nb * SELL_WAVES;   // one dot partial per wavefront
    }
    // Fused prolongation + residual of the polynomial post-smoothing on level l:
    // y = u + P e, L.r <- L.r - (K P) e (needs K P and the pre-smoothing residual in L.r).
    template <typename VT> void post_res_fused(int l, const VT *e, const VT *u, VT *y)
    {
        Level &L = lev[l];
        const DevMat &A = L.KP;
        unsigned nb = (unsigned)((A.nslices + SELL_WAVES - 1) / SELL_WAVES);
        if (l == 0) prof_begin();
        if (A.idx16)
            hipLaunchKernelGGL((k_sell_post_res<VT, uint16_t>), dim3(nb), dim3(256), 0, stream, A.sv<VT, uint16_t>(),
                               e, u, (VT *)L.r, L.agg, L.pc<VT>(), y);
        else
            hipLaunchKernelGGL((k_sell_post_res<VT, int32_t>), dim3(nb), dim3(256), 0, stream, A.sv<VT, int32_t>(),
                               e, u, (VT *)L.r, L.agg, L.pc<VT>(), y);
        HIPCHK(hipGetLastError());
        if (l == 0) {
            double bytes = (double)A.nnz * sizeof(VT) + A.index_bytes + (double)sizeof(VT) * lev[1].n +
                           (double)sizeof(VT) * A.n * 5 + 4.0 * A.n;   // u, pc, r read, r and y written, agg
            prof_end(bytes, AMG_PASS_KP);
        }
    }
    void finalize(unsigned nblk, int op, int slot = 0)
    {
        hipLaunchKernelGGL(k_finalize, dim3(1), dim3(FIN_THREADS), 0, stream, partial, (int)nblk, sc, op, slot);
        HIPCHK(hipGetLastError());
    }
    unsigned dot_partials(int64_t m, const double *a, const double *b, const double *c)
    {
        unsigned g = vgrid(m);
        hipLaunchKernelGGL(k_dot2, dim3(g), dim3(256), 0, stream, m, a, b, c, partial);
        HIPCHK(hipGetLastError());
        return g;
    }
    void dot2(int64_t m, const double *a, const double *b, const double *c, int op, int slot = 0)
    {
        finalize(dot_partials(m, a, b, c), op, slot);
    }
    unsigned vc_nb = 0;   // partial blocks left by the last V-cycle's dots
    template <typename DT, typename ST> void copy(int64_t m, const ST *s, DT *d)
    {
        hipLaunchKernelGGL((k_copy<DT, ST>), dim3(vgrid(m)), dim3(256), 0, stream, m, s, d);
        HIPCHK(hipGetLastError());
    }

    // ---- smoothing steps (Sec. 3 eq. (smoother)) ----------------------------
    // u_out = u_in + M (f - K u_in) with M = D^{-1} (l1-Jacobi) or the degree-4
    // polynomial p(D^{-1}K) D^{-1}.  At level 0 the last sweep may write the
    // FP64 output with dot partials (dots != 0).
    template <typename VT, typename FT, typename OT>
    void sweep(int l, const FT *f, const VT *uin, OT *uout, int ndot, const double *g0, const double *g1)
    {
        Level &L = lev[l];
        if (!L.poly_on) {
            if (ndot == 2) sell<VT, FT, OT, EPI_SMOOTH, 2>(l, uin, f, L.invd<VT>(), uout, g0, g1);
            else if (ndot == 1) sell<VT, FT, OT, EPI_SMOOTH, 1>(l, uin, f, L.invd<VT>(), uout, g0, g1);
            else sell<VT, FT, OT, EPI_SMOOTH, 0>(l, uin, f, L.invd<VT>(), uout, g0, g1);
            if (ndot) vc_nb = sell_blocks(l) * SELL_WAVES;
            return;
        }
        VT *res = (VT *)L.r, *c = (VT *)L.c, *c2 = (VT *)L.c2;
        sell<VT, FT, VT, EPI_RESID, 0>(l, uin, f, L.invd<VT>(), res, nullptr, nullptr);
        const VT *cr = poly_apply<VT, VT>(l, res, c, c2);
        finish_sweep<VT, OT>(l, uin, cr, uout, ndot, g0, g1);
    }
    // Horner from zero: c = a3 D^{-1} r, then c = a_k D^{-1} r + D^{-1} K c.
    template <typename VT, typename FT> VT *poly_apply(int l, const FT *rr, VT *&c, VT *&c2)
    {
        Level &L = lev[l];
        hipLaunchKernelGGL((k_scale_coef<VT, FT>), dim3(nblocks(L.n)), dim3(256), 0, stream, L.n, L.invd<VT>(), rr,
                           c, (VT)L.poly[3]);
        HIPCHK(hipGetLastError());
        for (int k = 2; k >= 0; k--) {
            sell<VT, FT, VT, EPI_POLY, 0>(l, c, rr, L.invd<VT>(), c2, nullptr, nullptr, (VT)L.poly[k]);
            std::swap(c, c2);
        }
        return c;
    }
    template <typename VT, typename OT>
    void finish_sweep(int l, const VT *uin, const VT *c, OT *uout, int ndot, const double *g0, const double *g1)
    {
        Level &L = lev[l];
        hipLaunchKernelGGL((k_add<VT, OT>), dim3(nblocks(L.n)), dim3(256), 0, stream, L.n, uin, c, uout);
        HIPCHK(hipGetLastError());
        if (ndot) vc_nb = dot_partials(L.n, (const double *)uout, g0, g1);
    }

    // ---- the V-cycle (Sec. 3, steps 1-5, recursively) -----------------------
    // Level l solves approximately K_l u = f with a zero initial guess and
    // returns where the result lives.  At level 0, the last post-smoothing sweep
    // writes zout (FP64) and the dot partials for the Krylov scalars.
    template <typename VT, typename FT>
    VT *vlevel(int l, const FT *f, double *zout, int ndot, const double *g0, const double *g1, bool u_ready)
    {
        TxRange tx(level_label(l));
        Level &L = lev[l];
        VT *u = (VT *)L.u, *u2 = (VT *)L.u2;
        // 1. pre-smoothing from the zero guess
        if (!u_ready) {
            if (L.poly_on) {
                VT *c = (VT *)L.c, *c2 = (VT *)L.c2;
                VT *res = poly_apply<VT, FT>(l, f, c, c2);
                copy<VT, VT>(L.n, res, u);
            } else {
                hipLaunchKernelGGL((k_scale<VT, FT>), dim3(nblocks(L.n)), dim3(256), 0, stream, L.n, L.invd<VT>(),
                                   f, u);
                HIPCHK(hipGetLastError());
            }
        } else if (L.poly_on) {
            // the restriction wrote a3 D^{-1} f into u: finish Horner from there
            VT *c = u, *c2 = (VT *)L.c2;
            for (int k = 2; k >= 0; k--) {
                sell<VT, FT, VT, EPI_POLY, 0>(l, c, f, L.invd<VT>(), c2, nullptr, nullptr, (VT)L.poly[k]);
                std::swap(c, c2);
            }
            if (c != u) copy<VT, VT>(L.n, c, u);
        }
        for (int s = 1; s < prm.nu_pre; s++) {
            sweep<VT, FT, VT>(l, f, u, u2, 0, nullptr, nullptr);
            std::swap(u, u2);
        }
        // 2. residual and restriction (fused with the coarse pre-smoothing)
        sell<VT, FT, VT, EPI_RESID, 0>(l, u, f, L.invd<VT>(), (VT *)L.r, nullptr, nullptr);
        Level &C = lev[l + 1];
        const bool coarsest = (l + 1 == nlev - 1);
        const VT a3 = C.poly_on ? (VT)C.poly[3] : (VT)1;
        hipLaunchKernelGGL((k_restrict<VT>), dim3(nblocks(C.n)), dim3(256), 0, stream, C.n, L.mw, L.members,
                           L.pc<VT>(), (const VT *)L.r, (VT *)C.f, coarsest ? nullptr : C.invd<VT>(),
                           coarsest ? nullptr : (VT *)C.u, a3);
        HIPCHK(hipGetLastError());
        // 3. coarse solve
        VT *e;
        if (coarsest) {
            e = (VT *)C.u;
            hipLaunchKernelGGL((k_coarse_solve<VT>), dim3(1), dim3(256), 0, stream, nL, ldL, Linv, LinvT,
                               (const VT *)C.f, e);
            HIPCHK(hipGetLastError());
        } else if (l + 1 == tail_start && tail_usable()) {
            e = run_tail<VT>(false);
        } else {
            e = vlevel<VT, VT>(l + 1, (const VT *)C.f, nullptr, 0, nullptr, nullptr, true);
        }
        // 4. + 5.: with l1-Jacobi the prolongation is fused into the first
        // post-smoothing sweep through K P (f - K (u + P e) = r - (K P) e)
        int s0 = 1;
        if (!L.poly_on && prm.nu_post >= 1 && L.KP.soff && fuse_post) {
            if (zout && prm.nu_post == 1) {
                vc_nb = post_fused<VT, double>(l, e, u, zout, ndot, g0, g1);
                return nullptr;
            }
            post_fused<VT, VT>(l, e, u, u2, 0, nullptr, nullptr);
            std::swap(u, u2);
            s0 = 2;
        } else if (L.poly_on && prm.nu_post >= 1 && L.KP.soff && fuse_post) {
            // polynomial smoother: the first step's residual f - K (u + P e) = r - (K P) e
            VT *c = (VT *)L.c, *c2 = (VT *)L.c2;
            post_res_fused<VT>(l, e, u, u2);
            std::swap(u, u2);
            const VT *cr = poly_apply<VT, VT>(l, (const VT *)L.r, c, c2);
            if (zout && prm.nu_post == 1) {
                finish_sweep<VT, double>(l, u, cr, zout, ndot, g0, g1);
                return nullptr;
            }
            finish_sweep<VT, VT>(l, u, cr, u2, 0, nullptr, nullptr);
            std::swap(u, u2);
            s0 = 2;
        } else {
            hipLaunchKernelGGL((k_prolong<VT>), dim3(nblocks(L.n)), dim3(256), 0, stream, L.n, L.agg, L.pc<VT>(), e, u);
            HIPCHK(hipGetLastError());
        }
        for (int s = s0; s <= prm.nu_post; s++) {
            if (zout && s == prm.nu_post) {
                sweep<VT, FT, double>(l, f, u, zout, ndot, g0, g1);
                return nullptr;
            }
            sweep<VT, FT, VT>(l, f, u, u2, 0, nullptr, nullptr);
            std::swap(u, u2);
        }
        if (zout) {
            copy<double, VT>(L.n, u, zout);
            if (ndot) vc_nb = dot_partials(L.n, zout, g0, g1);
            return nullptr;
        }
        return u;
    }

    // ---- the smoothed-aggregation form (Sec. 3.1 variants, Sec. 3.2, Sec. 5.1) --
    // Any of: fourth-kind Chebyshev smoother, smoothed prolongator, CG coarse
    // solver.  FP64, single vector.
    bool general_vcycle() const { return prm.smoother == 2 || prm.smooth_prolong || prm.coarse_solver == 1; }

    void coarsest_solve(const double *f, double *e)
    {
        if (prm.coarse_solver == 1)
            hipLaunchKernelGGL(k_coarse_cg, dim3(1), dim3(CG_THREADS), 0, stream, nL, cg_rp, cg_ci, cg_v, cg_dj, f,
                               e, prm.coarse_tol, prm.coarse_itmax);
        else
            hipLaunchKernelGGL((k_coarse_solve<double>), dim3(1), dim3(256), 0, stream, nL, ldL, Linv, LinvT, f, e);
        HIPCHK(hipGetLastError());
    }

    // One Chebyshev matrix pass over K_l (modes of k_sell_cheb).
    template <int MODE>
    void cheb(int l, const double *x, const double *f, double *r, double *u, double *dn, double a, double b,
              int first)
    {
        const Level &L = lev[l];
        const DevMat &A = L.A;
        if (A.lpr) {
            const unsigned g = (unsigned)((A.n * A.lpr + 255) / 256);
#define CSR_CHEB(LP) hipLaunchKernelGGL((k_csr_cheb<LP, MODE>), dim3(g), dim3(256), 0, stream, A.n, A.crp, A.cci, \
                                        A.cv, x, f, r, L.invd64, u, dn, a, b, first)
            switch (A.lpr) {
            case 8: CSR_CHEB(8); break;
            case 16: CSR_CHEB(16); break;
            case 32: CSR_CHEB(32); break;
            default: CSR_CHEB(64); break;
            }
#undef CSR_CHEB
            HIPCHK(hipGetLastError());
            return;
        }
        unsigned nb = (unsigned)((A.nslices + SELL_WAVES - 1) / SELL_WAVES);
        if (l == 0) prof_begin();
        if (A.idx16)
            hipLaunchKernelGGL((k_sell_cheb<uint16_t, MODE>), dim3(nb), dim3(256), 0, stream,
                               A.sv<double, uint16_t>(), x, f, r, L.invd64, u, dn, a, b, first);
        else
            hipLaunchKernelGGL((k_sell_cheb<int32_t, MODE>), dim3(nb), dim3(256), 0, stream,
                               A.sv<double, int32_t>(), x, f, r, L.invd64, u, dn, a, b, first);
        HIPCHK(hipGetLastError());
        if (l == 0) {
            // vectors: MODE 0 reads x (gathered once), f, invd and writes r, dn;
            // MODES 1/2 read x, r or f, u unless first, and write u, r; MODE 1
            // also reads invd and writes dn
            const int nvec = MODE == 0 ? 5 : (first ? 4 : 5) + (MODE == 1 ? 2 : 0);
            prof_end(pass_bytes(8, nvec), AMG_PASS_OTHER);
        }
    }

    // Level l of the V-cycle in this form; returns where the result lives
    // (level 0 writes zout with the dot partials instead).
    double *vgen(int l, const double *f, double *zout, int ndot, const double *g0, const double *g1)
    {
        Level &L = lev[l];
        double *u = (double *)L.u, *u2 = (double *)L.u2, *d = (double *)L.c, *d2 = (double *)L.c2;
        double *r = (double *)L.r;
        const bool ch = prm.smoother == 2;
        const int k = prm.cheb_degree;
        const unsigned g = nblocks(L.n);
        // 1. pre-smoothing from the zero guess, leaving r = f - K u
        if (ch) {
            hipLaunchKernelGGL((k_scale_coef<double, double>), dim3(g), dim3(256), 0, stream, L.n, L.invd64, f, d,
                               4.0 / 3.0);
            HIPCHK(hipGetLastError());
            for (int j = 1; j < k; j++) {
                cheb<1>(l, d, f, r, u, d2, (2.0 * j - 1.0) / (2.0 * j + 3.0), (8.0 * j + 4.0) / (2.0 * j + 3.0),
                        j == 1);
                std::swap(d, d2);
            }
            cheb<2>(l, d, f, r, u, nullptr, 0.0, 0.0, k == 1);
        } else {
            hipLaunchKernelGGL((k_scale<double, double>), dim3(g), dim3(256), 0, stream, L.n, L.invd64, f, u);
            HIPCHK(hipGetLastError());
            for (int s = 1; s < prm.nu_pre; s++) {
                sweep<double, double, double>(l, f, u, u2, 0, nullptr, nullptr);
                std::swap(u, u2);
            }
            sell<double, double, double, EPI_RESID, 0>(l, u, f, L.invd64, r, nullptr, nullptr);
        }
        // 2. restriction f_c = P^T r
        Level &C = lev[l + 1];
        const bool coarsest = (l + 1 == nlev - 1);
        if (L.Rm.built()) {
            apply<EPI_SPMV>(L.Rm, r, nullptr, (double *)C.f);
        } else {
            hipLaunchKernelGGL((k_restrict<double>), dim3(nblocks(C.n)), dim3(256), 0, stream, C.n, L.mw,
                               L.members, L.pc64, (const double *)r, (double *)C.f, nullptr, nullptr, 1.0);
            HIPCHK(hipGetLastError());
        }
        // 3. coarse correction
        double *e;
        if (coarsest) {
            e = (double *)C.u;
            coarsest_solve((const double *)C.f, e);
        } else {
            e = vgen(l + 1, (const double *)C.f, nullptr, 0, nullptr, nullptr);
        }
        // 4. prolongation u += P e
        if (L.Pm.built()) {
            apply<EPI_ADD>(L.Pm, e, u, u2);
            std::swap(u, u2);
        } else {
            hipLaunchKernelGGL((k_prolong<double>), dim3(g), dim3(256), 0, stream, L.n, L.agg, L.pc64, e, u);
            HIPCHK(hipGetLastError());
        }
        // 5. post-smoothing
        if (ch) {
            cheb<0>(l, u, f, r, nullptr, d, 0.0, 4.0 / 3.0, 0);
            for (int j = 1; j < k; j++) {
                cheb<1>(l, d, f, r, u, d2, (2.0 * j - 1.0) / (2.0 * j + 3.0), (8.0 * j + 4.0) / (2.0 * j + 3.0), 0);
                std::swap(d, d2);
            }
            if (zout) {
                hipLaunchKernelGGL((k_add<double, double>), dim3(g), dim3(256), 0, stream, L.n, u, d, zout);
                HIPCHK(hipGetLastError());
                if (ndot) vc_nb = dot_partials(L.n, zout, g0, g1);
                return nullptr;
            }
            hipLaunchKernelGGL((k_add<double, double>), dim3(g), dim3(256), 0, stream, L.n, u, d, u2);
            HIPCHK(hipGetLastError());
            return u2;
        }
        for (int s = 1; s <= prm.nu_post; s++) {
            if (zout && s == prm.nu_post) {
                sweep<double, double, double>(l, f, u, zout, ndot, g0, g1);
                return nullptr;
            }
            sweep<double, double, double>(l, f, u, u2, 0, nullptr, nullptr);
            std::swap(u, u2);
        }
        if (zout) {
            copy<double, double>(L.n, u, zout);
            if (ndot) vc_nb = dot_partials(L.n, zout, g0, g1);
            return nullptr;
        }
        return u;
    }

    // z = B r; when ndot > 0 the partials of (z, g0) [and (z, g1)] are left in
    // `partial` and the number of blocks to finalize is returned.
    unsigned vcycle(const double *rin, double *zout, int ndot, const double *g0, const double *g1)
    {
        vc_nb = 0;
        if (general_vcycle()) {
            if (nlev == 1) {
                coarsest_solve(rin, zout);
                if (ndot) vc_nb = dot_partials(n, zout, g0, g1);
            } else {
                vgen(0, rin, zout, ndot, g0, g1);
            }
            return vc_nb;
        }
        if (nlev == 1) {
            hipLaunchKernelGGL((k_coarse_solve<double>), dim3(1), dim3(256), 0, stream, nL, ldL, Linv, LinvT, rin,
                               zout);
            HIPCHK(hipGetLastError());
            if (ndot) vc_nb = dot_partials(n, zout, g0, g1);
            return vc_nb;
        }
        if (fp32()) vlevel<float, double>(0, rin, zout, ndot, g0, g1, false);
        else vlevel<double, double>(0, rin, zout, ndot, g0, g1, false);
        return vc_nb;
    }

    // ---- batched (16 columns) ------------------------------------------------
    void blk_alloc()
    {
        if (bR) return;
        const size_t vsz = fp32() ? sizeof(float) : sizeof(double);
        for (int l = 0; l < nlev; l++) {
            Level &L = lev[l];
            size_t nn = (size_t)L.n * NB * vsz;
            L.bf = alloc<char>(nn); L.bu = alloc<char>(nn); L.bu2 = alloc<char>(nn);
            L.br = alloc<char>(nn); L.bc = alloc<char>(nn); L.bc2 = alloc<char>(nn);
        }
        size_t nb = (size_t)n * NB;
        bR = alloc<double>(nb); bZ = alloc<double>(nb); bP = alloc<double>(nb);
        bQ = alloc<double>(nb); bU = alloc<double>(nb); bF = alloc<double>(nb);
        bY = alloc<double>((size_t)std::max(nL, 1) * NB);
        bsc = alloc<double>(B_NSLOTS * NB);
        bpartial = alloc<double>((size_t)partial_cap * NB);
        bstrided = alloc<double>((size_t)2 * NB * FIN_THREADS);
        bgram = alloc<double>((size_t)GRAM_BLOCKS * 512);
        bcoef = alloc<double>(256);
        bgsave = alloc<double>(256);
        if (tail_start > 0) tail_dev_blk = fp32() ? tail_descriptors<float>(true) : tail_descriptors<double>(true);
        HIPCHK(hipHostMalloc((void **)&hbsc, B_NSLOTS * NB * sizeof(double), hipHostMallocDefault));
    }
    unsigned blk_grid(const DevMat &B) const
    {
        int64_t wpb = blk_threads / 64;
        int64_t g = (B.nslices + wpb - 1) / wpb;
        return (unsigned)std::max<int64_t>(1, std::min<int64_t>(g, blk_threads == 512 ? 2048 : 4096));
    }
    template <typename VT, typename FT, typename OT, int EPI, int NDOT, int LPR>
    unsigned launch_sellb(const DevMat &B, const VT *x, const FT *f, const VT *invd, OT *y, const double *g0,
                          const double *g1, VT coef)
    {
        unsigned g = blk_grid(B);
        if (B.idx16)
            hipLaunchKernelGGL((k_sellb<VT, FT, OT, uint16_t, EPI, NDOT, LPR>), dim3(g), dim3(blk_threads), 0, stream,
                               B.sv<VT, uint16_t>(), x, f, invd, y, g0, g1, bpartial, coef);
        else
            hipLaunchKernelGGL((k_sellb<VT, FT, OT, int32_t, EPI, NDOT, LPR>), dim3(g), dim3(blk_threads), 0, stream,
                               B.sv<VT, int32_t>(), x, f, invd, y, g0, g1, bpartial, coef);
        return g;
    }
    // Block matrix pass on level l; returns the number of dot-partial blocks.
    template <typename VT, typename FT, typename OT, int EPI, int NDOT>
    unsigned sell_blk(int l, const VT *x, const FT *f, const VT *invd, OT *y, const double *g0, const double *g1,
                      VT coef = 1)
    {
        const DevMat &A = lev[l].A;
        const DevMat &B = lev[l].Ab;
        unsigned nb;
        if (l == 0) prof_begin();
        if (blk_win > 0 && A.nshared > 0 && A.shrun && A.val<VT>()) {
            // stencil image: staged x windows, blk_win rows per lane; the grid
            // is padded to a multiple of the XCD count (XCD-aware slice order)
            const unsigned lgrid = sell_blocks(l);
            const unsigned grid = xcd_grid(lgrid);
            nb = lgrid * SELL_WAVES;   // dot partials: one per wavefront of a logical block
#define BLKW(IT, R) hipLaunchKernelGGL((k_sellw_blk<VT, FT, OT, IT, EPI, NDOT, R>), dim3(grid), dim3(256), 0, stream, \
                                       A.sv<VT, IT>(), x, f, invd, y, g0, g1, bpartial, coef)
#define BLKWS(IT, R) hipLaunchKernelGGL((k_sellws_blk<VT, FT, OT, IT, EPI, NDOT, R>), dim3(grid), dim3(256), 0, \
                                        stream, A.sv<VT, IT>(), x, f, invd, y, g0, g1, bpartial, coef)
            if ((blk_share & (sizeof(VT) == 8 ? 1 : 2)) && A.wgtab) {
                if (A.idx16) {
                    if (blk_win == 2) BLKWS(uint16_t, 2);
                    else BLKWS(uint16_t, 4);
                } else {
                    if (blk_win == 2) BLKWS(int32_t, 2);
                    else BLKWS(int32_t, 4);
                }
            } else if (A.idx16) {
                if (blk_win == 2) BLKW(uint16_t, 2);
                else BLKW(uint16_t, 4);
            } else {
                if (blk_win == 2) BLKW(int32_t, 2);
                else BLKW(int32_t, 4);
            }
#undef BLKW
#undef BLKWS
        } else if (blk_lpr > 1 && B.soff && B.val<VT>()) {
            nb = blk_lpr == 4   ? launch_sellb<VT, FT, OT, EPI, NDOT, 4>(B, x, f, invd, y, g0, g1, coef)
                 : blk_lpr == 8 ? launch_sellb<VT, FT, OT, EPI, NDOT, 8>(B, x, f, invd, y, g0, g1, coef)
                                : launch_sellb<VT, FT, OT, EPI, NDOT, 16>(B, x, f, invd, y, g0, g1, coef);
        } else {
            const unsigned grid = sell_blocks(l);
            nb = grid * SELL_WAVES;   // dot partials: one per wavefront
#define BLK1(KER, IT) hipLaunchKernelGGL((KER<VT, FT, OT, IT, EPI, NDOT>), dim3(grid), dim3(256), 0, stream, \
                                         A.sv<VT, IT>(), x, f, invd, y, g0, g1, bpartial, coef)
            if (A.idx16) BLK1(k_sell_blk, uint16_t);
            else BLK1(k_sell_blk, int32_t);
#undef BLK1
        }
        HIPCHK(hipGetLastError());
        if (l == 0) {
            // 16 columns: matrix once, 16 vectors of each kind
            const DevMat &M = lev[0].A;
            // 16 columns: matrix once; X read and Y written once; F for the
            // residual, smoother and polynomial passes; invd per row; the FP64
            // dot partners (SpMV: G1 with two dots; smoother: G0, G1)
            const bool usesF = EPI == EPI_RESID || EPI == EPI_SMOOTH || EPI == EPI_POLY;
            const int ndp = EPI == EPI_SPMV ? (NDOT >= 2 ? 1 : 0) : EPI == EPI_SMOOTH ? NDOT : 0;
            double bytes = (double)M.nnz * sizeof(VT) + M.index_bytes +
                           (double)NB * M.n * (sizeof(VT) + sizeof(OT) + (usesF ? sizeof(FT) : 0) + 8.0 * ndp) +
                           ((EPI == EPI_SMOOTH || EPI == EPI_POLY) ? (double)sizeof(VT) * M.n : 0.0);
            prof_end(bytes, pass_kind(EPI));
        }
        return nb;
    }
    void bfinalize(unsigned nblk, int op, double tol = 0.0)
    {
        // many partials (one per wavefront of a level-0 pass): the strided sums
        // of the single final block over a wide grid first
        const double *st = nullptr;
        if (nblk > 4 * FIN_THREADS) {
            hipLaunchKernelGGL(k_bfin_strided, dim3(2 * NB * FIN_THREADS / 256), dim3(256), 0, stream, bpartial,
                               (int)nblk, bstrided);
            st = bstrided;
        }
        hipLaunchKernelGGL(k_bfinalize, dim3(1), dim3(FIN_THREADS), 0, stream, bpartial, (int)nblk, bsc, op, tol, st);
        HIPCHK(hipGetLastError());
    }
    // grid of the element-parallel block vector kernels (a multiple of 16 threads)
    unsigned bgrid(int64_t rows) const
    {
        return (unsigned)std::max<int64_t>(1, std::min<int64_t>(4096, (rows * NB + 255) / 256));
    }
    template <typename VT> void coarse_blk(const VT *f, VT *e)
    {
        const unsigned g = (unsigned)((nL + 256 / NB - 1) / (256 / NB));
        hipLaunchKernelGGL((k_coarse_solve_blk<VT>), dim3(g), dim3(256), 0, stream, nL, ldL, Linv, LinvT, f, bY, e, 0);
        hipLaunchKernelGGL((k_coarse_solve_blk<VT>), dim3(g), dim3(256), 0, stream, nL, ldL, Linv, LinvT, f, bY, e, 1);
        HIPCHK(hipGetLastError());
    }
    unsigned bdot_partials(int64_t m, const double *a, const double *b, const double *c)
    {
        unsigned g = bgrid(m);
        hipLaunchKernelGGL(k_dot2_blk, dim3(g), dim3(256), 0, stream, m, a, b, c, bpartial);
        HIPCHK(hipGetLastError());
        return g;
    }
    // Block fused prolongation + first post-smoothing sweep; returns the dot-partial blocks.
    template <typename VT, typename OT>
    unsigned bpost_fused(int l, const VT *E, const VT *U, OT *Y, int ndot, const double *g0, const double *g1)
    {
        Level &L = lev[l];
        const bool multi = blk_lpr > 1 && L.KPb.soff;
        const DevMat &A = multi ? L.KPb : L.KP;
        unsigned nb = multi ? blk_grid(A) : (unsigned)((A.nslices + SELL_WAVES - 1) / SELL_WAVES);
        unsigned thr = multi ? (unsigned)blk_threads : 256u;
        if (l == 0) prof_begin();
#define BPOST(KERN, IT, IDX)                                                                                    \
    hipLaunchKernelGGL(KERN, dim3(nb), dim3(thr), 0, stream, A.sv<VT, IT>(), E, U, (const VT *)L.br, L.invd<VT>(), \
                       L.agg, L.pc<VT>(), Y, g0, g1, bpartial)
#define BPOST_ND(IT, IDX, ND)                                                                                   \
    do {                                                                                                        \
        if (!multi) BPOST((k_sell_blk_post<VT, OT, IT, ND>), IT, IDX);                                          \
        else if (blk_lpr == 4) BPOST((k_sellb_post<VT, OT, IT, ND, 4>), IT, IDX);                               \
        else if (blk_lpr == 8) BPOST((k_sellb_post<VT, OT, IT, ND, 8>), IT, IDX);                               \
        else BPOST((k_sellb_post<VT, OT, IT, ND, 16>), IT, IDX);                                                \
    } while (0)
        if (A.idx16) {
            if (ndot == 2) BPOST_ND(uint16_t, A.d16, 2);
            else if (ndot == 1) BPOST_ND(uint16_t, A.d16, 1);
            else BPOST_ND(uint16_t, A.d16, 0);
        } else {
            if (ndot == 2) BPOST_ND(int32_t, A.c32, 2);
            else if (ndot == 1) BPOST_ND(int32_t, A.c32, 1);
            else BPOST_ND(int32_t, A.c32, 0);
        }
#undef BPOST_ND
#undef BPOST
        HIPCHK(hipGetLastError());
        if (l == 0) {
            double bytes = (double)A.nnz * sizeof(VT) + A.index_bytes + (double)NB * sizeof(VT) * lev[1].n + (double)NB * sizeof(VT) * A.n * 2 +
                           (double)sizeof(VT) * A.n * 2 + 4.0 * A.n + (double)NB * sizeof(OT) * A.n +
                           8.0 * NB * A.n * ndot;
            prof_end(bytes, AMG_PASS_KP);
        }
        return multi ? nb : nb * SELL_WAVES;   // one-lane kernel: a dot partial per wavefront
    }
    template <typename VT, typename FT> VT *bpoly_apply(int l, const FT *rr, VT *&c, VT *&c2)
    {
        Level &L = lev[l];
        hipLaunchKernelGGL((k_scale_blk<VT, FT>), dim3(nblocks(L.n)), dim3(256), 0, stream, L.n, L.invd<VT>(), rr,
                           c, (VT)L.poly[3]);
        HIPCHK(hipGetLastError());
        for (int k = 2; k >= 0; k--) {
            sell_blk<VT, FT, VT, EPI_POLY, 0>(l, c, rr, L.invd<VT>(), c2, nullptr, nullptr, (VT)L.poly[k]);
            std::swap(c, c2);
        }
        return c;
    }
    template <typename VT, typename FT, typename OT>
    void bsweep(int l, const FT *f, const VT *uin, OT *uout, int ndot, const double *g0, const double *g1)
    {
        Level &L = lev[l];
        if (!L.poly_on) {
            unsigned nb;
            if (ndot == 2) nb = sell_blk<VT, FT, OT, EPI_SMOOTH, 2>(l, uin, f, L.invd<VT>(), uout, g0, g1);
            else if (ndot == 1) nb = sell_blk<VT, FT, OT, EPI_SMOOTH, 1>(l, uin, f, L.invd<VT>(), uout, g0, g1);
            else nb = sell_blk<VT, FT, OT, EPI_SMOOTH, 0>(l, uin, f, L.invd<VT>(), uout, g0, g1);
            if (ndot) vc_nb = nb;
            return;
        }
        VT *res = (VT *)L.br, *c = (VT *)L.bc, *c2 = (VT *)L.bc2;
        sell_blk<VT, FT, VT, EPI_RESID, 0>(l, uin, f, L.invd<VT>(), res, nullptr, nullptr);
        const VT *cr = bpoly_apply<VT, VT>(l, res, c, c2);
        hipLaunchKernelGGL((k_add_blk<VT, OT>), dim3(nblocks(L.n * NB)), dim3(256), 0, stream, L.n, uin, cr, uout);
        HIPCHK(hipGetLastError());
        if (ndot) vc_nb = bdot_partials(L.n, (const double *)uout, g0, g1);
    }
    template <typename VT, typename FT>
    VT *vlevel_blk(int l, const FT *f, double *zout, int ndot, const double *g0, const double *g1, bool u_ready)
    {
        TxRange tx(level_label(l));
        Level &L = lev[l];
        VT *u = (VT *)L.bu, *u2 = (VT *)L.bu2;
        if (!u_ready) {
            if (L.poly_on) {
                VT *c = (VT *)L.bc, *c2 = (VT *)L.bc2;
                VT *res = bpoly_apply<VT, FT>(l, f, c, c2);
                hipLaunchKernelGGL((k_copy<VT, VT>), dim3(vgrid(L.n * NB)), dim3(256), 0, stream, L.n * NB,
                                   (const VT *)res, u);
            } else {
                hipLaunchKernelGGL((k_scale_blk<VT, FT>), dim3(nblocks(L.n)), dim3(256), 0, stream, L.n,
                                   L.invd<VT>(), f, u, (VT)1);
            }
            HIPCHK(hipGetLastError());
        } else if (L.poly_on) {
            VT *c = u, *c2 = (VT *)L.bc2;
            for (int k = 2; k >= 0; k--) {
                sell_blk<VT, FT, VT, EPI_POLY, 0>(l, c, f, L.invd<VT>(), c2, nullptr, nullptr, (VT)L.poly[k]);
                std::swap(c, c2);
            }
            if (c != u) copy<VT, VT>(L.n * NB, c, u);
        }
        for (int s = 1; s < prm.nu_pre; s++) {
            bsweep<VT, FT, VT>(l, f, u, u2, 0, nullptr, nullptr);
            std::swap(u, u2);
        }
        sell_blk<VT, FT, VT, EPI_RESID, 0>(l, u, f, L.invd<VT>(), (VT *)L.br, nullptr, nullptr);
        Level &C = lev[l + 1];
        const bool coarsest = (l + 1 == nlev - 1);
        const VT a3 = C.poly_on ? (VT)C.poly[3] : (VT)1;
        hipLaunchKernelGGL((k_restrict_blk<VT>), dim3(nblocks(C.n)), dim3(256), 0, stream, C.n, L.mw, L.members,
                           L.pc<VT>(), (const VT *)L.br, (VT *)C.bf, coarsest ? nullptr : C.invd<VT>(),
                           coarsest ? nullptr : (VT *)C.bu, a3);
        HIPCHK(hipGetLastError());
        VT *e;
        if (coarsest) {
            e = (VT *)C.bu;
            coarse_blk<VT>((const VT *)C.bf, e);
        } else if (l + 1 == tail_start && tail_usable()) {
            e = run_tail<VT>(true);
        } else {
            e = vlevel_blk<VT, VT>(l + 1, (const VT *)C.bf, nullptr, 0, nullptr, nullptr, true);
        }
        int s0 = 1;
        if (!L.poly_on && prm.nu_post >= 1 && L.KP.soff && fuse_post) {
            if (zout && prm.nu_post == 1) {
                vc_nb = bpost_fused<VT, double>(l, e, u, zout, ndot, g0, g1);
                return nullptr;
            }
            bpost_fused<VT, VT>(l, e, u, u2, 0, nullptr, nullptr);
            std::swap(u, u2);
            s0 = 2;
        } else {
            hipLaunchKernelGGL((k_prolong_blk<VT>), dim3(nblocks(L.n)), dim3(256), 0, stream, L.n, L.agg, L.pc<VT>(),
                               e, u);
            HIPCHK(hipGetLastError());
        }
        for (int s = s0; s <= prm.nu_post; s++) {
            if (zout && s == prm.nu_post) {
                bsweep<VT, FT, double>(l, f, u, zout, ndot, g0, g1);
                return nullptr;
            }
            bsweep<VT, FT, VT>(l, f, u, u2, 0, nullptr, nullptr);
            std::swap(u, u2);
        }
        if (zout) {
            copy<double, VT>(L.n * NB, u, zout);
            if (ndot) vc_nb = bdot_partials(L.n, zout, g0, g1);
            return nullptr;
        }
        return u;
    }
    unsigned vcycle_blk(const double *rin, double *zout, int ndot, const double *g0, const double *g1)
    {
        vc_nb = 0;
        if (nlev == 1) {
            coarse_blk<double>(rin, zout);
            if (ndot) vc_nb = bdot_partials(n, zout, g0, g1);
            return vc_nb;
        }
        if (fp32()) vlevel_blk<float, double>(0, rin, zout, ndot, g0, g1, false);
        else vlevel_blk<double, double>(0, rin, zout, ndot, g0, g1, false);
        return vc_nb;
    }
};

// ---------------------------------------------------------------------------

static amg_status build_device(amg_ctx *c, const CsrView &K0)
{
    HostHierarchy &H = c->host;
    c->lev.resize(c->nlev);
    const bool fp32 = c->fp32();
    const size_t vsz = fp32 ? sizeof(float) : sizeof(double);
    for (int l = 0; l < c->nlev; l++) {
        auto &hl = H.lev[l];
        Level &L = c->lev[l];
        L.n = hl.n;
        L.nnz = hl.nnz;
        const bool coarsest = (l == c->nlev - 1);
        if (!coarsest || l == 0) {
            CsrView K = l == 0 ? K0 : amgiga::view(hl.K);
            // the Chebyshev passes of coarse levels may take the CSR image
            if (c->prm.smoother == 2 && l > 0) L.A = c->upload_image(K);
            else L.A = c->upload_sell(K, SLICE, (l == 0) || !fp32, fp32);
        }
        L.invd64 = c->upload(hl.invd);
        if (fp32) {
            std::vector<float> t(hl.invd.begin(), hl.invd.end());
            L.invd32 = c->upload(t);
        }
        if (!coarsest) {
            if (c->general_vcycle()) {
                if (!hl.P.rp.empty()) {
                    L.Pm = c->upload_image(amgiga::view(hl.P), H.lev[l + 1].n);
                    L.Rm = c->upload_image(amgiga::view(hl.PT), hl.n);
                }
            } else {
                CsrView K = l == 0 ? K0 : amgiga::view(hl.K);
                amgiga::Csr kp = amgiga::kp_product(K, H.lev[l + 1].n, hl.agg.data(), hl.pc.data());
                L.KP = c->upload_sell(amgiga::view(kp), SLICE, !fp32, fp32, H.lev[l + 1].n);
            }
            L.agg = c->upload(hl.agg);
            L.pc64 = c->upload(hl.pc);
            if (fp32) {
                std::vector<float> t(hl.pc.begin(), hl.pc.end());
                L.pc32 = c->upload(t);
            }
            int64_t nc = H.lev[l + 1].n;
            L.mw = hl.max_members;
            std::vector<int32_t> mem((size_t)(nc * L.mw), -1);
            std::vector<int> fill(nc, 0);
            for (int64_t i = 0; i < hl.n; i++) {
                int32_t I = hl.agg[i];
                mem[(size_t)I * L.mw + fill[I]++] = (int32_t)i;
            }
            L.members = c->upload(mem);
        }
        size_t nn = (size_t)hl.n;
        L.f = c->alloc<char>(nn * vsz);
        L.u = c->alloc<char>(nn * vsz);
        L.u2 = c->alloc<char>(nn * vsz);
        L.r = c->alloc<char>(nn * vsz);
        L.c = c->alloc<char>(nn * vsz);
        L.c2 = c->alloc<char>(nn * vsz);
    }
    // coarsest level: CSR and 1 / k_ii for the CG coarse solver, or the dense
    // Cholesky factor on the device, then the inverse factor
    if (c->prm.coarse_solver == 1) {
        auto &hl = H.lev.back();
        CsrView K = c->nlev == 1 ? K0 : amgiga::view(hl.K);
        if (K.n > CG_MAXN || K.nnz() >= (int64_t(1) << 31)) {
            set_err("coarsest level too large for the CG coarse solver");
            return AMG_ERR_ARG;
        }
        std::vector<int32_t> rp32(K.n + 1);
        std::vector<double> dj(K.n, 0.0);
        for (int64_t i = 0; i <= K.n; i++) rp32[i] = (int32_t)K.rp[i];
        for (int64_t i = 0; i < K.n; i++)
            for (int64_t k = K.rp[i]; k < K.rp[i + 1]; k++)
                if (K.ci[k] == i) dj[i] = 1.0 / K.v[k];
        c->cg_rp = c->upload(rp32);
        c->cg_ci = c->upload(std::vector<int32_t>(K.ci, K.ci + K.nnz()));
        c->cg_v = c->upload(std::vector<double>(K.v, K.v + K.nnz()));
        c->cg_dj = c->upload(dj);
        c->nL = (int)K.n;
        c->ldL = 0;
    } else {
        auto &hl = H.lev.back();
        int nl = (int)hl.n;
        int npad = (nl + 15) / 16 * 16;
        std::vector<double> A((size_t)npad * npad, 0.0);
        for (int i = 0; i < nl; i++)
            for (int j = 0; j <= i; j++) A[(size_t)i * npad + j] = H.coarse_lower[(size_t)i * nl + j];
        for (int i = nl; i < npad; i++) A[(size_t)i * npad + i] = 1.0;
        double *dA = c->upload(A);
        int *dst = c->alloc<int>(1);
        HIPCHK(hipMemsetAsync(dst, 0, sizeof(int), c->stream));
        hipLaunchKernelGGL(k_chol_mfma, dim3(1), dim3(256), 0, c->stream, npad, dA, dst);
        HIPCHK(hipGetLastError());
        int hst = 0;
        HIPCHK(hipMemcpyAsync(&hst, dst, sizeof(int), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
        if (hst) {
            set_err("coarsest matrix is not SPD (non-positive Cholesky pivot)");
            return AMG_ERR_NOT_SPD;
        }
        c->nL = nl;
        c->ldL = npad;
        c->Linv = c->alloc<double>((size_t)npad * npad);
        c->LinvT = c->alloc<double>((size_t)npad * npad);
        hipLaunchKernelGGL(k_tri_inv, dim3((nl + 255) / 256), dim3(256), 0, c->stream, nl, npad, dA, c->Linv,
                           c->LinvT);
        HIPCHK(hipGetLastError());
    }
    c->n = H.lev[0].n;
    c->r = c->alloc<double>(c->n);
    c->z = c->alloc<double>(c->n);
    c->p = c->alloc<double>(c->n);
    c->q = c->alloc<double>(c->n);
    c->partial_cap = 2 * std::max<int64_t>(4096, SELL_WAVES * c->sell_blocks(0));
    c->partial = c->alloc<double>(c->partial_cap);
    c->sc = c->alloc<double>(S_NSLOTS);
    HIPCHK(hipHostMalloc((void **)&c->hsc, S_NSLOTS * sizeof(double), hipHostMallocDefault));
    HIPCHK(hipEventCreateWithFlags(&c->ev_iter, hipEventDisableTiming));
    c->choose_tail();
    c->tune_xwin();
    if (c->prm.nrhs > 1) c->tune_blocks(K0);
    HIPCHK(hipStreamSynchronize(c->stream));
    return AMG_OK;
}

extern "C" {

amg_status amg_params_default(amg_params *p)
{
    if (!p) { set_err("NULL params"); return AMG_ERR_ARG; }
    p->sweeps_per_level = 2;
    p->max_coarse = 200;
    p->max_levels = 40;
    p->nu_pre = 1;
    p->nu_post = 1;
    p->vcycle_fp32 = 0;
    p->smoother = 0;
    p->krylov = 0;
    p->match_positive_only = 0;
    p->itmax = 1000;
    p->nrhs = 1;
    p->slice_offsets = 1;
    p->smooth_prolong = 0;
    p->cheb_degree = 8;
    p->coarse_solver = 0;
    p->coarse_itmax = 30;
    p->omega = 4.0 / 3.0;
    p->coarse_tol = 1e-4;
    p->setup_device = 0;
    p->bootstrap_sweeps = 0;
    return AMG_OK;
}

const char *amg_last_error(void) { return g_err.c_str(); }

static amg_status setup_common(int64_t n, const int64_t *row_ptr, const int32_t *col, const double *val,
                               const double *w, const amg_params *prm, void *hip_stream, int host_only,
                               amg_ctx **out)
{
    TxRange tx("amg_setup");
    g_err.clear();
    if (!out) { set_err("NULL out"); return AMG_ERR_ARG; }
    *out = nullptr;
    amg_params P;
    amg_params_default(&P);
    if (prm) P = *prm;
    if (P.sweeps_per_level < 1 || P.sweeps_per_level > 3 || P.max_coarse < 1 || P.max_coarse > 2000 ||
        P.max_levels < 1 || P.nu_pre < 1 || P.nu_post < 0 || P.itmax < 1 || P.krylov < 0 || P.krylov > 2 ||
        P.nrhs < 1 || P.nrhs > NB ||
        P.smoother < 0 || P.smoother > 2 || P.slice_offsets < 0 || P.slice_offsets > 1 ||
        P.smooth_prolong < 0 || P.smooth_prolong > 1 || P.cheb_degree < 1 || P.cheb_degree > 64 ||
        P.coarse_solver < 0 || P.coarse_solver > 1 || P.coarse_itmax < 1 || P.coarse_itmax > 1000 ||
        !(P.omega > 0.0 && P.omega <= 2.0) || !(P.coarse_tol >= 0.0 && std::isfinite(P.coarse_tol)) ||
        P.setup_device < 0 || P.setup_device > 1 || P.bootstrap_sweeps < 0 || P.bootstrap_sweeps > 1000) {
        set_err("parameter out of range");
        return AMG_ERR_ARG;
    }
    if (P.smoother == 2 || P.smooth_prolong || P.coarse_solver == 1) {
        if (P.vcycle_fp32 || P.nrhs != 1 || P.smoother == 1 || (P.smoother == 2 && (P.nu_pre != 1 || P.nu_post != 1))) {
            set_err("smoother 2, smooth_prolong and coarse_solver 1 take the FP64 single-vector V-cycle "
                    "(vcycle_fp32 0, nrhs 1, smoother 0 or 2, one Chebyshev step before and after)");
            return AMG_ERR_ARG;
        }
    }
    if (n <= 0 || !row_ptr || !col || !val) { set_err("n <= 0 or NULL CSR array"); return AMG_ERR_ARG; }
    if (P.bootstrap_sweeps > 0 && !w) { set_err("bootstrap_sweeps needs the random start in w"); return AMG_ERR_ARG; }
    if (P.setup_device && (host_only || P.smooth_prolong)) {
        set_err("setup_device needs a device context and the tentative prolongator (smooth_prolong 0)");
        return AMG_ERR_ARG;
    }
    if (!host_only && n >= (int64_t(1) << 29)) {
        // vector gathers use 32-bit byte offsets
        set_err("the device path takes at most 2^29 - 1 rows");
        return AMG_ERR_ARG;
    }
    CsrView K0{n, row_ptr, col, val};
    std::string err;
    if (amgiga::validate_csr(K0, err)) { set_err(err); return AMG_ERR_ARG; }
    if (w)
        for (int64_t i = 0; i < n; i++)
            if (!std::isfinite(w[i])) { set_err("non-finite test vector"); return AMG_ERR_ARG; }
    std::unique_ptr<amg_ctx> c;
    try {
        c.reset(new amg_ctx());
        c->prm = P;
        c->host_only = host_only;
        c->stream = (hipStream_t)hip_stream;
        amgiga::SetupParams sp;
        sp.sweeps = P.sweeps_per_level;
        sp.max_coarse = P.max_coarse;
        sp.max_levels = P.max_levels;
        sp.positive_only = P.match_positive_only;
        sp.smooth = P.smooth_prolong;
        sp.omega = P.omega;
        sp.coarse_dense = P.coarse_solver == 0;
        sp.bootstrap = P.bootstrap_sweeps;
        int rc;
        if (P.setup_device) {
            HIPCHK(hipGetDevice(&c->device));
            rc = amgiga::build_hierarchy_on_device(K0, w, sp, c->host, err, (void *)c->stream, &c->setup_info);
        } else {
            rc = amgiga::build_hierarchy(K0, w, sp, c->host, err);
        }
        if (rc) { set_err(err); return (amg_status)rc; }
        c->nlev = (int)c->host.lev.size();
        if (!host_only) {
            HIPCHK(hipGetDevice(&c->device));
            amg_status st = build_device(c.get(), K0);
            if (st != AMG_OK) return st;
        }
    } catch (Fail &f) {
        return f.st;
    } catch (std::bad_alloc &) {
        set_err("host allocation failed");
        return AMG_ERR_OOM;
    }
    *out = c.release();
    return AMG_OK;
}

amg_status amg_setup(int64_t n, const int64_t *row_ptr, const int32_t *col, const double *val, const double *w,
                     const amg_params *prm, void *hip_stream, amg_ctx **out)
{
    return setup_common(n, row_ptr, col, val, w, prm, hip_stream, 0, out);
}

amg_status amg_setup_host(int64_t n, const int64_t *row_ptr, const int32_t *col, const double *val,
                          const double *w, const amg_params *prm, amg_ctx **out)
{
    return setup_common(n, row_ptr, col, val, w, prm, nullptr, 1, out);
}

amg_status amg_sell_spmv_host(int64_t n, int64_t ncols, const int64_t *row_ptr, const int32_t *col,
                              const double *val, int C, int layout, const double *x, double *y,
                              int64_t *shared_slices, int64_t *stored)
{
    g_err.clear();
    if (n <= 0 || ncols <= 0 || !row_ptr || !col || !val || !x || !y || (C != 4 && C != 8 && C != 16 && C != 32 &&
        C != 64) || layout < 0 || layout > 4 || (layout >= 1 && layout != 2 && ncols != n) ||
        (layout >= 3 && C != SLICE)) {
        set_err("bad size, NULL array, slice height or layout");
        return AMG_ERR_ARG;
    }
    for (int64_t i = 0; i < n; i++) {
        if (row_ptr[i + 1] < row_ptr[i]) { set_err("row_ptr not ascending"); return AMG_ERR_ARG; }
        for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; k++)
            if (col[k] < 0 || col[k] >= ncols || (k > row_ptr[i] && col[k] <= col[k - 1])) {
                set_err("columns out of range or not ascending");
                return AMG_ERR_ARG;
            }
    }
    CsrView K{n, row_ptr, col, val};
    std::string err;
    const int st = amgiga::sell_spmv_walk(K, ncols, C, layout, x, y, shared_slices, stored, err);
    if (st != 0) set_err(err);
    return (amg_status)st;
}

amg_status amg_match(int64_t n, const int64_t *row_ptr, const int32_t *col, const double *val, const double *w,
                     int positive_only, int32_t *mate)
{
    g_err.clear();
    if (n <= 0 || !row_ptr || !col || !val || !mate) { set_err("n <= 0 or NULL array"); return AMG_ERR_ARG; }
    CsrView K{n, row_ptr, col, val};
    std::string err;
    if (amgiga::validate_csr(K, err)) { set_err(err); return AMG_ERR_ARG; }
    std::vector<double> ones;
    if (!w) { ones.assign(n, 1.0); w = ones.data(); }
    amgiga::suitor_match(K, w, positive_only, mate);
    return AMG_OK;
}

void amg_destroy(amg_ctx *c) { delete c; }

static amg_status solve_impl(amg_ctx *c, const double *F, double *u_user, double tol, int *iters, double *relres,
                             double *relres_true)
{
    TxRange tx("pcg_solve");
    const int64_t n = c->n;
    c->hist.clear();
    const bool flex = c->prm.krylov >= 1;
    const int itmax = c->prm.itmax;
    const bool graph = c->use_graph && !c->prof;
    amg_ctx::OnGraphStream on(c, graph);
    hipStream_t st = c->stream;
    double *u = u_user;
    if (graph) {
        if (!c->uw) c->uw = c->alloc<double>(n);
        u = c->uw;
        c->copy<double, double>(n, u_user, u);
    }
    c->evused = 0;
    c->evbytes.clear();
    hipLaunchKernelGGL((k_fill<double>), dim3(1), dim3(256), 0, st, (int64_t)S_NSLOTS, 0.0, c->sc);
    HIPCHK(hipGetLastError());
    // r = F - K u ; (F, F) ; (r, r)
    c->sell<double, double, double, EPI_RESID, 0>(0, u, F, c->lev[0].invd64, c->r, nullptr, nullptr);
    c->dot2(n, F, F, nullptr, FIN_STORE, S_FF);
    c->dot2(n, c->r, c->r, nullptr, FIN_STORE, S_RR);
    HIPCHK(hipMemcpyAsync(c->hsc, c->sc, S_NSLOTS * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    const double ff = c->hsc[S_FF];
    if (!std::isfinite(ff)) { set_err("non-finite right-hand side"); return AMG_ERR_ARG; }
    if (iters) *iters = 0;
    if (ff == 0.0) {
        hipLaunchKernelGGL((k_fill<double>), dim3(vgrid(n)), dim3(256), 0, st, n, 0.0, u_user);
        HIPCHK(hipStreamSynchronize(st));
        if (relres) *relres = 0.0;
        if (relres_true) *relres_true = 0.0;
        return AMG_OK;
    }
    const double nF = std::sqrt(ff);
    double rr = c->hsc[S_RR];
    c->hist.push_back(std::sqrt(rr) / nF);
    amg_status status = AMG_NOT_CONVERGED;
    int k = 0;
    // iteration body, part A: q = K p, (p, q) [, (p, r)] -> alpha;
    // u += alpha p, r -= alpha q, (r, r); scalars to the host
    auto partA = [&]() {
        if (flex) c->sell<double, double, double, EPI_SPMV, 2>(0, c->p, nullptr, nullptr, c->q, nullptr, c->r);
        else c->sell<double, double, double, EPI_SPMV, 1>(0, c->p, nullptr, nullptr, c->q, nullptr, nullptr);
        c->finalize(c->sell_blocks(0) * SELL_WAVES, flex ? FIN_PQ_FCG : FIN_PQ_CG);
        unsigned g = vgrid(n);
        hipLaunchKernelGGL(k_cg_update, dim3(g), dim3(256), 0, c->stream, n, c->sc, u, c->r, c->p, c->q, c->partial);
        HIPCHK(hipGetLastError());
        c->finalize(g, FIN_STORE, S_RR);
        HIPCHK(hipMemcpyAsync(c->hsc, c->sc, S_NSLOTS * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    };
    // part B: z = B r, beta, p = z + beta p
    auto partB = [&]() {
        unsigned nb2 = c->vcycle(c->r, c->z, 1, flex ? c->q : c->r, nullptr);
        c->finalize(nb2, flex ? FIN_ZQ_FCG : FIN_RZ_CG);
        hipLaunchKernelGGL(k_cg_pupdate, dim3(vgrid(n)), dim3(256), 0, c->stream, n, c->sc, c->z, c->p);
        HIPCHK(hipGetLastError());
    };
    if (std::sqrt(rr) <= tol * nF) {
        status = AMG_OK;
    } else {
        // z = B r ; (r, z) ; p = z
        unsigned nb = c->vcycle(c->r, c->z, flex ? 0 : 1, c->r, nullptr);
        if (!flex) c->finalize(nb, FIN_RZ0);
        c->copy<double, double>(n, c->z, c->p);
        if (graph && !c->gA[flex]) {
            c->gA[flex] = c->capture(partA);
            c->gB[flex] = c->capture(partB);
        }
        for (k = 1; k <= itmax; k++) {
            TxRange txi("pcg iteration");
            if (graph) HIPCHK(hipGraphLaunch(c->gA[flex], st));
            else partA();
            HIPCHK(hipEventRecord(c->ev_iter, st));
            // speculative: next preconditioned direction while the host tests convergence
            if (k < itmax) {
                if (graph) HIPCHK(hipGraphLaunch(c->gB[flex], st));
                else partB();
            }
            HIPCHK(hipEventSynchronize(c->ev_iter));
            if (c->hsc[S_FLAG] != 0.0) {
                status = AMG_ERR_BREAKDOWN;
                k = k - 1;
                set_err("CG breakdown: (p, K p) <= 0 or (r, B r) <= 0 or non-finite");
                break;
            }
            rr = c->hsc[S_RR];
            c->hist.push_back(std::sqrt(rr) / nF);
            if (std::sqrt(rr) <= tol * nF) { status = AMG_OK; break; }
        }
        if (k > itmax) k = itmax;
    }
    if (graph) c->copy<double, double>(n, u, u_user);
    HIPCHK(hipStreamSynchronize(st));
    c->prof_collect();
    if (iters) *iters = k;
    if (relres) *relres = std::sqrt(rr) / nF;
    if (relres_true) {
        int saved = c->prof;
        c->prof = 0;
        c->sell<double, double, double, EPI_RESID, 0>(0, u, F, c->lev[0].invd64, c->r, nullptr, nullptr);
        c->prof = saved;
        c->dot2(n, c->r, c->r, nullptr, FIN_STORE, S_TMP);
        HIPCHK(hipMemcpyAsync(c->hsc, c->sc, S_NSLOTS * sizeof(double), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        *relres_true = std::sqrt(c->hsc[S_TMP]) / nF;
    }
    return status;
}

amg_status pcg_solve(amg_ctx *c, const double *F, double *u, double tol, int *iters, double *relres,
                     double *relres_true)
{
    g_err.clear();
    if (!c || !F || !u || !(tol >= 0.0)) { set_err("NULL argument or tol < 0"); return AMG_ERR_ARG; }
    if (c->host_only) { set_err("context was built by amg_setup_host"); return AMG_ERR_STATE; }
    if (F == u) { set_err("F and u alias"); return AMG_ERR_ARG; }
    try {
        return solve_impl(c, F, u, tol, iters, relres, relres_true);
    } catch (Fail &f) {
        return f.st;
    }
}

// Block flexible CG over the batch (krylov = 2): one block of up to 16 columns
// shares every Krylov step, alpha = G^{-1} P^T R, beta = -G^{-1} Q^T Z with
// G = P^T Q over the active columns (blockcg.h).
static amg_status solve_block_impl(amg_ctx *c, int nrhs, const double *F, double *U, double tol, int *iters,
                                   double *relres)
{
    TxRange tx("pcg_solve_batched (block CG)");
    const int64_t n = c->n;
    const int itmax = c->prm.itmax;
    hipStream_t st = c->stream;
    c->blk_alloc();
    c->evused = 0;
    c->evbytes.clear();
    hipLaunchKernelGGL((k_fill<double>), dim3(1), dim3(256), 0, st, (int64_t)(B_NSLOTS * NB), 0.0, c->bsc);
    if (nrhs < NB)
        hipLaunchKernelGGL((k_fill<double>), dim3(1), dim3(256), 0, st, (int64_t)(NB - nrhs), 1.0,
                           c->bsc + B_DONE * NB + nrhs);
    hipLaunchKernelGGL(k_pack_blk, dim3(nblocks(n)), dim3(256), 0, st, n, nrhs, F, c->bF);
    hipLaunchKernelGGL(k_pack_blk, dim3(nblocks(n)), dim3(256), 0, st, n, nrhs, (const double *)U, c->bU);
    HIPCHK(hipGetLastError());
    c->sell_blk<double, double, double, EPI_RESID, 0>(0, c->bU, c->bF, c->lev[0].invd64, c->bR, nullptr, nullptr);
    c->bfinalize(c->bdot_partials(n, c->bF, c->bF, nullptr), BF_FF, tol);
    c->bfinalize(c->bdot_partials(n, c->bR, c->bR, nullptr), BF_RR0);
    HIPCHK(hipMemcpyAsync(c->hbsc, c->bsc, B_NSLOTS * NB * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    for (int j = 0; j < nrhs; j++)
        if (!std::isfinite(c->hbsc[B_FF * NB + j])) { set_err("non-finite right-hand side"); return AMG_ERR_ARG; }
    auto all_stopped = [&]() {
        for (int j = 0; j < nrhs; j++)
            if (c->hbsc[B_DONE * NB + j] == 0.0 && c->hbsc[B_FLAG * NB + j] == 0.0) return false;
        return true;
    };
    double *P = c->bP, *Q = c->bQ;
    if (!all_stopped()) {
        c->vcycle_blk(c->bR, c->bZ, 0, nullptr, nullptr);
        c->copy<double, double>(n * NB, c->bZ, P);
        const unsigned g = c->bgrid(n);
        for (int k = 1; k <= itmax; k++) {
            // Q = K P ; alpha ; X += P alpha, R -= Q alpha ; (R, R) per column
            Q = (P == c->bP) ? c->bQ : c->bP;
            c->sell_blk<double, double, double, EPI_SPMV, 0>(0, P, nullptr, nullptr, Q, nullptr, nullptr);
            hipLaunchKernelGGL(k_gram2, dim3(GRAM_BLOCKS), dim3(256), 0, st, n, P, Q, c->bR, c->bgram);
            hipLaunchKernelGGL(k_bcg_small, dim3(1), dim3(1024), 0, st, GRAM_BLOCKS, c->bgram, c->bsc, c->bgsave,
                               c->bcoef, 0);
            hipLaunchKernelGGL(k_bcg_xr, dim3(g), dim3(256), 0, st, n, c->bcoef, c->bU, c->bR, P, Q, c->bpartial);
            HIPCHK(hipGetLastError());
            c->bfinalize(g, BF_RR);
            HIPCHK(hipMemcpyAsync(c->hbsc, c->bsc, B_NSLOTS * NB * sizeof(double), hipMemcpyDeviceToHost, st));
            HIPCHK(hipEventRecord(c->ev_iter, st));
            if (k < itmax) {
                // Z = B R ; beta = -G^{-1} Q^T Z ; P = Z + P beta (into the buffer Q held)
                c->vcycle_blk(c->bR, c->bZ, 0, nullptr, nullptr);
                hipLaunchKernelGGL(k_gram2, dim3(GRAM_BLOCKS), dim3(256), 0, st, n, Q, c->bZ, nullptr, c->bgram);
                hipLaunchKernelGGL(k_bcg_small, dim3(1), dim3(1024), 0, st, GRAM_BLOCKS, c->bgram, c->bsc, c->bgsave,
                                   c->bcoef, 1);
                hipLaunchKernelGGL(k_bcg_p, dim3(g), dim3(256), 0, st, n, c->bcoef, c->bZ, P, Q);
                HIPCHK(hipGetLastError());
                P = Q;   // the new directions
            }
            HIPCHK(hipEventSynchronize(c->ev_iter));
            if (all_stopped()) break;
        }
    }
    hipLaunchKernelGGL(k_unpack_blk, dim3(nblocks(n)), dim3(256), 0, st, n, nrhs, (const double *)c->bU, U);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(c->hbsc, c->bsc, B_NSLOTS * NB * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    c->prof_collect();
    amg_status status = AMG_OK;
    for (int j = 0; j < nrhs; j++) {
        const double ff = c->hbsc[B_FF * NB + j];
        if (iters) iters[j] = (int)c->hbsc[B_ITERS * NB + j];
        if (relres) relres[j] = ff > 0.0 ? std::sqrt(c->hbsc[B_RR * NB + j]) / std::sqrt(ff) : 0.0;
        if (c->hbsc[B_FLAG * NB + j] != 0.0) {
            status = AMG_ERR_BREAKDOWN;
            set_err("block CG breakdown (Gram matrix not positive definite) in column " + std::to_string(j));
        } else if (c->hbsc[B_DONE * NB + j] == 0.0 && status == AMG_OK) {
            status = AMG_NOT_CONVERGED;
        }
    }
    return status;
}

static amg_status solve_batched_impl(amg_ctx *c, int nrhs, const double *F, double *U, double tol, int *iters,
                                     double *relres)
{
    TxRange tx("pcg_solve_batched");
    if (c->prm.krylov == 2) return solve_block_impl(c, nrhs, F, U, tol, iters, relres);
    const int64_t n = c->n;
    const bool flex = c->prm.krylov >= 1;
    const int itmax = c->prm.itmax;
    const bool graph = c->use_graph && !c->prof;
    amg_ctx::OnGraphStream on(c, graph);
    hipStream_t st = c->stream;
    c->blk_alloc();
    c->evused = 0;
    c->evbytes.clear();
    hipLaunchKernelGGL((k_fill<double>), dim3(1), dim3(256), 0, st, (int64_t)(B_NSLOTS * NB), 0.0, c->bsc);
    // columns beyond nrhs are done from the start
    if (nrhs < NB)
        hipLaunchKernelGGL((k_fill<double>), dim3(1), dim3(256), 0, st, (int64_t)(NB - nrhs), 1.0,
                           c->bsc + B_DONE * NB + nrhs);
    hipLaunchKernelGGL(k_pack_blk, dim3(nblocks(n)), dim3(256), 0, st, n, nrhs, F, c->bF);
    hipLaunchKernelGGL(k_pack_blk, dim3(nblocks(n)), dim3(256), 0, st, n, nrhs, (const double *)U, c->bU);
    HIPCHK(hipGetLastError());
    // R = F - K U ; (F_j, F_j) ; (R_j, R_j)
    c->sell_blk<double, double, double, EPI_RESID, 0>(0, c->bU, c->bF, c->lev[0].invd64, c->bR, nullptr, nullptr);
    c->bfinalize(c->bdot_partials(n, c->bF, c->bF, nullptr), BF_FF, tol);
    c->bfinalize(c->bdot_partials(n, c->bR, c->bR, nullptr), BF_RR0);
    HIPCHK(hipMemcpyAsync(c->hbsc, c->bsc, B_NSLOTS * NB * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    for (int j = 0; j < nrhs; j++)
        if (!std::isfinite(c->hbsc[B_FF * NB + j])) { set_err("non-finite right-hand side"); return AMG_ERR_ARG; }
    auto all_stopped = [&]() {
        for (int j = 0; j < nrhs; j++)
            if (c->hbsc[B_DONE * NB + j] == 0.0 && c->hbsc[B_FLAG * NB + j] == 0.0) return false;
        return true;
    };
    if (!all_stopped()) {
        unsigned nb = c->vcycle_blk(c->bR, c->bZ, flex ? 0 : 1, c->bR, nullptr);
        if (!flex) c->bfinalize(nb, BF_RZ0);
        c->copy<double, double>(n * NB, c->bZ, c->bP);
        auto partA = [&]() {
            unsigned nbq;
            if (flex) nbq = c->sell_blk<double, double, double, EPI_SPMV, 2>(0, c->bP, nullptr, nullptr, c->bQ, nullptr, c->bR);
            else nbq = c->sell_blk<double, double, double, EPI_SPMV, 1>(0, c->bP, nullptr, nullptr, c->bQ, nullptr, nullptr);
            c->bfinalize(nbq, flex ? BF_PQ_FCG : BF_PQ_CG);
            unsigned g = c->bgrid(n);
            hipLaunchKernelGGL(k_bcg_update, dim3(g), dim3(256), 0, c->stream, n, c->bsc, c->bU, c->bR, c->bP, c->bQ,
                               c->bpartial);
            HIPCHK(hipGetLastError());
            c->bfinalize(g, BF_RR);
            HIPCHK(hipMemcpyAsync(c->hbsc, c->bsc, B_NSLOTS * NB * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        };
        auto partB = [&]() {
            unsigned nb2 = c->vcycle_blk(c->bR, c->bZ, 1, flex ? c->bQ : c->bR, nullptr);
            c->bfinalize(nb2, flex ? BF_ZQ_FCG : BF_RZ_CG);
            hipLaunchKernelGGL(k_bcg_pupdate, dim3(c->bgrid(n)), dim3(256), 0, c->stream, n, c->bsc, c->bZ, c->bP);
            HIPCHK(hipGetLastError());
        };
        if (graph && !c->gbA[flex]) {
            c->gbA[flex] = c->capture(partA);
            c->gbB[flex] = c->capture(partB);
        }
        for (int k = 1; k <= itmax; k++) {
            if (graph) HIPCHK(hipGraphLaunch(c->gbA[flex], st));
            else partA();
            HIPCHK(hipEventRecord(c->ev_iter, st));
            if (k < itmax) {
                if (graph) HIPCHK(hipGraphLaunch(c->gbB[flex], st));
                else partB();
            }
            HIPCHK(hipEventSynchronize(c->ev_iter));
            if (all_stopped()) break;
        }
    }
    hipLaunchKernelGGL(k_unpack_blk, dim3(nblocks(n)), dim3(256), 0, st, n, nrhs, (const double *)c->bU, U);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(c->hbsc, c->bsc, B_NSLOTS * NB * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    c->prof_collect();
    amg_status status = AMG_OK;
    for (int j = 0; j < nrhs; j++) {
        const double ff = c->hbsc[B_FF * NB + j];
        if (iters) iters[j] = (int)c->hbsc[B_ITERS * NB + j];
        if (relres) relres[j] = ff > 0.0 ? std::sqrt(c->hbsc[B_RR * NB + j]) / std::sqrt(ff) : 0.0;
        if (c->hbsc[B_FLAG * NB + j] != 0.0) {
            status = AMG_ERR_BREAKDOWN;
            set_err("CG breakdown in column " + std::to_string(j));
        } else if (c->hbsc[B_DONE * NB + j] == 0.0 && status == AMG_OK) {
            status = AMG_NOT_CONVERGED;
        }
    }
    return status;
}

amg_status pcg_solve_batched(amg_ctx *c, int nrhs, const double *F, double *U, double tol, int *iters,
                             double *relres)
{
    g_err.clear();
    if (!c || !F || !U || F == U || !(tol >= 0.0) || nrhs < 1 || nrhs > NB) {
        set_err("NULL / aliased argument, tol < 0, or nrhs outside 1..16");
        return AMG_ERR_ARG;
    }
    if (c->host_only) { set_err("context was built by amg_setup_host"); return AMG_ERR_STATE; }
    if (c->general_vcycle()) {
        set_err("the batched solve takes the l1-Jacobi / polynomial forms with the tentative prolongator");
        return AMG_ERR_STATE;
    }
    try {
        return solve_batched_impl(c, nrhs, F, U, tol, iters, relres);
    } catch (Fail &f) {
        return f.st;
    }
}

amg_status amg_vcycle(amg_ctx *c, const double *r, double *z)
{
    g_err.clear();
    if (!c || !r || !z || r == z) { set_err("NULL or aliased argument"); return AMG_ERR_ARG; }
    if (c->host_only) { set_err("context was built by amg_setup_host"); return AMG_ERR_STATE; }
    try {
        c->vcycle(r, z, 0, nullptr, nullptr);
        HIPCHK(hipStreamSynchronize(c->stream));
    } catch (Fail &f) {
        return f.st;
    }
    return AMG_OK;
}

amg_status amg_spmv(amg_ctx *c, int level, const double *x, double *y)
{
    g_err.clear();
    if (!c || !x || !y || x == y) { set_err("NULL or aliased argument"); return AMG_ERR_ARG; }
    if (c->host_only) { set_err("context was built by amg_setup_host"); return AMG_ERR_STATE; }
    if (level < 0 || level >= c->nlev || (level == c->nlev - 1 && level > 0)) {
        set_err("level has no sparse device matrix");
        return AMG_ERR_ARG;
    }
    const DevMat &A = c->lev[level].A;
    if (!A.v64 && !A.cv) { set_err("level is held in FP32 only (vcycle_fp32)"); return AMG_ERR_ARG; }
    try {
        int saved = c->prof;
        c->prof = 0;
        if (A.lpr) c->apply<EPI_SPMV>(A, x, nullptr, y);
        else c->sell<double, double, double, EPI_SPMV, 0>(level, x, nullptr, nullptr, y, nullptr, nullptr);
        c->prof = saved;
        HIPCHK(hipStreamSynchronize(c->stream));
    } catch (Fail &f) {
        return f.st;
    }
    return AMG_OK;
}

amg_status amg_set_option(amg_ctx *c, int option, int value)
{
    if (!c) { set_err("NULL context"); return AMG_ERR_ARG; }
    switch (option) {
    case AMG_OPT_GRAPH: c->use_graph = value ? 1 : 0; break;
    case AMG_OPT_FUSE_POST: c->fuse_post = value ? 1 : 0; c->drop_graphs(); break;
    case AMG_OPT_TAIL: c->use_tail = value ? 1 : 0; c->drop_graphs(); break;
    case AMG_OPT_X_WINDOW:
        for (int l = 0; l < c->nlev; l++) {
            DevMat &A = c->lev[l].A;
            A.xwin = value && A.C == SLICE && A.nshared > 0 && A.shrun ? 1 : 0;
        }
        c->drop_graphs();
        break;
    case AMG_OPT_WINDOW_SHARE:
        if (value < 0 || value > 3) {
            set_err("AMG_OPT_WINDOW_SHARE takes a mask: 1 FP64-value passes, 2 FP32-value passes");
            return AMG_ERR_ARG;
        }
        c->blk_share = value;
        c->drop_graphs();
        break;
    case AMG_OPT_BLOCK_WINDOW:
        if (value != 0 && value != 2 && value != 4) {
            set_err("AMG_OPT_BLOCK_WINDOW takes 0 (off) or 2 or 4 rows per lane");
            return AMG_ERR_ARG;
        }
        c->blk_win = value;
        c->drop_graphs();
        break;
    default: set_err("unknown option"); return AMG_ERR_ARG;
    }
    return AMG_OK;
}

amg_status amg_get_residual_history(const amg_ctx *c, double *hist, int cap, int *count)
{
    if (!c || cap < 0 || (cap > 0 && !hist)) { set_err("NULL context or buffer, or cap < 0"); return AMG_ERR_ARG; }
    const int m = (int)c->hist.size();
    for (int k = 0; k < std::min(m, cap); k++) hist[k] = c->hist[(size_t)k];
    if (count) *count = m;
    return AMG_OK;
}

amg_status amg_get_option(const amg_ctx *c, int option, int *value)
{
    if (!c || !value) { set_err("NULL argument"); return AMG_ERR_ARG; }
    switch (option) {
    case AMG_OPT_GRAPH: *value = c->use_graph; break;
    case AMG_OPT_FUSE_POST: *value = c->fuse_post; break;
    case AMG_OPT_TAIL: *value = c->use_tail && c->tail_start > 0 ? c->tail_start : 0; break;
    case AMG_OPT_WINDOW_SHARE: *value = c->lev[0].A.wgtab ? c->blk_share : 0; break;
    case AMG_OPT_X_WINDOW: *value = c->nlev > 0 ? c->lev[0].A.xwin : 0; break;
    case AMG_OPT_BLOCK_WINDOW: *value = c->blk_win; break;
    default: set_err("unknown option"); return AMG_ERR_ARG;
    }
    return AMG_OK;
}

amg_status amg_get_batched_variant(const amg_ctx *c, int *lpr, int *threads)
{
    if (!c) { set_err("NULL context"); return AMG_ERR_ARG; }
    if (lpr) *lpr = c->blk_lpr;
    if (threads) *threads = c->blk_threads;
    return AMG_OK;
}

amg_status amg_set_batched_variant(amg_ctx *c, int lpr, int threads)
{
    if (!c || (threads != 256 && threads != 512) || (lpr != 1 && lpr != 4 && lpr != 8 && lpr != 16)) {
        set_err("lpr must be 1, 4, 8 or 16 and threads 256 or 512");
        return AMG_ERR_ARG;
    }
    if (lpr > 1 && c->blk_img_lpr != lpr) {
        set_err("no block images with that many lanes per row (built by amg_setup with prm.nrhs > 1 for the "
                "autotuner's choice only)");
        return AMG_ERR_ARG;
    }
    if (lpr == 1 && threads != 256) { set_err("the one-lane-per-row kernels use 256 threads"); return AMG_ERR_ARG; }
    c->blk_lpr = lpr;
    c->blk_threads = threads;
    c->drop_graphs();
    return AMG_OK;
}

static int poly_ok(const double *a)
{
    for (int s = 0; s <= 10000; s++) {
        double t = s / 10000.0;
        double e = 1.0 - t * (((a[3] * t + a[2]) * t + a[1]) * t + a[0]);
        if (!std::isfinite(e) || std::fabs(e) > 1.0) return 0;
        if (s > 0 && !(e < 1.0)) return 0;
    }
    return 1;
}

amg_status amg_set_poly_coeffs(amg_ctx *c, int level, const double coeffs[4])
{
    g_err.clear();
    if (!c || !coeffs || level < 0 || level >= c->nlev - 1) { set_err("bad level or NULL"); return AMG_ERR_ARG; }
    if (c->host_only) { set_err("context was built by amg_setup_host"); return AMG_ERR_STATE; }
    if (!poly_ok(coeffs)) {
        set_err("polynomial rejected: error polynomial leaves [-1, 1] or reaches 1 on (0, 1]");
        return AMG_NOT_CONVERGED;
    }
    Level &L = c->lev[level];
    for (int k = 0; k < 4; k++) L.poly[k] = coeffs[k];
    L.poly_on = c->prm.smoother == 1 ? 1 : 0;
    c->drop_graphs();
    return AMG_OK;
}

amg_status amg_get_level_info(const amg_ctx *c, int level, int64_t *n, int64_t *nnz)
{
    if (!c || !n || !nnz || level < -1 || level >= c->nlev) { set_err("bad level or NULL"); return AMG_ERR_ARG; }
    if (level == -1) {
        *n = c->nlev;
        int64_t t = 0;
        for (auto &L : c->host.lev) t += L.nnz;
        *nnz = t;
        return AMG_OK;
    }
    *n = c->host.lev[level].n;
    *nnz = c->host.lev[level].nnz;
    return AMG_OK;
}

amg_status amg_get_aggregates(const amg_ctx *c, int level, int32_t *agg, double *pc)
{
    if (!c || level < 0 || level >= c->nlev - 1) { set_err("bad level"); return AMG_ERR_ARG; }
    auto &L = c->host.lev[level];
    if (agg) std::memcpy(agg, L.agg.data(), L.agg.size() * sizeof(int32_t));
    if (pc) std::memcpy(pc, L.pc.data(), L.pc.size() * sizeof(double));
    return AMG_OK;
}

amg_status amg_get_coarse_matrix(const amg_ctx *c, int level, int64_t *row_ptr, int32_t *col, double *val)
{
    if (!c || level < 1 || level >= c->nlev) { set_err("level must be 1 .. levels-1"); return AMG_ERR_ARG; }
    auto &K = c->host.lev[level].K;
    if (row_ptr) std::memcpy(row_ptr, K.rp.data(), K.rp.size() * sizeof(int64_t));
    if (col) std::memcpy(col, K.ci.data(), K.ci.size() * sizeof(int32_t));
    if (val) std::memcpy(val, K.v.data(), K.v.size() * sizeof(double));
    return AMG_OK;
}

amg_status amg_get_setup_rounds(const amg_ctx *c, int *sweeps, int *rounds_total, int *rounds_max)
{
    if (!c) { set_err("NULL context"); return AMG_ERR_ARG; }
    if (sweeps) *sweeps = c->setup_info.sweeps;
    if (rounds_total) *rounds_total = c->setup_info.rounds_total;
    if (rounds_max) *rounds_max = c->setup_info.rounds_max;
    return AMG_OK;
}

amg_status amg_get_prolongator(const amg_ctx *c, int level, int64_t *nnz, int64_t *row_ptr, int32_t *col,
                               double *val)
{
    if (!c || level < 0 || level >= c->nlev - 1) { set_err("level must be 0 .. levels-2"); return AMG_ERR_ARG; }
    auto &P = c->host.lev[level].P;
    if (nnz) *nnz = P.rp.empty() ? 0 : P.nnz();
    if (P.rp.empty()) return AMG_OK;
    if (row_ptr) std::memcpy(row_ptr, P.rp.data(), P.rp.size() * sizeof(int64_t));
    if (col) std::memcpy(col, P.ci.data(), P.ci.size() * sizeof(int32_t));
    if (val) std::memcpy(val, P.v.data(), P.v.size() * sizeof(double));
    return AMG_OK;
}

amg_status amg_set_profiling(amg_ctx *c, int enable)
{
    if (!c) return AMG_ERR_ARG;
    c->prof = enable ? 1 : 0;
    c->prof_launches = 0;
    c->prof_ms = 0.0;
    c->prof_bytes = 0.0;
    for (int k = 0; k < AMG_PASS_KINDS; k++) {
        c->pk_launches[k] = 0;
        c->pk_ms[k] = 0.0;
        c->pk_bytes[k] = 0.0;
    }
    return AMG_OK;
}

amg_status amg_get_profile_pass(const amg_ctx *c, int kind, int64_t *launches, double *ms, double *bytes)
{
    if (!c || kind < 0 || kind >= AMG_PASS_KINDS) { set_err("NULL context or unknown pass kind"); return AMG_ERR_ARG; }
    if (launches) *launches = c->pk_launches[kind];
    if (ms) *ms = c->pk_ms[kind];
    if (bytes) *bytes = c->pk_bytes[kind];
    return AMG_OK;
}

amg_status amg_get_profile(amg_ctx *c, int64_t *launches, double *ms, double *bytes)
{
    if (!c) return AMG_ERR_ARG;
    if (launches) *launches = c->prof_launches;
    if (ms) *ms = c->prof_ms;
    if (bytes) *bytes = c->prof_bytes;
    return AMG_OK;
}

amg_status amg_get_format(const amg_ctx *c, int level, int *slice, int64_t *stored, int *index_bytes,
                          int64_t *shared_slices)
{
    if (!c || c->host_only || level < 0 || level >= c->nlev || (level == c->nlev - 1 && level > 0)) {
        set_err("level has no sparse device matrix");
        return AMG_ERR_ARG;
    }
    const DevMat &A = c->lev[level].A;
    if (slice) *slice = A.lpr ? -A.lpr : SLICE;
    if (stored) *stored = A.stored;
    if (index_bytes) *index_bytes = (A.idx16 && !A.lpr) ? 2 : 4;
    if (shared_slices) *shared_slices = A.nshared;
    return AMG_OK;
}

amg_status amg_iga_poisson_size(int d, int p, int n, int64_t *N, int64_t *nnz)
{
    if (d < 2 || d > 3 || p < 1 || p > 10 || n < 1 || n + p - 2 < 1 || !N || !nnz) {
        set_err("need d in {2,3}, 1 <= p <= 10, n + p > 2");
        return AMG_ERR_ARG;
    }
    amgiga::iga_size(d, p, n, N, nnz);
    return AMG_OK;
}

amg_status amg_iga_poisson(int d, int p, int n, int64_t *row_ptr, int32_t *col, double *val, double *F)
{
    if (!row_ptr || !col || !val) { set_err("NULL output"); return AMG_ERR_ARG; }
    if (amgiga::iga_poisson(d, p, n, row_ptr, col, val, F)) { set_err("bad d, p or n"); return AMG_ERR_ARG; }
    return AMG_OK;
}

amg_status amg_iga_cube_size(int p, int n, int64_t *N, int64_t *nnz)
{
    if (p < 1 || p > 10 || n < 1 || n + p < 3 || !N || !nnz) { set_err("need 1 <= p <= 10, n >= 1, n + p >= 3"); return AMG_ERR_ARG; }
    amgiga::iga_cube_size(p, n, N, nnz);
    return AMG_OK;
}

amg_status amg_iga_cube(int p, int n, int64_t *row_ptr, int32_t *col, double *val, double *F)
{
    if (!row_ptr || !col || !val) { set_err("NULL output"); return AMG_ERR_ARG; }
    if (amgiga::iga_cube(p, n, row_ptr, col, val, F)) { set_err("bad p or n"); return AMG_ERR_ARG; }
    return AMG_OK;
}

amg_status amg_level_features(const amg_ctx *c, int level, float *feat)
{
    if (!c || !feat || level < 0 || level >= c->nlev) { set_err("bad level or NULL"); return AMG_ERR_ARG; }
    const auto &L = c->host.lev[level];
    for (int k = 0; k < 6; k++) feat[k] = L.feat[k];
    const auto &L0 = c->host.lev[0];
    const double dens = ((double)L.nnz / (double)L.n) / ((double)L0.nnz / (double)L0.n);
    feat[6] = (float)(std::log10(dens) / 2.0);
    feat[7] = level + 1 < c->nlev ? (float)((double)c->host.lev[level + 1].n / (double)L.n) : 0.0f;
    return AMG_OK;
}

amg_status amg_mlp_forward(const uint16_t *w, const float *X, int B, float *Y, float *act, void *hip_stream)
{
    if (!w || !X || !Y || B < 1) { set_err("NULL argument or B < 1"); return AMG_ERR_ARG; }
    hipLaunchKernelGGL(k_mlp_fwd, dim3((B + 63) / 64), dim3(64), 0, (hipStream_t)hip_stream, w, X, B, Y, act);
    if (hipGetLastError() != hipSuccess) { set_err("launch failed"); return AMG_ERR_HIP; }
    return AMG_OK;
}

amg_status amg_mlp_backward(const uint16_t *w, const float *X, const float *act, const float *Y, const float *T,
                            int B, float *del, float *grad, float *loss, void *hip_stream)
{
    if (!w || !X || !act || !Y || !T || !del || !grad || B < 1) { set_err("NULL argument or B < 1"); return AMG_ERR_ARG; }
    hipStream_t st = (hipStream_t)hip_stream;
    hipLaunchKernelGGL(k_mlp_delta, dim3((B + 63) / 64), dim3(64), 0, st, w, act, Y, T, B, del);
    hipLaunchKernelGGL(k_mlp_grad, dim3((MLP_NPARAM + 255) / 256), dim3(256), 0, st, X, act, del, Y, T, B, grad, loss);
    if (hipGetLastError() != hipSuccess) { set_err("launch failed"); return AMG_ERR_HIP; }
    return AMG_OK;
}

// ---- the MLP gradient without allocation ----------------------------------
//
// Per-sample deltas of the backward pass in a file-scope device array instead
// of a caller workspace, for callers that cannot allocate device memory.  Each
// device holds its own copy of the array (until the process ends); host code
// reaches it only through the address hipGetSymbolAddress returns on that
// device, looked up once per device on the first call there.
constexpr int MLP_NOALLOC_MAX_B = AMG_MLP_NOALLOC_MAX_B;
static __device__ __align__(256) float scratch[(size_t)MLP_NOALLOC_MAX_B * MLP_DEL];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex scratch_mx;
float *scratch_ptr[MAX_DEVICES] = {};

// device address of this device's scratch array (nullptr and a message on error)
float *scratch_on_current_device()
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) {
        set_err("no current HIP device (or device index >= 64)");
        return nullptr;
    }
    std::lock_guard<std::mutex> g(scratch_mx);
    if (!scratch_ptr[dev]) {
        void *ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            set_err(std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
            return nullptr;
        }
        scratch_ptr[dev] = static_cast<float *>(ptr);
    }
    return scratch_ptr[dev];
}
}  // namespace

amg_status amg_mlp_backward_noalloc(const uint16_t *w, const float *X, const float *act, const float *Y,
                                    const float *T, int B, float *grad, float *loss, void *hip_stream)
{
    g_err.clear();
    if (!w || !X || !act || !Y || !T || !grad || B < 1) { set_err("NULL argument or B < 1"); return AMG_ERR_ARG; }
    if (B > MLP_NOALLOC_MAX_B) {
        set_err("B = " + std::to_string(B) + " exceeds the static workspace of " + std::to_string(MLP_NOALLOC_MAX_B) +
                " samples (use amg_mlp_backward with a workspace)");
        return AMG_ERR_ARG;
    }
    float *del = scratch_on_current_device();
    if (!del) return AMG_ERR_HIP;
    hipStream_t st = (hipStream_t)hip_stream;
    // k_mlp_delta writes every delta of samples 0..B-1 before k_mlp_grad reads
    // them (stream order), so nothing left by an earlier call is read
    hipLaunchKernelGGL(k_mlp_delta, dim3((B + 63) / 64), dim3(64), 0, st, w, act, Y, T, B, del);
    hipLaunchKernelGGL(k_mlp_grad, dim3((MLP_NPARAM + 255) / 256), dim3(256), 0, st, X, act, del, Y, T, B, grad, loss);
    if (hipGetLastError() != hipSuccess) { set_err("launch failed"); return AMG_ERR_HIP; }
    return AMG_OK;
}

amg_status amg_mlp_adam(float *master, uint16_t *w, const float *grad, float *m, float *v, int step, float lr,
                        void *hip_stream)
{
    if (!master || !w || (step > 0 && (!grad || !m || !v)) || step < 0) { set_err("NULL argument"); return AMG_ERR_ARG; }
    hipLaunchKernelGGL(k_mlp_adam, dim3((MLP_NPARAM + 255) / 256), dim3(256), 0, (hipStream_t)hip_stream, master, w,
                       grad, m, v, step, lr, 0.9f, 0.999f, 1e-8f);
    if (hipGetLastError() != hipSuccess) { set_err("launch failed"); return AMG_ERR_HIP; }
    return AMG_OK;
}

// Coefficients a_0..a_3 of g(t) = sum_k a_k t^{k+1} from its values y_j at the
// nodes t_j = (1 - cos(j pi/4))/2, j = 1..4: solve sum_k a_k t_j^{k+1} = y_j
// (4 x 4, Gaussian elimination with partial pivoting).
static void poly_from_node_values(const double y[4], double a[4])
{
    double M[4][5];
    for (int j = 0; j < 4; j++) {
        double t = 0.5 * (1.0 - std::cos((j + 1) * M_PI / 4.0)), tp = t;
        for (int k = 0; k < 4; k++) { M[j][k] = tp; tp *= t; }
        M[j][4] = y[j];
    }
    for (int c = 0; c < 4; c++) {
        int piv = c;
        for (int r = c + 1; r < 4; r++)
            if (std::fabs(M[r][c]) > std::fabs(M[piv][c])) piv = r;
        for (int k = 0; k < 5; k++) std::swap(M[c][k], M[piv][k]);
        for (int r = c + 1; r < 4; r++) {
            double f = M[r][c] / M[c][c];
            for (int k = c; k < 5; k++) M[r][k] -= f * M[c][k];
        }
    }
    for (int c = 3; c >= 0; c--) {
        double s = M[c][4];
        for (int k = c + 1; k < 4; k++) s -= M[c][k] * a[k];
        a[c] = s / M[c][c];
    }
}

amg_status amg_set_learned_poly(amg_ctx *c, const uint16_t *w_host, int *accepted, double *coeffs)
{
    g_err.clear();
    if (!c || !w_host) { set_err("NULL argument"); return AMG_ERR_ARG; }
    if (c->host_only) { set_err("context was built by amg_setup_host"); return AMG_ERR_STATE; }
    if (c->prm.smoother != 1) { set_err("context not built with the polynomial smoother (prm.smoother = 1)"); return AMG_ERR_STATE; }
    const int nl = c->nlev - 1;
    if (nl < 1) return AMG_OK;
    try {
        std::vector<float> X((size_t)nl * MLP_IN), Y((size_t)nl * MLP_OUT);
        for (int l = 0; l < nl; l++) amg_level_features(c, l, &X[(size_t)l * MLP_IN]);
        uint16_t *dw = dalloc<uint16_t>(MLP_NPARAM);
        float *dX = dalloc<float>(X.size()), *dY = dalloc<float>(Y.size());
        HIPCHK(hipMemcpy(dw, w_host, MLP_NPARAM * sizeof(uint16_t), hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(dX, X.data(), X.size() * sizeof(float), hipMemcpyHostToDevice));
        hipLaunchKernelGGL(k_mlp_fwd, dim3((nl + 63) / 64), dim3(64), 0, c->stream, dw, dX, nl, dY, (float *)nullptr);
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpyAsync(Y.data(), dY, Y.size() * sizeof(float), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
        (void)hipFree(dw); (void)hipFree(dX); (void)hipFree(dY);
        for (int l = 0; l < nl; l++) {
            double y[4], cf[4];
            for (int k = 0; k < 4; k++) y[k] = (double)Y[(size_t)l * MLP_OUT + k];
            poly_from_node_values(y, cf);
            if (coeffs) for (int k = 0; k < 4; k++) coeffs[l * 4 + k] = cf[k];
            int ok = poly_ok(cf);
            Level &L = c->lev[l];
            if (ok) { for (int k = 0; k < 4; k++) L.poly[k] = cf[k]; L.poly_on = 1; }
            else { L.poly[0] = 1.0; L.poly[1] = L.poly[2] = L.poly[3] = 0.0; L.poly_on = 0; }
            if (accepted) accepted[l] = ok;
        }
        c->drop_graphs();
    } catch (Fail &f) {
        return f.st;
    }
    return AMG_OK;
}

amg_status amg_iga_diffusion(int p, int n, int nk, const double *a, const int32_t *mk, int64_t *row_ptr,
                             int32_t *col, double *val, double *F)
{
    if (!row_ptr || !col || !val || (nk > 0 && (!a || !mk))) { set_err("NULL argument"); return AMG_ERR_ARG; }
    if (amgiga::iga_diffusion(p, n, nk, a, mk, row_ptr, col, val, F)) { set_err("bad p, n or nk"); return AMG_ERR_ARG; }
    return AMG_OK;
}

}  // extern "C"
