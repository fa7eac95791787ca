// Block (multi right-hand side) kernels of the batched solve: NB = 16 columns
// held row-major (X[row * 16 + j], 64 B per row in FP32, 128 B in FP64) so that
// one matrix entry, read once from HBM, multiplies 16 contiguous values.
//
// The matrix is the same SELL-64 image as the single-vector kernels (layout in
// kernels.h).  A wavefront covers a 64-row slice; with LPR lanes per row it
// walks the slice in LPR sub-slices of 64/LPR rows, each lane owning 16/LPR
// columns.  With one lane per row, every row sum, every matrix-pass dot
// partial and every vector update of a column uses the single-vector kernels'
// operation order, so a column of the block solve carries the same bits as the
// single solve; only the norms of the stopping test ((F,F), (r,r)), summed by
// the element-parallel vector kernels, take another order.
#pragma once
#include <type_traits>
#include "kernels.h"

namespace amgk {

constexpr int NB = 16;

// per-column scalar slots: sc[slot * NB + j]
enum BSlot { B_RZ = 0, B_PQ, B_RR, B_ALPHA, B_BETA, B_PR, B_ZQ, B_FF, B_FLAG, B_DONE, B_ITERS, B_THR, B_NSLOTS };
enum BFin { BF_FF = 0, BF_RR0, BF_RZ0, BF_PQ_CG, BF_PQ_FCG, BF_RR, BF_RZ_CG, BF_ZQ_FCG };

__device__ inline bool bactive(const double *sc, int j) { return sc[B_DONE * NB + j] == 0.0 && sc[B_FLAG * NB + j] == 0.0; }

// Sum over the 256-thread block of one value per thread and column, per column
// in the order of block_sum; results valid in thread 0 (out[NB]).
template <int NC>
__device__ inline void block_sum_cols(double (&v)[NC], double *lds /* 4 * NC */)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int j = 0; j < NC; j++) v[j] = wave_sum(v[j]);
    __syncthreads();
    if (lane == 0)
#pragma unroll
        for (int j = 0; j < NC; j++) lds[wid * NC + j] = v[j];
    __syncthreads();
    if (threadIdx.x == 0)
#pragma unroll
        for (int j = 0; j < NC; j++) v[j] = ((lds[j] + lds[NC + j]) + lds[2 * NC + j]) + lds[3 * NC + j];
}

template <typename T> struct BlkVec;
template <> struct BlkVec<float> {
    static __device__ inline void load(const float *p, float (&o)[NB])
    {
        const vf4 *q = reinterpret_cast<const vf4 *>(p);
#pragma unroll
        for (int h = 0; h < 4; h++) {
            vf4 t = q[h];
            o[4 * h] = t.x; o[4 * h + 1] = t.y; o[4 * h + 2] = t.z; o[4 * h + 3] = t.w;
        }
    }
};
template <> struct BlkVec<double> {
    static __device__ inline void load(const double *p, double (&o)[NB])
    {
        const vd2 *q = reinterpret_cast<const vd2 *>(p);
#pragma unroll
        for (int h = 0; h < 8; h++) {
            vd2 t = q[h];
            o[2 * h] = t.x; o[2 * h + 1] = t.y;
        }
    }
};

// Block matrix pass, lane = row (all 16 columns per lane).  Epilogues as k_sell:
//   EPI_SPMV : Y = K X;                 dots per column (X_j, Y_j), (X_j, G1_j)
//   EPI_RESID: Y = F - K X
//   EPI_SMOOTH: Y = X + D^{-1}(F - K X); dots per column (Y_j, G0_j), (Y_j, G1_j)
//   EPI_POLY : Y = a D^{-1} F + D^{-1} K X
// Partials: partial[(blockIdx.x * 2 + d) * NB + j].
template <typename VT, typename FT, typename OT, typename IT, int EPI, int NDOT>
__global__ __launch_bounds__(256) void k_sell_blk(const Sell<VT, IT> A, const VT *__restrict__ X,
                                                  const FT *__restrict__ F, const VT *__restrict__ invd,
                                                  OT *__restrict__ Y, const double *__restrict__ G0,
                                                  const double *__restrict__ G1, double *__restrict__ partial,
                                                  VT coef)
{
    __shared__ double lds[8 * NB];
    const int lane = threadIdx.x & 63, wid = wave_id();
    const int64_t s = (int64_t)blockIdx.x * SELL_WAVES + wid;
    double d0[NB], d1[NB];
#pragma unroll
    for (int j = 0; j < NB; j++) { d0[j] = 0.0; d1[j] = 0.0; }
    if (s < A.nslices) {
        const int64_t row = A.row_of(s * SLICE + lane);
        VT acc[NB];
#pragma unroll
        for (int j = 0; j < NB; j++) acc[j] = 0;
        sell_row<SLICE>(A, s, lane, [&](const VT *v, const int *c) {
#pragma unroll
            for (int t = 0; t < 8; t++) {
                VT xv[NB];
                BlkVec<VT>::load(X + (int64_t)c[t] * NB, xv);
#pragma unroll
                for (int j = 0; j < NB; j++) acc[j] = fma(v[t], xv[j], acc[j]);
            }
        });
        if (row >= 0) {
            const int64_t o = row * NB;
            if (EPI == EPI_SPMV) {
#pragma unroll
                for (int j = 0; j < NB; j++) {
                    Y[o + j] = (OT)acc[j];
                    if (NDOT >= 1) d0[j] = (double)X[o + j] * (double)acc[j];
                    if (NDOT >= 2) d1[j] = (double)X[o + j] * G1[o + j];
                }
            } else if (EPI == EPI_RESID) {
#pragma unroll
                for (int j = 0; j < NB; j++) Y[o + j] = (OT)((VT)F[o + j] - acc[j]);
            } else if (EPI == EPI_SMOOTH) {
                const VT di = invd[row];
#pragma unroll
                for (int j = 0; j < NB; j++) {
                    VT out = X[o + j] + di * ((VT)F[o + j] - acc[j]);
                    Y[o + j] = (OT)out;
                    if (NDOT >= 1) d0[j] = (double)out * G0[o + j];
                    if (NDOT >= 2) d1[j] = (double)out * G1[o + j];
                }
            } else {
                const VT di = invd[row];
#pragma unroll
                for (int j = 0; j < NB; j++) Y[o + j] = (OT)(coef * (di * (VT)F[o + j]) + di * acc[j]);
            }
        }
    }
    if (NDOT >= 1) {
        // one partial per wavefront and column, as the single-vector kernels
        const int64_t w = (int64_t)blockIdx.x * SELL_WAVES + wid;
#pragma unroll
        for (int j = 0; j < NB; j++) {
            const double t0 = wave_sum(d0[j]);
            const double t1 = NDOT >= 2 ? wave_sum(d1[j]) : 0.0;
            if (lane == 0) {
                partial[(2 * w) * NB + j] = t0;
                partial[(2 * w + 1) * NB + j] = t1;
            }
        }
    }
}

// ---- block matrix pass with staged x windows --------------------------------
//
// In a slice with shared column offsets, a run of consecutive offsets o, o+1,
// ..., o+L-1 (for a stencil matrix: the 2p+1 entries of one x-line, the same
// (y, z) displacement) makes lane r read rows row0 + r + o + t, t < L, of X:
// the 64 lanes together touch only the 64 + L - 1 consecutive rows
// row0 + o .. row0 + o + 62 + L.  The wave copies those rows (16 columns each)
// into its own LDS window once per run and every lane then reads its rows from
// LDS; without the window each entry of each row gathers a full 16-column row
// of X from the cache hierarchy (64 B in FP32, 128 B in FP64), the traffic
// that bounds the one-lane-per-row kernel.
//
// The copy is a direct global-to-LDS load (global_load_lds_dwordx4): no
// registers hold the window on its way, and the wave's instruction i writes
// 16-byte slots 64 i .. 64 i + 63 of the window in lane order.  The window is
// row-major with one pad slot per row (row w, 16-byte chunk c at slot
// w (CH + 1) + c, CH chunks per row): the lanes of one load instruction read
// consecutive chunks of consecutive rows (the pad slot takes the next row's
// first chunk, never read), and the stride CH + 1 puts the chunks a group of
// lanes reads for R-row blocks on distinct banks.
//
// Each row's entries are summed in ascending column order (the padding
// entries of a shared list, value 0, are skipped: an FMA with a zero product
// leaves a nonzero or +0 sum unchanged), so each column carries the
// single-vector kernels' bits.  Slices with per-row indices take k_sell_blk's
// gather path.
//
// Each wave owns two windows and alternates between them by run: the copy of
// run rho + 1 and the load of its values are in flight while run rho is summed.
// The order is kept by explicit waits: before a copy into a window, for every
// LDS read of the wave (lgkmcnt 0: the window's last reads were two runs
// back); before the sums of a run, for all of the wave's vector memory loads
// (vmcnt 0: that run's copy and values were issued one run earlier).
// Measured on the c4 level 0 (p = 3): the copies and value loads (14 per run
// in FP64) keep the texture address unit busy 86% of the pass, each 1 KB
// request missing L1 (an L2 round trip of ~600 cycles); the sums themselves
// take a third of the VALU time.

template <typename VT> struct Chunk16;
template <> struct Chunk16<double> {
    typedef vd2 type;
    static __device__ inline void unpack(type q, double *o) { o[0] = q.x; o[1] = q.y; }
};
template <> struct Chunk16<float> {
    typedef vf4 type;
    static __device__ inline void unpack(type q, float *o) { o[0] = q.x; o[1] = q.y; o[2] = q.z; o[3] = q.w; }
};

// One 16-byte value group of the window kernels.  FP64: a streaming load --
// the values pass once, and the block's X (128 B per row) would not stay in
// L2 and the memory-side cache beside them (measured: 10.5 -> 9.8 GB of HBM
// reads per c4 pass, 2.00 -> 1.94 ms).  FP32: a plain load -- a group holds
// four entries, so consecutive runs share their boundary group, which a
// streaming load fetches twice from HBM (measured: 4.2 -> 5.6 GB, 1.00 ->
// 1.16 ms).
template <typename VT, typename CT> __device__ __forceinline__ CT load_group(const CT *p)
{
    if constexpr (sizeof(VT) == 8) return __builtin_nontemporal_load(p);
    else return *p;
}

// An empty asm statement reading v: the compiler keeps v in its registers
// up to this point (device code only; the host pass never runs it).
template <typename T> __device__ __forceinline__ void keep_in_vgprs(const T &v)
{
#if defined(__HIP_DEVICE_COMPILE__)
    asm volatile("" : : "v"(v));
#endif
}

// Value held by lane i of each aligned group of R lanes (R = 2 or 4), to
// every lane of the group: one DPP quad permutation per 32 bits.
template <int R, int I> struct GroupPerm {
    static constexpr int ctrl = R == 4 ? (I | I << 2 | I << 4 | I << 6) : (I | I << 2 | (2 + I) << 4 | (2 + I) << 6);
};
template <int R, int I> __device__ __forceinline__ float group_bcast(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), GroupPerm<R, I>::ctrl, 0xF,
                                                              0xF, true));
}
template <int R, int I> __device__ __forceinline__ double group_bcast(double v)
{
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)u, GroupPerm<R, I>::ctrl, 0xF, 0xF, true);
    const uint32_t hi =
        (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)(u >> 32), GroupPerm<R, I>::ctrl, 0xF, 0xF, true);
    return __builtin_bit_cast(double, (uint64_t)lo | (uint64_t)hi << 32);
}
template <int R, typename VT> __device__ __forceinline__ VT group_bcast(VT v, int i)
{
    // i is a constant after unrolling: the switch folds
    switch (i) {
    case 0: return group_bcast<R, 0>(v);
    case 1: return group_bcast<R, 1>(v);
    case 2: return group_bcast<R, R == 4 ? 2 : 0>(v);
    default: return group_bcast<R, R == 4 ? 3 : 1>(v);
    }
}

// One run of L entries (a compile-time length, so that the sums run without
// branches) from a staged window, the run's values starting at entry OFF of
// the lane's first value group: window row R g + w serves row R g + i at
// entry w - i.  Wr points at the lane's first window read.
template <typename VT, int R, int NGR> struct WinRun {
    typedef typename Chunk16<VT>::type CT;
    static constexpr int G = 16 / (int)sizeof(VT), CH = NB / G, CPL = NB / R, CPC = CH / R, WS = CH + 1;
    template <int OFF, int L>
    static __device__ __forceinline__ void run(VT (&acc)[R][CPL], const CT *Wr, const CT (&vg)[NGR])
    {
        static_assert(OFF + L <= NGR * G, "run past its value groups");
        VT e[NGR * G];
#pragma unroll
        for (int j = 0; j < NGR; j++) Chunk16<VT>::unpack(vg[j], e + j * G);
#pragma unroll
        for (int w = 0; w < R + L - 1; w++) {
            VT xv[CPL];
#pragma unroll
            for (int cc = 0; cc < CPC; cc++) Chunk16<VT>::unpack(Wr[w * WS + cc * R], xv + cc * G);
#pragma unroll
            for (int i = 0; i < R; i++) {
                const int t = w - i;
                if (t >= 0 && t < L) {
                    const VT v = group_bcast<R>(e[OFF + t], i);
#pragma unroll
                    for (int j = 0; j < CPL; j++) acc[i][j] = fma(v, xv[j], acc[i][j]);
                }
            }
        }
    }
    template <int OFF>
    static __device__ __forceinline__ void len(VT (&acc)[R][CPL], const CT *Wr, const CT (&vg)[NGR], int L)
    {
        static_assert(WIN_LMAX == 7, "one case per run length");
        switch (L) {
        case 1: run<OFF, 1>(acc, Wr, vg); break;
        case 2: run<OFF, 2>(acc, Wr, vg); break;
        case 3: run<OFF, 3>(acc, Wr, vg); break;
        case 4: run<OFF, 4>(acc, Wr, vg); break;
        case 5: run<OFF, 5>(acc, Wr, vg); break;
        case 6: run<OFF, 6>(acc, Wr, vg); break;
        default: run<OFF, WIN_LMAX>(acc, Wr, vg); break;
        }
    }
};

// Register blocking: with R rows per lane, lane = g * R + q owns rows R g ..
// R g + R - 1 and 16 / R columns (16-byte chunks q, q + R, q + 2R, ... of each
// row), so a window row read from LDS serves the lane's rows at every offset
// that reaches it: R + L - 1 window reads per chunk and run instead of R L.
// Each lane loads the value groups of its own row (row0 + lane, one coalesced
// 16-byte load per group) and takes the other rows of its block from their
// lanes by DPP.  Per column the row sums keep ascending entry order and the
// dots keep the single-vector kernels' butterfly order (the row bits above
// log2 R are lane bits, the ones below are summed in registers, in the same
// order).
// Epilogue of the window kernels for the R rows (row0 + R g + i) and 16 / R
// columns (16-byte chunks q, q + R, ... of each row) a lane owns; the dot
// partials of the slice go to slot w_id.
template <typename VT, typename FT, typename OT, int EPI, int NDOT, int R>
__device__ __forceinline__ void win_epilogue(VT (&acc)[R][NB / R], int64_t row0, int64_t nrows, int g, int q,
                                             const VT *__restrict__ X, const FT *__restrict__ F,
                                             const VT *__restrict__ invd, OT *__restrict__ Y,
                                             const double *__restrict__ G0, const double *__restrict__ G1,
                                             double *__restrict__ partial, int64_t w_id, VT coef)
{
    constexpr int G = 16 / (int)sizeof(VT), CPL = NB / R;
    // epilogue: local column jj = cc * G + u is column (q + cc R) G + u
    double d0[R][CPL], d1[R][CPL];
#pragma unroll
    for (int i = 0; i < R; i++) {
        const int64_t rr = row0 + R * g + i;
        const bool live = rr < nrows;   // shared-offset slices are never sorted
        const VT di = (live && (EPI == EPI_SMOOTH || EPI == EPI_POLY)) ? invd[rr] : (VT)0;
#pragma unroll
        for (int jj = 0; jj < CPL; jj++) {
            d0[i][jj] = 0.0;
            d1[i][jj] = 0.0;
            if (!live) continue;
            const int64_t o = rr * NB + (q + (jj / G) * R) * G + jj % G;
            const VT a = acc[i][jj];
            if (EPI == EPI_SPMV) {
                Y[o] = (OT)a;
                if (NDOT >= 1) d0[i][jj] = (double)X[o] * (double)a;
                if (NDOT >= 2) d1[i][jj] = (double)X[o] * G1[o];
            } else if (EPI == EPI_RESID) {
                Y[o] = (OT)((VT)F[o] - a);
            } else if (EPI == EPI_SMOOTH) {
                VT out = X[o] + di * ((VT)F[o] - a);
                Y[o] = (OT)out;
                if (NDOT >= 1) d0[i][jj] = (double)out * G0[o];
                if (NDOT >= 2) d1[i][jj] = (double)out * G1[o];
            } else {
                Y[o] = (OT)(coef * (di * (VT)F[o]) + di * a);
            }
        }
    }
    if (NDOT >= 1) {
        // the single-vector butterfly over the 64 rows: row bits >= log2 R
        // across lanes (xor 32 .. R), then the bits below in registers
#pragma unroll
        for (int i = 0; i < R; i++)
#pragma unroll
            for (int jj = 0; jj < CPL; jj++)
                for (int o = 32; o >= R; o >>= 1) {
                    d0[i][jj] += __shfl_xor(d0[i][jj], o, 64);
                    if (NDOT >= 2) d1[i][jj] += __shfl_xor(d1[i][jj], o, 64);
                }
#pragma unroll
        for (int o = R / 2; o >= 1; o >>= 1) {
            double t0[R][CPL], t1[R][CPL];
#pragma unroll
            for (int i = 0; i < R; i++)
#pragma unroll
                for (int jj = 0; jj < CPL; jj++) {
                    t0[i][jj] = d0[i][jj] + d0[i ^ o][jj];
                    t1[i][jj] = d1[i][jj] + d1[i ^ o][jj];
                }
#pragma unroll
            for (int i = 0; i < R; i++)
#pragma unroll
                for (int jj = 0; jj < CPL; jj++) { d0[i][jj] = t0[i][jj]; d1[i][jj] = t1[i][jj]; }
        }
        if (g == 0)
#pragma unroll
            for (int jj = 0; jj < CPL; jj++) {
                const int j = (q + (jj / G) * R) * G + jj % G;
                partial[(2 * w_id) * NB + j] = d0[0][jj];
                partial[(2 * w_id + 1) * NB + j] = NDOT >= 2 ? d1[0][jj] : 0.0;
            }
    }
}

// Slice s of an image with per-row indices (or past the last slice: zero dot
// partials) in a wave of the window kernels: k_sell_blk's gather walk.
template <typename VT, typename FT, typename OT, typename IT, int EPI, int NDOT>
__device__ __forceinline__ void gather_slice(const Sell<VT, IT> &A, int64_t s, int lane, const VT *__restrict__ X,
                                             const FT *__restrict__ F, const VT *__restrict__ invd,
                                             OT *__restrict__ Y, const double *__restrict__ G0,
                                             const double *__restrict__ G1, double *__restrict__ partial,
                                             int64_t w_id, VT coef)
{
    double d0[NB], d1[NB];
#pragma unroll
    for (int j = 0; j < NB; j++) { d0[j] = 0.0; d1[j] = 0.0; }
    if (s < A.nslices) {
        const int64_t row = A.row_of(s * SLICE + lane);
        VT acc[NB];
#pragma unroll
        for (int j = 0; j < NB; j++) acc[j] = 0;
        sell_row<SLICE>(A, s, lane, [&](const VT *v, const int *c) {
#pragma unroll
            for (int t = 0; t < 8; t++) {
                VT xv[NB];
                BlkVec<VT>::load(X + (int64_t)c[t] * NB, xv);
#pragma unroll
                for (int j = 0; j < NB; j++) acc[j] = fma(v[t], xv[j], acc[j]);
            }
        });
        if (row >= 0) {
            const int64_t o = row * NB;
            if (EPI == EPI_SPMV) {
#pragma unroll
                for (int j = 0; j < NB; j++) {
                    Y[o + j] = (OT)acc[j];
                    if (NDOT >= 1) d0[j] = (double)X[o + j] * (double)acc[j];
                    if (NDOT >= 2) d1[j] = (double)X[o + j] * G1[o + j];
                }
            } else if (EPI == EPI_RESID) {
#pragma unroll
                for (int j = 0; j < NB; j++) Y[o + j] = (OT)((VT)F[o + j] - acc[j]);
            } else if (EPI == EPI_SMOOTH) {
                const VT di = invd[row];
#pragma unroll
                for (int j = 0; j < NB; j++) {
                    VT out = X[o + j] + di * ((VT)F[o + j] - acc[j]);
                    Y[o + j] = (OT)out;
                    if (NDOT >= 1) d0[j] = (double)out * G0[o + j];
                    if (NDOT >= 2) d1[j] = (double)out * G1[o + j];
                }
            } else {
                const VT di = invd[row];
#pragma unroll
                for (int j = 0; j < NB; j++) Y[o + j] = (OT)(coef * (di * (VT)F[o + j]) + di * acc[j]);
            }
        }
    }
    if (NDOT >= 1) {
#pragma unroll
        for (int j = 0; j < NB; j++) {
            const double t0 = wave_sum(d0[j]);
            const double t1 = NDOT >= 2 ? wave_sum(d1[j]) : 0.0;
            if (lane == 0) {
                partial[(2 * w_id) * NB + j] = t0;
                partial[(2 * w_id + 1) * NB + j] = t1;
            }
        }
    }
}

template <typename VT, typename FT, typename OT, typename IT, int EPI, int NDOT, int R>
__global__ __launch_bounds__(256) void k_sellw_blk(const Sell<VT, IT> A, const VT *__restrict__ X,
                                                   const FT *__restrict__ F, const VT *__restrict__ invd,
                                                   OT *__restrict__ Y, const double *__restrict__ G0,
                                                   const double *__restrict__ G1, double *__restrict__ partial,
                                                   VT coef)
{
    typedef typename Chunk16<VT>::type CT;
    constexpr int G = 16 / (int)sizeof(VT);           // values per 16-byte chunk (= SELL group)
    constexpr int CH = NB / G;                        // chunks per row of X
    constexpr int CPL = NB / R;                       // columns per lane
    constexpr int CPC = CH / R;                       // chunks per lane
    static_assert(CH % R == 0 && (R == 2 || R == 4), "R must be 2 or 4");
    constexpr int WS = CH + 1;                        // window row stride in chunks
    constexpr int NLD = (WIN_ROWS * WS + 63) / 64;    // copy instructions per window
    constexpr int WN = NLD * 64;                      // chunks per window
    constexpr int XROWS = (WN - 1) / CH + 1;          // rows of X one copy may touch
    constexpr int NGR = (WIN_LMAX + G - 1) / G + 1;   // value groups covering one run
    __shared__ CT win[SELL_WAVES * 2 * WN];   // two windows per wave
    const int lane = threadIdx.x & 63, wid = wave_id();
    // XCD-aware order (xcd_block): every XCD one contiguous range of slices,
    // whose windows overlap (x-lines and planes of the stencil) in its L2
    const int64_t lb = xcd_block((A.nslices + SELL_WAVES - 1) / SELL_WAVES);
    if (lb < 0) return;
    const int64_t s = lb * SELL_WAVES + wid;
    const int64_t w_id = s;
    const int64_t ib = s < A.nslices ? A.ibase[s] : 0;
    // the slice's runs, 64 per vector register (packed: offset << 4 | length;
    // a list without a run table has 0 first and takes the gather path)
    const int32_t *rt = A.shrun + (ib < 0 ? (-1 - ib) >> 1 : 0);
    const int64_t base = s < A.nslices ? A.soff[s] : 0;
    const int width = s < A.nslices ? (int)((A.soff[s + 1] - base) / SLICE) : 0;
    int32_t runs = (ib < 0 && lane < width) ? rt[lane] : 0;
    if (ib < 0 && __builtin_amdgcn_readfirstlane(runs) != 0) {
        const int g = lane / R, q = lane % R;
        VT acc[R][CPL];
#pragma unroll
        for (int i = 0; i < R; i++)
#pragma unroll
            for (int j = 0; j < CPL; j++) acc[i][j] = 0;
        const int64_t row0 = s * SLICE;
        const int hi = (int)(A.ncols - 1);   // rows below 2^29 (checked at set-up)
        CT *W = win + wid * 2 * WN;   // windows W and W + WN, alternating by run
        const CT *Xc = reinterpret_cast<const CT *>(X);
        const CT *Wr = W + R * g * WS + q;   // the lane's first window read
        const int gmax = (width - 1) / G;
        // the window of the run at offset o: rows row0 + o + w; slot 64 i + lane
        // holds chunk xc = slot - slot / WS past the window's first chunk
        auto copy = [&](int g0, CT *D) {
            if (g0 >= 0 && g0 + XROWS - 1 <= hi) {
                const CT *src = Xc + (int64_t)g0 * CH;
#pragma unroll
                for (int i = 0; i < NLD; i++) {
                    const int slot = i * 64 + lane;
                    lds_copy16(src + (slot - slot / WS), D + i * 64);
                }
            } else {
                // first and last slices: rows outside [0, hi] clamped (loaded,
                // never read)
#pragma unroll
                for (int i = 0; i < NLD; i++) {
                    const int slot = i * 64 + lane, xc = slot - slot / WS;
                    const int gr = min(max(g0 + xc / CH, 0), hi);
                    lds_copy16(Xc + (int64_t)gr * CH + xc % CH, D + i * 64);
                }
            }
        };
        // value groups of the lane's own row holding entries kr .. kr + WIN_LMAX
        // - 1 (groups past the slice clamped to its last one, unused)
        auto load_vals = [&](CT (&dst)[NGR], int kr) {
#pragma unroll
            for (int j = 0; j < NGR; j++) {
                const int gi = min(kr / G + j, gmax);
                const VT *p = A.val + base + (int64_t)gi * (G * SLICE) + lane * G;
                dst[j] = load_group<VT>(reinterpret_cast<const CT *>(p));
            }
        };
        // per run: wait for its window and values (issued one run ahead),
        // issue the next run's window into the other buffer and its values,
        // then sum this run while those are in flight
        int k = 0, rho = 0;
        int32_t pk = __builtin_amdgcn_readfirstlane(runs);
        auto step = [&](const CT (&vg)[NGR], CT (&vn)[NGR], auto BUFC) {
            constexpr int BUF = decltype(BUFC)::value;
            const int L = pk & 15;
            const int kn = k + L;
            rho++;
            if ((rho & 63) == 0) runs = (rho + lane < width) ? rt[rho + lane] : 0;
            const int32_t pn = kn < width ? __builtin_amdgcn_readlane(runs, rho & 63) : 0;
            // this run's window and values have arrived, and every LDS read of
            // the other window (two runs back) has returned
            __builtin_amdgcn_s_waitcnt(wait_vm(0));
            __builtin_amdgcn_s_waitcnt(WAIT_LGKM0);
            wave_lds_sync();
            if (pn != 0) copy((int)row0 + (pn >> 4), W + (1 - BUF) * WN);
            load_vals(vn, kn);
            typedef WinRun<VT, R, NGR> WR;
            const CT *Wb = Wr + BUF * WN;
            if (G == 2) {
                if (k & 1) WR::template len<1>(acc, Wb, vg, L);
                else WR::template len<0>(acc, Wb, vg, L);
            } else {
                switch (k & (G - 1)) {
                case 0: WR::template len<0>(acc, Wb, vg, L); break;
                case 1: WR::template len<1>(acc, Wb, vg, L); break;
                case 2: WR::template len<2 % G>(acc, Wb, vg, L); break;
                default: WR::template len<3 % G>(acc, Wb, vg, L); break;
                }
            }
            // the next run's value registers stay allocated through the sums
            // of every run length (a dead group would be reused, and its
            // register then waited for)
#pragma unroll
            for (int j = 0; j < NGR; j++) keep_in_vgprs(vn[j]);
            k = kn;
            pk = pn;
        };
        CT va[NGR], vb[NGR];
        copy((int)row0 + (pk >> 4), W);
        load_vals(va, 0);
        while (pk != 0) {
            step(va, vb, std::integral_constant<int, 0>());
            if (pk == 0) break;
            step(vb, va, std::integral_constant<int, 1>());
        }
        win_epilogue<VT, FT, OT, EPI, NDOT, R>(acc, row0, A.nrows, g, q, X, F, invd, Y, G0, G1, partial, w_id, coef);
        return;
    }
    gather_slice<VT, FT, OT, IT, EPI, NDOT>(A, s, lane, X, F, invd, Y, G0, G1, partial, w_id, coef);
}

// The same pass with windows shared by the four waves of a block: the block's
// slices and its stages come from the image's stage table (WgStages, built at
// set-up), every stage's WIN_WG_ROWS rows of X are copied once into the
// block's LDS (the four waves each issuing a share of the copy) and every
// wave whose next run lies in them sums that run from there.  With slices one
// grid line apart, the runs of neighbouring lines (y displacements) fall into
// the same windows: at c4 the block copies 0.39 of the rows its waves would
// copy alone.  Two windows alternate by stage; one block barrier per stage
// orders the copies (each wave waits for its own share, vmcnt 0, before the
// barrier) and the reads (all of a window's readers are past the barrier
// before the next copy into it is issued).  Sums, dots and epilogues are the
// per-wave kernel's, in the same order.
template <typename VT, typename FT, typename OT, typename IT, int EPI, int NDOT, int R>
__global__ __launch_bounds__(256, 4) void k_sellws_blk(const Sell<VT, IT> A, const VT *__restrict__ X,
                                                    const FT *__restrict__ F, const VT *__restrict__ invd,
                                                    OT *__restrict__ Y, const double *__restrict__ G0,
                                                    const double *__restrict__ G1, double *__restrict__ partial,
                                                    VT coef)
{
    typedef typename Chunk16<VT>::type CT;
    constexpr int G = 16 / (int)sizeof(VT);
    constexpr int CH = NB / G;
    constexpr int CPL = NB / R;
    static_assert(CH % R == 0 && (R == 2 || R == 4), "R must be 2 or 4");
    constexpr int WS = CH + 1;
    constexpr int NLD = (WIN_WG_ROWS * WS + 63) / 64;   // copy instructions per window (shared by the waves)
    constexpr int WN = NLD * 64;
    constexpr int XROWS = (WN - 1) / CH + 1;
    constexpr int NGR = (WIN_LMAX + G - 1) / G + 1;
    __shared__ CT win[2 * WN];
    const int lane = threadIdx.x & 63, wid = wave_id();
    const int64_t lb = xcd_block((A.nslices + SELL_WAVES - 1) / SELL_WAVES);
    if (lb < 0) return;   // the whole block
    const int32_t *wt = A.wgtab + lb * 8;
    const int64_t s = wt[wid];
    const int st0 = wt[4], nst = wt[5];
    const int64_t ib = s < A.nslices ? A.ibase[s] : 0;
    const int32_t *rt = A.shrun + (ib < 0 ? (-1 - ib) >> 1 : 0);
    const int64_t base = s < A.nslices ? A.soff[s] : 0;
    const int width = s < A.nslices ? (int)((A.soff[s + 1] - base) / SLICE) : 0;
    int32_t runs = (ib < 0 && lane < width) ? rt[lane] : 0;
    const bool mine = ib < 0 && __builtin_amdgcn_readfirstlane(runs) != 0;
    if (!mine) gather_slice<VT, FT, OT, IT, EPI, NDOT>(A, s, lane, X, F, invd, Y, G0, G1, partial, s, coef);
    if (nst == 0) return;   // the whole block
    const int g = lane / R, q = lane % R;
    VT acc[R][CPL];
#pragma unroll
    for (int i = 0; i < R; i++)
#pragma unroll
        for (int j = 0; j < CPL; j++) acc[i][j] = 0;
    const int64_t row0 = s * SLICE;
    const int hi = (int)(A.ncols - 1);
    const CT *Xc = reinterpret_cast<const CT *>(X);
    const CT *Wl = win + R * g * WS + q;   // the lane's first read in a window at row shift 0
    const int gmax = (width - 1) / G;
    // this wave's share of the copy of the window at row g0 into buffer D:
    // instructions i = wid, wid + 4, ...
    auto copy = [&](int g0, CT *D) {
        if (g0 >= 0 && g0 + XROWS - 1 <= hi) {
            const CT *src = Xc + (int64_t)g0 * CH;
#pragma unroll
            for (int i0 = 0; i0 < NLD; i0 += SELL_WAVES) {
                const int i = i0 + wid;
                if (i < NLD) {
                    const int slot = i * 64 + lane;
                    lds_copy16(src + (slot - slot / WS), D + i * 64);
                }
            }
        } else {
#pragma unroll
            for (int i0 = 0; i0 < NLD; i0 += SELL_WAVES) {
                const int i = i0 + wid;
                if (i < NLD) {
                    const int slot = i * 64 + lane, xc = slot - slot / WS;
                    const int gr = min(max(g0 + xc / CH, 0), hi);
                    lds_copy16(Xc + (int64_t)gr * CH + xc % CH, D + i * 64);
                }
            }
        }
    };
    auto load_vals = [&](CT (&dst)[NGR], int kr) {
#pragma unroll
        for (int j = 0; j < NGR; j++) {
            const int gi = min(kr / G + j, gmax);
            const VT *p = A.val + base + (int64_t)gi * (G * SLICE) + lane * G;
            dst[j] = load_group<VT>(reinterpret_cast<const CT *>(p));
        }
    };
    int k = 0, rho = 0;
    int32_t pk = mine ? __builtin_amdgcn_readfirstlane(runs) : 0;
    CT vg[NGR], vn[NGR];
    if (mine) load_vals(vg, 0);
    const int32_t *st = A.wgst + 2 * (int64_t)st0;
    copy(st[0], win);
    for (int t = 0; t < nst; t++) {
        // this wave's share of window t and its values have arrived; after the
        // barrier every share has, and every read of window t - 1 is done
        __builtin_amdgcn_s_waitcnt(wait_vm(0));
        __syncthreads();
        if (t + 1 < nst) copy(st[2 * (t + 1)], win + ((t + 1) & 1) * WN);
        const int me = (st[2 * t + 1] >> (8 * wid)) & 0xFF;
        if (me & 0x80) {
            const int L = pk & 15;
            const int kn = k + L;
            rho++;
            if ((rho & 63) == 0) runs = (rho + lane < width) ? rt[rho + lane] : 0;
            const int32_t pn = kn < width ? __builtin_amdgcn_readlane(runs, rho & 63) : 0;
            load_vals(vn, kn);
            typedef WinRun<VT, R, NGR> WR;
            const CT *Wb = Wl + (t & 1) * WN + (me & 0x7F) * WS;
            if (G == 2) {
                if (k & 1) WR::template len<1>(acc, Wb, vg, L);
                else WR::template len<0>(acc, Wb, vg, L);
            } else {
                switch (k & (G - 1)) {
                case 0: WR::template len<0>(acc, Wb, vg, L); break;
                case 1: WR::template len<1>(acc, Wb, vg, L); break;
                case 2: WR::template len<2 % G>(acc, Wb, vg, L); break;
                default: WR::template len<3 % G>(acc, Wb, vg, L); break;
                }
            }
#pragma unroll
            for (int j = 0; j < NGR; j++) vg[j] = vn[j];
            k = kn;
            pk = pn;
        }
    }
    if (mine) win_epilogue<VT, FT, OT, EPI, NDOT, R>(acc, row0, A.nrows, g, q, X, F, invd, Y, G0, G1, partial, s, coef);
}

// Block matrix pass with LPR lanes per row: the wave covers a slice of
// C = 64 / LPR rows of a SELL-C image (same group layout as SELL-64 with the
// slice height C), lane = (row r = lane / LPR, quarter q = lane % LPR), each
// lane owning RPL = 16 / LPR consecutive columns.  The LPR lanes of a row read
// the same matrix groups (one broadcast address) and together one contiguous
// 16-column row of X per entry, so every X load of the wave is C contiguous
// 64-byte (FP32) or 128-byte (FP64) runs.  Blocks of any multiple of 64
// threads walk the slices grid-stride; per column the dot partials are summed
// over the rows of a wave (butterfly over the row bits of the lane), then over
// the block's waves in order: partial[(blockIdx.x * 2 + d) * NB + j].
template <typename VT> struct RowLoad;
typedef float vf2 __attribute__((ext_vector_type(2)));
template <> struct RowLoad<float> {
    template <int RPL> static __device__ inline void load(const float *p, float (&o)[RPL])
    {
        if constexpr (RPL == 4) {
            vf4 t = *reinterpret_cast<const vf4 *>(p);
            o[0] = t.x; o[1] = t.y; o[2] = t.z; o[3] = t.w;
        } else if constexpr (RPL == 2) {
            vf2 t = *reinterpret_cast<const vf2 *>(p);
            o[0] = t.x; o[1] = t.y;
        } else {
#pragma unroll
            for (int j = 0; j < RPL; j++) o[j] = p[j];
        }
    }
};
template <> struct RowLoad<double> {
    template <int RPL> static __device__ inline void load(const double *p, double (&o)[RPL])
    {
        if constexpr (RPL % 2 == 0) {
#pragma unroll
            for (int h = 0; h < RPL / 2; h++) {
                vd2 t = reinterpret_cast<const vd2 *>(p)[h];
                o[2 * h] = t.x; o[2 * h + 1] = t.y;
            }
        } else {
#pragma unroll
            for (int j = 0; j < RPL; j++) o[j] = p[j];
        }
    }
};

template <typename VT, typename FT, typename OT, typename IT, int EPI, int NDOT, int LPR>
__global__ __launch_bounds__(512) void k_sellb(const Sell<VT, IT> A, const VT *__restrict__ X,
                                               const FT *__restrict__ F, const VT *__restrict__ invd,
                                               OT *__restrict__ Y, const double *__restrict__ G0,
                                               const double *__restrict__ G1, double *__restrict__ partial,
                                               VT coef)
{
    constexpr int C = 64 / LPR, RPL = NB / LPR;
    __shared__ double lds[2 * 8 * NB];
    const int lane = threadIdx.x & 63, wid = wave_id(), nw = blockDim.x >> 6;
    const int r = lane / LPR, q = lane % LPR;
    double d0[RPL], d1[RPL];
#pragma unroll
    for (int j = 0; j < RPL; j++) { d0[j] = 0.0; d1[j] = 0.0; }
    for (int64_t s = (int64_t)blockIdx.x * nw + wid; s < A.nslices; s += (int64_t)gridDim.x * nw) {
        const int64_t row = A.row_of(s * C + r);
        VT acc[RPL];
#pragma unroll
        for (int j = 0; j < RPL; j++) acc[j] = 0;
        sell_row<C>(A, s, r, [&](const VT *v, const int *c) {
#pragma unroll
            for (int t = 0; t < 8; t++) {
                VT xv[RPL];
                RowLoad<VT>::template load<RPL>(X + (int64_t)c[t] * NB + q * RPL, xv);
#pragma unroll
                for (int j = 0; j < RPL; j++) acc[j] = fma(v[t], xv[j], acc[j]);
            }
        });
        if (row >= 0) {
            const int64_t o = row * NB + q * RPL;
            if (EPI == EPI_SPMV) {
#pragma unroll
                for (int j = 0; j < RPL; j++) {
                    Y[o + j] = (OT)acc[j];
                    if (NDOT >= 1) d0[j] += (double)X[o + j] * (double)acc[j];
                    if (NDOT >= 2) d1[j] += (double)X[o + j] * G1[o + j];
                }
            } else if (EPI == EPI_RESID) {
#pragma unroll
                for (int j = 0; j < RPL; j++) Y[o + j] = (OT)((VT)F[o + j] - acc[j]);
            } else if (EPI == EPI_SMOOTH) {
                const VT di = invd[row];
#pragma unroll
                for (int j = 0; j < RPL; j++) {
                    VT out = X[o + j] + di * ((VT)F[o + j] - acc[j]);
                    Y[o + j] = (OT)out;
                    if (NDOT >= 1) d0[j] += (double)out * G0[o + j];
                    if (NDOT >= 2) d1[j] += (double)out * G1[o + j];
                }
            } else {
                const VT di = invd[row];
#pragma unroll
                for (int j = 0; j < RPL; j++) Y[o + j] = (OT)(coef * (di * (VT)F[o + j]) + di * acc[j]);
            }
        }
    }
    if (NDOT >= 1) {
#pragma unroll
        for (int j = 0; j < RPL; j++)
            for (int o = LPR; o < 64; o <<= 1) {
                d0[j] += __shfl_xor(d0[j], o, 64);
                d1[j] += __shfl_xor(d1[j], o, 64);
            }
        if (r == 0)
#pragma unroll
            for (int j = 0; j < RPL; j++) {
                lds[(wid * NB + q * RPL + j) * 2] = d0[j];
                lds[(wid * NB + q * RPL + j) * 2 + 1] = d1[j];
            }
        __syncthreads();
        if (threadIdx.x < 2 * NB) {
            const int j = threadIdx.x >> 1, d = threadIdx.x & 1;
            double t = 0.0;
            for (int w = 0; w < nw; w++) t += lds[(w * NB + j) * 2 + d];
            partial[(2 * blockIdx.x + d) * NB + j] = (d == 1 && NDOT < 2) ? 0.0 : t;
        }
    }
}

// Fused prolongation + first post-smoothing sweep for 16 columns (see
// k_sell_post): acc = (K P) E over the SELL-64 image of K P, one lane per row;
// Y = U + P E + D^{-1} (R - acc).  Per column the order of k_sell_post.
template <typename VT, typename OT, typename IT, int NDOT>
__global__ __launch_bounds__(256) void k_sell_blk_post(const Sell<VT, IT> A, const VT *__restrict__ E, const VT *__restrict__ U,
                                                       const VT *__restrict__ R, const VT *__restrict__ invd,
                                                       const int32_t *__restrict__ agg, const VT *__restrict__ pc,
                                                       OT *__restrict__ Y, const double *__restrict__ G0,
                                                       const double *__restrict__ G1, double *__restrict__ partial)
{
    __shared__ double lds[8 * NB];
    const int lane = threadIdx.x & 63, wid = wave_id();
    const int64_t s = (int64_t)blockIdx.x * SELL_WAVES + wid;
    double d0[NB], d1[NB];
#pragma unroll
    for (int j = 0; j < NB; j++) { d0[j] = 0.0; d1[j] = 0.0; }
    if (s < A.nslices) {
        const int64_t row = A.row_of(s * SLICE + lane);
        VT acc[NB];
#pragma unroll
        for (int j = 0; j < NB; j++) acc[j] = 0;
        sell_row<SLICE>(A, s, lane, [&](const VT *v, const int *c) {
#pragma unroll
            for (int t = 0; t < 8; t++) {
                VT xv[NB];
                BlkVec<VT>::load(E + (int64_t)c[t] * NB, xv);
#pragma unroll
                for (int j = 0; j < NB; j++) acc[j] = fma(v[t], xv[j], acc[j]);
            }
        });
        if (row >= 0) {
            const int64_t o = row * NB, a = (int64_t)agg[row] * NB;
            const VT di = invd[row], pi = pc[row];
#pragma unroll
            for (int j = 0; j < NB; j++) {
                VT out = post_update(U[o + j], pi, E[a + j], di, R[o + j], acc[j]);
                Y[o + j] = (OT)out;
                if (NDOT >= 1) d0[j] = (double)out * G0[o + j];
                if (NDOT >= 2) d1[j] = (double)out * G1[o + j];
            }
        }
    }
    if (NDOT >= 1) {
        // one partial per wavefront and column, as the single-vector kernels
        const int64_t w = (int64_t)blockIdx.x * SELL_WAVES + wid;
#pragma unroll
        for (int j = 0; j < NB; j++) {
            const double t0 = wave_sum(d0[j]);
            const double t1 = NDOT >= 2 ? wave_sum(d1[j]) : 0.0;
            if (lane == 0) {
                partial[(2 * w) * NB + j] = t0;
                partial[(2 * w + 1) * NB + j] = t1;
            }
        }
    }
}

// The same with LPR lanes per row on a SELL-(64/LPR) image of K P (layout and
// reductions of k_sellb).
template <typename VT, typename OT, typename IT, int NDOT, int LPR>
__global__ __launch_bounds__(512) void k_sellb_post(const Sell<VT, IT> A, const VT *__restrict__ E,
                                                    const VT *__restrict__ U, const VT *__restrict__ R,
                                                    const VT *__restrict__ invd, const int32_t *__restrict__ agg,
                                                    const VT *__restrict__ pc, OT *__restrict__ Y,
                                                    const double *__restrict__ G0, const double *__restrict__ G1,
                                                    double *__restrict__ partial)
{
    constexpr int C = 64 / LPR, RPL = NB / LPR;
    __shared__ double lds[2 * 8 * NB];
    const int lane = threadIdx.x & 63, wid = wave_id(), nw = blockDim.x >> 6;
    const int r = lane / LPR, q = lane % LPR;
    double d0[RPL], d1[RPL];
#pragma unroll
    for (int j = 0; j < RPL; j++) { d0[j] = 0.0; d1[j] = 0.0; }
    for (int64_t s = (int64_t)blockIdx.x * nw + wid; s < A.nslices; s += (int64_t)gridDim.x * nw) {
        const int64_t row = A.row_of(s * C + r);
        VT acc[RPL];
#pragma unroll
        for (int j = 0; j < RPL; j++) acc[j] = 0;
        sell_row<C>(A, s, r, [&](const VT *v, const int *c) {
#pragma unroll
            for (int t = 0; t < 8; t++) {
                VT xv[RPL];
                RowLoad<VT>::template load<RPL>(E + (int64_t)c[t] * NB + q * RPL, xv);
#pragma unroll
                for (int j = 0; j < RPL; j++) acc[j] = fma(v[t], xv[j], acc[j]);
            }
        });
        if (row >= 0) {
            const int64_t o = row * NB + q * RPL, a = (int64_t)agg[row] * NB + q * RPL;
            const VT di = invd[row], pi = pc[row];
#pragma unroll
            for (int j = 0; j < RPL; j++) {
                VT out = post_update(U[o + j], pi, E[a + j], di, R[o + j], acc[j]);
                Y[o + j] = (OT)out;
                if (NDOT >= 1) d0[j] += (double)out * G0[o + j];
                if (NDOT >= 2) d1[j] += (double)out * G1[o + j];
            }
        }
    }
    if (NDOT >= 1) {
#pragma unroll
        for (int j = 0; j < RPL; j++)
            for (int o = LPR; o < 64; o <<= 1) {
                d0[j] += __shfl_xor(d0[j], o, 64);
                d1[j] += __shfl_xor(d1[j], o, 64);
            }
        if (r == 0)
#pragma unroll
            for (int j = 0; j < RPL; j++) {
                lds[(wid * NB + q * RPL + j) * 2] = d0[j];
                lds[(wid * NB + q * RPL + j) * 2 + 1] = d1[j];
            }
        __syncthreads();
        if (threadIdx.x < 2 * NB) {
            const int j = threadIdx.x >> 1, d = threadIdx.x & 1;
            double t = 0.0;
            for (int w = 0; w < nw; w++) t += lds[(w * NB + j) * 2 + d];
            partial[(2 * blockIdx.x + d) * NB + j] = (d == 1 && NDOT < 2) ? 0.0 : t;
        }
    }
}

// ---- elementwise block kernels (one thread per row, 16 columns) ---------------

template <typename VT, typename FT>
__global__ void k_scale_blk(int64_t n, const VT *__restrict__ invd, const FT *__restrict__ f, VT *__restrict__ u,
                            VT coef)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const VT di = invd[i];
#pragma unroll
    for (int j = 0; j < NB; j++) u[i * NB + j] = coef * (di * (VT)f[i * NB + j]);
}

// coef == 1 keeps the l1 sweep's bits: 1 * (d * f) == d * f exactly.
template <typename VT>
__global__ void k_restrict_blk(int64_t nc, int mw, const int32_t *__restrict__ members, const VT *__restrict__ pc,
                               const VT *__restrict__ r, VT *__restrict__ fc, const VT *__restrict__ invdc,
                               VT *__restrict__ uc, VT coef)
{
#pragma clang fp contract(off)
    int64_t I = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (I >= nc) return;
    VT s[NB];
#pragma unroll
    for (int j = 0; j < NB; j++) s[j] = 0;
    for (int t = 0; t < mw; t++) {
        int m = members[I * mw + t];
        if (m < 0) break;
        const VT pm = pc[m];
#pragma unroll
        for (int j = 0; j < NB; j++) {
            VT prod = pm * r[(int64_t)m * NB + j];
            s[j] = s[j] + prod;
        }
    }
#pragma unroll
    for (int j = 0; j < NB; j++) fc[I * NB + j] = s[j];
    if (uc) {
        const VT di = invdc[I];
#pragma unroll
        for (int j = 0; j < NB; j++) uc[I * NB + j] = coef * (di * s[j]);
    }
}

template <typename VT>
__global__ void k_prolong_blk(int64_t n, const int32_t *__restrict__ agg, const VT *__restrict__ pc,
                              const VT *__restrict__ e, VT *__restrict__ u)
{
#pragma clang fp contract(off)
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const VT pi = pc[i];
    const int64_t a = (int64_t)agg[i] * NB;
#pragma unroll
    for (int j = 0; j < NB; j++) {
        VT prod = pi * e[a + j];
        u[i * NB + j] = u[i * NB + j] + prod;
    }
}

template <typename VT, typename OT>
__global__ void k_add_blk(int64_t n, const VT *__restrict__ x, const VT *__restrict__ c, OT *__restrict__ y)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n * NB) return;
    y[i] = (OT)(x[i] + c[i]);
}

// Coarsest level for 16 columns, in two launches over 16-row tiles (block =
// 16 rows x 16 columns, thread = one output element):
//   phase 0: Y = L^{-1} F,   phase 1: E = L^{-T} Y   (Y: global scratch, n x 16).
// Per element the single-vector kernel's order (k ascending), so each column
// equals k_coarse_solve's result.
template <typename VT>
__global__ __launch_bounds__(256) void k_coarse_solve_blk(int n, int ld, const double *__restrict__ Linv,
                                                          const double *__restrict__ LinvT, const VT *__restrict__ f,
                                                          double *__restrict__ Y, VT *__restrict__ e, int phase)
{
    const int j = threadIdx.x & (NB - 1);
    const int i = blockIdx.x * (256 / NB) + threadIdx.x / NB;
    if (i >= n) return;
    double s = 0.0;
    if (phase == 0) {
#pragma unroll 8
        for (int k = 0; k <= i; k++) s = fma(LinvT[(int64_t)k * ld + i], (double)f[(int64_t)k * NB + j], s);
        Y[(int64_t)i * NB + j] = s;
    } else {
#pragma unroll 8
        for (int k = i; k < n; k++) s = fma(Linv[(int64_t)k * ld + i], Y[(int64_t)k * NB + j], s);
        e[(int64_t)i * NB + j] = (VT)s;
    }
}

// Column-major (n x k, leading dimension n) <-> row-major block (n x NB).
__global__ void k_pack_blk(int64_t n, int k, const double *__restrict__ cm, double *__restrict__ rm)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
#pragma unroll
    for (int j = 0; j < NB; j++) rm[i * NB + j] = j < k ? cm[(int64_t)j * n + i] : 0.0;
}

__global__ void k_unpack_blk(int64_t n, int k, const double *__restrict__ rm, double *__restrict__ cm)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    for (int j = 0; j < k; j++) cm[(int64_t)j * n + i] = rm[i * NB + j];
}

// ---- element-parallel block vector kernels ----------------------------------
//
// Thread t of the grid handles the elements e = t, t + T, ... (T = threads in
// the grid, a multiple of 16) of the row-major N x 16 arrays, so a wave's load
// is 64 consecutive values and every thread keeps one column j = e % 16.  Dot
// partials per column: the thread's running sum, the 4 lanes of each column in
// a wave (butterfly over lane bits 4 and 5), then the block's waves in order:
// partial[(2 * blockIdx.x + d) * NB + j].

__device__ inline void blk_col_partials(double s0, double s1, double *lds /* 2 * 4 * NB */, double *partial)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    s0 += __shfl_xor(s0, 16, 64);
    s0 += __shfl_xor(s0, 32, 64);
    s1 += __shfl_xor(s1, 16, 64);
    s1 += __shfl_xor(s1, 32, 64);
    if (lane < NB) {
        lds[wid * NB + lane] = s0;
        lds[(4 + wid) * NB + lane] = s1;
    }
    __syncthreads();
    if (threadIdx.x < NB) {
        const int j = threadIdx.x;
        partial[(2 * blockIdx.x) * NB + j] = ((lds[j] + lds[NB + j]) + lds[2 * NB + j]) + lds[3 * NB + j];
        partial[(2 * blockIdx.x + 1) * NB + j] =
            ((lds[4 * NB + j] + lds[5 * NB + j]) + lds[6 * NB + j]) + lds[7 * NB + j];
    }
}

// per-column partials of (a, b) and (a, c) (c may be NULL)
__global__ __launch_bounds__(256) void k_dot2_blk(int64_t n, const double *__restrict__ a, const double *__restrict__ b,
                                                  const double *__restrict__ c, double *__restrict__ partial)
{
    __shared__ double lds[8 * NB];
    double s0 = 0.0, s1 = 0.0;
    const int64_t m = n * NB;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < m; e += (int64_t)gridDim.x * 256) {
        s0 = fma(a[e], b[e], s0);
        if (c) s1 = fma(a[e], c[e], s1);
    }
    blk_col_partials(s0, s1, lds, partial);
}

// u += alpha p ; r -= alpha q for the active columns; partials of (r, r).
__global__ __launch_bounds__(256) void k_bcg_update(int64_t n, const double *__restrict__ sc, double *__restrict__ u,
                                                    double *__restrict__ r, const double *__restrict__ p,
                                                    const double *__restrict__ q, double *__restrict__ partial)
{
    __shared__ double lds[8 * NB];
    const int j = threadIdx.x & (NB - 1);
    const bool act = bactive(sc, j);
    const double al = sc[B_ALPHA * NB + j];
    double s = 0.0;
    const int64_t m = n * NB;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < m; e += (int64_t)gridDim.x * 256) {
        double ri = r[e];
        if (act) {
            u[e] = fma(al, p[e], u[e]);
            ri = fma(-al, q[e], ri);
            r[e] = ri;
        }
        s = fma(ri, ri, s);
    }
    blk_col_partials(s, 0.0, lds, partial);
}

// p = z + beta p for the active columns
__global__ __launch_bounds__(256) void k_bcg_pupdate(int64_t n, const double *__restrict__ sc,
                                                     const double *__restrict__ z, double *__restrict__ p)
{
    const int j = threadIdx.x & (NB - 1);
    if (!bactive(sc, j)) return;
    const double be = sc[B_BETA * NB + j];
    const int64_t m = n * NB;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < m; e += (int64_t)gridDim.x * 256)
        p[e] = fma(be, p[e], z[e]);
}

// First stage of k_bfinalize for many partials: the strided sums that its
// thread t would form (partials t, t + FIN_THREADS, ... in ascending order),
// one grid thread per (t, dot, column): strided[(d * NB + j) * FIN_THREADS + t].
__global__ __launch_bounds__(256) void k_bfin_strided(const double *__restrict__ partial, int nblk,
                                                      double *__restrict__ strided)
{
    const int idx = blockIdx.x * 256 + threadIdx.x;   // < 2 * NB * FIN_THREADS
    const int j = idx % NB, d = (idx / NB) % 2, t = idx / (2 * NB);
    double s = 0.0;
    for (int b = t; b < nblk; b += FIN_THREADS) s += partial[(2 * b + d) * NB + j];
    strided[(d * NB + j) * FIN_THREADS + t] = s;
}

// Final per-column sums of the partials (index order) and the scalar
// recurrences, masks and iteration counters of the 16 independent solves.
// With strided != nullptr the per-thread strided sums come from
// k_bfin_strided (the same values).
__global__ __launch_bounds__(FIN_THREADS) void k_bfinalize(const double *__restrict__ partial, int nblk, double *sc,
                                                           int op, double tol, const double *__restrict__ strided)
{
    // per column the order of k_finalize: thread strides, butterfly, waves in order
    constexpr int NW = FIN_THREADS / 64;
    __shared__ double lds[2 * NW * NB];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    double s0[NB], s1[NB];
#pragma unroll
    for (int j = 0; j < NB; j++) { s0[j] = 0.0; s1[j] = 0.0; }
    if (strided) {
#pragma unroll
        for (int j = 0; j < NB; j++) {
            s0[j] = strided[j * FIN_THREADS + threadIdx.x];
            s1[j] = strided[(NB + j) * FIN_THREADS + threadIdx.x];
        }
    } else {
        for (int b = threadIdx.x; b < nblk; b += FIN_THREADS)
#pragma unroll
            for (int j = 0; j < NB; j++) { s0[j] += partial[(2 * b) * NB + j]; s1[j] += partial[(2 * b + 1) * NB + j]; }
    }
#pragma unroll
    for (int j = 0; j < NB; j++) { s0[j] = wave_sum(s0[j]); s1[j] = wave_sum(s1[j]); }
    if (lane == 0)
#pragma unroll
        for (int j = 0; j < NB; j++) { lds[wid * NB + j] = s0[j]; lds[(NW + wid) * NB + j] = s1[j]; }
    __syncthreads();
    // thread j: column j, its waves summed in order (the columns are independent)
    if (threadIdx.x >= NB) return;
    {
        const int j = threadIdx.x;
        double a = 0.0, b = 0.0;
        for (int w = 0; w < NW; w++) { a += lds[w * NB + j]; b += lds[(NW + w) * NB + j]; }
        double *F = sc + B_FLAG * NB + j, *D = sc + B_DONE * NB + j;
        switch (op) {
        case BF_FF:
            sc[B_FF * NB + j] = a;
            sc[B_THR * NB + j] = tol * sqrt(a);
            break;
        case BF_RR0:   // initial residual: converged columns are done before any update
            sc[B_RR * NB + j] = a;
            if (sc[B_FF * NB + j] == 0.0 || sqrt(a) <= sc[B_THR * NB + j]) *D = 1.0;
            break;
        case BF_RZ0:
            if (*D != 0.0) break;
            sc[B_RZ * NB + j] = a;
            if (!(a > 0.0) || !isfinite(a)) *F = 2.0;
            break;
        case BF_PQ_CG:
        case BF_PQ_FCG:
            if (*D != 0.0 || *F != 0.0) break;
            sc[B_PQ * NB + j] = a;
            if (op == BF_PQ_FCG) sc[B_PR * NB + j] = b;
            if (!(a > 0.0) || !isfinite(a)) *F = 1.0;
            else sc[B_ALPHA * NB + j] = (op == BF_PQ_FCG ? b : sc[B_RZ * NB + j]) / a;
            break;
        case BF_RR:   // one more completed update of this column
            if (*D != 0.0 || *F != 0.0) break;
            sc[B_RR * NB + j] = a;
            sc[B_ITERS * NB + j] += 1.0;
            if (sqrt(a) <= sc[B_THR * NB + j]) *D = 1.0;
            break;
        case BF_RZ_CG:
            if (*D != 0.0 || *F != 0.0) break;
            if (!(a > 0.0) || !isfinite(a)) *F = 2.0;
            else { sc[B_BETA * NB + j] = a / sc[B_RZ * NB + j]; sc[B_RZ * NB + j] = a; }
            break;
        case BF_ZQ_FCG:
            if (*D != 0.0 || *F != 0.0) break;
            sc[B_ZQ * NB + j] = a;
            if (!isfinite(a)) *F = 2.0;
            else sc[B_BETA * NB + j] = -a / sc[B_PQ * NB + j];
            break;
        }
    }
}

}  // namespace amgk
