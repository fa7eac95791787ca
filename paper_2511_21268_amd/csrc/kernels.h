// Device kernels of the solve phase (gfx950, wave64).
//
// Sparse matrices are held in a sliced-ELL layout (SELL-C: C consecutive rows
// per slice; C = 64 gives one slice per wavefront, lane = row): each slice
// stores width w_s entries per row, column-major across its C rows so that every
// load of the wave is one contiguous run.  Entries are interleaved in groups of
// G per lane so that each lane issues 16-byte loads: element (k, r) of a slice
// whose stream starts at element `base` lives at
//     base + (k / G) * C * G + r * G + (k % G),
// with G = 2 for FP64 values, 4 for FP32 values and int32 columns, and 8 for
// 16-bit column deltas.  A lane walks its row in ascending column order.
//
// A slice stores its columns in one of two ways.
//  * Shared offsets: when the column offsets (column - row) of all rows of the
//    slice fit in one ascending list no longer than the slice's widest row
//    (stencil-like matrices: the rows of a slice differ only at boundaries),
//    the list is stored once per slice and lane r of row `row` reads column
//    row + offset[k]; entries a row does not have hold the value 0 (their
//    column is clamped into [0, ncols)).  The index stream costs ~0 bytes per
//    entry.
//  * Per-row indices: 16-bit column deltas (the column is a running sum from
//    col0[row], the row's first column) when every gap fits, else int32
//    columns; padding holds value 0 and delta 0 (or the last column).
// w_s is the longer of the row lengths or the offset list, rounded up to 8.
// Images of matrices without shared offsets place the rows of each window of
// 4 slices in its slots by decreasing length (SELL-C-sigma with sigma = 4C), so
// that the slices of a window pad to similar widths; perm maps slot -> row.
//
// Every reduction is deterministic: fixed grid, butterfly within the wave, one
// partial per wavefront (matrix passes) or a fixed-order sum across the block's
// waves and one partial per block (vector kernels), and a single-block final
// sum in index order.  No floating-point atomics.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "layout.h"

namespace amgk {

typedef double vd2 __attribute__((ext_vector_type(2)));
typedef float vf4 __attribute__((ext_vector_type(4)));
typedef unsigned vu4 __attribute__((ext_vector_type(4)));
typedef int vi4 __attribute__((ext_vector_type(4)));

constexpr int SLICE = 64;
constexpr int SELL_WAVES = 4;          // slices (wavefronts) per 256-thread block
constexpr int XCDS = 8;                // accelerator complex dies sharing the grid (one L2 each)

// XCD-aware block order (used by the staged-window block kernel).  The
// hardware deals blocks to the XCDs round-robin (block b runs on XCD b % XCDS);
// block b takes logical block (b % XCDS) * per + b / XCDS, so every XCD works
// through one contiguous range of slices and the neighbouring rows its loads
// reach stay in that XCD's L2.  Grids are padded to a multiple of XCDS;
// xcd_block returns -1 for a padding block.  Dot partials are indexed by
// logical block, so the order of every sum does not depend on this mapping.
// (The single-vector matrix passes keep the plain order: measured the same.)
__device__ __forceinline__ int64_t xcd_block(int64_t nlb)
{
    const int64_t per = (nlb + XCDS - 1) / XCDS;
    const int64_t lb = (int64_t)(blockIdx.x % XCDS) * per + blockIdx.x / XCDS;
    return lb < nlb ? lb : -1;
}
inline unsigned xcd_grid(int64_t nlb) { return (unsigned)((nlb + XCDS - 1) / XCDS * XCDS); }
constexpr int RED_THREADS = 256;

enum Epi { EPI_SPMV = 0, EPI_RESID = 1, EPI_SMOOTH = 2, EPI_POLY = 3, EPI_ADD = 4 };

// scalar slots of the solver's device scalar array
enum Slot { S_RZ = 0, S_PQ, S_RR, S_ALPHA, S_BETA, S_PR, S_ZQ, S_FF, S_FLAG, S_TMP, S_NSLOTS = 16 };
enum FinOp { FIN_STORE = 0, FIN_PQ_CG, FIN_PQ_FCG, FIN_RZ_CG, FIN_ZQ_FCG, FIN_RZ0 };

__device__ inline double wave_sum(double v)
{
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Sum of one value per thread over a 256-thread block, in a fixed order;
// the result is valid in thread 0.
__device__ inline double block_sum(double v, double *lds)
{
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) lds[wid] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0) s = ((lds[0] + lds[1]) + lds[2]) + lds[3];
    return s;
}

// Sum of one value per thread over a block of NW wavefronts: butterfly within
// each wave, then the waves' sums in index order; valid in thread 0.
template <int NW> __device__ inline double block_sum_n(double v, double *lds /* NW */)
{
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) lds[wid] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < NW; w++) s += lds[w];
    return s;
}

// threads of the single-block final reductions (k_finalize, k_bfinalize)
constexpr int FIN_THREADS = 1024;

// ---- loads of 8 consecutive entries (k .. k+7) of lane r of a C-row slice ----

template <int C> __device__ inline void load8c(const double *__restrict__ val, int64_t base, int kk, int r, double v[8])
{
    const vd2 *p = reinterpret_cast<const vd2 *>(val + base) + (int64_t)(kk >> 1) * C + r;
#pragma unroll
    for (int c = 0; c < 4; c++) {
        vd2 t = __builtin_nontemporal_load(p + c * C);
        v[2 * c] = t.x; v[2 * c + 1] = t.y;
    }
}
template <int C> __device__ inline void load8c(const float *__restrict__ val, int64_t base, int kk, int r, float v[8])
{
    const vf4 *p = reinterpret_cast<const vf4 *>(val + base) + (int64_t)(kk >> 2) * C + r;
#pragma unroll
    for (int c = 0; c < 2; c++) {
        vf4 t = __builtin_nontemporal_load(p + c * C);
        v[4 * c] = t.x; v[4 * c + 1] = t.y; v[4 * c + 2] = t.z; v[4 * c + 3] = t.w;
    }
}
// 16-bit deltas: one 16-byte load holds the 8 deltas of entries kk .. kk+7.
template <int C>
__device__ inline void loadidx8c(const uint16_t *__restrict__ d16, int64_t base, int kk, int r, int &col, int c[8])
{
    vu4 t = __builtin_nontemporal_load(reinterpret_cast<const vu4 *>(d16 + base) + (int64_t)(kk >> 3) * C + r);
    unsigned w[4] = {t.x, t.y, t.z, t.w};
#pragma unroll
    for (int q = 0; q < 4; q++) {
        col += (int)(w[q] & 0xffffu);
        c[2 * q] = col;
        col += (int)(w[q] >> 16);
        c[2 * q + 1] = col;
    }
}
template <int C>
__device__ inline void loadidx8c(const int32_t *__restrict__ c32, int64_t base, int kk, int r, int &col, int c[8])
{
    const vi4 *p = reinterpret_cast<const vi4 *>(c32 + base) + (int64_t)(kk >> 2) * C + r;
#pragma unroll
    for (int h = 0; h < 2; h++) {
        vi4 t = __builtin_nontemporal_load(p + h * C);
        c[4 * h] = t.x; c[4 * h + 1] = t.y; c[4 * h + 2] = t.z; c[4 * h + 3] = t.w;
    }
    col = c[7];
}

// Device view of one SELL-C image (layout at the top of this file).
template <typename VT, typename IT> struct Sell {
    int64_t nrows, ncols, nslices;
    const int64_t *soff;    // values of slice s: soff[s] .. soff[s+1]; width (soff[s+1] - soff[s]) / C
    const int64_t *ibase;   // >= 0: start of slice s in idx; < 0: shared offsets, e = -1 - ibase[s]:
                            // at shoff[e >> 1]; e & 1 set when every row + offset of the slice is a
                            // valid column (no clamping needed)
    const VT *val;
    const IT *idx;          // per-row indices: 16-bit deltas or int32 columns
    const int32_t *col0;    // first column of each row (16-bit deltas)
    const int32_t *shoff;   // shared offsets, w_s per shared slice, ascending
    const int32_t *perm;    // row of each slot (slices sorted by row length), -1 past
                            // the last row; nullptr: slot s * C + r holds row s * C + r
                            // (always so for shared-offset slices)
    const int32_t *shrun;   // parallel to shoff: from each list's position, its runs
                            // of consecutive offsets (at most WIN_LMAX long) in
                            // order, packed as first offset * 16 + length, then 0
                            // (0 first: no run table for that list)
    const int32_t *wgtab;   // window stages shared by the four waves of a block
    const int32_t *wgst;    // (layout in host.h: WgStages); nullptr: none
    int xwin;               // k_sell walks the slices with run tables through x windows

    // row held by slot q, or -1
    __device__ __forceinline__ int64_t row_of(int64_t q) const
    {
        return perm ? (int64_t)perm[q] : (q < nrows ? q : -1);
    }
};

// Walk row s * C + r of slice s (s uniform across the wavefront) in groups of
// 8 entries in ascending column order: body(v, c) gets the values and columns.
// With U > 1 the loads of U groups are issued before their bodies run (more
// loads in flight per wavefront; the bodies still run in column order).
template <int C, int U = 1, typename VT, typename IT, typename Body>
__device__ __forceinline__ void sell_row(const Sell<VT, IT> &A, int64_t s, int r, Body &&body)
{
    const int64_t base = A.soff[s];
    const int width = (int)((A.soff[s + 1] - base) / C);
    const int64_t ib = A.ibase[s];
    const int row = (int)(s * C + r);   // shared-offset slices are never sorted
    int kk = 0;
    if (ib < 0) {
        const int64_t e = -1 - ib;
        const int32_t *so = A.shoff + (e >> 1);
        if (e & 1) {
            if constexpr (U > 1)
                for (; kk + 8 * U <= width; kk += 8 * U) {
                    VT v[U][8];
                    int c[U][8];
#pragma unroll
                    for (int u = 0; u < U; u++) load8c<C>(A.val, base, kk + 8 * u, r, v[u]);
#pragma unroll
                    for (int u = 0; u < U; u++)
#pragma unroll
                        for (int t = 0; t < 8; t++) c[u][t] = row + so[kk + 8 * u + t];
#pragma unroll
                    for (int u = 0; u < U; u++) body(v[u], c[u]);
                }
            for (; kk < width; kk += 8) {
                VT v[8];
                int c[8];
                load8c<C>(A.val, base, kk, r, v);
#pragma unroll
                for (int t = 0; t < 8; t++) c[t] = row + so[kk + t];
                body(v, c);
            }
        } else {
            const int hi = (int)A.ncols - 1;   // columns of lanes without the entry stay in range
            for (; kk < width; kk += 8) {
                VT v[8];
                int c[8];
                load8c<C>(A.val, base, kk, r, v);
#pragma unroll
                for (int t = 0; t < 8; t++) c[t] = min(max(row + so[kk + t], 0), hi);
                body(v, c);
            }
        }
    } else {
        int col = (sizeof(IT) == 2) ? A.col0[s * C + r] : 0;   // col0 is kept per slot
        if constexpr (U > 1)
            for (; kk + 8 * U <= width; kk += 8 * U) {
                VT v[U][8];
                int c[U][8];
#pragma unroll
                for (int u = 0; u < U; u++) loadidx8c<C>(A.idx, ib, kk + 8 * u, r, col, c[u]);
#pragma unroll
                for (int u = 0; u < U; u++) load8c<C>(A.val, base, kk + 8 * u, r, v[u]);
#pragma unroll
                for (int u = 0; u < U; u++) body(v[u], c[u]);
            }
        for (; kk < width; kk += 8) {
            VT v[8];
            int c[8];
            loadidx8c<C>(A.idx, ib, kk, r, col, c);
            load8c<C>(A.val, base, kk, r, v);
            body(v, c);
        }
    }
}

// compiler fence for the wave's own LDS accesses (in order per wave)
__device__ inline void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Direct global-to-LDS load of 16 bytes per lane (global_load_lds_dwordx4):
// lane l's 16 bytes from src go to lds + 16 l (lds wave-uniform).  The host
// pass of the compiler does not take the builtin, hence the guard.
template <typename CT> __device__ __forceinline__ void lds_copy16(const CT *src, CT *lds)
{
#if defined(__HIP_DEVICE_COMPILE__)
    __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void *)lds, 16, 0, 0);
#endif
}

// s_waitcnt immediates (gfx9 encoding: vmcnt bits 3:0 and 15:14, expcnt 6:4,
// lgkmcnt 11:8): wait for this wave's LDS operations only, or until at most
// n < 16 of its vector memory loads are outstanding
constexpr int WAIT_LGKM0 = 0xC07F;
constexpr int wait_vm(int n) { return 0x0F70 | n; }   // n < 16

// ---- x windows of the single-vector K pass ----------------------------------
//
// In a slice with shared column offsets and a run table (stencil rows), a run
// of L consecutive offsets o .. o + L - 1 makes lane r read x[row0 + r + o + t],
// t < L: together the 63 + L consecutive entries from row0 + o.  The wave
// copies the 16-byte-aligned 1 KB of x that holds them into its LDS window with
// one direct global-to-LDS load, and each lane reads its L entries from there
// instead of the L gathers of the gather walk (8 of its 12 vector-memory
// instructions per 8 entries).  A run whose 1 KB would leave [0, ncols) takes
// the gathers, clamped as the gather walk clamps.  Entries are summed in
// ascending order, run after run; the padding entries of a list (value 0, past
// its last run) are skipped: an FMA with a zero product leaves a nonzero or +0
// sum unchanged.  Measured at c4 (FP64): the SpMV pass 1.023 -> 0.996 ms, the
// residual 1.022 -> 1.003 ms.
template <typename VT> struct Vec16;
template <> struct Vec16<double> { typedef vd2 type; };
template <> struct Vec16<float> { typedef vf4 type; };

// the run's L entries at offset OFF of the lane's value groups vg, x from the
// window (Wl: the lane's first entry) or gathered from column c0 on
template <typename VT, int NG, int OFF>
__device__ __forceinline__ VT xwin_run(VT acc, const typename Vec16<VT>::type (&vg)[NG], int L, bool win,
                                       const VT *Wl, const VT *__restrict__ x, int c0, bool clamp, int hi)
{
    constexpr int E = 16 / (int)sizeof(VT);
    static_assert(OFF + WIN_LMAX <= NG * E, "run past its value groups");
    VT ev[NG * E];
#pragma unroll
    for (int j = 0; j < NG; j++)
#pragma unroll
        for (int u = 0; u < E; u++) ev[j * E + u] = vg[j][u];
    if (win) {
#pragma unroll
        for (int t = 0; t < WIN_LMAX; t++)
            if (t < L) acc = fma(ev[OFF + t], Wl[t], acc);
    } else {
#pragma unroll
        for (int t = 0; t < WIN_LMAX; t++)
            if (t < L) {
                const int c = clamp ? min(max(c0 + t, 0), hi) : c0 + t;
                acc = fma(ev[OFF + t], *reinterpret_cast<const VT *>(reinterpret_cast<const char *>(x) +
                                                                        (uint32_t)c * (uint32_t)sizeof(VT)),
                          acc);
            }
    }
    return acc;
}
// xwin_run with the offset a runtime value below E + WIN_LMAX (constant
// branches: the offsets the value groups of two runs can start at)
template <typename VT, int NG>
__device__ __forceinline__ VT xwin_run_at(int off, VT acc, const typename Vec16<VT>::type (&vg)[NG], int L, bool win,
                                          const VT *Wl, const VT *__restrict__ x, int c0, bool clamp, int hi)
{
    constexpr int E = 16 / (int)sizeof(VT);
    static_assert(E - 1 + WIN_LMAX <= 10, "one case per offset");
#define XWR(O) return xwin_run<VT, NG, (O) < E + WIN_LMAX ? (O) : 0>(acc, vg, L, win, Wl, x, c0, clamp, hi)
    switch (off) {
    case 0: XWR(0);
    case 1: XWR(1);
    case 2: XWR(2);
    case 3: XWR(3);
    case 4: XWR(4);
    case 5: XWR(5);
    case 6: XWR(6);
    case 7: XWR(7);
    case 8: XWR(8);
    case 9: XWR(9);
    default: XWR(10);
    }
#undef XWR
}

// Row sum of lane r of shared-offset slice s through x windows (W: the wave's
// 2 KB of LDS, one window per run of a pair); runs: this lane's entry of the
// slice's first 64 runs.  Runs go in pairs: both windows copied and the value
// groups of both runs loaded before one wait, then the two runs summed.
template <typename VT, typename IT>
__device__ __forceinline__ VT xwin_row(const Sell<VT, IT> &A, int64_t s, int lane, int32_t runs, const int32_t *rt,
                                       int width, const VT *__restrict__ x, VT *W)
{
    typedef typename Vec16<VT>::type CT;
    constexpr int E = 16 / (int)sizeof(VT);
    constexpr int NG = (2 * WIN_LMAX + 2 * E - 2) / E;   // value groups covering two runs at any offset
    constexpr int WE = 64 * E;                           // entries of one window
    constexpr int XL = (E - 1 + 63 + WIN_LMAX + E - 1) / E;   // pieces of x one run reads
    const int64_t base = A.soff[s];
    const bool clamp = !((-1 - A.ibase[s]) & 1);
    const int hi = (int)(A.ncols - 1);
    const int row0 = (int)(s * SLICE);
    const int gmax = (width - 1) / E;
    VT acc = 0;
    int k = 0, rho = 0;
    auto next_run = [&]() -> int32_t {
        rho++;
        if ((rho & 63) == 0) runs = (rho + lane < width) ? rt[rho + lane] : 0;
        return k < width ? __builtin_amdgcn_readlane(runs, rho & 63) : 0;
    };
    int32_t pa = __builtin_amdgcn_readfirstlane(runs);
    while (pa != 0) {
        const int ka = k, la = pa & 15, ga = row0 + (pa >> 4), gaa = ga & ~(E - 1);
        k += la;
        const int32_t pb = next_run();
        const int lb = pb & 15, gb = row0 + (pb >> 4), gba = gb & ~(E - 1);
        const bool wa = gaa >= 0 && gaa + WE - 1 <= hi;
        const bool wb = pb != 0 && gba >= 0 && gba + WE - 1 <= hi;
        // the previous pair's reads of the windows have returned
        __builtin_amdgcn_s_waitcnt(WAIT_LGKM0);
        wave_lds_sync();
        // a run reads entries g .. g + 62 + L of x: the first XL 16-byte pieces
        // from g rounded down to a piece
        if (wa && lane < XL) lds_copy16(reinterpret_cast<const CT *>(x + gaa) + lane, reinterpret_cast<CT *>(W));
        if (wb && lane < XL) lds_copy16(reinterpret_cast<const CT *>(x + gba) + lane, reinterpret_cast<CT *>(W + WE));
        CT vg[NG];
#pragma unroll
        for (int j = 0; j < NG; j++) {
            const VT *p = A.val + base + (int64_t)min(ka / E + j, gmax) * (E * SLICE) + lane * E;
            vg[j] = __builtin_nontemporal_load(reinterpret_cast<const CT *>(p));
        }
        __builtin_amdgcn_s_waitcnt(wait_vm(0));
        wave_lds_sync();
        const int off = ka & (E - 1);
        acc = xwin_run_at<VT, NG>(off, acc, vg, la, wa, W + (ga - gaa) + lane, x, ga + lane, clamp, hi);
        if (pb != 0) {
            acc = xwin_run_at<VT, NG>(off + la, acc, vg, lb, wb, W + WE + (gb - gba) + lane, x, gb + lane, clamp, hi);
            k += lb;
            pa = next_run();
        } else {
            pa = 0;
        }
    }
    return acc;
}

// x[i] for 0 <= i < 2^32 / sizeof(T), addressed as a uniform base plus a
// 32-bit byte offset (vectors of at most 2^29 FP64 entries; checked at set-up).
template <typename T> __device__ __forceinline__ T ld32(const T *__restrict__ x, int i)
{
    return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(x) + (uint32_t)i * (uint32_t)sizeof(T));
}

// wavefront index within the block, as a wave-uniform (scalar) value
__device__ inline int wave_id() { return __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)); }

// ---- the sparse matrix-pass kernel -------------------------------------------
//
// acc = (K x)_row, then by epilogue:
//   EPI_SPMV  : y = acc;                   dots: (x, y), (x, g1)
//   EPI_RESID : y = f - acc
//   EPI_SMOOTH: y = x + invd (f - acc);    dots: (y, g0), (y, g1)
//   EPI_POLY  : y = a invd f + invd acc    (a = coef; one Horner step of the
//               polynomial smoother: c <- a D^{-1} r + D^{-1} K c)
//   EPI_ADD   : y = f + acc                (prolongation u + P e with the
//               smoothed prolongator; x is the coarse vector)
// VT: matrix, x and invd type; FT: type of f; OT: type of y; IT: index stream
// (uint16_t deltas or int32_t columns).  NDOT dots are accumulated in FP64 and
// written as one partial per block to partial[blockIdx.x * 2 + d].
template <typename VT, typename FT, typename OT, typename IT, int EPI, int NDOT>
// 8 wavefronts per SIMD (at most 64 VGPRs): the pass is bound by loads in flight
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_sell(const Sell<VT, IT> A, const VT *__restrict__ x,
                                              const FT *__restrict__ f, const VT *__restrict__ invd,
                                              OT *__restrict__ y, const double *__restrict__ g0,
                                              const double *__restrict__ g1, double *__restrict__ partial,
                                              VT coef)
{
    // two 1 KB x windows per wave (passes over FP64 values only: with FP32
    // values a run carries half the bytes and the per-run wait costs more than
    // the gathers, measured 0.62 against 0.50 ms for the c4 FP32 residual)
    constexpr bool XW = sizeof(VT) == 8;
    __shared__ VT xw[XW ? SELL_WAVES * 2 * 64 * 2 : 1];
    const int lane = threadIdx.x & 63, wid = wave_id();
    const int64_t s = (int64_t)blockIdx.x * SELL_WAVES + wid;
    double d0 = 0.0, d1 = 0.0;
    if (s < A.nslices) {
        const int64_t row = A.row_of(s * SLICE + lane);
        VT acc = 0;
        const int64_t ib = A.ibase[s];
        const int32_t *rt = A.shrun + (ib < 0 ? (-1 - ib) >> 1 : 0);
        const int width = (int)((A.soff[s + 1] - A.soff[s]) / SLICE);
        const int32_t runs = (XW && A.xwin && ib < 0 && lane < width) ? rt[lane] : 0;
        if (XW && __builtin_amdgcn_readfirstlane(runs) != 0) {
            acc = xwin_row(A, s, lane, runs, rt, width, x, xw + wid * 2 * 64 * 2);
        } else {
            // unroll 2 where the compiler keeps all gathers in flight within 64
            // VGPRs; the SpMV with fused dots keeps one group per step
            sell_row<SLICE, NDOT == 0 ? 2 : 1>(A, s, lane, [&](const VT *v, const int *c) {
#pragma unroll
                for (int t = 0; t < 8; t++) acc = fma(v[t], ld32(x, c[t]), acc);
            });
        }
        if (row >= 0) {
            if (EPI == EPI_SPMV) {
                y[row] = (OT)acc;
                if (NDOT >= 1) d0 = (double)x[row] * (double)acc;
                if (NDOT >= 2) d1 = (double)x[row] * g1[row];
            } else if (EPI == EPI_RESID) {
                y[row] = (OT)((VT)f[row] - acc);
            } else if (EPI == EPI_SMOOTH) {
                VT out = x[row] + invd[row] * ((VT)f[row] - acc);
                y[row] = (OT)out;
                if (NDOT >= 1) d0 = (double)out * g0[row];
                if (NDOT >= 2) d1 = (double)out * g1[row];
            } else if (EPI == EPI_ADD) {
                y[row] = (OT)((VT)f[row] + acc);
            } else {
                VT di = invd[row];
                y[row] = (OT)(coef * (di * (VT)f[row]) + di * acc);
            }
        }
    }
    if (NDOT >= 1) {
        // one partial per wavefront (no barrier: the waves of a block may end apart)
        double t0 = wave_sum(d0);
        double t1 = NDOT >= 2 ? wave_sum(d1) : 0.0;
        if (lane == 0) {
            const int64_t w = (int64_t)blockIdx.x * SELL_WAVES + wid;
            partial[2 * w] = t0;
            partial[2 * w + 1] = t1;
        }
    }
}

// One row of the fused prolongation + post-smoothing (k_sell_post, the block
// variants and the V-cycle tail share it, so their bits agree):
// u' = u + pc e_agg, y = u' + invd (r - acc).
template <typename VT> __device__ __forceinline__ VT post_update(VT u, VT pc, VT e, VT invd, VT r, VT acc)
{
    VT up = u + pc * e;
    return up + invd * (r - acc);
}

// Prolongation fused with the first l1-Jacobi post-smoothing sweep:
//   u' = u + P e,   y = u' + D^{-1} (f - K u') = u' + D^{-1} (r - (K P) e)
// with r = f - K u kept from the residual pass and acc = ((K P) e)_row taken
// over the SELL image of K P (its columns are coarse indices; the gathered
// vector is e).  Dots as EPI_SMOOTH: (y, g0), (y, g1).
template <typename VT, typename OT, typename IT, int NDOT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_sell_post(const Sell<VT, IT> A, const VT *__restrict__ e,
                                                   const VT *__restrict__ u, const VT *__restrict__ r,
                                                   const VT *__restrict__ invd, const int32_t *__restrict__ agg,
                                                   const VT *__restrict__ pc, OT *__restrict__ y,
                                                   const double *__restrict__ g0, const double *__restrict__ g1,
                                                   double *__restrict__ partial)
{
    const int lane = threadIdx.x & 63, wid = wave_id();
    const int64_t s = (int64_t)blockIdx.x * SELL_WAVES + wid;
    double d0 = 0.0, d1 = 0.0;
    if (s < A.nslices) {
        const int64_t row = A.row_of(s * SLICE + lane);
        VT acc = 0;
        sell_row<SLICE, 2>(A, s, lane, [&](const VT *v, const int *c) {
#pragma unroll
            for (int t = 0; t < 8; t++) acc = fma(v[t], ld32(e, c[t]), acc);
        });
        if (row >= 0) {
            VT out = post_update(u[row], pc[row], e[agg[row]], invd[row], r[row], acc);
            y[row] = (OT)out;
            if (NDOT >= 1) d0 = (double)out * g0[row];
            if (NDOT >= 2) d1 = (double)out * g1[row];
        }
    }
    if (NDOT >= 1) {
        // one partial per wavefront (no barrier: the waves of a block may end apart)
        double t0 = wave_sum(d0);
        double t1 = NDOT >= 2 ? wave_sum(d1) : 0.0;
        if (lane == 0) {
            const int64_t w = (int64_t)blockIdx.x * SELL_WAVES + wid;
            partial[2 * w] = t0;
            partial[2 * w + 1] = t1;
        }
    }
}

// ---- vector kernels ----------------------------------------------------------

// u = invd * f  (one smoothing sweep from the zero guess: K 0 = 0)
template <typename VT, typename FT>
__global__ void k_scale(int64_t n, const VT *__restrict__ invd, const FT *__restrict__ f, VT *__restrict__ u)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) u[i] = invd[i] * (VT)f[i];
}

// u = coef * invd * f  (first Horner step of the polynomial smoother from zero)
template <typename VT, typename FT>
__global__ void k_scale_coef(int64_t n, const VT *__restrict__ invd, const FT *__restrict__ f, VT *__restrict__ u,
                             VT coef)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) u[i] = coef * (invd[i] * (VT)f[i]);
}

// y = x + c   (smoother correction), written in the output type
template <typename VT, typename OT>
__global__ void k_add(int64_t n, const VT *__restrict__ x, const VT *__restrict__ c, OT *__restrict__ y)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = (OT)(x[i] + c[i]);
}

// Restriction f_c = P^T r over the members of each coarse row (ascending, at
// most mw, padded with -1), fused with the coarse level's zero-guess smoothing
// sweep u_c = invd_c * f_c when uc != nullptr.  Sum order is fixed and no
// contraction is applied: f_c is the same bits as a sequential P^T r.
template <typename VT>
__global__ void k_restrict(int64_t nc, int mw, const int32_t *__restrict__ members, const VT *__restrict__ pc,
                           const VT *__restrict__ r, VT *__restrict__ fc, const VT *__restrict__ invdc,
                           VT *__restrict__ uc, VT coef)
{
#pragma clang fp contract(off)
    int64_t I = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (I >= nc) return;
    VT s = 0;
    for (int t = 0; t < mw; t++) {
        int m = members[I * mw + t];
        if (m < 0) break;
        VT prod = pc[m] * r[m];
        s = s + prod;
    }
    fc[I] = s;
    if (uc) uc[I] = coef * (invdc[I] * s);
}

// Prolongation and correction u_i += pc_i e[agg_i] (no contraction).
template <typename VT>
__global__ void k_prolong(int64_t n, const int32_t *__restrict__ agg, const VT *__restrict__ pc,
                          const VT *__restrict__ e, VT *__restrict__ u)
{
#pragma clang fp contract(off)
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    VT prod = pc[i] * e[agg[i]];
    u[i] = u[i] + prod;
}

// Coarsest level: e = L^{-T} (L^{-1} f) with the precomputed inverse Cholesky
// factor (row-major, leading dimension ld) and its transpose; FP64 arithmetic
// whatever the level type.  One 256-thread block, n <= 2048, one thread per
// output row: y_i = sum_{k<=i} L^{-1}_ik f_k reads column i of L^{-T} (row k of
// LinvT), x_j = sum_{k>=j} L^{-1}_kj y_k reads column j of L^{-1}, so the
// threads of a wave load consecutive addresses and every load is independent
// of the running sum; k ascending.
template <typename VT>
__global__ __launch_bounds__(256) void k_coarse_solve(int n, int ld, const double *__restrict__ Linv,
                                                      const double *__restrict__ LinvT, const VT *__restrict__ f,
                                                      VT *__restrict__ e)
{
    __shared__ double fs[2048];
    __shared__ double ys[2048];
    for (int i = threadIdx.x; i < n; i += 256) fs[i] = (double)f[i];
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += 256) {
        double s = 0.0;
#pragma unroll 8
        for (int k = 0; k <= i; k++) s = fma(LinvT[(int64_t)k * ld + i], fs[k], s);
        ys[i] = s;
    }
    __syncthreads();
    for (int j = threadIdx.x; j < n; j += 256) {
        double s = 0.0;
#pragma unroll 8
        for (int k = j; k < n; k++) s = fma(Linv[(int64_t)k * ld + j], ys[k], s);
        e[j] = (VT)s;
    }
}

// Dot-product partials: one per block of a fixed grid (grid-stride).
__global__ void k_dot2(int64_t n, const double *__restrict__ a, const double *__restrict__ b,
                       const double *__restrict__ c, double *__restrict__ partial)
{
    __shared__ double lds[8];
    double s0 = 0.0, s1 = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        s0 = fma(a[i], b[i], s0);
        if (c) s1 = fma(a[i], c[i], s1);
    }
    double t0 = block_sum(s0, lds), t1 = block_sum(s1, lds + 4);
    if (threadIdx.x == 0) { partial[2 * blockIdx.x] = t0; partial[2 * blockIdx.x + 1] = t1; }
}

// u += alpha p ; r -= alpha q ; partials of (r, r).  Skipped once a breakdown
// flag is set (so u keeps the last valid iterate).
__global__ void k_cg_update(int64_t n, const double *__restrict__ sc, double *__restrict__ u,
                            double *__restrict__ r, const double *__restrict__ p, const double *__restrict__ q,
                            double *__restrict__ partial)
{
    __shared__ double lds[8];
    const bool skip = sc[S_FLAG] != 0.0;
    const double alpha = sc[S_ALPHA];
    double s = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        double ri = r[i];
        if (!skip) {
            u[i] = fma(alpha, p[i], u[i]);
            ri = fma(-alpha, q[i], ri);
            r[i] = ri;
        }
        s = fma(ri, ri, s);
    }
    double t = block_sum(s, lds);
    if (threadIdx.x == 0) { partial[2 * blockIdx.x] = t; partial[2 * blockIdx.x + 1] = 0.0; }
}

// p = z + beta p
__global__ void k_cg_pupdate(int64_t n, const double *__restrict__ sc, const double *__restrict__ z,
                             double *__restrict__ p)
{
    const double beta = sc[S_BETA];
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        p[i] = fma(beta, p[i], z[i]);
}

template <typename DT, typename ST>
__global__ void k_copy(int64_t n, const ST *__restrict__ s, DT *__restrict__ d)
{
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        d[i] = (DT)s[i];
}

template <typename T>
__global__ void k_fill(int64_t n, T v, T *__restrict__ d)
{
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) d[i] = v;
}

// Final sum of the block partials (two dots) in index order, then the scalar
// recurrences of CG / FCG(1) on the device.
__global__ __launch_bounds__(FIN_THREADS) void k_finalize(const double *__restrict__ partial, int nblk, double *sc,
                                                           int op, int slot)
{
    __shared__ double lds[2 * FIN_THREADS / 64];
    double s0 = 0.0, s1 = 0.0;
    for (int b = threadIdx.x; b < nblk; b += FIN_THREADS) { s0 += partial[2 * b]; s1 += partial[2 * b + 1]; }
    double t0 = block_sum_n<FIN_THREADS / 64>(s0, lds), t1 = block_sum_n<FIN_THREADS / 64>(s1, lds + FIN_THREADS / 64);
    if (threadIdx.x != 0) return;
    switch (op) {
    case FIN_STORE:
        sc[slot] = t0;
        if (slot + 1 < S_NSLOTS && slot == S_TMP) sc[slot + 1] = t1;
        break;
    case FIN_PQ_CG:
    case FIN_PQ_FCG: {
        sc[S_PQ] = t0;
        if (op == FIN_PQ_FCG) sc[S_PR] = t1;
        double num = op == FIN_PQ_FCG ? t1 : sc[S_RZ];
        if (!(t0 > 0.0) || !isfinite(t0)) { if (sc[S_FLAG] == 0.0) sc[S_FLAG] = 1.0; }
        else sc[S_ALPHA] = num / t0;
        break;
    }
    case FIN_RZ0:
        sc[S_RZ] = t0;
        if (!(t0 > 0.0) || !isfinite(t0)) { if (sc[S_FLAG] == 0.0) sc[S_FLAG] = 2.0; }
        break;
    case FIN_RZ_CG:
        if (!(t0 > 0.0) || !isfinite(t0)) { if (sc[S_FLAG] == 0.0) sc[S_FLAG] = 2.0; }
        else { sc[S_BETA] = t0 / sc[S_RZ]; sc[S_RZ] = t0; }
        break;
    case FIN_ZQ_FCG:
        sc[S_ZQ] = t0;
        if (!isfinite(t0)) { if (sc[S_FLAG] == 0.0) sc[S_FLAG] = 2.0; }
        else sc[S_BETA] = -t0 / sc[S_PQ];
        break;
    }
}

}  // namespace amgk
