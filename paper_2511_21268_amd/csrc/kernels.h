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
    const int lane = threadIdx.x & 63, wid = wave_id();
    const int64_t s = (int64_t)blockIdx.x * SELL_WAVES + wid;
    double d0 = 0.0, d1 = 0.0;
    if (s < A.nslices) {
        const int64_t row = A.row_of(s * SLICE + lane);
        VT acc = 0;
        // unroll 2 where the compiler keeps all gathers in flight within 64
        // VGPRs; the SpMV with fused dots keeps one group per step
        sell_row<SLICE, NDOT == 0 ? 2 : 1>(A, s, lane, [&](const VT *v, const int *c) {
#pragma unroll
            for (int t = 0; t < 8; t++) acc = fma(v[t], ld32(x, c[t]), acc);
        });
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
