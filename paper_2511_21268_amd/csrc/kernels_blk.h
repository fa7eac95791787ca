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
                VT up = U[o + j] + pi * E[a + j];
                VT out = up + di * (R[o + j] - acc[j]);
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
                VT up = U[o + j] + pi * E[a + j];
                VT out = up + di * (R[o + j] - acc[j]);
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

// Final per-column sums of the partials (index order) and the scalar
// recurrences, masks and iteration counters of the 16 independent solves.
__global__ __launch_bounds__(FIN_THREADS) void k_bfinalize(const double *__restrict__ partial, int nblk, double *sc,
                                                           int op, double tol)
{
    // per column the order of k_finalize: thread strides, butterfly, waves in order
    constexpr int NW = FIN_THREADS / 64;
    __shared__ double lds[2 * NW * NB];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    double s0[NB], s1[NB];
#pragma unroll
    for (int j = 0; j < NB; j++) { s0[j] = 0.0; s1[j] = 0.0; }
    for (int b = threadIdx.x; b < nblk; b += FIN_THREADS)
#pragma unroll
        for (int j = 0; j < NB; j++) { s0[j] += partial[(2 * b) * NB + j]; s1[j] += partial[(2 * b + 1) * NB + j]; }
#pragma unroll
    for (int j = 0; j < NB; j++) { s0[j] = wave_sum(s0[j]); s1[j] = wave_sum(s1[j]); }
    if (lane == 0)
#pragma unroll
        for (int j = 0; j < NB; j++) { lds[wid * NB + j] = s0[j]; lds[(NW + wid) * NB + j] = s1[j]; }
    __syncthreads();
    if (threadIdx.x != 0) return;
#pragma unroll
    for (int j = 0; j < NB; j++) {
        double a = 0.0, b = 0.0;
        for (int w = 0; w < NW; w++) { a += lds[w * NB + j]; b += lds[(NW + w) * NB + j]; }
        s0[j] = a;
        s1[j] = b;
    }
    for (int j = 0; j < NB; j++) {
        const double a = s0[j], b = s1[j];
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
