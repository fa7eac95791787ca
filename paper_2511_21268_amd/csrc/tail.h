// The tail of the V-cycle in one persistent workgroup.
//
// The coarsest levels of a hierarchy are small (for 3D p = 3, n = 128: 2181,
// 560 and 144 rows), so their per-level kernels -- residual, restriction with
// the coarse zero-guess sweep, the coarse Cholesky solve, the fused
// prolongation + post-smoothing pass -- are launch-bound.  k_vtail runs all of
// them, level after level, in a single block of TAIL_THREADS threads, with a
// block barrier between dependent phases: the waves walk the slices of each
// level's SELL-64 images (lane = row, as k_sell and k_sell_post), the threads
// the coarse rows of each restriction and the rows of the coarse solve.
// Every row's arithmetic is the per-level kernels' (entries in ascending order,
// the same fused or unfused operations), so the results are bitwise theirs.
// Scope: l1-Jacobi with one pre- and one post-smoothing sweep and the fused
// K P post-smoothing (the set-up checks this before using the tail).
// k_vtail_blk is the same for the 16-column blocks of the batched solve.
#pragma once
#include "kernels.h"
#include "kernels_blk.h"

namespace amgk {

constexpr int TAIL_THREADS = 1024;
constexpr int TAIL_WAVES = TAIL_THREADS / 64;
constexpr int TAIL_MAX_COARSE = 2048;   // rows of the coarsest level held in LDS (single vector)

// One tail level: its matrix K and K P (SELL-64 images; one of the two index
// types in use), smoother and transfer data, and work vectors (single vector,
// or row-major 16-column blocks).
template <typename VT> struct TailLevel {
    Sell<VT, uint16_t> A16;
    Sell<VT, int32_t> A32;
    Sell<VT, uint16_t> P16;
    Sell<VT, int32_t> P32;
    int a16, p16, mw, pad;
    int64_t n;
    const VT *invd, *pc;
    const int32_t *agg, *members;
    VT *f, *u, *u2, *r;
};

template <typename VT> __device__ __forceinline__ VT restrict_sum(int mw, const int32_t *members, const VT *pc,
                                                                  const VT *r, int64_t I)
{
#pragma clang fp contract(off)
    VT s = 0;
    for (int t = 0; t < mw; t++) {
        int m = members[I * mw + t];
        if (m < 0) break;
        VT prod = pc[m] * r[m];
        s = s + prod;
    }
    return s;
}

template <typename VT, typename IT>
__device__ inline void tail_resid(const Sell<VT, IT> &A, const VT *f, const VT *u, VT *r)
{
    const int lane = threadIdx.x & 63, wid = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    for (int64_t s = wid; s < A.nslices; s += TAIL_WAVES) {
        const int64_t row = A.row_of(s * SLICE + lane);
        VT acc = 0;
        sell_row<SLICE>(A, s, lane, [&](const VT *v, const int *c) {
#pragma unroll
            for (int t = 0; t < 8; t++) acc = fma(v[t], ld32(u, c[t]), acc);
        });
        if (row >= 0) r[row] = f[row] - acc;
    }
}

template <typename VT, typename IT>
__device__ inline void tail_post(const Sell<VT, IT> &A, const VT *e, const VT *u, const VT *r, const VT *invd,
                                 const int32_t *agg, const VT *pc, VT *y)
{
    const int lane = threadIdx.x & 63, wid = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    for (int64_t s = wid; s < A.nslices; s += TAIL_WAVES) {
        const int64_t row = A.row_of(s * SLICE + lane);
        VT acc = 0;
        sell_row<SLICE>(A, s, lane, [&](const VT *v, const int *c) {
#pragma unroll
            for (int t = 0; t < 8; t++) acc = fma(v[t], ld32(e, c[t]), acc);
        });
        if (row >= 0) y[row] = post_update(u[row], pc[row], e[agg[row]], invd[row], r[row], acc);
    }
}

// T[0 .. nt-1]: the tail levels, finest first, each with u = invd f already
// (written by the restriction into the first one); fL, eL: right-hand side and
// solution of the coarsest level.  Output: T[0].u2.
template <typename VT>
__global__ __launch_bounds__(TAIL_THREADS) void k_vtail(const TailLevel<VT> *__restrict__ T, int nt, int nL, int ld,
                                                        const double *__restrict__ Linv,
                                                        const double *__restrict__ LinvT, VT *fL, VT *eL)
{
    __shared__ double fs[TAIL_MAX_COARSE];
    __shared__ double ys[TAIL_MAX_COARSE];
    for (int t = 0; t < nt; t++) {
        const TailLevel<VT> &L = T[t];
        if (L.a16) tail_resid(L.A16, L.f, L.u, L.r);
        else tail_resid(L.A32, L.f, L.u, L.r);
        __syncthreads();
        // restriction, fused with the next level's zero-guess sweep unless it is the coarsest
        const bool last = t + 1 == nt;
        const int64_t nc = last ? nL : T[t + 1].n;
        VT *fc = last ? fL : T[t + 1].f;
        for (int64_t I = threadIdx.x; I < nc; I += TAIL_THREADS) {
            const VT sI = restrict_sum(L.mw, L.members, L.pc, L.r, I);
            fc[I] = sI;
            if (!last) T[t + 1].u[I] = (VT)1 * (T[t + 1].invd[I] * sI);
        }
        __syncthreads();
    }
    // coarsest level: e = L^{-T} (L^{-1} f), k_coarse_solve's order
    for (int i = threadIdx.x; i < nL; i += TAIL_THREADS) fs[i] = (double)fL[i];
    __syncthreads();
    for (int i = threadIdx.x; i < nL; i += TAIL_THREADS) {
        double s = 0.0;
#pragma unroll 8
        for (int k = 0; k <= i; k++) s = fma(LinvT[(int64_t)k * ld + i], fs[k], s);
        ys[i] = s;
    }
    __syncthreads();
    for (int j = threadIdx.x; j < nL; j += TAIL_THREADS) {
        double s = 0.0;
#pragma unroll 8
        for (int k = j; k < nL; k++) s = fma(Linv[(int64_t)k * ld + j], ys[k], s);
        eL[j] = (VT)s;
    }
    __syncthreads();
    for (int t = nt - 1; t >= 0; t--) {
        const TailLevel<VT> &L = T[t];
        const VT *e = t + 1 < nt ? T[t + 1].u2 : eL;
        if (L.p16) tail_post(L.P16, e, L.u, L.r, L.invd, L.agg, L.pc, L.u2);
        else tail_post(L.P32, e, L.u, L.r, L.invd, L.agg, L.pc, L.u2);
        __syncthreads();
    }
}

// ---- the same for 16-column blocks ------------------------------------------

template <typename VT, typename IT>
__device__ inline void tail_resid_blk(const Sell<VT, IT> &A, const VT *F, const VT *U, VT *R)
{
    const int lane = threadIdx.x & 63, wid = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    for (int64_t s = wid; s < A.nslices; s += TAIL_WAVES) {
        const int64_t row = A.row_of(s * SLICE + lane);
        VT acc[NB];
#pragma unroll
        for (int j = 0; j < NB; j++) acc[j] = 0;
        sell_row<SLICE>(A, s, lane, [&](const VT *v, const int *c) {
#pragma unroll
            for (int t = 0; t < 8; t++) {
                VT xv[NB];
                BlkVec<VT>::load(U + (int64_t)c[t] * NB, xv);
#pragma unroll
                for (int j = 0; j < NB; j++) acc[j] = fma(v[t], xv[j], acc[j]);
            }
        });
        if (row >= 0)
#pragma unroll
            for (int j = 0; j < NB; j++) R[row * NB + j] = F[row * NB + j] - acc[j];
    }
}

template <typename VT, typename IT>
__device__ inline void tail_post_blk(const Sell<VT, IT> &A, const VT *E, const VT *U, const VT *R, const VT *invd,
                                     const int32_t *agg, const VT *pc, VT *Y)
{
    const int lane = threadIdx.x & 63, wid = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    for (int64_t s = wid; s < A.nslices; s += TAIL_WAVES) {
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
            for (int j = 0; j < NB; j++) Y[o + j] = post_update(U[o + j], pi, E[a + j], di, R[o + j], acc[j]);
        }
    }
}

// As k_vtail for 16 columns; Yc: global scratch of the coarse solve (nL x 16).
template <typename VT>
__global__ __launch_bounds__(TAIL_THREADS) void k_vtail_blk(const TailLevel<VT> *__restrict__ T, int nt, int nL,
                                                            int ld, const double *__restrict__ Linv,
                                                            const double *__restrict__ LinvT, VT *FL, VT *EL,
                                                            double *Yc)
{
    for (int t = 0; t < nt; t++) {
        const TailLevel<VT> &L = T[t];
        if (L.a16) tail_resid_blk(L.A16, L.f, L.u, L.r);
        else tail_resid_blk(L.A32, L.f, L.u, L.r);
        __syncthreads();
        const bool last = t + 1 == nt;
        const int64_t nc = last ? nL : T[t + 1].n;
        VT *fc = last ? FL : T[t + 1].f;
        for (int64_t I = threadIdx.x; I < nc; I += TAIL_THREADS) {
#pragma clang fp contract(off)
            VT s[NB];
#pragma unroll
            for (int j = 0; j < NB; j++) s[j] = 0;
            for (int q = 0; q < L.mw; q++) {
                int m = L.members[I * L.mw + q];
                if (m < 0) break;
                const VT pm = L.pc[m];
#pragma unroll
                for (int j = 0; j < NB; j++) {
                    VT prod = pm * L.r[(int64_t)m * NB + j];
                    s[j] = s[j] + prod;
                }
            }
#pragma unroll
            for (int j = 0; j < NB; j++) fc[I * NB + j] = s[j];
            if (!last) {
                const VT di = T[t + 1].invd[I];
#pragma unroll
                for (int j = 0; j < NB; j++) T[t + 1].u[I * NB + j] = (VT)1 * (di * s[j]);
            }
        }
        __syncthreads();
    }
    // coarsest level, k_coarse_solve_blk's order: Y = L^{-1} F, then E = L^{-T} Y
    for (int q = threadIdx.x; q < nL * NB; q += TAIL_THREADS) {
        const int i = q / NB, j = q % NB;
        double s = 0.0;
#pragma unroll 8
        for (int k = 0; k <= i; k++) s = fma(LinvT[(int64_t)k * ld + i], (double)FL[(int64_t)k * NB + j], s);
        Yc[(int64_t)i * NB + j] = s;
    }
    __syncthreads();
    for (int q = threadIdx.x; q < nL * NB; q += TAIL_THREADS) {
        const int i = q / NB, j = q % NB;
        double s = 0.0;
#pragma unroll 8
        for (int k = i; k < nL; k++) s = fma(Linv[(int64_t)k * ld + i], Yc[(int64_t)k * NB + j], s);
        EL[(int64_t)i * NB + j] = (VT)s;
    }
    __syncthreads();
    for (int t = nt - 1; t >= 0; t--) {
        const TailLevel<VT> &L = T[t];
        const VT *e = t + 1 < nt ? T[t + 1].u2 : EL;
        if (L.p16) tail_post_blk(L.P16, e, L.u, L.r, L.invd, L.agg, L.pc, L.u2);
        else tail_post_blk(L.P32, e, L.u, L.r, L.invd, L.agg, L.pc, L.u2);
        __syncthreads();
    }
}

}  // namespace amgk
