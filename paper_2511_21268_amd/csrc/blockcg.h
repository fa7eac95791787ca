// Kernels of the block flexible CG for up to NB = 16 right-hand sides (O'Leary's
// block CG with the coefficients of flexible CG): per iteration
//     Q = K P,  G = P^T Q,  alpha = G^{-1} P^T R,  X += P alpha,  R -= Q alpha,
//     Z = B R,  beta = -G^{-1} Q^T Z,  P = Z + P beta,
// over the columns still active (a converged column leaves the block).  Block
// vectors are the row-major N x 16 arrays of the batched solve.
#pragma once
#include "kernels_blk.h"

namespace amgk {

constexpr int GRAM_BLOCKS = 2048;  // fixed grid of the Gram-matrix partials (a multiple of 16)
static_assert(GRAM_BLOCKS % 16 == 0, "k_bcg_small sums the partials in groups of 16 blocks");

// Partials of A^T B and A^T C (16 x 16 each; C may be NULL): 16-row tiles of
// A, B, C staged in LDS; thread (i, j) = (t / 16, t % 16) accumulates
// A_ri B_rj over the block's rows in ascending order.  The tiles of a block
// are chunk = blockIdx.x, blockIdx.x + GRAM_BLOCKS, ...
__global__ __launch_bounds__(256) void k_gram2(int64_t n, const double *__restrict__ A, const double *__restrict__ B,
                                               const double *__restrict__ Cm, double *__restrict__ partial)
{
    __shared__ double as[16][NB], bs[16][NB], cs[16][NB];
    const int t = threadIdx.x, i = t >> 4, j = t & 15;
    double g1 = 0.0, g2 = 0.0;
    for (int64_t r0 = (int64_t)blockIdx.x * 16; r0 < n; r0 += (int64_t)gridDim.x * 16) {
        const int64_t row = r0 + i;
        const bool in = row < n;
        as[i][j] = in ? A[row * NB + j] : 0.0;
        bs[i][j] = in ? B[row * NB + j] : 0.0;
        if (Cm) cs[i][j] = in ? Cm[row * NB + j] : 0.0;
        __syncthreads();
#pragma unroll
        for (int rr = 0; rr < 16; rr++) {
            g1 = fma(as[rr][i], bs[rr][j], g1);
            if (Cm) g2 = fma(as[rr][i], cs[rr][j], g2);
        }
        __syncthreads();
    }
    partial[(int64_t)blockIdx.x * 512 + t] = g1;
    partial[(int64_t)blockIdx.x * 512 + 256 + t] = g2;
}

// Final Gram sums and the small solve on the active columns S (bactive):
//   mode 0: G = first Gram (stored in gsave), H = second (P^T R);
//           coef = G_SS^{-1} H_SS                       (alpha)
//   mode 1: G = gsave, W = first Gram (Q^T Z);
//           coef = -G_SS^{-1} W_SS                      (beta)
// The 2 x 256 entries are summed over the blocks by four thread groups, group q
// taking the blocks q, q + 4, ... (four interleaved chains per thread), then the
// four group sums in order.
// coef is 16 x 16 row-major (direction i, column j), zero outside S x S.  A
// non-positive pivot marks every active column broken (flag slot).
__global__ __launch_bounds__(1024) void k_bcg_small(int nblk, const double *__restrict__ partial, double *sc,
                                                    double *__restrict__ gsave, double *__restrict__ coef, int mode)
{
    __shared__ double G[256], H[256], L[256], Y[256];
    __shared__ double qa[4][256], qb[4][256];
    __shared__ int idx[NB];
    const int t = threadIdx.x & 255, q = threadIdx.x >> 8;
    // four independent chains per thread (blocks q, q+4, q+8, q+12 of each 16),
    // combined in a fixed order; nblk is a multiple of 16
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0, b0 = 0.0, b1 = 0.0, b2 = 0.0, b3 = 0.0;
    for (int k = q; k < nblk; k += 16) {
        const double *pk = partial + (int64_t)k * 512 + t;
        a0 += pk[0];        b0 += pk[256];
        a1 += pk[4 * 512];  b1 += pk[4 * 512 + 256];
        a2 += pk[8 * 512];  b2 += pk[8 * 512 + 256];
        a3 += pk[12 * 512]; b3 += pk[12 * 512 + 256];
    }
    double a = (a0 + a1) + (a2 + a3), b = (b0 + b1) + (b2 + b3);
    qa[q][t] = a;
    qb[q][t] = b;
    __syncthreads();
    if (threadIdx.x < 256) {
        a = ((qa[0][t] + qa[1][t]) + qa[2][t]) + qa[3][t];
        b = ((qb[0][t] + qb[1][t]) + qb[2][t]) + qb[3][t];
        if (mode == 0) {
            G[t] = a;
            gsave[t] = a;
            H[t] = b;
        } else {
            G[t] = gsave[t];
            H[t] = -a;
        }
        coef[t] = 0.0;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    int m = 0;
    for (int j = 0; j < NB; j++)
        if (bactive(sc, j)) idx[m++] = j;
    // Cholesky of G_SS
    for (int r = 0; r < m; r++)
        for (int c = 0; c <= r; c++) {
            double s = G[idx[r] * NB + idx[c]];
            for (int k = 0; k < c; k++) s -= L[r * NB + k] * L[c * NB + k];
            if (r == c) {
                if (!(s > 0.0) || !isfinite(s)) {
                    for (int z = 0; z < m; z++) sc[B_FLAG * NB + idx[z]] = 3.0;
                    return;
                }
                L[r * NB + r] = sqrt(s);
            } else {
                L[r * NB + c] = s / L[c * NB + c];
            }
        }
    // Y = G_SS^{-1} H_SS, column by column
    for (int c = 0; c < m; c++) {
        for (int r = 0; r < m; r++) {
            double s = H[idx[r] * NB + idx[c]];
            for (int k = 0; k < r; k++) s -= L[r * NB + k] * Y[k * NB + c];
            Y[r * NB + c] = s / L[r * NB + r];
        }
        for (int r = m - 1; r >= 0; r--) {
            double s = Y[r * NB + c];
            for (int k = r + 1; k < m; k++) s -= L[k * NB + r] * Y[k * NB + c];
            Y[r * NB + c] = s / L[r * NB + r];
        }
    }
    for (int r = 0; r < m; r++)
        for (int c = 0; c < m; c++) coef[idx[r] * NB + idx[c]] = Y[r * NB + c];
}

// X += P alpha ; R -= Q alpha over 16-row tiles: the tile's rows of P and Q are
// staged in LDS (one load per thread each), thread (row r, column j) of the
// tile forms sum_i P_ri alpha_ij in ascending i; per-column partials of (R, R)
// as k_bcg_update (the tiles of a block: blockIdx.x, + gridDim.x, ...).
__global__ __launch_bounds__(256) void k_bcg_xr(int64_t n, const double *__restrict__ alpha, double *__restrict__ X,
                                                double *__restrict__ R, const double *__restrict__ P,
                                                const double *__restrict__ Q, double *__restrict__ partial)
{
    __shared__ double al[256], ps[256], qs[256];
    __shared__ double lds[8 * NB];
    const int t = threadIdx.x, r = t >> 4, j = t & (NB - 1);
    al[t] = alpha[t];
    double s = 0.0;
    for (int64_t r0 = (int64_t)blockIdx.x * 16; r0 < n; r0 += (int64_t)gridDim.x * 16) {
        const int64_t row = r0 + r;
        const bool in = row < n;
        __syncthreads();
        ps[t] = in ? P[row * NB + j] : 0.0;
        qs[t] = in ? Q[row * NB + j] : 0.0;
        __syncthreads();
        if (in) {
            double dx = 0.0, dr = 0.0;
#pragma unroll
            for (int i = 0; i < NB; i++) {
                const double a = al[i * NB + j];
                dx = fma(ps[r * NB + i], a, dx);
                dr = fma(qs[r * NB + i], a, dr);
            }
            const int64_t e = row * NB + j;
            X[e] = X[e] + dx;
            const double ri = R[e] - dr;
            R[e] = ri;
            s = fma(ri, ri, s);
        }
    }
    blk_col_partials(s, 0.0, lds, partial);
}

// Pn = Z + P beta over 16-row tiles (P staged in LDS)
__global__ __launch_bounds__(256) void k_bcg_p(int64_t n, const double *__restrict__ beta, const double *__restrict__ Z,
                                               const double *__restrict__ P, double *__restrict__ Pn)
{
    __shared__ double be[256], ps[256];
    const int t = threadIdx.x, r = t >> 4, j = t & (NB - 1);
    be[t] = beta[t];
    for (int64_t r0 = (int64_t)blockIdx.x * 16; r0 < n; r0 += (int64_t)gridDim.x * 16) {
        const int64_t row = r0 + r;
        const bool in = row < n;
        __syncthreads();
        ps[t] = in ? P[row * NB + j] : 0.0;
        __syncthreads();
        if (in) {
            double acc = 0.0;
#pragma unroll
            for (int i = 0; i < NB; i++) acc = fma(ps[r * NB + i], be[i * NB + j], acc);
            Pn[row * NB + j] = Z[row * NB + j] + acc;
        }
    }
}

}  // namespace amgk
